// bs_hier.hip -- bottom-up generation of surfel approximations over a scene
// hierarchy (paper Sec. 3.4).
//
// The paper generates one approximation per complex subtree and, bottom-up,
// takes the surfels already chosen for a node's children as the node's
// initial candidate set instead of re-capturing its geometry.  Here a node's
// candidates are: for a leaf, its own rows of the caller's candidate array;
// for an inner node, the surfels its children chose (child after child, each
// child's picks in order).  Nodes of one level (one more than the deepest
// child) are independent, so a level is one batched ordering (the persistent
// work queue of bs_batch.hip, or the several-picks scan over all CUs when the
// level holds a single node); levels run one after another on the stream.
// Per level, three small kernels move data: the candidates' source rows
// (copied from the children's outputs, or the leaf's own rows), their
// positions (gathered from the caller's array), and after the ordering each
// pick's source row.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "bs_internal.h"
#include "bs_sample.h"

namespace bs {
namespace {

// A run of a level's candidate sources: `len` entries at level position
// `dst`, copied from the hierarchy's output sources at `src` (kind 0) or
// the rows src, src + 1, ... of the caller's array (kind 1, a leaf).
struct SrcRun {
    int64_t dst, src, len;
    int32_t kind, pad;
};

__global__ void build_sources_kernel(const SrcRun* __restrict__ runs, int nruns,
                                     const int32_t* __restrict__ out_src, int32_t* __restrict__ level_src) {
    for (int r = blockIdx.x; r < nruns; r += gridDim.x) {
        const SrcRun R = runs[r];
        for (int64_t i = threadIdx.x; i < R.len; i += blockDim.x)
            level_src[R.dst + i] = R.kind ? int32_t(R.src + i) : out_src[R.src + i];
    }
}

// Positions of a level's candidates; a source -1 (a child whose input was not
// finite) becomes a NaN position, so that the parent is flagged in turn.
__global__ void gather_positions_kernel(const float* __restrict__ pts, const int32_t* __restrict__ src,
                                        int64_t count, float* __restrict__ xyz) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int32_t s = src[i];
        const float nan = __builtin_nanf("");
        xyz[3 * i + 0] = s >= 0 ? pts[3 * int64_t(s) + 0] : nan;
        xyz[3 * i + 1] = s >= 0 ? pts[3 * int64_t(s) + 1] : nan;
        xyz[3 * i + 2] = s >= 0 ? pts[3 * int64_t(s) + 2] : nan;
    }
}

// After a level's ordering: the source row of every pick of its nodes.
struct NodeMap {
    int64_t out_off;   // the node's picks in the outputs
    int64_t cand_off;  // its candidates in the level arrays
    int64_t k;
};

__global__ void map_sources_kernel(const NodeMap* __restrict__ nodes, int nnodes, const int32_t* __restrict__ order,
                                   const int32_t* __restrict__ level_src, int32_t* __restrict__ out_src) {
    for (int j = blockIdx.x; j < nnodes; j += gridDim.x) {
        const NodeMap N = nodes[j];
        for (int64_t t = threadIdx.x; t < N.k; t += blockDim.x) {
            const int32_t o = order[N.out_off + t];
            out_src[N.out_off + t] = o >= 0 ? level_src[N.cand_off + o] : -1;
        }
    }
}

struct Level {
    std::vector<int> nodes;          // node numbers, in order
    std::vector<SrcRun> runs;
    std::vector<NodeMap> maps;
    int64_t count = 0;               // candidates of the level
    BatchPlan* plan = nullptr;       // several nodes: one batched ordering
    std::vector<int32_t*> io_order;  // per node of the level (filled at execute)
    std::vector<float*> io_radius;
    std::vector<uint32_t*> io_done;
};

template <class T>
T* carve(char* base, size_t& off, size_t count) {
    T* p = reinterpret_cast<T*>(base + off);
    off += align_up(std::max<size_t>(count, 1) * sizeof(T));
    return p;
}

}  // namespace

struct HierPlan {
    int m = 0;
    std::vector<int64_t> k, out_off, ncand;
    std::vector<uint64_t> seed;
    std::vector<Level> levels;
    int64_t total_k = 0, max_count = 0;
    size_t max_runs = 0, max_maps = 0, order_ws = 0;
    bs_tuning tuning{};
    bool has_tuning = false;
    std::mutex mu;
};

namespace {

// Workspace: the level arrays (sources, positions), the run and map tables,
// and the ordering workspace the largest level needs.
struct HierWs {
    int32_t* level_src;
    float* level_xyz;
    SrcRun* runs;
    NodeMap* maps;
    void* order_ws;
    size_t total;
};

HierWs hier_layout(const HierPlan& p, char* base) {
    HierWs w{};
    size_t off = 0;
    w.level_src = carve<int32_t>(base, off, size_t(p.max_count));
    w.level_xyz = carve<float>(base, off, size_t(p.max_count) * 3);
    w.runs = carve<SrcRun>(base, off, p.max_runs);
    w.maps = carve<NodeMap>(base, off, p.max_maps);
    w.order_ws = base ? base + off : nullptr;
    off += align_up(std::max<size_t>(p.order_ws, 1));
    w.total = off;
    return w;
}

void free_plan(HierPlan* p) {
    for (Level& L : p->levels)
        if (L.plan) batch_plan_free(L.plan);
    delete p;
}

}  // namespace
}  // namespace bs

using namespace bs;

extern "C" {

struct bs_hier_plan {
    bs::HierPlan* p;
};

int bs_hier_plan_create(int32_t m, const int32_t* h_parent, const int64_t* h_leaf_offsets, const int64_t* h_k,
                        const uint64_t* h_seed, const bs_tuning* tuning, bs_hier_plan** out) {
    if (!out) return set_error(BS_ERR_INVALID_ARG, "null plan pointer");
    *out = nullptr;
    if (m < 1 || !h_parent || !h_leaf_offsets || !h_k) return set_error(BS_ERR_INVALID_ARG, "null hierarchy arrays");
    if (h_leaf_offsets[0] != 0) return set_error(BS_ERR_INVALID_ARG, "leaf offsets must start at 0");
    if (tuning)
        for (int r : tuning->reserved)
            if (r) return set_error(BS_ERR_INVALID_ARG, "bad tuning struct");
    HierPlan* p = new HierPlan();
    p->m = m;
    p->k.assign(h_k, h_k + m);
    p->seed.assign(size_t(m), 0);
    if (h_seed) p->seed.assign(h_seed, h_seed + m);
    if (tuning) {
        p->tuning = *tuning;
        p->has_tuning = true;
    }
    std::vector<std::vector<int>> children(static_cast<size_t>(m));
    std::vector<int> depth(size_t(m), 0);
    p->ncand.assign(size_t(m), 0);
    for (int j = 0; j < m; ++j) {
        const int par = h_parent[j];
        const int64_t rows = h_leaf_offsets[j + 1] - h_leaf_offsets[j];
        if (rows < 0) {
            const int err = set_error(BS_ERR_INVALID_ARG, "leaf offsets decrease at node %d", j);
            free_plan(p);
            return err;
        }
        if (par != -1 && (par <= j || par >= m)) {
            const int err = set_error(BS_ERR_INVALID_ARG, "node %d: parent %d must be -1 or a later node", j, par);
            free_plan(p);
            return err;
        }
        if (par >= 0) children[size_t(par)].push_back(j);
    }
    if (h_leaf_offsets[m] >= (int64_t(1) << 31)) {
        const int err = set_error(BS_ERR_INVALID_ARG, "%lld candidate rows >= 2^31", (long long)h_leaf_offsets[m]);
        free_plan(p);
        return err;
    }
    p->out_off.assign(size_t(m) + 1, 0);
    for (int j = 0; j < m; ++j) p->out_off[size_t(j) + 1] = p->out_off[size_t(j)] + p->k[size_t(j)];
    p->total_k = p->out_off[size_t(m)];
    if (p->total_k >= (int64_t(1) << 31)) {
        const int err = set_error(BS_ERR_INVALID_ARG, "%lld picks in total >= 2^31", (long long)p->total_k);
        free_plan(p);
        return err;
    }
    for (int j = 0; j < m; ++j) {
        const int64_t rows = h_leaf_offsets[j + 1] - h_leaf_offsets[j];
        if (children[size_t(j)].empty()) {
            p->ncand[size_t(j)] = rows;
        } else {
            if (rows != 0) {
                const int err = set_error(BS_ERR_INVALID_ARG, "node %d has children and %lld own rows", j, (long long)rows);
                free_plan(p);
                return err;
            }
            int d = 0;
            for (int c : children[size_t(j)]) {
                p->ncand[size_t(j)] += p->k[size_t(c)];
                d = std::max(d, depth[size_t(c)] + 1);
            }
            depth[size_t(j)] = d;
        }
        if (p->k[size_t(j)] < 0 || p->k[size_t(j)] > p->ncand[size_t(j)]) {
            const int err = set_error(BS_ERR_INVALID_ARG, "node %d: k=%lld outside [0, %lld candidates]", j,
                             (long long)p->k[size_t(j)], (long long)p->ncand[size_t(j)]);
            free_plan(p);
            return err;
        }
        if (p->ncand[size_t(j)] >= (int64_t(1) << 31)) {
            const int err = set_error(BS_ERR_INVALID_ARG, "node %d: too many candidates", j);
            free_plan(p);
            return err;
        }
    }
    const int nlev = 1 + *std::max_element(depth.begin(), depth.end());
    p->levels.resize(size_t(nlev));
    for (int j = 0; j < m; ++j) p->levels[size_t(depth[size_t(j)])].nodes.push_back(j);
    const float target = (tuning && tuning->cell_points > 0.f) ? tuning->cell_points : 8.f;
    for (Level& L : p->levels) {
        std::vector<int64_t> offs(1, 0), ks;
        std::vector<uint64_t> seeds;
        for (int j : L.nodes) {
            const int64_t base = L.count;
            if (children[size_t(j)].empty()) {
                if (p->ncand[size_t(j)] > 0)
                    L.runs.push_back(SrcRun{base, h_leaf_offsets[j], p->ncand[size_t(j)], 1, 0});
            } else {
                int64_t at = base;
                for (int c : children[size_t(j)]) {
                    if (p->k[size_t(c)] > 0) L.runs.push_back(SrcRun{at, p->out_off[size_t(c)], p->k[size_t(c)], 0, 0});
                    at += p->k[size_t(c)];
                }
            }
            L.maps.push_back(NodeMap{p->out_off[size_t(j)], base, p->k[size_t(j)]});
            L.count += p->ncand[size_t(j)];
            offs.push_back(L.count);
            ks.push_back(p->k[size_t(j)]);
            seeds.push_back(p->seed[size_t(j)]);
        }
        p->max_count = std::max(p->max_count, L.count);
        p->max_runs = std::max(p->max_runs, L.runs.size());
        p->max_maps = std::max(p->max_maps, L.maps.size());
        size_t need = 0;
        if (L.nodes.size() == 1) {
            const int j = L.nodes[0];
            if (p->k[size_t(j)] > 0)
                need = bs_workspace_size(p->ncand[size_t(j)], p->k[size_t(j)], tuning);
            if (p->k[size_t(j)] > 0 && need == 0) {
                const int err = set_error(BS_ERR_UNSUPPORTED, "node %d: no single-object plan for %lld candidates", j,
                                 (long long)p->ncand[size_t(j)]);
                free_plan(p);
                return err;
            }
            const size_t sneed = bs_sample_workspace_size(p->ncand[size_t(j)]);
            need = std::max(need, sneed);
        } else {
            const int rc = batch_plan_create(offs.data(), ks.data(), seeds.data(), int32_t(L.nodes.size()), target,
                                             tuning ? tuning->batch_wide : 0, tuning ? tuning->groups : 0,
                                             &L.plan);
            if (rc != BS_OK) {
                free_plan(p);
                return rc;
            }
            // an inner node's candidates are its children's surfels, compact
            // groups whose Morton-prefix cells are uneven: cut them
            if (&L != &p->levels.front()) batch_set_split_cells(L.plan, true);
            need = batch_workspace_bytes(L.plan);
        }
        p->order_ws = std::max(p->order_ws, need);
    }
    *out = new bs_hier_plan{p};
    return BS_OK;
}

size_t bs_hier_workspace_size(const bs_hier_plan* plan) {
    return plan ? hier_layout(*plan->p, nullptr).total : 0;
}

int64_t bs_hier_total_k(const bs_hier_plan* plan) { return plan ? plan->p->total_k : 0; }

int bs_hier_out_offsets(const bs_hier_plan* plan, int64_t* h_out_offsets) {
    if (!plan || !h_out_offsets) return set_error(BS_ERR_INVALID_ARG, "null argument");
    for (int j = 0; j <= plan->p->m; ++j) h_out_offsets[j] = plan->p->out_off[size_t(j)];
    return BS_OK;
}

int bs_hier_plan_execute(bs_hier_plan* plan, const float* d_points, const bs_sampler* sampler,
                         int32_t* d_out_order, float* d_out_radius, int32_t* d_out_source, void* d_workspace,
                         size_t workspace_bytes, void* stream) {
    if (!plan) return set_error(BS_ERR_INVALID_ARG, "null plan");
    HierPlan& p = *plan->p;
    if (p.total_k == 0) return BS_OK;
    if (!d_points || !d_out_order || !d_out_source) return set_error(BS_ERR_INVALID_ARG, "null points or outputs");
    const size_t need = bs_hier_workspace_size(plan);
    if (!d_workspace || workspace_bytes < need)
        return set_error(BS_ERR_INVALID_ARG, "workspace %zu bytes < %zu needed", workspace_bytes, need);
    if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
        return set_error(BS_ERR_INVALID_ARG, "workspace not %zu-byte aligned", kAlign);
    bs_sampler sp{};
    if (sampler) {
        for (int r : sampler->reserved)
            if (r) return set_error(BS_ERR_INVALID_ARG, "sampler: reserved fields must be zero");
        sp = *sampler;
    }
    std::lock_guard<std::mutex> lk(p.mu);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const HierWs w = hier_layout(p, static_cast<char*>(d_workspace));
    for (Level& L : p.levels) {
        if (L.count == 0 && L.maps.empty()) continue;
        hipError_t e = hipSuccess;
        if (!L.runs.empty()) {
            e = hipMemcpyAsync(w.runs, L.runs.data(), L.runs.size() * sizeof(SrcRun), hipMemcpyHostToDevice, st);
            if (e != hipSuccess) return set_error(BS_ERR_HIP, "runs: %s", hipGetErrorString(e));
            hipLaunchKernelGGL(build_sources_kernel, dim3(unsigned(std::min<size_t>(L.runs.size(), 4096))), dim3(256),
                               0, st, w.runs, int(L.runs.size()), d_out_source, w.level_src);
            const int64_t gb = std::min<int64_t>((L.count + 255) / 256, 16384);
            hipLaunchKernelGGL(gather_positions_kernel, dim3(unsigned(std::max<int64_t>(gb, 1))), dim3(256), 0, st,
                               d_points, w.level_src, L.count, w.level_xyz);
            if ((e = hipGetLastError()) != hipSuccess) return set_error(BS_ERR_HIP, "%s", hipGetErrorString(e));
        }
        int rc = BS_OK;
        if (!L.plan) {  // one node: the single-object path over all CUs
            const int j = L.nodes[0];
            const int64_t n = p.ncand[size_t(j)], k = p.k[size_t(j)];
            int32_t* oo = d_out_order + p.out_off[size_t(j)];
            float* orr = d_out_radius ? d_out_radius + p.out_off[size_t(j)] : nullptr;
            if (k > 0) {
                if (sampler)
                    rc = bs_sample(w.level_xyz, n, k, p.seed[size_t(j)], -1, &sp, oo, orr, nullptr, w.order_ws,
                                   p.order_ws, stream);
                else
                    rc = order_impl(w.level_xyz, n, k, p.seed[size_t(j)], -1, oo, orr, nullptr, nullptr, w.order_ws,
                                    p.order_ws, p.has_tuning ? &p.tuning : nullptr, stream);
            }
        } else {
            L.io_order.resize(L.nodes.size());
            L.io_radius.resize(L.nodes.size());
            L.io_done.assign(L.nodes.size(), nullptr);
            for (size_t i = 0; i < L.nodes.size(); ++i) {
                const int j = L.nodes[i];
                L.io_order[i] = d_out_order + p.out_off[size_t(j)];
                L.io_radius[i] = d_out_radius ? d_out_radius + p.out_off[size_t(j)] : nullptr;
            }
            batch_set_job_io(L.plan, L.io_order, L.io_radius, L.io_done);
            if (sampler)
                rc = batch_plan_execute_sample(L.plan, sp.sample_size, sp.growth_rounds, sp.vicinity, w.level_xyz,
                                               nullptr, nullptr, nullptr, w.order_ws, p.order_ws, st);
            else
                rc = batch_plan_execute(L.plan, w.level_xyz, nullptr, nullptr, w.order_ws, p.order_ws, st);
        }
        if (rc != BS_OK) return rc;
        e = hipMemcpyAsync(w.maps, L.maps.data(), L.maps.size() * sizeof(NodeMap), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return set_error(BS_ERR_HIP, "maps: %s", hipGetErrorString(e));
        hipLaunchKernelGGL(map_sources_kernel, dim3(unsigned(std::min<size_t>(L.maps.size(), 4096))), dim3(256), 0, st,
                           w.maps, int(L.maps.size()), d_out_order, w.level_src, d_out_source);
        if ((e = hipGetLastError()) != hipSuccess) return set_error(BS_ERR_HIP, "%s", hipGetErrorString(e));
    }
    return BS_OK;
}

void bs_hier_plan_destroy(bs_hier_plan* plan) {
    if (!plan) return;
    free_plan(plan->p);
    delete plan;
}

}  // extern "C"
