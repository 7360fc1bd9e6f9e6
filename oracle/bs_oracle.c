/*
 * bs_oracle.c -- CPU oracle for the exact greedy permutation of surfel
 * candidates ("Progressive Blue Surfels", Brandt, Jaehn, Fischer and
 * Meyer auf der Heide, arXiv 1904.08225).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the package's smoke check and the
 * benchmark's CPU-baseline leg do.  It shares no code, header, table or
 * helper with the HIP path.
 *
 * What it computes (paper, Sec. 3.2 "Progressive Sampling" and Sec. 3.3):
 *   The goal sequence is a greedy permutation (farthest-first traversal,
 *   Related Work paragraph citing Eppstein et al. and Eldar et al.): start
 *   from a random surfel, then repeatedly append the remaining candidate
 *   whose distance to all previously chosen surfels is largest, and remove
 *   it from the candidate set; stop after the desired count or when the set
 *   is exhausted.  "Distance to all chosen surfels" is read as the distance
 *   to the NEAREST chosen surfel (max-min, the r-net reading of Sec. 4.1).
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - arithmetic is IEEE binary32, round to nearest even, no contraction:
 *       d2(a,b) = ((dx*dx + dy*dy) + dz*dz),  dx = a.x - b.x, ...
 *     compiled with -ffp-contract=off on SSE2 (no x87 excess precision);
 *   - the argmax runs on d2 (not on its square root), lowest index wins ties;
 *   - radius[t] = sqrtf(d2 of order[t] to its nearest earlier pick), the
 *     covering radius of the t-prefix; radius[0] = +inf;
 *   - a picked candidate is never picked again, even at distance 0;
 *   - the random start is the first output of SplitMix64 (Steele, Lea and
 *     Flood, OOPSLA 2014) seeded with `seed`, reduced modulo n;
 *   - non-finite coordinates: order[:] = -1, radius[:] = NaN.
 *
 * Functions:
 *   oracle_splitmix64_first  SplitMix64 first output, from its definition.
 *   oracle_start_index       start = first output mod n.
 *   oracle_greedy32          plain O(n k) FP32 greedy (the oracle proper).
 *   oracle_greedy64          the same algorithm in binary64.
 *   oracle_along_order64     binary64 nearest-earlier distance along a given
 *                            order (for the FP64 error bound).
 *   oracle_greedy32_grid     an exact, faster variant of oracle_greedy32 that
 *                            skips provably unaffected candidates using a
 *                            uniform grid with a conservative binary64 bound
 *                            and a max segment tree over cells.  It is pinned
 *                            bit-exact to oracle_greedy32 by the test suite
 *                            and exists only so that large inputs can be
 *                            checked in seconds.
 *   oracle_greedy32_grid_h   the same with the cell side given (for pins that
 *                            place points on cell boundaries).
 *   oracle_oct_encode        octahedral code of a normal (2 x snorm16).
 *   oracle_emit_surfels      the ordered 20-byte surfel records of a prefix.
 *   oracle_median_nn         r_m: median nearest-neighbour distance within
 *                            the first p_m ordered surfels (Sec. 4.1).
 *   oracle_prefix_length     p(r) = p_m (r_m / r)^2, rounded up, in [1, k].
 *   oracle_philox4x32_10     the counter-based generator the sampler draws
 *                            from (Salmon et al., SC'11), from its definition.
 *   oracle_sample32          the paper's randomized progressive sampler
 *                            (Sec. 3.2), rounds of ~200 random candidates.
 *   oracle_prefix_nn         each prefix surfel's distance to its nearest
 *                            other prefix surfel (the Sec. 3.3 quality
 *                            measure of a prefix).
 *   oracle_capture_view      camera of one of the eight capture views.
 *   oracle_capture32         the initial surfel set of Sec. 3.1: the first
 *                            surface hit of every pixel of eight orthographic
 *                            views from the bounding-box corners.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_BAD_ARG -1
#define ORACLE_NO_MEM -2
#define ORACLE_NONFINITE 1

/* ---------------------------------------------------------------- start */

uint64_t oracle_splitmix64_first(uint64_t seed)
{
    /* SplitMix64: state advances by the golden-ratio increment, the output
     * is the advanced state passed through the variant-13 mix. */
    uint64_t z = seed + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int64_t oracle_start_index(uint64_t seed, int64_t n)
{
    if (n <= 0) return -1;
    return (int64_t)(oracle_splitmix64_first(seed) % (uint64_t)n);
}

/* ------------------------------------------------------------ distances */

static float d2_f32(const float* a, const float* b)
{
    float dx = a[0] - b[0];
    float dy = a[1] - b[1];
    float dz = a[2] - b[2];
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float s = xx + yy;
    return s + zz;
}

static double d2_f64(const double* a, const double* b)
{
    double dx = a[0] - b[0];
    double dy = a[1] - b[1];
    double dz = a[2] - b[2];
    return (dx * dx + dy * dy) + dz * dz;
}

static int all_finite(const float* P, int64_t n)
{
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!isfinite(P[i])) return 0;
    return 1;
}

static void fill_nonfinite(int32_t* order, float* radius, int64_t k)
{
    for (int64_t t = 0; t < k; ++t) {
        order[t] = -1;
        if (radius) radius[t] = NAN;
    }
}

/* ------------------------------------------------------ plain FP32 greedy */

/*
 * Plain greedy permutation in binary32.  P is AoS [n][3].  Writes k entries
 * of order and (optionally) radius.  Optional per-update statistics, each
 * of length k-1 (entry u describes the update with the u-th pick, u=0..k-2):
 *   n_live[u]  live candidates after that pick,
 *   n_ball[u]  live candidates strictly closer to the pick than the pick's
 *              own covering radius (d2 < m(pick)),
 *   n_dec[u]   min-distances that strictly decreased.
 */
int oracle_greedy32(const float* P, int64_t n, int64_t k, int64_t start,
                    int32_t* order, float* radius,
                    int64_t* n_live, int64_t* n_ball, int64_t* n_dec)
{
    if (k == 0) return ORACLE_OK;
    if (!P || !order || n < 1 || k < 0 || k > n || start < 0 || start >= n)
        return ORACLE_BAD_ARG;
    if (!all_finite(P, n)) {
        fill_nonfinite(order, radius, k);
        return ORACLE_NONFINITE;
    }
    float* m = (float*)malloc(sizeof(float) * (size_t)n);
    unsigned char* sel = (unsigned char*)calloc((size_t)n, 1);
    if (!m || !sel) { free(m); free(sel); return ORACLE_NO_MEM; }

    int64_t c = start;
    float mc = INFINITY;            /* covering radius^2 of the pick */
    sel[c] = 1;
    order[0] = (int32_t)c;
    if (radius) radius[0] = INFINITY;
    for (int64_t i = 0; i < n; ++i) m[i] = INFINITY;

    for (int64_t t = 1; t <= k; ++t) {
        /* update every live candidate with the newest pick c */
        if (t < k) {
            int64_t live = 0, ball = 0, dec = 0;
            for (int64_t i = 0; i < n; ++i) {
                if (sel[i]) continue;
                float d = d2_f32(P + 3 * i, P + 3 * c);
                ++live;
                if (d < mc) ++ball;
                if (d < m[i]) { m[i] = d; ++dec; }
            }
            if (n_live) n_live[t - 1] = live;
            if (n_ball) n_ball[t - 1] = ball;
            if (n_dec) n_dec[t - 1] = dec;
        }
        if (t == k) break;
        /* select: largest min-distance, lowest index on ties */
        int64_t best = -1;
        for (int64_t i = 0; i < n; ++i) {
            if (sel[i]) continue;
            if (best < 0 || m[i] > m[best]) best = i;
        }
        c = best;
        mc = m[c];
        sel[c] = 1;
        order[t] = (int32_t)c;
        if (radius) radius[t] = sqrtf(mc);
    }
    free(m);
    free(sel);
    return ORACLE_OK;
}

/* ------------------------------------------------------------ FP64 greedy */

int oracle_greedy64(const double* P, int64_t n, int64_t k, int64_t start,
                    int32_t* order, double* radius)
{
    if (k == 0) return ORACLE_OK;
    if (!P || !order || n < 1 || k < 0 || k > n || start < 0 || start >= n)
        return ORACLE_BAD_ARG;
    double* m = (double*)malloc(sizeof(double) * (size_t)n);
    unsigned char* sel = (unsigned char*)calloc((size_t)n, 1);
    if (!m || !sel) { free(m); free(sel); return ORACLE_NO_MEM; }
    int64_t c = start;
    sel[c] = 1;
    order[0] = (int32_t)c;
    if (radius) radius[0] = INFINITY;
    for (int64_t i = 0; i < n; ++i) m[i] = INFINITY;
    for (int64_t t = 1; t < k; ++t) {
        for (int64_t i = 0; i < n; ++i) {
            if (sel[i]) continue;
            double d = d2_f64(P + 3 * i, P + 3 * c);
            if (d < m[i]) m[i] = d;
        }
        int64_t best = -1;
        for (int64_t i = 0; i < n; ++i) {
            if (sel[i]) continue;
            if (best < 0 || m[i] > m[best]) best = i;
        }
        c = best;
        sel[c] = 1;
        order[t] = (int32_t)c;
        if (radius) radius[t] = sqrt(m[c]);
    }
    free(m);
    free(sel);
    return ORACLE_OK;
}

/*
 * r64[t] = sqrt(min_{j<t} d2_64(P[order[t]], P[order[j]])), r64[0] = +inf,
 * evaluated in binary64 on coordinates widened exactly from binary32.
 */
int oracle_along_order64(const float* P, int64_t n, const int32_t* order,
                         int64_t k, double* r64)
{
    if (k == 0) return ORACLE_OK;
    if (!P || !order || !r64 || k < 0 || k > n) return ORACLE_BAD_ARG;
    double* Q = (double*)malloc(sizeof(double) * 3 * (size_t)k);
    if (!Q) return ORACLE_NO_MEM;
    for (int64_t t = 0; t < k; ++t) {
        int64_t o = order[t];
        if (o < 0 || o >= n) { free(Q); return ORACLE_BAD_ARG; }
        Q[3 * t + 0] = (double)P[3 * o + 0];
        Q[3 * t + 1] = (double)P[3 * o + 1];
        Q[3 * t + 2] = (double)P[3 * o + 2];
    }
    r64[0] = INFINITY;
    for (int64_t t = 1; t < k; ++t) {
        double best = INFINITY;
        for (int64_t j = 0; j < t; ++j) {
            double d = d2_f64(Q + 3 * t, Q + 3 * j);
            if (d < best) best = d;
        }
        r64[t] = sqrt(best);
    }
    free(Q);
    return ORACLE_OK;
}

/* ------------------------------------------ exact grid-accelerated greedy */

typedef struct {
    int64_t begin, end;      /* range in the cell-sorted index list */
    double lo[3], hi[3];     /* exact box of the member coordinates */
    int64_t gx, gy, gz;      /* integer cell coordinates */
} ocell;

static uint64_t cell_hash_key(int64_t gx, int64_t gy, int64_t gz)
{
    return ((uint64_t)(gx & 0x1FFFFF) << 42) | ((uint64_t)(gy & 0x1FFFFF) << 21) |
           (uint64_t)(gz & 0x1FFFFF);
}

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 33)) * 0xff51afd7ed558ccdull;
    z = (z ^ (z >> 33)) * 0xc4ceb9fe1a85ec53ull;
    return z ^ (z >> 33);
}

typedef struct { uint64_t key; int64_t cell; int64_t i; } osort_rec;

static int cmp_rec(const void* a, const void* b)
{
    const osort_rec* x = (const osort_rec*)a;
    const osort_rec* y = (const osort_rec*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->i < y->i ? -1 : (x->i > y->i);
}

/* selection key: larger d2 first, then lower index; 0 = no live member */
static uint64_t sel_key(float d2, int64_t i)
{
    uint32_t b;
    memcpy(&b, &d2, 4);
    return ((uint64_t)b << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)i);
}

/*
 * Same result as oracle_greedy32 (bit for bit), faster on large inputs.
 * A candidate's min-distance can only drop if its binary32 distance to the
 * pick is below its own min-distance, which is at most the pick's m(c).  A
 * cell is skipped when the binary64 distance from the pick to the cell's
 * exact member box, shrunk by a relative margin of 1e-5 (binary32 rounding
 * of d2 is within 5 * 2^-24 relative, plus underflow of order 1e-38), is at
 * least m(c).  `target` is the desired mean number of points per cell;
 * `cell_side` > 0 fixes the cell side instead (at most 1e6 cells per axis)
 * and always walks the cells within `span` (without it, a span box holding
 * more cells than are occupied makes every cell a box-test candidate).
 *
 * Which cells are looked at: those within `span` cells of the pick's cell
 * along every axis.  A cell further away lies, along one axis, more than
 * (span - 1e-9) * h from the pick (cell indices are floors of binary64
 * quotients below 1e6, off by far less than 1e-9 of a cell).  span is
 * chosen so that distance exceeds rr = sqrt((m(c) + 1e-37) / (1 - 1e-5)),
 * the same margin as the box test: such a point's binary32 d2 cannot fall
 * below m(c), so skipping its cell changes no min-distance and no count.
 */
int oracle_greedy32_grid_h(const float* P, int64_t n, int64_t k, int64_t start,
                           int32_t* order, float* radius, double target,
                           double cell_side, int64_t* n_ball)
{
    if (k == 0) return ORACLE_OK;
    if (!P || !order || n < 1 || k < 0 || k > n || start < 0 || start >= n)
        return ORACLE_BAD_ARG;
    if (!all_finite(P, n)) {
        fill_nonfinite(order, radius, k);
        return ORACLE_NONFINITE;
    }
    if (!(target >= 1.0)) target = 12.0;

    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double v = P[3 * i + a];
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) if (hi[a] - lo[a] > ext) ext = hi[a] - lo[a];
    if (!(ext > 0.0)) ext = 1.0;

    osort_rec* rec = (osort_rec*)malloc(sizeof(osort_rec) * (size_t)n);
    if (!rec) return ORACLE_NO_MEM;

    /* pick the cell side h: start from a volume-filling guess and refine by
     * the observed occupancy (surfaces occupy far fewer cells) */
    double h = cell_side > 0.0 ? cell_side : ext / cbrt((double)n / target);
    if (cell_side > 0.0 && ext / h > 1.0e6) { free(rec); return ORACLE_BAD_ARG; }
    int64_t ncell = 0;
    for (int iter = 0; iter < 3; ++iter) {
        if (ext / h > 1.0e6) h = ext / 1.0e6;
        for (int64_t i = 0; i < n; ++i) {
            int64_t g[3];
            for (int a = 0; a < 3; ++a) g[a] = (int64_t)floor(((double)P[3 * i + a] - lo[a]) / h);
            rec[i].key = cell_hash_key(g[0], g[1], g[2]);
            rec[i].i = i;
        }
        qsort(rec, (size_t)n, sizeof(osort_rec), cmp_rec);
        ncell = 0;
        for (int64_t i = 0; i < n; ++i)
            if (i == 0 || rec[i].key != rec[i - 1].key) ++ncell;
        double per = (double)n / (double)ncell;
        if (cell_side > 0.0 || iter == 2 || (per > 0.5 * target && per < 2.0 * target)) break;
        h *= sqrt(target / per);
    }

    ocell* cells = (ocell*)malloc(sizeof(ocell) * (size_t)ncell);
    int64_t* cell_of = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* members = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t hcap = 1;
    while (hcap < 2 * ncell) hcap <<= 1;
    int64_t* htab = (int64_t*)malloc(sizeof(int64_t) * (size_t)hcap);
    uint64_t* hkey = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)hcap);
    int64_t tsize = 1;
    while (tsize < ncell) tsize <<= 1;
    uint64_t* tree = (uint64_t*)calloc(2 * (size_t)tsize, sizeof(uint64_t));
    float* m = (float*)malloc(sizeof(float) * (size_t)n);
    unsigned char* sel = (unsigned char*)calloc((size_t)n, 1);
    int64_t* visit = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
    if (!cells || !cell_of || !members || !htab || !hkey || !tree || !m || !sel || !visit) {
        free(rec); free(cells); free(cell_of); free(members); free(htab); free(hkey);
        free(tree); free(m); free(sel); free(visit);
        return ORACLE_NO_MEM;
    }
    for (int64_t i = 0; i < hcap; ++i) htab[i] = -1;

    int64_t ci = -1;
    for (int64_t r = 0; r < n; ++r) {
        int64_t i = rec[r].i;
        if (r == 0 || rec[r].key != rec[r - 1].key) {
            ++ci;
            ocell* C = &cells[ci];
            C->begin = r;
            for (int a = 0; a < 3; ++a) { C->lo[a] = INFINITY; C->hi[a] = -INFINITY; }
            C->gx = (int64_t)floor(((double)P[3 * i + 0] - lo[0]) / h);
            C->gy = (int64_t)floor(((double)P[3 * i + 1] - lo[1]) / h);
            C->gz = (int64_t)floor(((double)P[3 * i + 2] - lo[2]) / h);
            uint64_t key = rec[r].key;
            uint64_t s = mix64(key) & (uint64_t)(hcap - 1);
            while (htab[s] >= 0) s = (s + 1) & (uint64_t)(hcap - 1);
            htab[s] = ci;
            hkey[s] = key;
        }
        ocell* C = &cells[ci];
        C->end = r + 1;
        members[r] = i;
        cell_of[i] = ci;
        for (int a = 0; a < 3; ++a) {
            double v = P[3 * i + a];
            if (v < C->lo[a]) C->lo[a] = v;
            if (v > C->hi[a]) C->hi[a] = v;
        }
    }
    free(rec);

    for (int64_t i = 0; i < n; ++i) m[i] = INFINITY;

    int64_t c = start;
    float mc = INFINITY;
    sel[c] = 1;
    order[0] = (int32_t)c;
    if (radius) radius[0] = INFINITY;

    for (int64_t t = 1; t < k; ++t) {
        const float* pc = P + 3 * c;
        double pcd[3] = {pc[0], pc[1], pc[2]};
        /* gather the cells that may contain an affected candidate */
        int64_t nvisit = 0;
        double rr = sqrt(((double)mc + 1e-37) / (1.0 - 1e-5));
        int64_t span = isinf(rr) ? INT64_MAX : (int64_t)floor(rr / h) + 2;
        double boxes = (double)(2 * (double)span + 1);
        boxes = boxes * boxes * boxes;
        if (isinf(rr) || (cell_side <= 0.0 && boxes >= (double)ncell)) {
            for (int64_t q = 0; q < ncell; ++q) visit[nvisit++] = q;
        } else {
            int64_t g0 = (int64_t)floor((pcd[0] - lo[0]) / h);
            int64_t g1 = (int64_t)floor((pcd[1] - lo[1]) / h);
            int64_t g2 = (int64_t)floor((pcd[2] - lo[2]) / h);
            for (int64_t a = g0 - span; a <= g0 + span; ++a)
                for (int64_t b = g1 - span; b <= g1 + span; ++b)
                    for (int64_t e = g2 - span; e <= g2 + span; ++e) {
                        if (a < 0 || b < 0 || e < 0) continue;
                        uint64_t key = cell_hash_key(a, b, e);
                        uint64_t s = mix64(key) & (uint64_t)(hcap - 1);
                        while (htab[s] >= 0) {
                            if (hkey[s] == key) { visit[nvisit++] = htab[s]; break; }
                            s = (s + 1) & (uint64_t)(hcap - 1);
                        }
                    }
        }
        int64_t ball = 0;
        int64_t own = cell_of[c];
        for (int64_t v = 0; v < nvisit; ++v) {
            int64_t q = visit[v];
            ocell* C = &cells[q];
            if (q != own && !isinf(rr)) {
                double bd = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double g = 0.0;
                    if (pcd[a] < C->lo[a]) g = C->lo[a] - pcd[a];
                    else if (pcd[a] > C->hi[a]) g = pcd[a] - C->hi[a];
                    bd += g * g;
                }
                if (bd * (1.0 - 1e-5) - 1e-37 >= (double)mc) continue;
            }
            uint64_t best = 0;
            for (int64_t r = C->begin; r < C->end; ++r) {
                int64_t i = members[r];
                if (sel[i]) continue;
                float d = d2_f32(P + 3 * i, pc);
                if (d < mc) ++ball;
                if (d < m[i]) m[i] = d;
                uint64_t kk = sel_key(m[i], i);
                if (kk > best) best = kk;
            }
            int64_t node = tsize + q;
            tree[node] = best;
            for (node >>= 1; node >= 1; node >>= 1) {
                uint64_t l = tree[2 * node], rgt = tree[2 * node + 1];
                tree[node] = l > rgt ? l : rgt;
            }
        }
        if (n_ball) n_ball[t - 1] = ball;
        uint64_t top = tree[1];
        c = (int64_t)(0xFFFFFFFFu - (uint32_t)(top & 0xFFFFFFFFu));
        mc = m[c];
        sel[c] = 1;
        order[t] = (int32_t)c;
        if (radius) radius[t] = sqrtf(mc);
    }

    free(cells); free(cell_of); free(members); free(htab); free(hkey);
    free(tree); free(m); free(sel); free(visit);
    return ORACLE_OK;
}

int oracle_greedy32_grid(const float* P, int64_t n, int64_t k, int64_t start,
                         int32_t* order, float* radius, double target,
                         int64_t* n_ball)
{
    return oracle_greedy32_grid_h(P, n, k, start, order, radius, target, 0.0, n_ball);
}

/* -------------------------------------------- ordered surfel buffer (a6) */
/*
 * The paper stores an approximation as one contiguous vertex buffer of
 * surfels (position, normal, material), ordered so that any prefix is a
 * level of detail (Sec. 3, and the per-surfel size that Table 1 implies:
 * 20 bytes).  It does not say how the normal and colour are packed.
 * Readings (listed in the design notes):
 *   record = x, y, z as binary32 (12 bytes), the normal as an octahedral
 *   code of two signed 16-bit normalised integers (4 bytes), and the colour
 *   as r, g, b, a bytes with a = 255 (4 bytes), little-endian;
 *   octahedral map (Meyer et al. 2010, "On floating-point normal vectors";
 *   survey by Cigolle et al. 2014): p = (n.x, n.y) / (|n.x| + |n.y| + |n.z|),
 *   folded for n.z < 0 to ((1 - |p.y|) sgn(p.x), (1 - |p.x|) sgn(p.y)) with
 *   sgn(0) = +1; each component to round-to-nearest-even(clamp(p, -1, 1) *
 *   32767) in binary32 without contraction;
 *   a normal whose |n.x| + |n.y| + |n.z| is zero or not finite, or no normal
 *   array, codes as (0, 0); no colour array gives 255, 255, 255, 255;
 *   an order entry outside [0, n) (a non-finite input's -1) gives a NaN
 *   position, normal code (0, 0) and colour 0, 0, 0, 0.
 */
static float sgn_nz(float v) { return v >= 0.0f ? 1.0f : -1.0f; }

static int16_t snorm16(float v)
{
    float c = v < -1.0f ? -1.0f : (v > 1.0f ? 1.0f : v);
    return (int16_t)lrintf(c * 32767.0f);
}

void oracle_oct_encode(const float* nrm, int16_t* out)
{
    float ax = fabsf(nrm[0]), ay = fabsf(nrm[1]), az = fabsf(nrm[2]);
    float s = ax + ay;
    float l1 = s + az;
    if (!(l1 > 0.0f) || !isfinite(l1)) {
        out[0] = 0;
        out[1] = 0;
        return;
    }
    float px = nrm[0] / l1;
    float py = nrm[1] / l1;
    if (nrm[2] < 0.0f) {
        float qx = (1.0f - fabsf(py)) * sgn_nz(px);
        float qy = (1.0f - fabsf(px)) * sgn_nz(py);
        px = qx;
        py = qy;
    }
    out[0] = snorm16(px);
    out[1] = snorm16(py);
}

int oracle_emit_surfels(const float* P, const float* N, const uint8_t* C, int64_t n, const int32_t* order,
                        int64_t k, uint8_t* out)
{
    if (k < 0 || (k > 0 && (!P || !order || !out))) return ORACLE_BAD_ARG;
    for (int64_t t = 0; t < k; ++t) {
        uint8_t* r = out + 20 * t;
        int64_t i = order[t];
        float pos[3];
        int16_t code[2] = {0, 0};
        uint8_t col[4] = {0, 0, 0, 0};
        if (i < 0 || i >= n) {
            pos[0] = pos[1] = pos[2] = NAN;
        } else {
            memcpy(pos, P + 3 * i, 12);
            if (N) oracle_oct_encode(N + 3 * i, code);
            if (C) {
                col[0] = C[3 * i];
                col[1] = C[3 * i + 1];
                col[2] = C[3 * i + 2];
                col[3] = 255;
            } else {
                col[0] = col[1] = col[2] = col[3] = 255;
            }
        }
        memcpy(r, pos, 12);
        memcpy(r + 12, code, 4);
        memcpy(r + 16, col, 4);
    }
    return ORACLE_OK;
}

/* ---------------------------------------------- prefix length estimate */
/*
 * Sec. 4.1: every prefix of a greedy permutation is an r-net; the prefix
 * length for a surfel radius r is estimated as p(r) = p_m (r_m / r)^2, with
 * r_m the median, over the first p_m ordered surfels, of each one's minimum
 * distance to the other surfels of that prefix.  Readings: distances in
 * binary32 with the fixed d2 above and a correctly rounded sqrtf; the median
 * of an even count is the binary32 mean 0.5f * (a + b) of the two middle
 * values; p(r) is rounded up (the minimal length) and clamped to [1, k].
 */
static int cmp_f32(const void* a, const void* b)
{
    float x = *(const float*)a, y = *(const float*)b;
    return (x > y) - (x < y);
}

int oracle_median_nn(const float* P, int64_t n, const int32_t* order, int64_t pm, float* out_rm)
{
    if (pm < 2 || !P || !order || !out_rm) return ORACLE_BAD_ARG;
    for (int64_t a = 0; a < pm; ++a)
        if (order[a] < 0 || order[a] >= n) return ORACLE_BAD_ARG;
    float* nn = (float*)malloc(sizeof(float) * (size_t)pm);
    if (!nn) return ORACLE_NO_MEM;
    for (int64_t a = 0; a < pm; ++a) {
        float m = INFINITY;
        for (int64_t b = 0; b < pm; ++b) {
            if (b == a) continue;
            float d = d2_f32(P + 3 * (int64_t)order[a], P + 3 * (int64_t)order[b]);
            if (d < m) m = d;
        }
        nn[a] = sqrtf(m);
    }
    qsort(nn, (size_t)pm, sizeof(float), cmp_f32);
    if (pm % 2) *out_rm = nn[pm / 2];
    else *out_rm = 0.5f * (nn[pm / 2 - 1] + nn[pm / 2]);
    free(nn);
    return ORACLE_OK;
}

int64_t oracle_prefix_length(double r, double r_m, int64_t pm, int64_t k)
{
    if (k < 1) return 0;
    if (!(r > 0.0)) return k;
    double p = ceil((double)pm * (r_m / r) * (r_m / r));
    if (!(p >= 1.0)) return 1;
    return p > (double)k ? k : (int64_t)p;
}

int oracle_oct_encode_n(const float* N, int64_t n, int16_t* out)
{
    if (n < 0 || (n > 0 && (!N || !out))) return ORACLE_BAD_ARG;
    for (int64_t i = 0; i < n; ++i) oracle_oct_encode(N + 3 * i, out + 2 * i);
    return ORACLE_OK;
}

/* ------------------------------------------- randomized sampler (Sec. 3.2) */
/*
 * Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): a 4 x 32-bit counter and a 2 x 32-bit key; each
 * of the 10 rounds multiplies counter words 0 and 2 by the round constants
 * 0xD2511F53 and 0xCD9E8D57 into 64-bit products and mixes the halves with
 * words 1 and 3 and the key; the key grows by the Weyl increments
 * 0x9E3779B9 and 0xBB67AE85 between rounds.
 */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/*
 * The paper's randomized approximation of the greedy permutation (Sec. 3.2):
 * remove a random start surfel and output it; then, round after round, draw
 * a random sample of the remaining input set, append the sample member whose
 * distance to all surfels chosen before is largest and remove it from the
 * input; optionally remove sample members in close vicinity of the chosen
 * surfels; stop after k surfels or when the input set is empty.  Heuristic:
 * after every K rounds one more surfel is taken from each sample.
 *
 * Readings (the paper does not fix them; listed in the design notes):
 *   - start = SplitMix64(seed) mod n (as the exact ordering);
 *   - the sample of round i (i = 0 for the first round after the start):
 *     slot j = 0 .. S-1 tries up to 16 draws a = 0, 1, ...: the first output
 *     word u of Philox4x32-10 with counter (i, j, a, 0) and key (seed low,
 *     seed high 32 bits) names candidate floor(u * n / 2^32); the slot takes
 *     the first draw that names a remaining candidate (else stays empty).
 *     The sample is the set of the slots' candidates (a candidate named twice
 *     counts once);
 *   - S = 0 means the whole remaining set (the exact greedy permutation);
 *   - a round whose slots all stayed empty takes the remaining candidate with
 *     the largest distance (the whole input as its sample);
 *   - "distance to all surfels chosen before" is the binary32 squared
 *     distance to the nearest chosen surfel (the fixed d2 above, so ties and
 *     radii follow the exact ordering's rules); largest wins, lowest index on
 *     ties; radius[t] = sqrtf of that squared distance;
 *   - round i takes q_i = 1 + floor(i / K) picks (K < 0: always one), one
 *     after another from the same sample, each the member farthest from all
 *     surfels chosen so far, including the round's earlier picks;
 *   - vicinity v > 0: after the round's picks, every remaining sample member
 *     whose squared distance to the nearest chosen surfel is below
 *     (v * v) * d1, d1 the squared distance of the round's first pick, is
 *     removed from the input (binary32); v = 0 removes nothing;
 *   - the output may end early (input set empty, only with v > 0): count
 *     picks are made, entries count .. k-1 get order -3 and radius NaN.
 * The distance of every remaining candidate to the chosen set is kept for
 * all candidates (a plain O(n) update per pick), which is the definition.
 */
int oracle_sample32(const float* P, int64_t n, int64_t k, uint64_t seed, int64_t start,
                    int32_t S, int32_t K, float vicinity,
                    int32_t* order, float* radius, int64_t* out_count)
{
    if (out_count) *out_count = 0;
    if (k == 0) return ORACLE_OK;
    if (!P || !order || n < 1 || k < 0 || k > n || start < 0 || start >= n || S < 0 ||
        !(vicinity >= 0.0f) || (S == 0 && vicinity > 0.0f) || n >= ((int64_t)1 << 31))
        return ORACLE_BAD_ARG;
    if (!all_finite(P, n)) {
        fill_nonfinite(order, radius, k);
        return ORACLE_NONFINITE;
    }
    float* m = (float*)malloc(sizeof(float) * (size_t)n);
    unsigned char* alive = (unsigned char*)malloc((size_t)n);
    int64_t* sample = (int64_t*)malloc(sizeof(int64_t) * (size_t)(S > 0 ? S : 1));
    if (!m || !alive || !sample) { free(m); free(alive); free(sample); return ORACLE_NO_MEM; }
    for (int64_t i = 0; i < n; ++i) { m[i] = INFINITY; alive[i] = 1; }
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};

    /* the start: output it, remove it, distances of the rest to it */
    int64_t t = 1, remaining = n - 1;
    int64_t c = start;
    order[0] = (int32_t)c;
    if (radius) radius[0] = INFINITY;
    alive[c] = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!alive[i]) continue;
        float d = d2_f32(P + 3 * i, P + 3 * c);
        if (d < m[i]) m[i] = d;
    }
    for (int64_t round = 0; t < k && remaining > 0; ++round) {
        int64_t ns = 0;
        int whole = S == 0;
        if (!whole) {
            for (int32_t j = 0; j < S; ++j) {
                for (uint32_t a = 0; a < 16; ++a) {
                    const uint32_t ctr[4] = {(uint32_t)round, (uint32_t)j, a, 0u};
                    uint32_t u[4];
                    oracle_philox4x32_10(ctr, key, u);
                    int64_t idx = (int64_t)(((uint64_t)u[0] * (uint64_t)n) >> 32);
                    if (!alive[idx]) continue;
                    int dup = 0;
                    for (int64_t q = 0; q < ns; ++q) if (sample[q] == idx) dup = 1;
                    if (!dup) sample[ns++] = idx;
                    break;
                }
            }
            if (ns == 0) whole = 1;  /* no draw hit: the whole input this round */
        }
        int64_t q = K < 0 ? 1 : 1 + round / (K > 0 ? K : 1);
        if (whole && S > 0) q = 1;
        float d_first = 0.0f;
        for (int64_t p = 0; p < q && t < k; ++p) {
            int64_t best = -1;
            if (whole) {
                for (int64_t i = 0; i < n; ++i)
                    if (alive[i] && (best < 0 || m[i] > m[best])) best = i;
            } else {
                for (int64_t s2 = 0; s2 < ns; ++s2) {
                    int64_t i = sample[s2];
                    if (!alive[i]) continue;
                    if (best < 0 || m[i] > m[best] || (m[i] == m[best] && i < best)) best = i;
                }
            }
            if (best < 0) break;
            if (p == 0) d_first = m[best];
            c = best;
            order[t] = (int32_t)c;
            if (radius) radius[t] = sqrtf(m[c]);
            alive[c] = 0;
            --remaining;
            ++t;
            for (int64_t i = 0; i < n; ++i) {
                if (!alive[i]) continue;
                float d = d2_f32(P + 3 * i, P + 3 * c);
                if (d < m[i]) m[i] = d;
            }
        }
        if (vicinity > 0.0f && !whole) {
            const float thr = (vicinity * vicinity) * d_first;
            for (int64_t s2 = 0; s2 < ns; ++s2) {
                int64_t i = sample[s2];
                if (alive[i] && m[i] < thr) { alive[i] = 0; --remaining; }
            }
        }
    }
    if (out_count) *out_count = t;
    for (int64_t u = t; u < k; ++u) {
        order[u] = -3;
        if (radius) radius[u] = NAN;
    }
    free(m); free(alive); free(sample);
    return ORACLE_OK;
}

/*
 * Sec. 3.3 measures how evenly a prefix of an ordering covers the surface by
 * each prefix surfel's distance to its nearest other surfel of the prefix.
 * out[a] = sqrtf(min over b != a of d2(P[order[a]], P[order[b]])), a < p,
 * binary32 with the fixed d2; +inf when p = 1.
 */
int oracle_prefix_nn(const float* P, int64_t n, const int32_t* order, int64_t p, float* out)
{
    if (p < 1 || !P || !order || !out) return ORACLE_BAD_ARG;
    for (int64_t a = 0; a < p; ++a)
        if (order[a] < 0 || order[a] >= n) return ORACLE_BAD_ARG;
    for (int64_t a = 0; a < p; ++a) {
        const float* pa = P + 3 * (int64_t)order[a];
        float best = INFINITY;
        for (int64_t b = 0; b < p; ++b) {
            if (b != a) {
                float d = d2_f32(pa, P + 3 * (int64_t)order[b]);
                if (d < best) best = d;
            }
        }
        out[a] = sqrtf(best);
    }
    return ORACLE_OK;
}

/* ----------------------------------------- visible-surface capture (Sec. 3.1) */
/*
 * The paper captures a node's visible surface by rendering it from the eight
 * corners of its bounding box with orthographic projection towards the box
 * centre, into buffers of position, normal and colour; every covered pixel
 * becomes a candidate surfel.  Here the node is a set of analytic primitives
 * (sphere: radius a; box: half extents a, b, c; cylinder along local z:
 * radius a, half height b; world = rot * local + center) and each pixel's
 * candidate is the first primitive surface its ray meets (the visibility a
 * rasterizer computes at the pixel centre).  Readings (design notes):
 *   - box centre c = 0.5 (lo + hi), s = half the box diagonal; view v
 *     (bits x, y, z of v choose hi over lo) looks along d = (c - corner) /
 *     |c - corner|; image axes u = d x (0,0,1) normalised (d x (0,1,0) if
 *     that is shorter than 1e-6) and w = u x d; the image is the square of
 *     side 2 s around c, R x R pixels; pixel (i, j) (i along u) shoots from
 *     c + a u + b w - 2 s d with a = ((2 i + 1) / R - 1) s, b likewise from j;
 *   - the hit is the smallest t > 0 over the primitives, lowest primitive
 *     index on equal t; position o + t d, normal rot * local normal (unit);
 *     colour the primitive's;
 *   - candidates in view order, then row j, then column i;
 *   - every value in binary32 with the operation order written below.
 * A view whose corner is the centre (an empty box) contributes nothing.
 */
static float dot3f(const float* a, const float* b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

/* view v: out[0..2] d, [3..5] u, [6..8] w, [9..11] c, [12] s; returns 0 if degenerate */
int oracle_capture_view(const float* lo, const float* hi, int v, float* out)
{
    float c[3], e[3], dv[3], d[3], u[3], w[3];
    for (int a = 0; a < 3; ++a) {
        c[a] = 0.5f * (lo[a] + hi[a]);
        e[a] = hi[a] - lo[a];
        float corner = ((v >> a) & 1) ? hi[a] : lo[a];
        dv[a] = c[a] - corner;
    }
    float s = 0.5f * sqrtf(dot3f(e, e));
    float L = sqrtf(dot3f(dv, dv));
    if (!(L > 0.0f)) return 0;
    for (int a = 0; a < 3; ++a) d[a] = dv[a] / L;
    u[0] = d[1];
    u[1] = -d[0];
    u[2] = 0.0f;
    float lu = sqrtf(dot3f(u, u));
    if (!(lu >= 1e-6f)) {
        u[0] = -d[2];
        u[1] = 0.0f;
        u[2] = d[0];
        lu = sqrtf(dot3f(u, u));
    }
    for (int a = 0; a < 3; ++a) u[a] = u[a] / lu;
    w[0] = u[1] * d[2] - u[2] * d[1];
    w[1] = u[2] * d[0] - u[0] * d[2];
    w[2] = u[0] * d[1] - u[1] * d[0];
    for (int a = 0; a < 3; ++a) {
        out[a] = d[a];
        out[3 + a] = u[a];
        out[6 + a] = w[a];
        out[9 + a] = c[a];
    }
    out[12] = s;
    return 1;
}

/* local = rot^T (p - center) for a point, rot^T p for a direction */
static void to_local(const float* rot, const float* p, float* q)
{
    q[0] = (rot[0] * p[0] + rot[3] * p[1]) + rot[6] * p[2];
    q[1] = (rot[1] * p[0] + rot[4] * p[1]) + rot[7] * p[2];
    q[2] = (rot[2] * p[0] + rot[5] * p[1]) + rot[8] * p[2];
}

/* first hit t > 0 of the local ray ol + t dl with primitive (kind, prm);
 * returns 0 on a miss, else t and the local unit normal */
static int hit_local(int kind, const float* prm, const float* ol, const float* dl, float* t_out, float* nl)
{
    if (kind == 0) { /* sphere: from the ray's closest approach to the centre */
        float r = prm[0];
        float a = dot3f(dl, dl);
        float t0 = -dot3f(ol, dl) / a;
        float p0[3] = {ol[0] + t0 * dl[0], ol[1] + t0 * dl[1], ol[2] + t0 * dl[2]};
        float h2 = r * r - dot3f(p0, p0);
        if (h2 < 0.0f) return 0;
        float t = t0 - sqrtf(h2 / a);
        if (!(t > 0.0f)) return 0;
        for (int k = 0; k < 3; ++k) nl[k] = (ol[k] + t * dl[k]) / r;
        *t_out = t;
        return 1;
    }
    if (kind == 1) { /* box: slabs */
        float tn = -INFINITY, tf = INFINITY;
        int axis = -1;
        for (int k = 0; k < 3; ++k) {
            float h = prm[k];
            if (dl[k] == 0.0f) {
                if (ol[k] < -h || ol[k] > h) return 0;
                continue;
            }
            float t1 = (-h - ol[k]) / dl[k];
            float t2 = (h - ol[k]) / dl[k];
            float lo = t1 < t2 ? t1 : t2;
            float hi = t1 < t2 ? t2 : t1;
            if (lo > tn) { tn = lo; axis = k; }
            if (hi < tf) tf = hi;
        }
        if (axis < 0 || !(tn <= tf) || !(tn > 0.0f)) return 0;
        nl[0] = nl[1] = nl[2] = 0.0f;
        nl[axis] = dl[axis] > 0.0f ? -1.0f : 1.0f;
        *t_out = tn;
        return 1;
    }
    if (kind == 2) { /* cylinder along z: lateral surface and two caps */
        float r = prm[0], h = prm[1];
        float best = INFINITY;
        int side = -1;
        float a = dl[0] * dl[0] + dl[1] * dl[1];
        if (a > 0.0f) { /* lateral: from the closest approach to the axis */
            float t0 = -(ol[0] * dl[0] + ol[1] * dl[1]) / a;
            float x0 = ol[0] + t0 * dl[0];
            float y0 = ol[1] + t0 * dl[1];
            float h2 = r * r - (x0 * x0 + y0 * y0);
            if (h2 >= 0.0f) {
                float t = t0 - sqrtf(h2 / a);
                float z = ol[2] + t * dl[2];
                if (t > 0.0f && z >= -h && z <= h) { best = t; side = 0; }
            }
        }
        if (dl[2] != 0.0f) {
            for (int cap = 0; cap < 2; ++cap) {
                float zc = cap ? h : -h;
                float t = (zc - ol[2]) / dl[2];
                float x = ol[0] + t * dl[0];
                float y = ol[1] + t * dl[1];
                if (t > 0.0f && (x * x + y * y) <= r * r && t < best) { best = t; side = 1 + cap; }
            }
        }
        if (side < 0) return 0;
        if (side == 0) {
            float x = ol[0] + best * dl[0];
            float y = ol[1] + best * dl[1];
            nl[0] = x / r;
            nl[1] = y / r;
            nl[2] = 0.0f;
        } else {
            nl[0] = 0.0f;
            nl[1] = 0.0f;
            nl[2] = side == 2 ? 1.0f : -1.0f;
        }
        *t_out = best;
        return 1;
    }
    return 0;
}

/*
 * Primitives: kind[P] (0 sphere, 1 box, 2 cylinder), center[P][3],
 * rot[P][9] (row-major, local -> world), prm[P][3], rgb[P][3].  Outputs of
 * capacity 8 R^2: pos, nrm (float [][3]), col (uint8 [][3]); *count.
 */
int oracle_capture32(const int32_t* kind, const float* center, const float* rot, const float* prm,
                     const uint8_t* rgb, int64_t P, const float* lo, const float* hi, int32_t R,
                     float* pos, float* nrm, uint8_t* col, int64_t* count)
{
    if (P < 0 || R < 1 || !lo || !hi || !pos || !nrm || !col || !count) return ORACLE_BAD_ARG;
    int64_t n = 0;
    for (int v = 0; v < 8; ++v) {
        float cam[13];
        if (!oracle_capture_view(lo, hi, v, cam)) continue;
        const float *d = cam, *u = cam + 3, *w = cam + 6, *c = cam + 9;
        float s = cam[12];
        float s2 = 2.0f * s;
        for (int32_t j = 0; j < R; ++j) {
            float fb = (float)(2 * j + 1) / (float)R - 1.0f;
            float b = fb * s;
            for (int32_t i = 0; i < R; ++i) {
                float fa = (float)(2 * i + 1) / (float)R - 1.0f;
                float a = fa * s;
                float o[3];
                for (int k = 0; k < 3; ++k) o[k] = ((c[k] + a * u[k]) + b * w[k]) - s2 * d[k];
                float tbest = INFINITY;
                int64_t pbest = -1;
                float nbest[3] = {0, 0, 0};
                for (int64_t q = 0; q < P; ++q) {
                    const float* R9 = rot + 9 * q;
                    float oc[3] = {o[0] - center[3 * q], o[1] - center[3 * q + 1], o[2] - center[3 * q + 2]};
                    float ol[3], dl[3], nl[3], t;
                    to_local(R9, oc, ol);
                    to_local(R9, d, dl);
                    if (!hit_local(kind[q], prm + 3 * q, ol, dl, &t, nl)) continue;
                    if (t < tbest) {
                        tbest = t;
                        pbest = q;
                        nbest[0] = (R9[0] * nl[0] + R9[1] * nl[1]) + R9[2] * nl[2];
                        nbest[1] = (R9[3] * nl[0] + R9[4] * nl[1]) + R9[5] * nl[2];
                        nbest[2] = (R9[6] * nl[0] + R9[7] * nl[1]) + R9[8] * nl[2];
                    }
                }
                if (pbest < 0) continue;
                for (int k = 0; k < 3; ++k) {
                    pos[3 * n + k] = o[k] + tbest * d[k];
                    nrm[3 * n + k] = nbest[k];
                    col[3 * n + k] = rgb[3 * pbest + k];
                }
                ++n;
            }
        }
    }
    *count = n;
    return ORACLE_OK;
}
