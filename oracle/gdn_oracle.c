/*
 * CPU oracle for the adaptive dual-weight gravitational denoiser
 * (arxiv 2512.10386, Section 3).
 *
 * TEST INFRASTRUCTURE ONLY: the plain, obviously-correct reference the HIP
 * path is compared against. It shares no code with the HIP library. Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may use it.
 *
 * The steps follow the paper's order:
 *   octree partition (Sec. 3, octree paragraph)
 *   -> leaf bounding-box volume (Eq. 10) -> adaptive voxel size (Eq. 11)
 *   -> voxel occupancy filter P1 (Eq. 12)
 *   -> kNN on P1, r_K and density (Eq. 13) -> percentile cut P2 (Eq. 14)
 *   -> per-leaf median density (Eq. 16) -> dual-weight score (Eq. 15-21)
 *   -> per-leaf top-lambda retention and union of leaves (Eq. 22).
 *
 * Readings taken where the paper is silent:
 *   - octree root = cube of side S = largest bbox extent at the bbox minimum;
 *     21-bit-per-axis Morton keys, x in the lowest bit; a node splits while it
 *     holds more than leaf_cap points and is above the depth limit;
 *   - voxel grid origin = minimum corner of the leaf's point bbox; h is
 *     rounded to fp32; h == 0 (flat leaf) makes the whole leaf one voxel;
 *     voxel indices are clamped to [0, 2^21-1];
 *   - kNN candidates of a leaf = P1 points of the 27 same-level octree cells
 *     around it (halo from adjacent cells); the point itself is excluded;
 *     ties are broken by original index;
 *   - fewer than k candidates -> "insufficient": r = +inf, density 0;
 *   - q is in percent with MATLAB prctile semantics, applied per leaf;
 *   - the median of Eq. 16 is taken per leaf over P1;
 *   - the score sums over the P1 kNN graph; the kernel is 1/(d^2+eps);
 *   - top-lambda keeps ceil(lambda*|P2|) points per leaf by (score desc,
 *     index asc); a NaN score ranks below every number.
 *
 * parity pins: every function here is pinned by a CPU test (see tests/),
 * against brute force, closed forms or the textbook definition it follows.
 */
#include "gdn_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MORTON_BITS 21
#define QMAX ((1u << MORTON_BITS) - 1u)
#define NO_NBR 0xFFFFFFFFu

void orc_default_params(orc_params *p)
{
    /* K, rho_percentile and min_vox_count are the paper's defaults
     * (Sec. 4.3.1); the rest are unvalued in the paper. */
    p->k = 12;
    p->leaf_cap = 512;
    p->min_leaf_side = 0.0;
    p->beta = 1.0;
    p->min_vox_count = 4;
    p->rho_percentile = 0.2;
    p->alpha = 1.0;
    p->sigma = 1.0;
    p->eps = 1e-12;
    p->keep_ratio = 0.98;
    p->gamma = 2.0;
    p->log_threshold = NAN;
    p->stages = 7;
}

static int params_ok(const orc_params *p)
{
    if (p->k < 1 || p->k > 64) return 0;
    if (p->leaf_cap < 1) return 0;
    if (!(p->beta > 0.0) || !isfinite(p->beta)) return 0;
    if (p->min_vox_count < 1) return 0;
    if (!(p->rho_percentile >= 0.0 && p->rho_percentile <= 100.0)) return 0;
    if (!(p->alpha >= 0.0) || !isfinite(p->alpha)) return 0;
    if (!(p->sigma > 0.0) || !isfinite(p->sigma)) return 0;
    if (!(p->eps >= 0.0) || !isfinite(p->eps)) return 0;
    if (!(p->keep_ratio > 0.0 && p->keep_ratio <= 1.0)) return 0;
    if (isnan(p->min_leaf_side)) return 0;
    if (!(p->gamma >= 0.0) || !isfinite(p->gamma)) return 0;
    if (isinf(p->log_threshold)) return 0;
    if (p->stages < 0 || p->stages > 7) return 0;
    return 1;
}

/* ---------------------------------------------------------------- Morton */

/* Bit b of each axis goes to key bit 3b (x), 3b+1 (y), 3b+2 (z). */
uint64_t orc_morton_interleave(uint32_t qx, uint32_t qy, uint32_t qz)
{
    uint64_t key = 0;
    for (int b = 0; b < MORTON_BITS; ++b) {
        key |= (uint64_t)((qx >> b) & 1u) << (3 * b);
        key |= (uint64_t)((qy >> b) & 1u) << (3 * b + 1);
        key |= (uint64_t)((qz >> b) & 1u) << (3 * b + 2);
    }
    return key;
}

/* Quantise one coordinate onto the 2^21 grid of the root cube. */
static uint32_t quantise(float x, float lo, double scale)
{
    double q = floor(((double)x - (double)lo) * scale);
    if (!(q >= 0.0)) q = 0.0;
    if (q > (double)QMAX) q = (double)QMAX;
    return (uint32_t)q;
}

/* ------------------------------------------------------------ small sorts */

typedef struct { uint64_t key; uint32_t idx; } key_idx;

static int cmp_key_idx(const void *a, const void *b)
{
    const key_idx *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static int cmp_f32_desc(const void *a, const void *b)
{
    float x = *(const float *)a, y = *(const float *)b;
    return x > y ? -1 : (x < y ? 1 : 0);
}

static int cmp_f64_asc(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

typedef struct { double f; uint32_t idx; } score_idx;

/* score descending, NaN last, then original index ascending */
static int cmp_score(const void *a, const void *b)
{
    const score_idx *x = a, *y = b;
    int xn = isnan(x->f), yn = isnan(y->f);
    if (xn != yn) return xn ? 1 : -1;
    if (!xn) {
        if (x->f > y->f) return -1;
        if (x->f < y->f) return 1;
    }
    return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

/* --------------------------------------------------------------- octree */

typedef struct {
    uint32_t begin, end, level;
    uint64_t prefix;
} leaf_t;

typedef struct {
    const uint64_t *skey;  /* keys in sorted order */
    int32_t cap;
    int dmax;
    leaf_t *leaves;
    int64_t n_leaves;
} tree_ctx;

/* A node (level d, key prefix) covering sorted positions [b, e) is split
 * into its 8 children while it holds more than cap points and d < dmax;
 * otherwise it is a leaf. Children are visited in octal-digit order, so
 * leaves come out in Morton order. */
static void split_node(tree_ctx *t, int d, uint64_t prefix, uint32_t b, uint32_t e)
{
    if ((int64_t)(e - b) > (int64_t)t->cap && d < t->dmax) {
        int shift = 3 * (MORTON_BITS - (d + 1));
        uint32_t s = b;
        for (uint64_t c = 0; c < 8; ++c) {
            uint64_t child = prefix * 8u + c;
            uint32_t u = s;
            while (u < e && (t->skey[u] >> shift) == child) ++u;
            if (u > s) split_node(t, d + 1, child, s, u);
            s = u;
        }
    } else if (e > b) {
        leaf_t *L = &t->leaves[t->n_leaves++];
        L->begin = b;
        L->end = e;
        L->level = (uint32_t)d;
        L->prefix = prefix;
    }
}

/* Deepest level whose cell side S*2^-d is still >= min_side. */
static int depth_limit(double S, double min_side)
{
    if (!(min_side > 0.0)) return MORTON_BITS;
    int d = 0;
    while (d < MORTON_BITS && ldexp(S, -(d + 1)) >= min_side) ++d;
    return d;
}

/* ------------------------------------------------------------- top-k */

static int pair_less(float da, uint32_t ia, float db, uint32_t ib)
{
    return da < db || (da == db && ia < ib);
}

/* Keep the k smallest (d2, idx) pairs seen so far, ascending. */
static void topk_push(float *bd, uint32_t *bi, int *cnt, int k, float d2, uint32_t j)
{
    int pos;
    if (*cnt == k) {
        if (!pair_less(d2, j, bd[k - 1], bi[k - 1])) return;
        pos = k - 1;
    } else {
        pos = (*cnt)++;
    }
    while (pos > 0 && pair_less(d2, j, bd[pos - 1], bi[pos - 1])) {
        bd[pos] = bd[pos - 1];
        bi[pos] = bi[pos - 1];
        --pos;
    }
    bd[pos] = d2;
    bi[pos] = j;
}

/* ------------------------------------------------------------- halo block */

/* Point i's cell at the level whose shift is sh lies within one cell of c on
 * every axis. Cells outside [0, 2^d) hold no points, so the block is clipped
 * at the grid border without a separate test. */
static int in_block(const uint32_t *q, int64_t i, int sh, const int64_t *c)
{
    int64_t px = (int64_t)(q[3 * i] >> sh), py = (int64_t)(q[3 * i + 1] >> sh), pz = (int64_t)(q[3 * i + 2] >> sh);
    return llabs(px - c[0]) <= 1 && llabs(py - c[1]) <= 1 && llabs(pz - c[2]) <= 1;
}

/* ------------------------------------------------------------ percentile */

/* MATLAB prctile places the i-th smallest of n values at percentile
 * 100*(i-0.5)/n and interpolates linearly in between, clamping outside.
 * Keeping the values >= prctile(v, q) therefore keeps exactly the values
 * >= the c-th smallest, with c = ceil(n*q/100 + 0.5) clamped to [1, n]. */
int64_t orc_percentile_rank(int64_t n, double q)
{
    if (n <= 0) return 0;
    double c = ceil((double)n * q / 100.0 + 0.5);
    if (c < 1.0) c = 1.0;
    if (c > (double)n) c = (double)n;
    return (int64_t)c;
}

/* ----------------------------------------------------------- the pipeline */

int orc_denoise(const float *xyz, int64_t n, const orc_params *p, orc_out *o)
{
    if (!params_ok(p) || n < 0 || n > (int64_t)0x7FFFFFFF) return -1;
    const int K = p->k;
    o->n_kept = 0;
    o->n_leaves = 0;
    o->pairs = 0;
#ifdef _OPENMP
    o->threads = omp_get_max_threads();
#else
    o->threads = 1;
#endif
    if (n == 0) return 0;

    /* Frame bounding box (Eq. 2 applied to the whole frame): the octree root
     * is the cube of side S = the largest extent, at the minimum corner. */
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = xyz[a];
    for (int64_t i = 1; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            float v = xyz[3 * i + a];
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    double S = 0.0;
    for (int a = 0; a < 3; ++a) {
        double H = (double)hi[a] - (double)lo[a];
        if (H > S) S = H;
    }
    if (S == 0.0) S = 1.0;
    const double scale = 2097152.0 / S;

    /* Morton keys and the sorted order (key, original index). */
    uint32_t *q = malloc(sizeof(uint32_t) * 3 * (size_t)n);
    key_idx *ki = malloc(sizeof(key_idx) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) q[3 * i + a] = quantise(xyz[3 * i + a], lo[a], scale);
        ki[i].key = orc_morton_interleave(q[3 * i], q[3 * i + 1], q[3 * i + 2]);
        ki[i].idx = (uint32_t)i;
        if (o->key) o->key[i] = ki[i].key;
    }
    qsort(ki, (size_t)n, sizeof(key_idx), cmp_key_idx);
    uint64_t *skey = malloc(sizeof(uint64_t) * (size_t)n);
    uint32_t *sidx = malloc(sizeof(uint32_t) * (size_t)n);
    for (int64_t s = 0; s < n; ++s) {
        skey[s] = ki[s].key;
        sidx[s] = ki[s].idx;
        if (o->order) o->order[s] = ki[s].idx;
    }
    free(ki);

    /* Octree partition into leaves (Sec. 3). */
    tree_ctx t;
    t.skey = skey;
    t.cap = p->leaf_cap;
    t.dmax = depth_limit(S, p->min_leaf_side);
    t.leaves = malloc(sizeof(leaf_t) * (size_t)n);
    t.n_leaves = 0;
    split_node(&t, 0, 0, 0, (uint32_t)n);
    const int64_t NL = t.n_leaves;
    leaf_t *L = t.leaves;
    o->n_leaves = NL;

    uint32_t *leaf_of = malloc(sizeof(uint32_t) * (size_t)n);
    for (int64_t l = 0; l < NL; ++l)
        for (uint32_t s = L[l].begin; s < L[l].end; ++s) leaf_of[sidx[s]] = (uint32_t)l;

    /* Per leaf: bbox volume (Eq. 10), voxel size (Eq. 11), occupancy and the
     * filter n(voxel(p)) >= n_v (Eq. 12). */
    uint32_t *occ = malloc(sizeof(uint32_t) * (size_t)n);
    uint8_t *p1 = calloc((size_t)n, 1);
    float *leaf_h = malloc(sizeof(float) * (size_t)NL);
    for (int64_t l = 0; l < NL; ++l) {
        uint32_t b = L[l].begin, e = L[l].end, nt = e - b;
        float mn[3], mx[3];
        for (int a = 0; a < 3; ++a) mn[a] = mx[a] = xyz[3 * (size_t)sidx[b] + a];
        for (uint32_t s = b; s < e; ++s)
            for (int a = 0; a < 3; ++a) {
                float v = xyz[3 * (size_t)sidx[s] + a];
                if (v < mn[a]) mn[a] = v;
                if (v > mx[a]) mx[a] = v;
            }
        double Hx = (double)mx[0] - (double)mn[0];
        double Hy = (double)mx[1] - (double)mn[1];
        double Hz = (double)mx[2] - (double)mn[2];
        double V = (Hx * Hy) * Hz;
        float h32 = (float)(p->beta * cbrt(V / (double)nt));
        if (!(h32 > 0.0f) || !isfinite(h32)) h32 = 0.0f;
        leaf_h[l] = h32;
        if (h32 == 0.0f) {
            for (uint32_t s = b; s < e; ++s) occ[sidx[s]] = nt;
        } else {
            /* voxel id (vx, vy, vz) packed 21 bits per axis; count by sorting */
            uint64_t *vk = malloc(sizeof(uint64_t) * nt);
            for (uint32_t s = b; s < e; ++s) {
                uint64_t v[3];
                for (int a = 0; a < 3; ++a) {
                    double f = floor(((double)xyz[3 * (size_t)sidx[s] + a] - (double)mn[a]) / (double)h32);
                    if (!(f >= 0.0)) f = 0.0;
                    if (f > (double)QMAX) f = (double)QMAX;
                    v[a] = (uint64_t)f;
                }
                vk[s - b] = v[0] | (v[1] << 21) | (v[2] << 42);
            }
            uint64_t *sorted = malloc(sizeof(uint64_t) * nt);
            memcpy(sorted, vk, sizeof(uint64_t) * nt);
            qsort(sorted, nt, sizeof(uint64_t), cmp_u64);
            for (uint32_t s = b; s < e; ++s) {
                uint64_t x = vk[s - b];
                /* count of x in the sorted list: two binary searches */
                uint32_t lo_i = 0, hi_i = nt;
                while (lo_i < hi_i) { uint32_t m = (lo_i + hi_i) / 2; if (sorted[m] < x) lo_i = m + 1; else hi_i = m; }
                uint32_t first = lo_i;
                hi_i = nt;
                while (lo_i < hi_i) { uint32_t m = (lo_i + hi_i) / 2; if (sorted[m] <= x) lo_i = m + 1; else hi_i = m; }
                occ[sidx[s]] = lo_i - first;
            }
            free(sorted);
            free(vk);
        }
        for (uint32_t s = b; s < e; ++s)
            p1[sidx[s]] = !(p->stages & 1) || occ[sidx[s]] >= (uint32_t)p->min_vox_count;
    }

    /* Candidate set of each leaf: the P1 points whose level-d cell lies in
     * the 3x3x3 block of cells around the leaf's cell (level d = the leaf's
     * level; cell coordinates = the 21-bit grid coordinates shifted down by
     * 21 - d). Leaves are independent, so both passes run in parallel over
     * leaves; the offsets between them are a plain prefix sum. */
    int *cell_sh = malloc(sizeof(int) * (size_t)(NL > 0 ? NL : 1));
    int64_t *cell = malloc(sizeof(int64_t) * 3 * (size_t)(NL > 0 ? NL : 1));
    for (int64_t l = 0; l < NL; ++l) {
        cell_sh[l] = MORTON_BITS - (int)L[l].level;
        uint32_t f = sidx[L[l].begin];
        for (int a = 0; a < 3; ++a) cell[3 * l + a] = (int64_t)(q[3 * (size_t)f + a] >> cell_sh[l]);
    }
    int64_t *cand_off = malloc(sizeof(int64_t) * (size_t)(NL + 1));
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t l = 0; l < NL; ++l) {
        int64_t cnt = 0;
        for (int64_t i = 0; i < n; ++i)
            if (p1[i] && in_block(q, i, cell_sh[l], cell + 3 * l)) ++cnt;
        cand_off[l + 1] = cnt;
    }
    cand_off[0] = 0;
    for (int64_t l = 0; l < NL; ++l) cand_off[l + 1] += cand_off[l];
    uint32_t *cand = malloc(sizeof(uint32_t) * (size_t)(cand_off[NL] > 0 ? cand_off[NL] : 1));
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t l = 0; l < NL; ++l) {
        int64_t w = cand_off[l];
        for (int64_t i = 0; i < n; ++i)
            if (p1[i] && in_block(q, i, cell_sh[l], cell + 3 * l)) cand[w++] = (uint32_t)i;
        if (o->leaf_ncand) o->leaf_ncand[l] = (uint32_t)(cand_off[l + 1] - cand_off[l]);
    }
    free(cell_sh);
    free(cell);

    /* Queries: the P1 points of each leaf. */
    uint32_t *queries = malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *qleaf = malloc(sizeof(uint32_t) * (size_t)n);
    int64_t nq = 0;
    uint64_t pairs = 0;
    for (int64_t l = 0; l < NL; ++l) {
        uint64_t n1 = 0;
        for (uint32_t s = L[l].begin; s < L[l].end; ++s)
            if (p1[sidx[s]]) { queries[nq] = sidx[s]; qleaf[nq] = (uint32_t)l; ++nq; ++n1; }
        uint64_t c = (uint64_t)(cand_off[l + 1] - cand_off[l]);
        if (n1 > 0) pairs += n1 * (c - 1);
    }
    o->pairs = pairs;

    /* kNN over the candidate set (Sec. 3, N_K(i), d_ij, r_K,i) and the
     * density of Eq. 13, in FP64 from the fp32 coordinates. */
    uint32_t *nbr_i = malloc(sizeof(uint32_t) * (size_t)n * K);
    float *nbr_d = malloc(sizeof(float) * (size_t)n * K);
    int *nbr_cnt = calloc((size_t)n, sizeof(int));
    float *r2k = malloc(sizeof(float) * (size_t)n);
    double *r64 = malloc(sizeof(double) * (size_t)n);
    double *rho = calloc((size_t)n, sizeof(double));
    uint8_t *insufficient = calloc((size_t)n, 1);
    const double PI = 3.14159265358979323846;

#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t qi = 0; qi < nq; ++qi) {
        uint32_t i = queries[qi], l = qleaf[qi];
        float xi = xyz[3 * (size_t)i], yi = xyz[3 * (size_t)i + 1], zi = xyz[3 * (size_t)i + 2];
        float *bd = nbr_d + (size_t)i * K;
        uint32_t *bi = nbr_i + (size_t)i * K;
        int cnt = 0;
        for (int64_t c = cand_off[l]; c < cand_off[l + 1]; ++c) {
            uint32_t j = cand[c];
            if (j == i) continue;
            float dx = xyz[3 * (size_t)j] - xi;
            float dy = xyz[3 * (size_t)j + 1] - yi;
            float dz = xyz[3 * (size_t)j + 2] - zi;
            float d2 = (dx * dx + dy * dy) + dz * dz;
            topk_push(bd, bi, &cnt, K, d2, j);
        }
        nbr_cnt[i] = cnt;
        for (int m = cnt; m < K; ++m) { bd[m] = INFINITY; bi[m] = NO_NBR; }
        if (cnt < K) {
            insufficient[i] = 1;
            r2k[i] = INFINITY;
            r64[i] = INFINITY;
            rho[i] = 0.0;
        } else {
            r2k[i] = bd[K - 1];
            double m2 = 0.0;
            for (int m = 0; m < K; ++m) {
                uint32_t j = bi[m];
                double dx = (double)xyz[3 * (size_t)j] - (double)xi;
                double dy = (double)xyz[3 * (size_t)j + 1] - (double)yi;
                double dz = (double)xyz[3 * (size_t)j + 2] - (double)zi;
                double d2 = dx * dx + dy * dy + dz * dz;
                if (d2 > m2) m2 = d2;
            }
            r64[i] = sqrt(m2);
            rho[i] = (double)K / ((4.0 / 3.0) * PI * (r64[i] * r64[i] * r64[i]));
        }
    }

    /* Per leaf: percentile cut (Eq. 14) and median density (Eq. 16). */
    uint8_t *p2 = calloc((size_t)n, 1);
    double *rho_med = malloc(sizeof(double) * (size_t)NL);
    {
        float *rv = malloc(sizeof(float) * (size_t)n);
        double *dv = malloc(sizeof(double) * (size_t)n);
        for (int64_t l = 0; l < NL; ++l) {
            int64_t n1 = 0;
            for (uint32_t s = L[l].begin; s < L[l].end; ++s) {
                uint32_t i = sidx[s];
                if (!p1[i]) continue;
                rv[n1] = r2k[i];
                dv[n1] = rho[i];
                ++n1;
            }
            rho_med[l] = 0.0;
            if (n1 == 0) {
                if (o->leaf_n1) o->leaf_n1[l] = 0;
                continue;
            }
            qsort(rv, (size_t)n1, sizeof(float), cmp_f32_desc);
            int64_t c = orc_percentile_rank(n1, p->rho_percentile);
            float cut = rv[c - 1];
            qsort(dv, (size_t)n1, sizeof(double), cmp_f64_asc);
            rho_med[l] = (n1 % 2) ? dv[(n1 - 1) / 2] : (dv[n1 / 2 - 1] + dv[n1 / 2]) / 2.0;
            for (uint32_t s = L[l].begin; s < L[l].end; ++s) {
                uint32_t i = sidx[s];
                if (p1[i] && !insufficient[i] && (!(p->stages & 2) || r2k[i] <= cut)) p2[i] = 1;
            }
            if (o->leaf_n1) o->leaf_n1[l] = (uint32_t)n1;
        }
        free(rv);
        free(dv);
    }

    /* Dual-weight gravitational score, Eq. 21 (= Eq. 15 with Eq. 17, 19, 20),
     * summed over N_K(i) in (d2, index) order. A zero bandwidth (all k
     * neighbours coincide with i) gives d = 0 and the Gaussian factor 1.
     * The kernel of Eq. 20 is taken to the power gamma/2 (gamma = 2: Eq. 20). */
    double *score = malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) score[i] = -1.0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        if (!p2[i] || !(p->stages & 4)) continue;
        double med = rho_med[leaf_of[i]];
        double den = med * med + p->eps;
        double xi = xyz[3 * i], yi = xyz[3 * i + 1], zi = xyz[3 * i + 2];
        double sr = p->sigma * r64[i];
        double F = 0.0;
        for (int m = 0; m < K; ++m) {
            uint32_t j = nbr_i[(size_t)i * K + m];
            double dx = (double)xyz[3 * (size_t)j] - xi;
            double dy = (double)xyz[3 * (size_t)j + 1] - yi;
            double dz = (double)xyz[3 * (size_t)j + 2] - zi;
            double d2 = dx * dx + dy * dy + dz * dz;
            double w_den = pow(rho[i] * rho[j] / den, p->alpha / 2.0);
            double w_dis = (d2 == 0.0) ? 1.0 : exp(-d2 / (2.0 * sr * sr));
            double kern = (p->gamma == 2.0) ? 1.0 / (d2 + p->eps) : pow(d2 + p->eps, -p->gamma / 2.0);
            F += w_den * w_dis * kern;
        }
        score[i] = F;
    }

    /* Top-lambda per leaf, then the union of leaves (Eq. 22). */
    uint8_t *stage = calloc((size_t)n, 1);
    uint8_t *keep = calloc((size_t)n, 1);
    {
        score_idx *sv = malloc(sizeof(score_idx) * (size_t)n);
        for (int64_t l = 0; l < NL; ++l) {
            int64_t n2 = 0;
            for (uint32_t s = L[l].begin; s < L[l].end; ++s) {
                uint32_t i = sidx[s];
                if (p1[i]) stage[i] = 1;
                if (p2[i]) { stage[i] = 2; sv[n2].f = score[i]; sv[n2].idx = i; ++n2; }
            }
            int64_t m = 0;
            if (!(p->stages & 4)) {
                /* A3 disabled: every P2 point is kept */
                for (int64_t r = 0; r < n2; ++r) {
                    stage[sv[r].idx] = 3;
                    keep[sv[r].idx] = 1;
                }
                m = n2;
            } else if (!isnan(p->log_threshold)) {
                /* threshold mode: ln F_i >= threshold, no ranking */
                for (int64_t r = 0; r < n2; ++r) {
                    if (log(sv[r].f) >= p->log_threshold) {
                        stage[sv[r].idx] = 3;
                        keep[sv[r].idx] = 1;
                        ++m;
                    }
                }
            } else if (n2 > 0) {
                double mf = ceil(p->keep_ratio * (double)n2);
                m = (int64_t)mf;
                if (m > n2) m = n2;
                qsort(sv, (size_t)n2, sizeof(score_idx), cmp_score);
                for (int64_t r = 0; r < m; ++r) { stage[sv[r].idx] = 3; keep[sv[r].idx] = 1; }
            }
            if (o->leaf_n2) o->leaf_n2[l] = (uint32_t)n2;
            if (o->leaf_m) o->leaf_m[l] = (uint32_t)m;
        }
        free(sv);
    }

    /* Outputs in original order. */
    int64_t nk = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (keep[i]) {
            if (o->kept_idx) o->kept_idx[nk] = (uint32_t)i;
            ++nk;
        }
    }
    o->n_kept = nk;
    for (int64_t i = 0; i < n; ++i) {
        if (o->leaf_of) o->leaf_of[i] = leaf_of[i];
        if (o->occ) o->occ[i] = occ[i];
        if (o->p1) o->p1[i] = p1[i];
        if (o->p2) o->p2[i] = p2[i];
        if (o->stage) o->stage[i] = stage[i];
        if (o->keep) o->keep[i] = keep[i];
        if (o->score) o->score[i] = score[i];
        if (p1[i]) {
            if (o->r2k) o->r2k[i] = r2k[i];
            if (o->rho) o->rho[i] = rho[i];
            if (o->nbr_idx) memcpy(o->nbr_idx + (size_t)i * K, nbr_i + (size_t)i * K, sizeof(uint32_t) * K);
            if (o->nbr_d2) memcpy(o->nbr_d2 + (size_t)i * K, nbr_d + (size_t)i * K, sizeof(float) * K);
        }
    }
    for (int64_t l = 0; l < NL; ++l) {
        if (o->leaf_begin) o->leaf_begin[l] = L[l].begin;
        if (o->leaf_end) o->leaf_end[l] = L[l].end;
        if (o->leaf_level) o->leaf_level[l] = L[l].level;
        if (o->leaf_prefix) o->leaf_prefix[l] = L[l].prefix;
        if (o->leaf_h) o->leaf_h[l] = leaf_h[l];
        if (o->leaf_rho_med) o->leaf_rho_med[l] = rho_med[l];
    }

    free(q); free(skey); free(sidx); free(t.leaves); free(leaf_of); free(occ); free(p1);
    free(leaf_h); free(cand_off); free(cand); free(queries); free(qleaf);
    free(nbr_i); free(nbr_d); free(nbr_cnt); free(r2k); free(r64); free(rho);
    free(insufficient); free(p2); free(rho_med); free(score); free(stage); free(keep);
    return 0;
}

/* ------------------------------------------------------------- score fit */

/* Score-fit loss and gradient. The score follows Eq. 21 with the kernel
 * exponent gamma; its derivatives are taken term by term:
 *   d/dalpha ln t_ij = (1/2) ln(rho_i rho_j / (rho_med^2 + eps))     (Eq. 17)
 *   d/dsigma ln t_ij = d_ij^2 / (sigma^3 r_K,i^2)                    (Eq. 18, 19)
 *   d/dgamma ln t_ij = -(1/2) ln(d_ij^2 + eps)                        (Eq. 20)
 * so dF_i/dtheta = sum_j t_ij d/dtheta ln t_ij, and with p_i = sigmoid(z_i),
 * dL/dz_i = (p_i - y_i) / |terms|, dz_i/dtheta = (dF_i/dtheta) / (T F_i),
 * dz_i/dtau = -1/T. Terms with t_ij = 0 (a zero density) add nothing. */
int orc_fit_loss_grad(const float *xyz, int64_t n, int k, double eps, const orc_out *o,
                      const uint8_t *label, double alpha, double sigma, double gamma,
                      double tau, double T, double *out)
{
    if (!(T > 0.0) || !(sigma > 0.0)) return -1;
    double L = 0.0, ga = 0.0, gs = 0.0, gg = 0.0, gt = 0.0, cnt = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!o->p2[i]) continue;
        double xi = xyz[3 * i], yi = xyz[3 * i + 1], zi = xyz[3 * i + 2];
        /* r_K,i in FP64: the largest neighbour distance (as for Eq. 13) */
        double m2 = 0.0;
        for (int m = 0; m < k; ++m) {
            uint32_t j = o->nbr_idx[(size_t)i * k + m];
            double dx = (double)xyz[3 * (size_t)j] - xi;
            double dy = (double)xyz[3 * (size_t)j + 1] - yi;
            double dz = (double)xyz[3 * (size_t)j + 2] - zi;
            double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 > m2) m2 = d2;
        }
        double r2 = m2;
        double med = o->leaf_rho_med[o->leaf_of[i]];
        double F = 0.0, dFa = 0.0, dFs = 0.0, dFg = 0.0;
        for (int m = 0; m < k; ++m) {
            uint32_t j = o->nbr_idx[(size_t)i * k + m];
            double dx = (double)xyz[3 * (size_t)j] - xi;
            double dy = (double)xyz[3 * (size_t)j + 1] - yi;
            double dz = (double)xyz[3 * (size_t)j + 2] - zi;
            double d2 = dx * dx + dy * dy + dz * dz;
            double ratio = o->rho[i] * o->rho[j] / (med * med + eps);
            double w_den = pow(ratio, alpha / 2.0);
            double w_dis = (d2 == 0.0) ? 1.0 : exp(-d2 / (2.0 * sigma * sigma * r2));
            double kern = pow(d2 + eps, -gamma / 2.0);
            double t = w_den * w_dis * kern;
            if (t == 0.0) continue;
            F += t;
            dFa += t * 0.5 * log(ratio);
            if (d2 != 0.0) dFs += t * d2 / (sigma * sigma * sigma * r2);
            dFg += t * (-0.5 * log(d2 + eps));
        }
        if (!(F > 0.0) || isinf(F)) continue;
        double y = label[i] ? 0.0 : 1.0;
        double z = (log(F) - tau) / T;
        double p = 1.0 / (1.0 + exp(-z));
        /* BCE(sigmoid(z), y) = log(1 + e^z) - y z, written without overflow */
        L += (z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z))) - y * z;
        double g = (p - y) / T;
        ga += g * dFa / F;
        gs += g * dFs / F;
        gg += g * dFg / F;
        gt += -g;
        cnt += 1.0;
    }
    double c = cnt > 0.0 ? cnt : 1.0;
    out[0] = L / c;
    out[1] = ga / c;
    out[2] = gs / c;
    out[3] = gg / c;
    out[4] = gt / c;
    out[5] = cnt;
    return 0;
}

/* ------------------------------------------------------ evaluation (Eq. 29, 30) */

int orc_nearest(const float *a, int64_t na, const float *b, int64_t nb, uint32_t *idx, float *d2)
{
    if (nb <= 0) return -1;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t i = 0; i < na; ++i) {
        float best = INFINITY;
        uint32_t bi = 0;
        for (int64_t j = 0; j < nb; ++j) {
            float dx = b[3 * j] - a[3 * i];
            float dy = b[3 * j + 1] - a[3 * i + 1];
            float dz = b[3 * j + 2] - a[3 * i + 2];
            float d = (dx * dx + dy * dy) + dz * dz;
            if (d < best) {
                best = d;
                bi = (uint32_t)j;
            }
        }
        idx[i] = bi;
        d2[i] = best;
    }
    return 0;
}

/* mean over a of the FP64 squared distance to its nearest point of b */
static double mean_nearest_d2(const float *a, int64_t na, const float *b, int64_t nb)
{
    uint32_t *idx = malloc(sizeof(uint32_t) * (size_t)na);
    float *d2 = malloc(sizeof(float) * (size_t)na);
    orc_nearest(a, na, b, nb, idx, d2);
    double s = 0.0;
    for (int64_t i = 0; i < na; ++i) {
        uint32_t j = idx[i];
        double dx = (double)b[3 * (size_t)j] - (double)a[3 * i];
        double dy = (double)b[3 * (size_t)j + 1] - (double)a[3 * i + 1];
        double dz = (double)b[3 * (size_t)j + 2] - (double)a[3 * i + 2];
        s += dx * dx + dy * dy + dz * dz;
    }
    free(idx);
    free(d2);
    return s / (double)na;
}

int orc_eval_metrics(const float *clean, int64_t nc, const float *den, int64_t nd, double *out)
{
    if (nc <= 0 || nd <= 0) return -1;
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = clean[a];
    for (int64_t i = 1; i < nc; ++i)
        for (int a = 0; a < 3; ++a) {
            if (clean[3 * i + a] < lo[a]) lo[a] = clean[3 * i + a];
            if (clean[3 * i + a] > hi[a]) hi[a] = clean[3 * i + a];
        }
    double m2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double e = (double)hi[a] - (double)lo[a];
        m2 += e * e;
    }
    out[0] = mean_nearest_d2(clean, nc, den, nd);
    out[1] = mean_nearest_d2(den, nd, clean, nc);
    out[2] = out[0] + out[1];
    out[3] = 10.0 * log10(m2 / out[0]);
    return 0;
}
