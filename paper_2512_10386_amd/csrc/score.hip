// Density (Eq. 13), the per-leaf percentile cut (Eq. 14) and median density
// (Eq. 16), the dual-weight gravitational score (Eq. 15-21), the per-leaf
// top-lambda rule and the union of the leaves' kept points (Eq. 22).
#include <climits>

#include "kernels.hpp"
#include "scan.hpp"

namespace gdn {

constexpr uint32_t NO_NBR = 0xFFFFFFFFu;
constexpr double PI_D = 3.14159265358979323846;

// ---------------------------------------------------------------- density
//
// r_K,i = the largest FP64 distance to the k neighbours; rho_i = K / (4/3 pi r^3).
// A point with fewer than k candidates has rho = 0 (r = inf).

__global__ __launch_bounds__(256) void density_kernel(Plan P, const float* __restrict__ xyz, int k,
                                                      double half_alpha) {
    const uint32_t np1 = P.ctr->n_p1;
    for (uint32_t qi = blockIdx.x * blockDim.x + threadIdx.x; qi < np1; qi += gridDim.x * blockDim.x) {
        const uint32_t i = __float_as_uint(P.cand4[qi].w);
        const double xi = xyz[3 * (size_t)i], yi = xyz[3 * (size_t)i + 1], zi = xyz[3 * (size_t)i + 2];
        const uint32_t* nb = P.nbr + (size_t)qi * k;
        double rho, r64;
        if (nb[k - 1] == NO_NBR) {
            rho = 0.0;
            r64 = INFINITY;
        } else {
            double m2 = 0.0;
            for (int r = 0; r < k; ++r) {
                const uint32_t j = nb[r];
                if (j >= P.n) continue;
                const double dx = (double)xyz[3 * (size_t)j] - xi;
                const double dy = (double)xyz[3 * (size_t)j + 1] - yi;
                const double dz = (double)xyz[3 * (size_t)j + 2] - zi;
                const double d2 = dx * dx + dy * dy + dz * dz;
                if (d2 > m2) m2 = d2;
            }
            r64 = sqrt(m2);
            rho = (double)k / ((4.0 / 3.0) * PI_D * (r64 * r64 * r64));
        }
        P.rho_c[qi] = rho;
        P.r64_c[qi] = r64;
        P.rho_o[i] = rho;
        P.gpow_o[i] = pow(rho, half_alpha);
    }
}

void launch_density(const Plan& P, const Params& prm, const float* xyz, hipStream_t st) {
    unsigned blocks = (P.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(density_kernel, dim3(blocks), dim3(256), 0, st, P, xyz, prm.k, prm.alpha / 2.0);
}

// ---------------------------------------------------------------- block radix select

// Wave 0 finds the histogram bin holding ascending rank r; out = {bin, count below it}.
__device__ __forceinline__ void find_bin(const uint32_t* hist, uint32_t r, uint32_t* out) {
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const uint32_t h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
        const uint32_t s = h0 + h1 + h2 + h3;
        const uint32_t inc = wave_incl_scan(s);
        const uint32_t ex = inc - s;
        if (ex <= r && r < inc) {
            uint32_t acc = ex;
            int b = 4 * lane;
            if (r >= acc + h0) {
                acc += h0; ++b;
                if (r >= acc + h1) {
                    acc += h1; ++b;
                    if (r >= acc + h2) { acc += h2; ++b; }
                }
            }
            out[0] = (uint32_t)b;
            out[1] = acc;
        }
    }
}

// Value of ascending rank r (0-based, r < cnt) among get(0..cnt-1), by 8-bit
// MSD passes over LDS histograms. Whole block must call it.
template <typename T, class Get>
__device__ T block_select(Get get, uint32_t cnt, uint32_t r, uint32_t* s_hist, uint32_t* s_sel) {
    constexpr int BITS = 8 * (int)sizeof(T);
    T prefix = 0, mask = 0;
    for (int shift = BITS - 8; shift >= 0; shift -= 8) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) s_hist[i] = 0u;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
            const T v = get(i);
            if ((v & mask) == prefix) atomicAdd(&s_hist[(uint32_t)(v >> shift) & 255u], 1u);
        }
        __syncthreads();
        find_bin(s_hist, r, s_sel);
        __syncthreads();
        r -= s_sel[1];
        prefix |= (T)s_sel[0] << shift;
        mask |= (T)255 << shift;
        __syncthreads();
    }
    return prefix;
}

struct R2Bits {
    const float* r2k;
    uint32_t qb;
    __device__ uint32_t operator()(uint32_t i) const { return __float_as_uint(r2k[qb + i]); }
};
struct RhoBits {
    const double* rho;
    uint32_t qb;
    __device__ unsigned long long operator()(uint32_t i) const {
        return (unsigned long long)__double_as_longlong(rho[qb + i]);
    }
};

// ---------------------------------------------------------------- percentile + median
//
// Per leaf over Q_t = P1 of the leaf (n1 points): MATLAB prctile keeps the
// densities >= the c-th smallest, c = ceil(n1*q/100 + 0.5) clamped to [1, n1];
// density falls as r grows, so P2 keeps r^2 <= the c-th largest fp32 r^2 (and
// drops points with fewer than k candidates). The median of the densities is
// the middle value, or the mean of the two middle values for even n1.

__global__ __launch_bounds__(SEL_BLOCK) void leaf_select_kernel(Plan P, Params prm) {
    __shared__ uint32_t s_hist[256];
    __shared__ uint32_t s_sel[2];
    const uint32_t nl = P.ctr->n_leaves;
    const int k = prm.k;
    for (uint32_t t = blockIdx.x; t < nl; t += gridDim.x) {
        const uint32_t qb = P.p1pos[P.leaf_begin[t]], qe = P.p1pos[P.leaf_begin[t + 1]];
        const uint32_t n1 = qe - qb;
        if (n1 == 0) {
            if (threadIdx.x == 0) { P.leaf_rho_med[t] = 0.0; P.leaf_r2cut[t] = 0.0f; }
            continue;
        }
        double cd = ceil((double)n1 * prm.rho_percentile / 100.0 + 0.5);
        if (cd < 1.0) cd = 1.0;
        if (cd > (double)n1) cd = (double)n1;
        const uint32_t c = (uint32_t)cd;
        const float cut = __uint_as_float(block_select<uint32_t>(R2Bits{P.r2k, qb}, n1, n1 - c, s_hist, s_sel));
        double med;
        if (n1 & 1u) {
            med = __longlong_as_double((long long)block_select<unsigned long long>(RhoBits{P.rho_c, qb}, n1, (n1 - 1) / 2, s_hist, s_sel));
        } else {
            const double a = __longlong_as_double((long long)block_select<unsigned long long>(RhoBits{P.rho_c, qb}, n1, n1 / 2 - 1, s_hist, s_sel));
            const double b = __longlong_as_double((long long)block_select<unsigned long long>(RhoBits{P.rho_c, qb}, n1, n1 / 2, s_hist, s_sel));
            med = (a + b) / 2.0;
        }
        const double den = med * med + prm.eps;
        const double ha = prm.alpha / 2.0;
        for (uint32_t i = threadIdx.x; i < n1; i += blockDim.x) {
            const uint32_t qi = qb + i;
            const bool insufficient = P.nbr[(size_t)qi * k + (k - 1)] == NO_NBR;
            P.p2[qi] = (!insufficient && P.r2k[qi] <= cut) ? 1 : 0;
            P.afac_c[qi] = pow(P.rho_c[qi] / den, ha);
        }
        if (threadIdx.x == 0) { P.leaf_rho_med[t] = med; P.leaf_r2cut[t] = cut; }
        __syncthreads();
    }
}

void launch_leaf_select(const Plan& P, const Params& prm, hipStream_t st) {
    unsigned blocks = P.n < 2048 ? P.n : 2048;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(leaf_select_kernel, dim3(blocks), dim3(SEL_BLOCK), 0, st, P, prm);
}

// ---------------------------------------------------------------- score
//
// F_i = sum over N_K(i) of (rho_i rho_j / (rho_med^2 + eps))^(alpha/2)
//       * exp(-d_ij^2 / (2 (sigma r_K,i)^2)) / (d_ij^2 + eps), in FP64, with the
// density weight factored as afac_i * rho_j^(alpha/2). A neighbour at d = 0
// gets the Gaussian factor 1 (also when r_K,i = 0).

__global__ __launch_bounds__(256) void score_kernel(Plan P, const float* __restrict__ xyz, int k, double sigma,
                                                    double eps) {
    const uint32_t np1 = P.ctr->n_p1;
    for (uint32_t qi = blockIdx.x * blockDim.x + threadIdx.x; qi < np1; qi += gridDim.x * blockDim.x) {
        if (!P.p2[qi]) continue;
        const uint32_t i = __float_as_uint(P.cand4[qi].w);
        const double xi = xyz[3 * (size_t)i], yi = xyz[3 * (size_t)i + 1], zi = xyz[3 * (size_t)i + 2];
        const double sr = sigma * P.r64_c[qi];
        const double a = P.afac_c[qi];
        const uint32_t* nb = P.nbr + (size_t)qi * k;
        double F = 0.0;
        for (int r = 0; r < k; ++r) {
            const uint32_t j = nb[r];
            if (j >= P.n) continue;
            const double dx = (double)xyz[3 * (size_t)j] - xi;
            const double dy = (double)xyz[3 * (size_t)j + 1] - yi;
            const double dz = (double)xyz[3 * (size_t)j + 2] - zi;
            const double d2 = dx * dx + dy * dy + dz * dz;
            const double w_den = a * P.gpow_o[j];
            const double w_dis = (d2 == 0.0) ? 1.0 : exp(-d2 / (2.0 * sr * sr));
            const double kern = 1.0 / (d2 + eps);
            F += w_den * w_dis * kern;
        }
        P.score_c[qi] = F;
    }
}

void launch_score(const Plan& P, const Params& prm, const float* xyz, hipStream_t st) {
    unsigned blocks = (P.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(score_kernel, dim3(blocks), dim3(256), 0, st, P, xyz, prm.k, prm.sigma, prm.eps);
}

// ---------------------------------------------------------------- top-lambda
//
// Per leaf keep m = min(n2, ceil(lambda * n2)) points of P2 by (score desc,
// original index asc); a NaN score ranks below every number. The m-th largest
// score key is found by radix select, remaining ties by a select on indices.

struct ScoreKey {
    const double* score;
    const uint8_t* p2;
    uint32_t qb;
    __device__ unsigned long long operator()(uint32_t i) const {
        const uint32_t qi = qb + i;
        if (!p2[qi]) return 0ull;
        const double f = score[qi];
        if (isnan(f)) return 1ull;
        return (unsigned long long)__double_as_longlong(f) + 2ull;
    }
};
struct TieIdx {
    ScoreKey key;
    const float4* cand4;
    unsigned long long theta;
    __device__ uint32_t operator()(uint32_t i) const {
        return key(i) == theta ? __float_as_uint(cand4[key.qb + i].w) : 0xFFFFFFFFu;
    }
};

__global__ __launch_bounds__(SEL_BLOCK) void topl_kernel(Plan P, double lambda) {
    __shared__ uint32_t s_hist[256];
    __shared__ uint32_t s_sel[2];
    __shared__ uint32_t s_cnt;
    const uint32_t nl = P.ctr->n_leaves;
    for (uint32_t t = blockIdx.x; t < nl; t += gridDim.x) {
        const uint32_t qb = P.p1pos[P.leaf_begin[t]], qe = P.p1pos[P.leaf_begin[t + 1]];
        const uint32_t n1 = qe - qb;
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        uint32_t c = 0;
        for (uint32_t i = threadIdx.x; i < n1; i += blockDim.x) c += P.p2[qb + i];
        c = wave_sum(c);
        if ((threadIdx.x & 63) == 0 && c) atomicAdd(&s_cnt, c);
        __syncthreads();
        const uint32_t n2 = s_cnt;
        uint32_t m = 0;
        if (n2 > 0) {
            const double mf = ceil(lambda * (double)n2);
            m = mf >= (double)n2 ? n2 : (uint32_t)mf;
        }
        const ScoreKey key{P.score_c, P.p2, qb};
        unsigned long long theta = ~0ull;
        uint32_t idx_cut = 0;
        if (m > 0) {
            theta = block_select<unsigned long long>(key, n1, n1 - m, s_hist, s_sel);
            if (threadIdx.x == 0) s_cnt = 0;
            __syncthreads();
            uint32_t g = 0;
            for (uint32_t i = threadIdx.x; i < n1; i += blockDim.x) g += key(i) > theta ? 1u : 0u;
            g = wave_sum(g);
            if ((threadIdx.x & 63) == 0 && g) atomicAdd(&s_cnt, g);
            __syncthreads();
            const uint32_t need = m - s_cnt;
            idx_cut = block_select<uint32_t>(TieIdx{key, P.cand4, theta}, n1, need - 1, s_hist, s_sel);
        }
        for (uint32_t i = threadIdx.x; i < n1; i += blockDim.x) {
            const uint32_t qi = qb + i;
            uint8_t st = 1;
            if (P.p2[qi]) {
                const unsigned long long kv = key(i);
                const uint32_t oi = __float_as_uint(P.cand4[qi].w);
                const bool kept = m > 0 && (kv > theta || (kv == theta && oi <= idx_cut));
                st = kept ? 3 : 2;
            }
            P.stage_c[qi] = st;
        }
        if (threadIdx.x == 0) P.leaf_m[t] = m;
        __syncthreads();
    }
}

void launch_topl(const Plan& P, const Params& prm, hipStream_t st) {
    unsigned blocks = P.n < 2048 ? P.n : 2048;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(topl_kernel, dim3(blocks), dim3(SEL_BLOCK), 0, st, P, prm.keep_ratio);
}

// ---------------------------------------------------------------- outputs

__global__ __launch_bounds__(256) void outputs_kernel(Plan P, uint8_t* keep, float* score, uint8_t* stage) {
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < P.n; s += gridDim.x * blockDim.x) {
        const uint32_t i = P.idx_a[s];
        uint8_t st = 0;
        float sc = -1.0f;
        if (P.p1[s]) {
            const uint32_t qi = P.p1pos[s];
            st = P.stage_c[qi];
            if (st >= 2) sc = (float)P.score_c[qi];
        }
        keep[i] = st == 3;
        score[i] = sc;
        if (stage) stage[i] = st;
    }
}

struct KeepGet {
    const uint8_t* keep;
    __device__ uint32_t operator()(uint32_t i) const { return keep[i]; }
};
struct KeepEmit {
    uint32_t* kept_idx;
    __device__ void operator()(uint32_t i, uint32_t ex, uint32_t f) const {
        if (f) kept_idx[ex] = i;
    }
};
struct KeepFin {
    Counters* c;
    int64_t* n_kept;
    __device__ void operator()(uint32_t total) const {
        c->n_kept = total;
        *n_kept = (int64_t)total;
    }
};

void launch_outputs(const Plan& P, uint8_t* keep, float* score, uint8_t* stage, uint32_t* kept_idx,
                    int64_t* n_kept, hipStream_t st) {
    unsigned blocks = (P.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(outputs_kernel, dim3(blocks), dim3(256), 0, st, P, keep, score, stage);
    launch_scan(KeepGet{keep}, KeepEmit{kept_idx}, KeepFin{P.ctr, n_kept}, nullptr, P.n,
                P.scan_status + 2 * (size_t)P.scan_tiles, &P.ctr->scan_tile_ctr[2], &P.ctr->status, st);
}

__global__ void write_zero_count_kernel(int64_t* n_kept) { *n_kept = 0; }

void launch_write_zero_count(int64_t* n_kept, hipStream_t st) {
    hipLaunchKernelGGL(write_zero_count_kernel, dim3(1), dim3(1), 0, st, n_kept);
}

}  // namespace gdn
