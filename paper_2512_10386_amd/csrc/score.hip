// Density (Eq. 13), the per-leaf percentile cut (Eq. 14) and median density
// (Eq. 16), the dual-weight gravitational score (Eq. 15-21), the per-leaf
// top-lambda rule and the union of the leaves' kept points (Eq. 22).
#include <climits>
#include <cmath>

#include "kernels.hpp"
#include "scan.hpp"
#include "wave.hpp"

namespace gdn {

constexpr uint32_t NO_NBR = 0xFFFFFFFFu;
constexpr double PI_D = 3.14159265358979323846;

// ---------------------------------------------------------------- density
//
// r_K,i = the largest FP64 distance to the k neighbours; rho_i = K / (4/3 pi r^3).
// A point with fewer than k candidates has rho = 0 (r = inf).
//
// The score gathers its neighbours one lane each: a wave holds 64 / kp
// queries, kp = k rounded up to a power of two, lane r of a segment takes
// neighbour r, and a segment reduction adds the terms.

__device__ __forceinline__ uint32_t pow2_at_least(uint32_t k) {
    uint32_t p = 1;
    while (p < k) p <<= 1;
    return p;
}

__device__ __forceinline__ double seg_sum(double v, uint32_t kp) {
    for (uint32_t o = kp >> 1; o > 0; o >>= 1) v += __shfl_xor(v, (int)o, 64);
    return v;
}

// x^(alpha/2) of the density weight (Eq. 17): the square root for the
// default alpha = 1 (a few instructions instead of a general FP64 power; the
// two agree to an ulp), pow otherwise. The select kernels are instantiated
// for either, so each holds only the code it runs.
template <bool SQRT>
__device__ __forceinline__ double pow_ha(double x, double ha) {
    if constexpr (SQRT) return sqrt(x);
    else return pow(x, ha);
}

// Density of P1 query qi. The list is sorted by fp32 d2, and fp32 d2 is
// within ~6e-7 relative of the exact value, so only the neighbours whose fp32
// d2 is within 2^-16 of the k-th can hold the FP64 maximum. Usually that is
// the k-th alone (the (k-1)-th lies below), read from the dense record the
// kNN writes; otherwise walk the list down from the k-th and stop at the
// first one below. Stores r^2_K, rho and r densely (the selects run it for
// their leaf's points, so the density needs no launch of its own).
struct Dens {
    float r2;
    double rho, r64;
    bool short_list;  // fewer than k candidates
};

// What the density of a query starts from: its k-th neighbour record and the
// coordinates of the query and of that neighbour (the query's again when it
// has none), all loaded at once.
struct DensIn {
    uint4 kr;
    float4 cq, cj;
};
__device__ __forceinline__ DensIn density_load(const Plan& P, uint32_t qi) {
    DensIn d;
    d.kr = P.krec[qi];
    d.cq = P.cand4[qi];
    d.cj = P.cand4[d.kr.x < P.n ? d.kr.x : qi];
    return d;
}

__device__ __forceinline__ Dens density_finish(const Plan& P, uint32_t k, uint32_t qi, const DensIn& in) {
    const uint4 kr = in.kr;
    const uint32_t jk = kr.x;
    Dens out;
    out.r2 = __uint_as_float(kr.z);
    out.short_list = jk == NO_NBR;
    if (out.short_list) {
        out.rho = 0.0;
        out.r64 = INFINITY;
    } else {
        // the query's coordinates: cand4 holds bit copies of the input
        const double xi = in.cq.x, yi = in.cq.y, zi = in.cq.z;
        // a neighbour's sorted copy of the input coordinates
        auto d2_of = [&](const float4 cj) -> double {
            const double dx = (double)cj.x - xi;
            const double dy = (double)cj.y - yi;
            const double dz = (double)cj.z - zi;
            return dx * dx + dy * dy + dz * dz;
        };
        auto d2_to = [&](uint32_t j) -> double { return d2_of(P.cand4[j]); };
        const float thr = out.r2 * (1.0f - 1.0f / 65536.0f);
        double m2 = 0.0;
        if (k == 1u || __uint_as_float(kr.y) < thr) {
            if (jk < P.n) m2 = fmax(m2, d2_of(in.cj));
        } else {
            const uint32_t* nb = P.nbr + (size_t)qi * k;
            const float* d2 = P.nbr_d2 + (size_t)qi * k;
            for (int r = (int)k - 1; r >= 0; --r) {
                if (d2[r] < thr) break;
                const uint32_t j = nb[r];
                if (j >= P.n) continue;
                const double v = d2_to(j);
                if (v > m2) m2 = v;
            }
        }
        out.r64 = sqrt(m2);
        out.rho = (double)k / ((4.0 / 3.0) * PI_D * (out.r64 * out.r64 * out.r64));
    }
    P.r2k[qi] = out.r2;
    P.rho_c[qi] = out.rho;
    P.r64_c[qi] = out.r64;
    return out;
}

__device__ __forceinline__ Dens density_at(const Plan& P, const float* __restrict__ xyz, uint32_t k, uint32_t qi) {
    (void)xyz;
    return density_finish(P, k, qi, density_load(P, qi));
}

// ---------------------------------------------------------------- block radix select

// Wave 0 finds the histogram bin holding ascending rank r; out = {bin, count
// below it, count in it}.
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
            out[2] = hist[b];
        }
    }
}

// Value of ascending rank r (0-based, r < cnt) among get(0..cnt-1), by 8-bit
// MSD passes over LDS histograms; once the selected bin holds a single value,
// that value is the answer and is fetched directly. Whole block must call it.
// s_sel needs SEL_SCRATCH words.
constexpr int SEL_SCRATCH = 6;

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
        const bool single = s_sel[2] == 1u;
        __syncthreads();
        if (single && shift > 0) {
            // exactly one value carries this prefix
            for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
                const T v = get(i);
                if ((v & mask) == prefix) {
                    s_sel[3] = (uint32_t)v;
                    if constexpr (sizeof(T) > 4) s_sel[4] = (uint32_t)((unsigned long long)v >> 32);
                }
            }
            __syncthreads();
            T out = (T)s_sel[3];
            if constexpr (sizeof(T) > 4) out |= (T)((unsigned long long)s_sel[4] << 32);
            __syncthreads();
            return out;
        }
    }
    return prefix;
}

// Given a = the value of ascending rank r, the value of rank r + 1: a again
// if more than r + 1 values are <= a, else the smallest value above a.
template <typename T, class Get>
__device__ T block_next_rank(Get get, uint32_t cnt, uint32_t r, T a, uint32_t* s_sel) {
    __shared__ uint32_t s_le[SEL_BLOCK / 64];
    __shared__ T s_mn[SEL_BLOCK / 64];
    uint32_t le = 0;
    T mn = ~(T)0;
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
        const T v = get(i);
        if (v <= a) ++le;
        else if (v < mn) mn = v;
    }
    for (int o = 32; o > 0; o >>= 1) {
        le += (uint32_t)__shfl_xor((int)le, o, 64);
        const T x = (T)__shfl_xor(mn, o, 64);
        mn = x < mn ? x : mn;
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_le[w] = le;
        s_mn[w] = mn;
    }
    __syncthreads();
    uint32_t L = 0;
    T M = ~(T)0;
    for (int q = 0; q < SEL_BLOCK / 64; ++q) {
        L += s_le[q];
        M = s_mn[q] < M ? s_mn[q] : M;
    }
    __syncthreads();
    (void)s_sel;
    return L > r + 1u ? a : M;
}

template <typename T>
struct LdsBits {
    const T* v;
    __device__ T operator()(uint32_t i) const { return v[i]; }
};

constexpr uint32_t SEL_LDS_MAX = 2048;  // leaves up to this size are selected from LDS
constexpr uint32_t SEL_BATCH_MAX = 1024;  // leaves up to this size: each thread loads its points at once
constexpr uint32_t SMALL_LEAF = 256;    // leaves up to this size: one wave (4 values per lane), no LDS
constexpr uint32_t SMALL_PATH_MIN_N = 1u << 20;  // the wave path is used above this many points
constexpr uint32_t PACKED_OUT_MIN_N = 1u << 20;  // above: outputs scattered as packed records

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

// A block's leaves are t = its index (mod the stride). They are examined
// SEL_BLOCK at a time, one per thread (one round of loads instead of a chain
// of them), and those the block must handle (with `small`, the ones above
// SMALL_LEAF P1 points; otherwise all) are listed in order in s_list.
// Returns the count; whole block.
__device__ uint32_t block_leaf_round(const Plan& P, uint32_t base, uint32_t nl, bool small, uint32_t* s_list,
                                     uint32_t* s_scan, uint32_t stride) {
    const uint32_t ti = base + threadIdx.x * stride;
    uint32_t take = 0;
    if (ti < nl)
        take = small ? (P.p1pos[P.leaf_begin[ti + 1]] - P.p1pos[P.leaf_begin[ti]] > SMALL_LEAF ? 1u : 0u) : 1u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(take, s_scan, &tot);
    if (take) s_list[ex] = ti;
    __syncthreads();
    return tot;
}

// ---------------------------------------------------------------- percentile + median
//
// Per leaf over Q_t = P1 of the leaf (n1 points): MATLAB prctile keeps the
// densities >= the c-th smallest, c = ceil(n1*q/100 + 0.5) clamped to [1, n1];
// density falls as r grows, so P2 keeps r^2 <= the c-th largest fp32 r^2 (and
// drops points with fewer than k candidates). The median of the densities is
// the middle value, or the mean of the two middle values for even n1.

template <class RG>
__device__ float leaf_cut(RG r2, uint32_t n1, double q, uint32_t* s_hist, uint32_t* s_sel) {
    double cd = ceil((double)n1 * q / 100.0 + 0.5);
    if (cd < 1.0) cd = 1.0;
    if (cd > (double)n1) cd = (double)n1;
    const uint32_t c = (uint32_t)cd;
    return __uint_as_float(block_select<uint32_t>(r2, n1, n1 - c, s_hist, s_sel));
}

template <class HG>
__device__ void leaf_median(HG rho, uint32_t n1, double* med, uint32_t* s_hist, uint32_t* s_sel) {
    if (n1 & 1u) {
        *med = __longlong_as_double((long long)block_select<unsigned long long>(rho, n1, (n1 - 1) / 2, s_hist, s_sel));
    } else {
        const unsigned long long ab = block_select<unsigned long long>(rho, n1, n1 / 2 - 1, s_hist, s_sel);
        const unsigned long long bb = block_next_rank<unsigned long long>(rho, n1, n1 / 2 - 1, ab, s_sel);
        *med = (__longlong_as_double((long long)ab) + __longlong_as_double((long long)bb)) / 2.0;
    }
}

// Two workgroups per leaf, side by side: role 0 (even blocks) finds the
// percentile cut and writes P2, role 1 (odd blocks) the median, the weight
// factors and the density powers. Both compute the leaf's densities (the
// same values, stored twice); the two selects, each a chain of
// barrier-separated passes, then run at the same time instead of in turn.
template <bool SQRT>
__global__ __launch_bounds__(SEL_BLOCK) void leaf_select_kernel(Plan P, Params prm, bool small,
                                                               const float* __restrict__ xyz) {
    __shared__ uint32_t s_hist[256];
    __shared__ uint32_t s_sel[SEL_SCRATCH];
    __shared__ uint32_t s_r2[SEL_LDS_MAX];
    __shared__ unsigned long long s_rho[SEL_LDS_MAX];
    __shared__ uint32_t s_list[SEL_BLOCK];
    __shared__ uint32_t s_lscan[SEL_BLOCK / 64 + 1];
    const uint32_t nl = P.ctr->n_leaves;
    const int k = prm.k;
    const uint32_t role = blockIdx.x & 1u, bx = blockIdx.x >> 1, gx = gridDim.x >> 1;
    for (uint32_t base = bx; base < nl; base += gx * SEL_BLOCK) {
    const uint32_t nlist = block_leaf_round(P, base, nl, small, s_list, s_lscan, gx);
    for (uint32_t li = 0; li < nlist; ++li) {
        const uint32_t t = s_list[li];
        const uint32_t qb = P.p1pos[P.leaf_begin[t]], qe = P.p1pos[P.leaf_begin[t + 1]];
        const uint32_t n1 = qe - qb;
        if (small && n1 <= SMALL_LEAF) continue;  // leaf_select_small_kernel
        if (n1 == 0) {
            if (threadIdx.x == 0) {
                if (role == 0u) P.leaf_r2cut[t] = 0.0f;
                else P.leaf_rho_med[t] = 0.0;
            }
            continue;
        }
        float cut = 0.0f;
        double med = 0.0;
        if (n1 <= SEL_BATCH_MAX) {
            // point i = threadIdx.x + u * SEL_BLOCK of the leaf in slot u of
            // each thread, every load of a pass issued first (a slot past n1
            // loads the last point and is dropped)
            constexpr int SU = SEL_BATCH_MAX / SEL_BLOCK;
            {
                DensIn din[SU];
#pragma unroll
                for (int u = 0; u < SU; ++u)
                    din[u].kr = P.krec[qb + min(threadIdx.x + (uint32_t)u * SEL_BLOCK, n1 - 1u)];
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const uint32_t qi = qb + min(threadIdx.x + (uint32_t)u * SEL_BLOCK, n1 - 1u);
                    din[u].cq = P.cand4[qi];
                    din[u].cj = P.cand4[din[u].kr.x < P.n ? din[u].kr.x : qi];
                }
                // (an empty statement taking the loaded values keeps the compiler
                // from moving each load into the branch of its slot)
#pragma unroll
                for (int u = 0; u < SU; ++u) asm volatile("" ::"v"(din[u].kr.x), "v"(din[u].cq.x), "v"(din[u].cj.x));
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const uint32_t i = threadIdx.x + (uint32_t)u * SEL_BLOCK;
                    if (i >= n1) break;
                    const Dens dn = density_finish(P, (uint32_t)k, qb + i, din[u]);
                    if (role == 0u) s_r2[i] = __float_as_uint(dn.r2);
                    else s_rho[i] = (unsigned long long)__double_as_longlong(dn.rho);
                }
            }
            __syncthreads();
            if (role == 0u) {
                cut = leaf_cut(LdsBits<uint32_t>{s_r2}, n1, prm.rho_percentile, s_hist, s_sel);
                uint32_t kx[SU];
#pragma unroll
                for (int u = 0; u < SU; ++u) kx[u] = P.krec[qb + min(threadIdx.x + (uint32_t)u * SEL_BLOCK, n1 - 1u)].x;
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const uint32_t i = threadIdx.x + (uint32_t)u * SEL_BLOCK;
                    if (i >= n1) break;
                    P.p2[qb + i] = (kx[u] != NO_NBR && __uint_as_float(s_r2[i]) <= cut) ? 1 : 0;
                }
                if (threadIdx.x == 0) P.leaf_r2cut[t] = cut;
            } else {
                leaf_median(LdsBits<unsigned long long>{s_rho}, n1, &med, s_hist, s_sel);
                const double den = med * med + prm.eps;
                const double ha = prm.alpha / 2.0;
                double r64[SU];
#pragma unroll
                for (int u = 0; u < SU; ++u) r64[u] = P.r64_c[qb + min(threadIdx.x + (uint32_t)u * SEL_BLOCK, n1 - 1u)];
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const uint32_t i = threadIdx.x + (uint32_t)u * SEL_BLOCK;
                    if (i >= n1) break;
                    const double rho = __longlong_as_double((long long)s_rho[i]);
                    const double sr = prm.sigma * r64[u];
                    P.afac_c[qb + i] = make_double2(pow_ha<SQRT>(rho / den, ha), 1.0 / (2.0 * sr * sr));
                    // rho_j^(alpha/2) of Eq. 17's factored density weight, by P1 position
                    P.gpow_p[qb + i] = pow_ha<SQRT>(rho, ha);
                }
                if (threadIdx.x == 0) P.leaf_rho_med[t] = med;
            }
            __syncthreads();
            continue;
        }
        if (n1 <= SEL_LDS_MAX) {
            for (uint32_t i = threadIdx.x; i < n1; i += blockDim.x) {
                const Dens dn = density_at(P, xyz, (uint32_t)k, qb + i);
                if (role == 0u) s_r2[i] = __float_as_uint(dn.r2);
                else s_rho[i] = (unsigned long long)__double_as_longlong(dn.rho);
            }
            __syncthreads();
            if (role == 0u) cut = leaf_cut(LdsBits<uint32_t>{s_r2}, n1, prm.rho_percentile, s_hist, s_sel);
            else leaf_median(LdsBits<unsigned long long>{s_rho}, n1, &med, s_hist, s_sel);
        } else {
            for (uint32_t i = threadIdx.x; i < n1; i += blockDim.x) (void)density_at(P, xyz, (uint32_t)k, qb + i);
            __syncthreads();
            if (role == 0u) cut = leaf_cut(R2Bits{P.r2k, qb}, n1, prm.rho_percentile, s_hist, s_sel);
            else leaf_median(RhoBits{P.rho_c, qb}, n1, &med, s_hist, s_sel);
        }
        // same thread-to-point mapping as the density loop: each thread reads back its own stores
        if (role == 0u) {
            for (uint32_t i = threadIdx.x; i < n1; i += blockDim.x) {
                const uint32_t qi = qb + i;
                const bool insufficient = P.krec[qi].x == NO_NBR;
                P.p2[qi] = (!insufficient && P.r2k[qi] <= cut) ? 1 : 0;
            }
            if (threadIdx.x == 0) P.leaf_r2cut[t] = cut;
        } else {
            const double den = med * med + prm.eps;
            const double ha = prm.alpha / 2.0;
            for (uint32_t i = threadIdx.x; i < n1; i += blockDim.x) {
                const uint32_t qi = qb + i;
                const double sr = prm.sigma * P.r64_c[qi];
                P.afac_c[qi] = make_double2(pow_ha<SQRT>(P.rho_c[qi] / den, ha), 1.0 / (2.0 * sr * sr));
                // rho_j^(alpha/2) of Eq. 17's factored density weight, by P1 position
                P.gpow_p[qi] = pow_ha<SQRT>(P.rho_c[qi], ha);
            }
            if (threadIdx.x == 0) P.leaf_rho_med[t] = med;
        }
        __syncthreads();
    }
    __syncthreads();  // s_list is refilled by the next round
    }
}

// Leaves with at most SMALL_LEAF (= 256) P1 points: one wave each, no block
// barriers. The values sit as point i of the leaf in register i / 64 of lane
// i % 64 (padding ~0). Up to 64 values are sorted descending across the wave
// by a bitonic network (DPP exchanges) and ranks read from the sorted order;
// larger leaves use the wave radix select (fewer instructions than a
// 256-value network).
struct WaveVals {
    unsigned long long v[4];
};

__device__ __forceinline__ unsigned long long wave_rank_value(WaveVals w, uint32_t n1, uint32_t lane, uint32_t r,
                                                              uint32_t* hist) {
    // ascending rank r (0-based, r < n1) of the n1 values; the padding sorts first
    if (n1 <= 64u) {
        const unsigned long long s = sort64_desc_dir(w.v[0], lane);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)s, 63 - (int)r);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(s >> 32), 63 - (int)r);
        return ((unsigned long long)hi << 32) | lo;
    }
    return wave_select(w.v, n1, r, lane, hist);
}

// Given a = the value of ascending rank r, the value of rank r + 1: a again
// if more than r + 1 values are <= a, else the smallest value above a.
__device__ __forceinline__ unsigned long long wave_next_rank(const WaveVals& w, uint32_t n1, uint32_t lane, uint32_t r,
                                                             unsigned long long a) {
    uint32_t le = 0;
    unsigned long long mn = ~0ull;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool in = (uint32_t)j * 64u + lane < n1;
        le += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(in && w.v[j] <= a));
        if (in && w.v[j] > a && w.v[j] < mn) mn = w.v[j];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long x = (unsigned long long)__shfl_xor((long long)mn, off, 64);
        mn = x < mn ? x : mn;
    }
    return le > r + 1u ? a : mn;
}

template <bool SQRT>
__global__ __launch_bounds__(256) void leaf_select_small_kernel(Plan P, Params prm, const float* __restrict__ xyz) {
    __shared__ uint32_t s_hist[4][256];
    uint32_t* const hist = s_hist[threadIdx.x >> 6];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    const uint32_t nl = P.ctr->n_leaves;
    const int k = prm.k;
    const double ha = prm.alpha / 2.0;
    for (uint32_t t = wid; t < nl; t += nw) {
        const uint32_t qb = P.p1pos[P.leaf_begin[t]], qe = P.p1pos[P.leaf_begin[t + 1]];
        const uint32_t n1 = qe - qb;
        if (n1 > SMALL_LEAF) continue;
        if (n1 == 0) {
            if (lane == 0) { P.leaf_rho_med[t] = 0.0; P.leaf_r2cut[t] = 0.0f; }
            continue;
        }
        WaveVals r2v, rhov;
        double r64v[4];
        bool shortv[4];
        // every load of the four points first (a slot past n1 loads the last
        // point and is dropped): the stores of one point's density would
        // otherwise hold the next point's loads back
        DensIn din[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) din[j].kr = P.krec[qb + min((uint32_t)j * 64u + lane, n1 - 1u)];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t qi = qb + min((uint32_t)j * 64u + lane, n1 - 1u);
            din[j].cq = P.cand4[qi];
            din[j].cj = P.cand4[din[j].kr.x < P.n ? din[j].kr.x : qi];
        }
        // (an empty statement taking the loaded values keeps the compiler from
        // moving each load into the branch of its slot)
#pragma unroll
        for (int j = 0; j < 4; ++j) asm volatile("" ::"v"(din[j].kr.x), "v"(din[j].cq.x), "v"(din[j].cj.x));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t i = (uint32_t)j * 64u + lane;
            r2v.v[j] = ~0ull;
            rhov.v[j] = ~0ull;
            r64v[j] = 0.0;
            shortv[j] = true;
            if (i < n1) {
                const Dens dn = density_finish(P, (uint32_t)k, qb + i, din[j]);
                r2v.v[j] = (unsigned long long)__float_as_uint(dn.r2);
                rhov.v[j] = (unsigned long long)__double_as_longlong(dn.rho);
                r64v[j] = dn.r64;
                shortv[j] = dn.short_list;
            }
        }
        double cd = ceil((double)n1 * prm.rho_percentile / 100.0 + 0.5);
        if (cd < 1.0) cd = 1.0;
        if (cd > (double)n1) cd = (double)n1;
        const uint32_t c = (uint32_t)cd;
        const float cut = __uint_as_float((uint32_t)wave_rank_value(r2v, n1, lane, n1 - c, hist));
        double med;
        if (n1 & 1u) {
            med = __longlong_as_double((long long)wave_rank_value(rhov, n1, lane, (n1 - 1) / 2, hist));
        } else {
            const unsigned long long ab = wave_rank_value(rhov, n1, lane, n1 / 2 - 1, hist);
            const unsigned long long bb = wave_next_rank(rhov, n1, lane, n1 / 2 - 1, ab);
            med = (__longlong_as_double((long long)ab) + __longlong_as_double((long long)bb)) / 2.0;
        }
        const double den = med * med + prm.eps;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t i = (uint32_t)j * 64u + lane;
            if (i >= n1) continue;
            const uint32_t qi = qb + i;
            const double rho = __longlong_as_double((long long)rhov.v[j]);
            P.p2[qi] = (!shortv[j] && __uint_as_float((uint32_t)r2v.v[j]) <= cut) ? 1 : 0;
            const double sr = prm.sigma * r64v[j];
            P.afac_c[qi] = make_double2(pow_ha<SQRT>(rho / den, ha), 1.0 / (2.0 * sr * sr));
            P.gpow_p[qi] = pow_ha<SQRT>(rho, ha);
        }
        if (lane == 0) { P.leaf_rho_med[t] = med; P.leaf_r2cut[t] = cut; }
    }
}

void launch_leaf_select(const Plan& P, const Params& prm, const float* xyz, hipStream_t st) {
    // the wave path pays off for the many small leaves of large batches
    const bool small = P.n > SMALL_PATH_MIN_N;
    const bool sq = prm.alpha == 1.0;
    if (small) {
        unsigned wb = (P.n / 128 + 3) / 4;
        if (wb > 8192) wb = 8192;
        hipLaunchKernelGGL(sq ? leaf_select_small_kernel<true> : leaf_select_small_kernel<false>, dim3(wb), dim3(256),
                           0, st, P, prm, xyz);
    }
    unsigned blocks = P.n < 2048 ? P.n : 2048;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(sq ? leaf_select_kernel<true> : leaf_select_kernel<false>, dim3(2 * blocks), dim3(SEL_BLOCK), 0,
                       st, P, prm, small, xyz);
}

// ---------------------------------------------------------------- score
//
// F_i = sum over N_K(i) of (rho_i rho_j / (rho_med^2 + eps))^(alpha/2)
//       * exp(-d_ij^2 / (2 (sigma r_K,i)^2)) / (d_ij^2 + eps), in FP64, with the
// density weight factored as afac_i * rho_j^(alpha/2) and the Gaussian
// exponent as d^2 * c_i, c_i = 1 / (2 (sigma r_K,i)^2), both per query from the
// select kernel. A neighbour at d = 0 gets the Gaussian factor 1 (also when
// r_K,i = 0). The k terms are summed by a fixed pairwise tree (lane r holds
// term r), not left to right.

// Instantiated for the plain kernel exponent gamma = 2 (Eq. 20, one
// division) and the general power: a kernel holding both paths needs more
// registers and runs slower even when the power is never taken. PAIR: each
// wave takes two tiles of queries per step, so the loads of both (the
// neighbour lists, then the neighbours' coordinates and density powers) are
// in flight together; it pays on large inputs, where the step count per wave
// is high, and costs a little on a single frame.
constexpr uint32_t SCORE_PAIR_MIN_N = 1u << 20;

template <bool G2, bool PAIR>
__global__ __launch_bounds__(256) void score_kernel(Plan P, int kk, double eps, double gamma) {
    const uint32_t np1 = P.ctr->n_p1;
    const uint32_t k = (uint32_t)kk, kp = pow2_at_least(k), qpw = 64u / kp;
    const uint32_t lane = threadIdx.x & 63u, seg = lane / kp, r = lane % kp;
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    // the query's flag, neighbour index, coordinates and factors, issued
    // together; j = none for idle lanes and queries outside P2
    auto fetch = [&](uint32_t q0, uint32_t& qi, uint32_t& j, bool& live, float4& a, double2& af) {
        qi = q0 + seg;
        j = 0xFFFFFFFFu;
        live = false;
        if (qi < np1) {
            live = P.p2[qi] != 0;
            if (r < k) j = P.nbr[(size_t)qi * k + r];
            a = P.cand4[qi];
            af = P.afac_c[qi];
        }
        if (!live) j = 0xFFFFFFFFu;
    };
    // term r of the query's sum: the neighbour's coordinates (bit copies of
    // the input, in P1 order) and density power
    auto term_of = [&](const float4& c, double gp, const float4& a, const double2& af) -> double {
        const double dx = (double)c.x - (double)a.x;
        const double dy = (double)c.y - (double)a.y;
        const double dz = (double)c.z - (double)a.z;
        const double d2 = dx * dx + dy * dy + dz * dz;
        const double w_den = af.x * gp;
        const double w_dis = (d2 == 0.0) ? 1.0 : exp(-(d2 * af.y));
        double kern;
        if constexpr (G2) kern = 1.0 / (d2 + eps);
        else kern = pow(d2 + eps, -gamma / 2.0);
        return w_den * w_dis * kern;
    };
    if constexpr (PAIR) {
        // XCD-aware: the query tiles go in chunks of C consecutive tiles,
        // chunk c to the blocks b with b % 8 = c % 8 (the dispatcher hands
        // blocks to the eight XCDs in turn), so the neighbours a chunk gathers
        // (mostly within a few hundred P1 positions) stay in one XCD's L2:
        // half the HBM fetch of interleaved tiles, at the same speed. Whole
        // eighths per XCD fetched as little but balanced the uneven P2 tiles
        // worse (+5% time).
        constexpr uint32_t C = 64;
        const uint32_t wv = threadIdx.x >> 6, tq = qpw * (blockDim.x >> 6);
        const uint32_t T = (np1 + tq - 1) / tq;
        const uint32_t xcd = blockIdx.x % 8u, bi = blockIdx.x / 8u, nb = gridDim.x / 8u;
        // this XCD's i-th tile; the loop runs while the chunk of i can hold tiles
        auto tile_of = [&](uint32_t i) { return ((i / C) * 8u + xcd) * C + i % C; };
        const uint32_t t_hi = T;
        for (uint32_t i = bi; ((i / C) * 8u + xcd) * C < T || tile_of(i + nb) < T; i += 2u * nb) {
            const uint32_t t = tile_of(i);
            uint32_t qi0, j0, qi1, j1;
            bool l0, l1;
            float4 a0, a1, c0{}, c1{};
            double2 f0, f1;
            double g0 = 0.0, g1 = 0.0;
            fetch(t < t_hi ? t * tq + wv * qpw : np1, qi0, j0, l0, a0, f0);
            const uint32_t t1 = tile_of(i + nb);
            fetch(t1 < t_hi ? t1 * tq + wv * qpw : np1, qi1, j1, l1, a1, f1);
            if (j0 < P.n) { c0 = P.cand4[j0]; g0 = P.gpow_p[j0]; }
            if (j1 < P.n) { c1 = P.cand4[j1]; g1 = P.gpow_p[j1]; }
            const double F0 = seg_sum(j0 < P.n ? term_of(c0, g0, a0, f0) : 0.0, kp);
            const double F1 = seg_sum(j1 < P.n ? term_of(c1, g1, a1, f1) : 0.0, kp);
            if (l0 && r == 0) P.score_c[qi0] = F0;
            if (l1 && r == 0) P.score_c[qi1] = F1;
        }
    } else {
        for (uint32_t q0 = wid * qpw; q0 < np1; q0 += nw * qpw) {
            uint32_t qi, j;
            bool live;
            float4 a;
            double2 af;
            fetch(q0, qi, j, live, a, af);
            const double F = seg_sum(j < P.n ? term_of(P.cand4[j], P.gpow_p[j], a, af) : 0.0, kp);
            if (live && r == 0) P.score_c[qi] = F;
        }
    }
}

void launch_score(const Plan& P, const Params& prm, hipStream_t st) {
    uint32_t kp = 1;
    while (kp < (uint32_t)prm.k) kp <<= 1;
    const uint64_t waves = ((uint64_t)P.n * kp + 63) / 64;
    unsigned blocks = (unsigned)((waves + 3) / 4);
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    const bool pair = P.n > SCORE_PAIR_MIN_N;
    if (pair) blocks = (blocks + 7u) & ~7u;  // a whole number of blocks per XCD
    const bool g2 = prm.gamma == 2.0;
    auto kern = g2 ? (pair ? score_kernel<true, true> : score_kernel<true, false>)
                   : (pair ? score_kernel<false, true> : score_kernel<false, false>);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, st, P, prm.k, prm.eps, prm.gamma);
}

// ---------------------------------------------------------------- top-lambda
//
// Per leaf keep m = min(n2, ceil(lambda * n2)) points of P2 by (score desc,
// original index asc); a NaN score ranks below every number. The m-th largest
// score key is found by radix select, remaining ties by a select on indices.

__device__ __forceinline__ unsigned long long score_key(bool p2, double f) {
    if (!p2) return 0ull;
    if (isnan(f)) return 1ull;
    return (unsigned long long)__double_as_longlong(f) + 2ull;
}
struct ScoreKey {
    const double* score;
    const uint8_t* p2;
    uint32_t qb;
    __device__ unsigned long long operator()(uint32_t i) const {
        const uint32_t qi = qb + i;
        return p2[qi] ? score_key(true, score[qi]) : 0ull;
    }
};

// theta = the m-th largest key, idx_cut = the largest original index kept
// among the keys equal to theta.
template <class KG, class IG>
__device__ void topl_cut(KG key, IG tie_idx_of, uint32_t n1, uint32_t m, unsigned long long* theta,
                         uint32_t* idx_cut, uint32_t* s_hist, uint32_t* s_sel, uint32_t* s_cnt) {
    const unsigned long long th = block_select<unsigned long long>(key, n1, n1 - m, s_hist, s_sel);
    uint32_t* const s_eq = s_sel + SEL_SCRATCH - 1;  // free between selects
    if (threadIdx.x == 0) { *s_cnt = 0; *s_eq = 0; }
    __syncthreads();
    uint32_t g = 0, e = 0;
    for (uint32_t i = threadIdx.x; i < n1; i += blockDim.x) {
        const unsigned long long kv = key(i);
        g += kv > th ? 1u : 0u;
        e += kv == th ? 1u : 0u;
    }
    g = wave_sum(g);
    e = wave_sum(e);
    if ((threadIdx.x & 63) == 0 && g) atomicAdd(s_cnt, g);
    if ((threadIdx.x & 63) == 0 && e) atomicAdd(s_eq, e);
    __syncthreads();
    const uint32_t need = m - *s_cnt;
    if (*s_eq == need) {
        // every key equal to theta is kept (the usual case: one such key)
        *idx_cut = 0xFFFFFFFFu;
    } else {
        auto tie = [&](uint32_t i) -> uint32_t { return key(i) == th ? tie_idx_of(i) : 0xFFFFFFFFu; };
        *idx_cut = block_select<uint32_t>(tie, n1, need - 1, s_hist, s_sel);
    }
    *theta = th;
}

struct CandIdx {
    const float4* cand4;
    uint32_t qb;
    __device__ uint32_t operator()(uint32_t i) const { return __float_as_uint(cand4[qb + i].w); }
};

// Optional outputs (single frames, every leaf handled here): keep, score and
// stage in input order for every point of each leaf, as outputs_kernel
// writes them, so that pass is not needed.
struct ToplOut {
    uint8_t* keep;
    float* score;
    uint8_t* stage;
    __device__ void put(uint32_t i, uint8_t st, double sc) const {
        keep[i] = st == 3;
        score[i] = st >= 2 ? (float)sc : -1.0f;
        if (stage) stage[i] = st;
    }
};

__global__ __launch_bounds__(SEL_BLOCK) void topl_kernel(Plan P, double lambda, bool small, ToplOut out) {
    __shared__ uint32_t s_hist[256];
    __shared__ uint32_t s_sel[SEL_SCRATCH];
    __shared__ uint32_t s_cnt;
    __shared__ unsigned long long s_key[SEL_LDS_MAX];
    __shared__ uint32_t s_idx[SEL_LDS_MAX];
    __shared__ uint32_t s_list[SEL_BLOCK];
    __shared__ uint32_t s_lscan[SEL_BLOCK / 64 + 1];
    const uint32_t nl = P.ctr->n_leaves;
    for (uint32_t base = blockIdx.x; base < nl; base += gridDim.x * SEL_BLOCK) {
    const uint32_t nlist = block_leaf_round(P, base, nl, small, s_list, s_lscan, gridDim.x);
    for (uint32_t li = 0; li < nlist; ++li) {
        const uint32_t t = s_list[li];
        const uint32_t lb = P.leaf_begin[t], le = P.leaf_begin[t + 1];
        const uint32_t qb = P.p1pos[lb], qe = P.p1pos[le];
        const uint32_t n1 = qe - qb;
        if (small && n1 <= SMALL_LEAF) continue;  // topl_small_kernel
        // outputs of the leaf's points outside P1 (stage 0): for leaves of up to
        // 4 * SEL_BLOCK points their flags and indices are read here, beside
        // the P1 reads below, and written once those are in
        constexpr int NU = 4;
        const uint32_t nt = le - lb;
        const bool outs_b = out.keep && nt <= (uint32_t)NU * SEL_BLOCK;
        uint32_t f1[NU], oi[NU];
        if (outs_b) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const uint32_t s = lb + min(threadIdx.x + (uint32_t)u * SEL_BLOCK, nt - 1u);
                f1[u] = P.p1[s];
                oi[u] = P.idx_a[s];
            }
        }
        auto put_outside_p1 = [&]() {
            if (outs_b) {
#pragma unroll
                for (int u = 0; u < NU; ++u)
                    if (threadIdx.x + (uint32_t)u * SEL_BLOCK < nt && !f1[u]) out.put(oi[u], 0, 0.0);
            } else if (out.keep) {
                for (uint32_t s = lb + threadIdx.x; s < le; s += SEL_BLOCK)
                    if (!P.p1[s]) out.put(P.idx_a[s], 0, 0.0);
            }
        };
        if (n1 == 0) {
            put_outside_p1();
            if (threadIdx.x == 0) P.leaf_m[t] = 0;
            continue;
        }
        if (n1 <= SEL_BATCH_MAX) {
            // point i = threadIdx.x + u * SEL_BLOCK of the leaf in slot u of
            // each thread: every load first (a slot past n1 loads the last
            // point and is dropped), keys and indices staged in LDS and kept
            // in registers for the stage codes, |P2| counted on the way
            constexpr int SU = SEL_BATCH_MAX / SEL_BLOCK;
            uint32_t p2v[SU], ix[SU];
            double sv[SU];
            if (threadIdx.x == 0) s_cnt = 0;
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const uint32_t qi = qb + min(threadIdx.x + (uint32_t)u * SEL_BLOCK, n1 - 1u);
                p2v[u] = P.p2[qi];
                sv[u] = P.score_c[qi];
                ix[u] = __float_as_uint(P.cand4[qi].w);
            }
            // (an empty statement taking the loaded values keeps the compiler
            // from moving each load into the branch of its slot)
#pragma unroll
            for (int u = 0; u < SU; ++u) asm volatile("" ::"v"(p2v[u]), "v"(sv[u]), "v"(ix[u]));
            put_outside_p1();
            unsigned long long kv[SU];
            uint32_t c = 0;
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const uint32_t i = threadIdx.x + (uint32_t)u * SEL_BLOCK;
                kv[u] = score_key(p2v[u] != 0u, sv[u]);
                if (i < n1) {
                    s_key[i] = kv[u];
                    s_idx[i] = ix[u];
                    c += p2v[u] != 0u ? 1u : 0u;
                }
            }
            c = wave_sum(c);
            __syncthreads();  // s_cnt cleared
            if ((threadIdx.x & 63) == 0 && c) atomicAdd(&s_cnt, c);
            __syncthreads();
            const uint32_t n2 = s_cnt;
            uint32_t m = 0;
            if (n2 > 0) {
                const double mf = ceil(lambda * (double)n2);
                m = mf >= (double)n2 ? n2 : (uint32_t)mf;
            }
            unsigned long long theta = ~0ull;
            uint32_t idx_cut = 0;
            if (m > 0)
                topl_cut(LdsBits<unsigned long long>{s_key}, LdsBits<uint32_t>{s_idx}, n1, m, &theta, &idx_cut,
                         s_hist, s_sel, &s_cnt);
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const uint32_t i = threadIdx.x + (uint32_t)u * SEL_BLOCK;
                if (i >= n1) break;
                uint8_t st = 1;
                if (p2v[u]) {
                    const bool kept = m > 0 && (kv[u] > theta || (kv[u] == theta && ix[u] <= idx_cut));
                    st = kept ? 3 : 2;
                }
                P.stage_c[qb + i] = st;
                if (out.keep) out.put(ix[u], st, sv[u]);
            }
            if (threadIdx.x == 0) P.leaf_m[t] = m;
            __syncthreads();
            continue;
        }
        // larger leaves
        put_outside_p1();
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
            if (n1 <= SEL_LDS_MAX) {
                for (uint32_t i = threadIdx.x; i < n1; i += blockDim.x) {
                    s_key[i] = key(i);
                    s_idx[i] = __float_as_uint(P.cand4[qb + i].w);
                }
                __syncthreads();
                topl_cut(LdsBits<unsigned long long>{s_key}, LdsBits<uint32_t>{s_idx}, n1, m, &theta, &idx_cut,
                         s_hist, s_sel, &s_cnt);
            } else {
                topl_cut(key, CandIdx{P.cand4, qb}, n1, m, &theta, &idx_cut, s_hist, s_sel, &s_cnt);
            }
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
            if (out.keep) out.put(__float_as_uint(P.cand4[qi].w), st, st >= 2 ? P.score_c[qi] : 0.0);
        }
        if (threadIdx.x == 0) P.leaf_m[t] = m;
        __syncthreads();
    }
    __syncthreads();  // s_list is refilled by the next round
    }
}

// Small leaves: theta = the m-th largest key from a wave sort; keys above it
// are kept, and among the keys equal to it the `need` smallest indices.
__global__ __launch_bounds__(256) void topl_small_kernel(Plan P, double lambda) {
    __shared__ uint32_t s_hist[4][256];
    uint32_t* const hist = s_hist[threadIdx.x >> 6];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    const uint32_t nl = P.ctr->n_leaves;
    for (uint32_t t = wid; t < nl; t += nw) {
        const uint32_t qb = P.p1pos[P.leaf_begin[t]], qe = P.p1pos[P.leaf_begin[t + 1]];
        const uint32_t n1 = qe - qb;
        if (n1 > SMALL_LEAF) continue;
        WaveVals kv;
        uint32_t oi[4];
        uint32_t n2 = 0;
        // flags, scores and indices of the four points read at once (a slot
        // past n1 reads the last point and is dropped; an empty leaf reads none)
        uint32_t p2v[4] = {0u, 0u, 0u, 0u}, ixv[4] = {0u, 0u, 0u, 0u};
        double sv[4] = {0.0, 0.0, 0.0, 0.0};
        if (n1 > 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t qi = qb + min((uint32_t)j * 64u + lane, n1 - 1u);
                p2v[j] = P.p2[qi];
                sv[j] = P.score_c[qi];
                ixv[j] = __float_as_uint(P.cand4[qi].w);
            }
            // (an empty statement taking the loaded values keeps the compiler
            // from moving each load into the branch of its slot)
#pragma unroll
            for (int j = 0; j < 4; ++j) asm volatile("" ::"v"(p2v[j]), "v"(sv[j]), "v"(ixv[j]));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t i = (uint32_t)j * 64u + lane;
            const bool in = i < n1;
            kv.v[j] = in ? score_key(p2v[j] != 0u, sv[j]) : 0ull;
            oi[j] = in ? ixv[j] : 0xFFFFFFFFu;
            n2 += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(in && p2v[j] != 0u));
        }
        uint32_t m = 0;
        if (n2 > 0) {
            const double mf = ceil(lambda * (double)n2);
            m = mf >= (double)n2 ? n2 : (uint32_t)mf;
        }
        unsigned long long theta = ~0ull;
        uint32_t need = 0;
        bool ties_cut = false;
        if (m > 0) {
            WaveVals srt = kv;
            if (n1 <= 64u) {
                srt.v[0] = sort64_desc(srt.v[0], lane);
                const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)srt.v[0], (int)m - 1);
                const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(srt.v[0] >> 32), (int)m - 1);
                theta = ((unsigned long long)hi << 32) | lo;
            } else {
                theta = wave_select(kv.v, n1, n1 - m, lane, hist);  // the m-th largest
            }
            uint32_t greater = 0, equal = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool in = (uint32_t)j * 64u + lane < n1;
                greater += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(in && kv.v[j] > theta));
                equal += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(in && kv.v[j] == theta));
            }
            need = m - greater;
            ties_cut = equal > need;
        }
        // ties at theta ranked by original index (whole-wave ballots)
        uint32_t below[4] = {0u, 0u, 0u, 0u};
        if (ties_cut) {
#pragma unroll
            for (int j2 = 0; j2 < 4; ++j2) {
                unsigned long long e = __builtin_amdgcn_ballot_w64((uint32_t)j2 * 64u + lane < n1 && kv.v[j2] == theta);
                while (e) {
                    const int l = __ffsll((long long)e) - 1;
                    e &= e - 1ull;
                    const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)oi[j2], l);
#pragma unroll
                    for (int j = 0; j < 4; ++j) below[j] += o < oi[j] ? 1u : 0u;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t i = (uint32_t)j * 64u + lane;
            const bool kept = m > 0 && (kv.v[j] > theta || (kv.v[j] == theta && (!ties_cut || below[j] < need)));
            if (i < n1) P.stage_c[qb + i] = p2v[j] ? (kept ? 3 : 2) : 1;
        }
        if (lane == 0) P.leaf_m[t] = m;
    }
}

// Threshold mode: a P2 point is kept iff ln F >= thr (no ranking, no leaves).
__global__ __launch_bounds__(256) void threshold_kernel(Plan P, double thr) {
    const uint32_t np1 = P.ctr->n_p1;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < np1; q += gridDim.x * blockDim.x)
        P.stage_c[q] = P.p2[q] ? (log(P.score_c[q]) >= thr ? 3 : 2) : 1;
}

// Score module switched off: every P2 point is kept, none is scored.
__global__ __launch_bounds__(256) void keep_p2_kernel(Plan P) {
    const uint32_t np1 = P.ctr->n_p1;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < np1; q += gridDim.x * blockDim.x) {
        P.stage_c[q] = P.p2[q] ? 3 : 1;
        P.score_c[q] = -1.0;
    }
}

void launch_keep_p2(const Plan& P, hipStream_t st) {
    unsigned blocks = (P.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(keep_p2_kernel, dim3(blocks), dim3(256), 0, st, P);
}

bool launch_topl(const Plan& P, const Params& prm, uint8_t* keep, float* score, uint8_t* stage, hipStream_t st) {
    if (!std::isnan(prm.log_thr)) {
        unsigned blocks = (P.n + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        if (blocks == 0) blocks = 1;
        hipLaunchKernelGGL(threshold_kernel, dim3(blocks), dim3(256), 0, st, P, prm.log_thr);
        return false;
    }
    const bool small = P.n > SMALL_PATH_MIN_N;
    if (small) {
        unsigned wb = (P.n / 128 + 3) / 4;
        if (wb > 8192) wb = 8192;
        hipLaunchKernelGGL(topl_small_kernel, dim3(wb), dim3(256), 0, st, P, prm.keep_ratio);
    }
    unsigned blocks = P.n < 2048 ? P.n : 2048;
    if (blocks == 0) blocks = 1;
    // up to 2^20 points every leaf passes through topl_kernel, which then
    // writes the outputs too (large inputs scatter them as packed records)
    const bool write = !small && P.n <= PACKED_OUT_MIN_N;
    const ToplOut out{write ? keep : nullptr, score, stage};
    hipLaunchKernelGGL(topl_kernel, dim3(blocks), dim3(SEL_BLOCK), 0, st, P, prm.keep_ratio, small, out);
    return write;
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

// Large inputs: the outputs go out in two steps. outputs_pack_kernel
// scatters one 8-byte record per point to its original index (one random
// line per point instead of one per output array), and the keep scan, which
// reads every point in input order anyway, writes the three output arrays
// from the records as it loads them (coalesced). Each XCD takes one eighth of
// the positions, so the lines of a frame's records are written whole in one
// XCD's L2.
__global__ __launch_bounds__(256) void outputs_pack_kernel(Plan P) {
    const XcdPart R = xcd_part(P.n);
    for (uint32_t s = R.first; s < R.end; s += R.step) {
        uint32_t st = 0;
        float sc = -1.0f;
        if (P.p1[s]) {
            const uint32_t qi = P.p1pos[s];
            st = P.stage_c[qi];
            if (st >= 2) sc = (float)P.score_c[qi];
        }
        P.outrec[P.idx_a[s]] = make_uint2(__float_as_uint(sc), st);
    }
}

struct PackedKeepGet {
    const uint2* rec;
    uint8_t* keep;
    float* score;
    uint8_t* stage;
    __device__ uint32_t operator()(uint32_t i) const {
        const uint2 r = rec[i];
        const uint32_t k = r.y == 3u ? 1u : 0u;
        keep[i] = (uint8_t)k;
        score[i] = __uint_as_float(r.x);
        if (stage) stage[i] = (uint8_t)r.y;
        return k;
    }
};
template <>
struct ScanGetWrites<PackedKeepGet> {
    static constexpr bool value = true;
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

// Batches: the scan records each point's count of kept points before it;
// kept point i of frame f then lands at kept_idx[foff[f] + its rank within
// the frame] as the frame-local index i - foff[f].
struct BatchKeepEmit {
    uint32_t* keep_ex;
    __device__ void operator()(uint32_t i, uint32_t ex, uint32_t) const { keep_ex[i] = ex; }
};
struct BatchKeepFin {
    Counters* c;
    uint32_t* keep_ex;
    uint32_t n;
    __device__ void operator()(uint32_t total) const {
        c->n_kept = total;
        keep_ex[n] = total;
    }
};

__global__ __launch_bounds__(256) void kept_frames_kernel(Plan P, const uint8_t* keep, uint32_t* kept_idx,
                                                          int64_t* n_kept) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
    for (uint32_t i = tid; i < P.n; i += nt) {
        if (keep[i]) {
            const uint32_t f = P.fid[i], fs = P.foff[f];
            kept_idx[fs + (P.keep_ex[i] - P.keep_ex[fs])] = i - fs;
        }
    }
    for (uint32_t f = tid; f < P.nf; f += nt) n_kept[f] = (int64_t)(P.keep_ex[P.foff[f + 1]] - P.keep_ex[P.foff[f]]);
}

void launch_outputs(const Plan& P, uint8_t* keep, float* score, uint8_t* stage, uint32_t* kept_idx,
                    int64_t* n_kept, hipStream_t st, bool written) {
    unsigned blocks = (P.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    uint32_t* const sstat = P.scan_status + 2 * (size_t)P.scan_tiles;
    if (P.n > PACKED_OUT_MIN_N) {
        hipLaunchKernelGGL(outputs_pack_kernel, dim3(xcd_grid(blocks)), dim3(256), 0, st, P);
        const PackedKeepGet get{P.outrec, keep, score, stage};
        if (P.nf == 1)
            launch_scan(get, KeepEmit{kept_idx}, KeepFin{P.ctr, n_kept}, nullptr, P.n, sstat, &P.ctr->status, st);
        else
            launch_scan(get, BatchKeepEmit{P.keep_ex}, BatchKeepFin{P.ctr, P.keep_ex, P.n}, nullptr, P.n, sstat,
                        &P.ctr->status, st);
    } else {
        if (!written) hipLaunchKernelGGL(outputs_kernel, dim3(blocks), dim3(256), 0, st, P, keep, score, stage);
        if (P.nf == 1)
            launch_scan(KeepGet{keep}, KeepEmit{kept_idx}, KeepFin{P.ctr, n_kept}, nullptr, P.n, sstat,
                        &P.ctr->status, st);
        else
            launch_scan(KeepGet{keep}, BatchKeepEmit{P.keep_ex}, BatchKeepFin{P.ctr, P.keep_ex, P.n}, nullptr, P.n,
                        sstat, &P.ctr->status, st);
    }
    if (P.nf > 1) hipLaunchKernelGGL(kept_frames_kernel, dim3(blocks), dim3(256), 0, st, P, keep, kept_idx, n_kept);
}

__global__ void write_zero_counts_kernel(int64_t* n_kept, uint32_t nf) {
    for (uint32_t f = threadIdx.x; f < nf; f += blockDim.x) n_kept[f] = 0;
}

void launch_write_zero_count(int64_t* n_kept, uint32_t nf, hipStream_t st) {
    hipLaunchKernelGGL(write_zero_counts_kernel, dim3(1), dim3(256), 0, st, n_kept, nf);
}

}  // namespace gdn
