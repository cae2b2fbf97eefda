// Leaf-local brute-force kNN with halo candidates (Sec. 3: N_K(i), d_ij and
// r_K,i on the voxel-filtered set P1).
//
// One wave per work item (64 queries, one per lane); the candidate stream
// has wave-uniform addresses and comes through the scalar cache. Squared distances are fp32 (dx*dx + dy*dy) + dz*dz without
// contraction, so the neighbour sets are exact. Each lane keeps its k best
// (d2, original index) pairs as sorted 64-bit keys (d2 bits << 32 | index) in
// registers, updated by a fully unrolled insertion network; a list of KMAX
// slots serves any k <= KMAX by parking KMAX - k sentinel keys (-1) in front.
//
// Bound (knn_bound_kernel, once per query tile): tau = the largest d2 to k
// points next to the query in Morton order inside its own leaf; then, over a
// window of the leaf's points around the tile, count the candidates under
// tau * 2^(-m/2) and keep the smallest such threshold still holding k of them.
// Those are candidates, so the k-th nearest distance is <= tau: the scan's
// list starts as k placeholder keys (tau, 0xFFFFFFFF) and only candidates with
// d2 <= tau can ever enter it. The result is unchanged; the insertion path
// runs far less.
//
// Leaves with many candidates are split into chunks processed by different
// workgroups; each writes its partial list and the last chunk of a query tile
// to finish (arrival counter, device-scope fences, no waiting) inserts the
// other chunks' entries into its own list.
#include <climits>

#include "kernels.hpp"

namespace gdn {

constexpr uint32_t NONE32 = 0xFFFFFFFFu;

__device__ __forceinline__ float dist2(const float4 q, const float4 c) {
    const float dx = c.x - q.x, dy = c.y - q.y, dz = c.z - q.z;
    return (dx * dx + dy * dy) + dz * dz;
}

template <int KMAX>
__device__ __forceinline__ void topk_insert(long long (&a)[KMAX], const long long key) {
#pragma unroll
    for (int i = KMAX - 1; i >= 1; --i) {
        const long long lo = key < a[i] ? key : a[i];
        a[i] = a[i - 1] > lo ? a[i - 1] : lo;
    }
    a[0] = key < a[0] ? key : a[0];
}

template <int KMAX>
__device__ __forceinline__ void try_insert(long long (&a)[KMAX], float& worst, const float d,
                                           const float cw, const uint32_t self) {
    const uint32_t ci = __float_as_uint(cw);
    // sign bit cleared: keys stay >= 0 even for a NaN distance (non-finite input)
    const long long key = ((long long)(__float_as_uint(d) & 0x7FFFFFFFu) << 32) | (long long)ci;
    if (key < a[KMAX - 1] && ci != self) {
        topk_insert<KMAX>(a, key);
        worst = __uint_as_float((uint32_t)((unsigned long long)a[KMAX - 1] >> 32));
    }
}

// A list entry is real unless it is the empty key or a tau placeholder.
__device__ __forceinline__ bool real_entry(long long v) {
    return v != LLONG_MAX && (uint32_t)v != NONE32;
}

__device__ __forceinline__ void write_final(const Plan& P, uint32_t qi, int k, int r, long long v) {
    const bool ok = real_entry(v);
    const float d = ok ? __uint_as_float((uint32_t)((unsigned long long)v >> 32)) : INFINITY;
    P.nbr[(size_t)qi * k + r] = ok ? (uint32_t)v : NONE32;
    P.nbr_d2[(size_t)qi * k + r] = d;
    if (r == k - 1) P.r2k[qi] = d;
}

constexpr int BOUND_MARGIN = 64;   // window reaches this far on each side of a query
constexpr int BOUND_LEVELS = 10;   // thresholds tau * 2^(-m/2), m = 1..10

// tau for query qi (one lane): -1 when the leaf has <= k P1 points.
__device__ float query_bound(const float4* __restrict__ cand4, uint32_t qb, uint32_t qe, uint32_t qi, int k) {
    if (qe - qb <= (uint32_t)k) return -1.0f;
    const float4 q = cand4[qi];
    uint32_t s0 = (qi - qb > (uint32_t)(k / 2)) ? qi - (uint32_t)(k / 2) : qb;
    if (s0 + (uint32_t)k + 1u > qe) s0 = qe - (uint32_t)k - 1u;
    float tau = 0.0f;
    for (uint32_t j = s0; j <= s0 + (uint32_t)k; ++j)
        if (j != qi) tau = fmaxf(tau, dist2(q, cand4[j]));
    float th[BOUND_LEVELS];
    uint32_t cnt[BOUND_LEVELS];
    float f = tau;
#pragma unroll
    for (int m = 0; m < BOUND_LEVELS; ++m) {
        f = f * 0.70710678f;
        th[m] = f;
        cnt[m] = 0;
    }
    const uint32_t wlo = (qi - qb > (uint32_t)BOUND_MARGIN) ? qi - (uint32_t)BOUND_MARGIN : qb;
    const uint32_t whi = min(qe, qi + (uint32_t)BOUND_MARGIN + 1u);
    for (uint32_t j = wlo; j < whi; ++j) {
        const float d = dist2(q, cand4[j]);
        const uint32_t notself = (j != qi) ? 1u : 0u;
#pragma unroll
        for (int m = 0; m < BOUND_LEVELS; ++m) cnt[m] += (d <= th[m]) ? notself : 0u;
    }
    float best = tau;
#pragma unroll
    for (int m = 0; m < BOUND_LEVELS; ++m)
        if (cnt[m] >= (uint32_t)k) best = th[m];
    return best;
}

// One wave per query tile (the chunk-0 item of each tile).
__global__ __launch_bounds__(256) void knn_bound_kernel(Plan P, const float4* __restrict__ cand4, int k) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t n_items = P.ctr->n_items;
    for (uint32_t it = wave; it < n_items; it += nwaves) {
        const KnnItem w = P.items[it];
        if (w.chunk != 0) continue;
        const uint32_t t = w.leaf;
        const uint32_t qb = P.p1pos[P.leaf_begin[t]], qe = P.p1pos[P.leaf_begin[t + 1]];
        const uint32_t qi = w.q0 + lane;
        if (qi < w.q1) P.tau_c[qi] = query_bound(cand4, qb, qe, qi, k);
    }
}

template <int KMAX>
__device__ __forceinline__ void test4(long long (&a)[KMAX], float& worst, const uint32_t self, const bool vq,
                                      const float d0, const float d1, const float d2, const float d3,
                                      const float w0, const float w1, const float w2, const float w3) {
    const float dm = fminf(fminf(d0, d1), fminf(d2, d3));
    if (vq && !(dm > worst)) {
        try_insert<KMAX>(a, worst, d0, w0, self);
        try_insert<KMAX>(a, worst, d1, w1, self);
        try_insert<KMAX>(a, worst, d2, w2, self);
        try_insert<KMAX>(a, worst, d3, w3, self);
    }
}

template <int KMAX>
__device__ __forceinline__ void scan4(long long (&a)[KMAX], float& worst, const float4 q, const uint32_t self,
                                      const bool vq, const float4 c0, const float4 c1, const float4 c2,
                                      const float4 c3) {
    const float d0 = dist2(q, c0), d1 = dist2(q, c1), d2 = dist2(q, c2), d3 = dist2(q, c3);
    const float dm = fminf(fminf(d0, d1), fminf(d2, d3));
    if (vq && !(dm > worst)) {
        try_insert<KMAX>(a, worst, d0, c0.w, self);
        try_insert<KMAX>(a, worst, d1, c1.w, self);
        try_insert<KMAX>(a, worst, d2, c2.w, self);
        try_insert<KMAX>(a, worst, d3, c3.w, self);
    }
}

// One wave per work item; waves of a block are independent. Item scalars and
// the candidate stream have wave-uniform addresses, so they come through the
// scalar cache into SGPRs and feed the VALU directly.
template <int KMAX>
__global__ __launch_bounds__(256) void knn_kernel(Plan P, const float4* __restrict__ cand4, int k) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t n_items = P.ctr->n_items;
    for (;;) {
        uint32_t got = 0;
        if (lane == 0) got = atomicAdd(&P.ctr->knn_next, 1u);
        const uint32_t it = __builtin_amdgcn_readfirstlane(__shfl(got, 0, 64));
        if (it >= n_items) break;
        const KnnItem w = P.items[it];
        const uint32_t t = w.leaf;
        const uint32_t nr = P.leaf_nr[t];
        const uint32_t ncand = P.leaf_ncand[t], nch = P.leaf_nch[t], cc = P.leaf_cc[t];
        const uint32_t qb = P.p1pos[P.leaf_begin[t]];
        const uint32_t qi = w.q0 + lane;
        const bool vq = qi < w.q1;
        const float4 q = vq ? cand4[qi] : make_float4(0.f, 0.f, 0.f, 0.f);
        const uint32_t self = __float_as_uint(q.w);
        const float tb = vq ? P.tau_c[qi] : -1.0f;
        const bool has_tau = tb >= 0.0f;
        const long long init =
            has_tau ? (((long long)(__float_as_uint(tb) & 0x7FFFFFFFu) << 32) | (long long)NONE32) : LLONG_MAX;
        long long a[KMAX];
#pragma unroll
        for (int r = 0; r < KMAX; ++r) a[r] = (r < KMAX - k) ? -1ll : init;
        float worst = has_tau ? tb : __uint_as_float(0x7FFFFFFFu);  // NaN: no bound yet

        // walk the chunk [c_lo, c_hi) of the leaf's concatenated candidate ranges
        const uint32_t c_lo = w.chunk * cc;
        const uint32_t c_hi = min(ncand, c_lo + cc);
        uint32_t pre = 0;
        for (uint32_t r = 0; r < nr && pre < c_hi; ++r) {
            const uint2 R = P.leaf_ranges[(size_t)t * HALO + r];
            const uint32_t len = R.y - R.x;
            const uint32_t s = max(c_lo, pre), e = min(c_hi, pre + len);
            if (s < e) {
                const float4* cp = cand4 + (R.x + (s - pre));
                const float4* const cend = cand4 + (R.x + (e - pre));
                if (cp + 8 <= cend) {
                    // software pipeline: the next 8 candidates are requested
                    // after this group's distances, so their scalar loads are
                    // in flight while this group is tested
                    float4 n0 = cp[0], n1 = cp[1], n2 = cp[2], n3 = cp[3];
                    float4 n4 = cp[4], n5 = cp[5], n6 = cp[6], n7 = cp[7];
                    for (;;) {
                        const float d0 = dist2(q, n0), d1 = dist2(q, n1), d2 = dist2(q, n2), d3 = dist2(q, n3);
                        const float d4 = dist2(q, n4), d5 = dist2(q, n5), d6 = dist2(q, n6), d7 = dist2(q, n7);
                        const float w0 = n0.w, w1 = n1.w, w2 = n2.w, w3 = n3.w;
                        const float w4 = n4.w, w5 = n5.w, w6 = n6.w, w7 = n7.w;
                        cp += 8;
                        const bool more = cp + 8 <= cend;
                        __builtin_amdgcn_sched_barrier(0);
                        if (more) {
                            n0 = cp[0]; n1 = cp[1]; n2 = cp[2]; n3 = cp[3];
                            n4 = cp[4]; n5 = cp[5]; n6 = cp[6]; n7 = cp[7];
                        }
                        __builtin_amdgcn_sched_barrier(0);
                        test4<KMAX>(a, worst, self, vq, d0, d1, d2, d3, w0, w1, w2, w3);
                        test4<KMAX>(a, worst, self, vq, d4, d5, d6, d7, w4, w5, w6, w7);
                        if (!more) break;
                    }
                }
                for (; cp < cend; ++cp) {
                    const float4 c0 = cp[0];
                    const float d0 = dist2(q, c0);
                    if (vq && !(d0 > worst)) try_insert<KMAX>(a, worst, d0, c0.w, self);
                }
            }
            pre += len;
        }

        bool write_out = nch == 1;
        if (nch > 1) {
            // partial lists of a tile, laid out [chunk][r][query]: coalesced
            const uint32_t m = w.q1 - w.q0;
            long long* tb_ = (long long*)P.plist + ((size_t)P.leaf_plist[t] + (size_t)(w.q0 - qb) * nch) * (size_t)k;
            if (vq) {
#pragma unroll
                for (int r = 0; r < KMAX; ++r)
                    if (r >= KMAX - k) tb_[((size_t)w.chunk * k + (r - (KMAX - k))) * m + lane] = a[r];
            }
            __threadfence();
            uint32_t last = 0;
            if (lane == 0) last = (atomicAdd(&P.tile_done[w.grp], 1u) == nch - 1u) ? 1u : 0u;
            last = __builtin_amdgcn_readfirstlane(__shfl(last, 0, 64));
            if (last) {
                // last chunk of this tile to finish: insert the other chunks'
                // entries (sorted; stop at the first that cannot enter)
                __threadfence();
                write_out = true;
                if (vq) {
                    for (uint32_t c = 0; c < nch; ++c) {
                        if (c == w.chunk) continue;
                        for (int r = 0; r < k; ++r) {
                            const long long v = tb_[((size_t)c * k + r) * m + lane];
                            if (!real_entry(v) || !(v < a[KMAX - 1])) break;
                            topk_insert<KMAX>(a, v);
                        }
                    }
                }
            }
        }
        if (write_out && vq) {
#pragma unroll
            for (int r = 0; r < KMAX; ++r)
                if (r >= KMAX - k) write_final(P, qi, k, r - (KMAX - k), a[r]);
        }
    }
}

template <int KMAX>
static void launch_knn_t(const Plan& P, int k, int num_cus, hipStream_t st) {
    const unsigned blocks = (unsigned)(num_cus > 0 ? num_cus : 256) * 4u;
    hipLaunchKernelGGL(knn_kernel<KMAX>, dim3(blocks), dim3(256), 0, st, P, (const float4*)P.cand4, k);
}

void launch_knn_bound(const Plan& P, int k, int num_cus, hipStream_t st) {
    const unsigned blocks = (unsigned)(num_cus > 0 ? num_cus : 256) * 4u;
    hipLaunchKernelGGL(knn_bound_kernel, dim3(blocks), dim3(256), 0, st, P, (const float4*)P.cand4, k);
}

void launch_knn(const Plan& P, int k, int num_cus, hipStream_t st) {
    if (k <= 8) launch_knn_t<8>(P, k, num_cus, st);
    else if (k <= 16) launch_knn_t<16>(P, k, num_cus, st);
    else if (k <= 32) launch_knn_t<32>(P, k, num_cus, st);
    else launch_knn_t<64>(P, k, num_cus, st);
}

}  // namespace gdn
