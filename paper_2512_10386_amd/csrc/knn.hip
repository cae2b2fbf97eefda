// Leaf-local brute-force kNN with halo candidates (Sec. 3: N_K(i), d_ij and
// r_K,i on the voxel-filtered set P1).
//
// Work item = (leaf, up to 16 queries, candidate chunk), one wave each.
// Lane-per-candidate: each lane holds 8 candidates of a 512-candidate block
// (coalesced loads, the next block prefetched), reused for the item's 16
// queries, whose coordinates are wave-uniform (scalar loads). Squared
// distances are fp32 (dx*dx + dy*dy) + dz*dz without contraction, so the
// neighbour sets are exact.
//
// Each query keeps, in LDS, its k best (d2, original index) keys (d2 bits <<
// 32 | index), sorted, one per lane when loaded, and a pending buffer of up
// to 64 candidates (their P1 positions, 4 bytes each: the keys are rebuilt
// when the buffer is merged, which halves the LDS a wave needs). A candidate block is tested against the query's current k-th
// distance with one compare per lane; the candidates that pass are appended
// to the pending buffer (ballot + lane rank). A full buffer, and the buffer
// at the end of the chunk, is merged into the list: the 64 pending keys are
// sorted descending by a wave-wide bitonic network, the elementwise minimum
// with the ascending list holds the 64 smallest keys of both as a bitonic
// sequence, and six more exchange steps sort it. The list keeps the first k.
// When k <= 32, buffers holding at most 32 keys at the end of an item are
// merged on 32-lane halves, two queries at once (15 + 5 exchange steps for
// both instead of 21 + 6 for one).
//
// Bound: knn_bound_kernel gives each query tau >= its k-th squared distance
// (from k of its own candidates), so its list starts as k placeholder keys
// (tau, 0xFFFFFFFF) and only candidates with d2 <= tau can ever enter. The
// result is unchanged.
//
// Leaves with many candidates are split into chunks processed as separate
// items; each writes its partial lists, which knn_merge_kernel combines after
// this kernel. (Combining them here would need device-scope release/acquire
// between waves, which on this chip writes back the L2 of the releasing XCD
// on every chunk.)
#include <climits>

#include "kernels.hpp"
#include "wave.hpp"

namespace gdn {

constexpr uint32_t NONE32 = 0xFFFFFFFFu;
constexpr unsigned long long KEY_EMPTY = (unsigned long long)LLONG_MAX;
constexpr int QPW = KNN_TQ;  // queries per wave item
constexpr int CPL = 8;       // candidates per lane per block
constexpr int CBLK = 64 * CPL;
constexpr int PEND = 64;     // pending keys per query
constexpr int PEND_HALF = 32;  // pending keys a half-wave merge takes (k <= 32)
constexpr uint32_t KNN_POS_MIN_N = 1u << 20;  // above: pending buffers of positions

__device__ __forceinline__ float dist2(const float4 q, const float4 c) {
    const float dx = c.x - q.x, dy = c.y - q.y, dz = c.z - q.z;
    return (dx * dx + dy * dy) + dz * dz;
}

// A list entry is real unless it is the empty key or a tau placeholder.
__device__ __forceinline__ bool real_entry(unsigned long long v) {
    return v != KEY_EMPTY && (uint32_t)v != NONE32;
}

__device__ __forceinline__ unsigned long long make_key(float d, uint32_t idx) {
    // sign bit cleared: keys stay >= 0 even for a NaN distance (non-finite input)
    return ((unsigned long long)(__float_as_uint(d) & 0x7FFFFFFFu) << 32) | idx;
}

__device__ __forceinline__ unsigned long long read_lane64(unsigned long long v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long shfl64(unsigned long long v, int src_lane) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src_lane, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src_lane, 64);
    return ((unsigned long long)hi << 32) | lo;
}

// ---------------------------------------------------------------- bound

constexpr int BOUND_MARGIN = 64;   // window reaches this far on each side of a query
constexpr int BOUND_SPLIT = 8;     // adjacent lanes sharing one query's distances
// Threshold ladders: tau * 2^(-m/2), m = 1..10, for single frames; tau * 2^-m,
// m = 1..5, above 1M points (small leaves: the coarser ladder costs the bound
// less than it costs the kNN there).
constexpr uint32_t BOUND_COARSE_MIN_N = 1u << 20;
constexpr int BOUND_Q = 128;       // queries per block (BOUND_Q * BOUND_SPLIT threads)
static_assert(BOUND_Q % KNN_GRP == 0, "a bound block covers whole culling groups");

// tau: the largest d2 to the k points next to the query in Morton order inside
// [qb, qe), a run of candidates holding the query; then, over the run's points
// within BOUND_MARGIN positions, count those under each rung of the ladder
// (LEVELS rungs, each the previous times STEP) and keep the smallest threshold
// still holding k. -1 when the run has <= k points.
// The BOUND_SPLIT lanes of a query each take every BOUND_SPLIT-th point and
// combine their maxima and counts (exact, so tau does not depend on the
// split); every lane of the wave calls this, `run` false for idle ones.
template <int LEVELS, class Pts>
__device__ float query_bound(Pts cand4, uint32_t qb, uint32_t qe, uint32_t qi, int k, uint32_t sub, bool live) {
    constexpr float STEP = LEVELS == 10 ? 0.70710678f : 0.5f;
    static_assert(LEVELS == 10 || LEVELS == 5, "ladder");
    const bool run = live && qe - qb > (uint32_t)k;
    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t s0 = 0, s1 = 0, wlo = 0, whi = 0;
    if (run) {
        q = cand4[qi];
        s0 = (qi - qb > (uint32_t)(k / 2)) ? qi - (uint32_t)(k / 2) : qb;
        if (s0 + (uint32_t)k + 1u > qe) s0 = qe - (uint32_t)k - 1u;
        s1 = s0 + (uint32_t)k + 1u;
        wlo = (qi - qb > (uint32_t)BOUND_MARGIN) ? qi - (uint32_t)BOUND_MARGIN : qb;
        whi = min(qe, qi + (uint32_t)BOUND_MARGIN + 1u);
    }
    float tau = 0.0f;
    for (uint32_t j = s0 + sub; j < s1; j += BOUND_SPLIT)
        if (j != qi) tau = fmaxf(tau, dist2(q, cand4[j]));
#pragma unroll
    for (int o = 1; o < BOUND_SPLIT; o <<= 1) tau = fmaxf(tau, __shfl_xor(tau, o, 64));
    float th[LEVELS];
    uint32_t cnt[LEVELS];
    float f = tau;
#pragma unroll
    for (int m = 0; m < LEVELS; ++m) {
        f = f * STEP;
        th[m] = f;
        cnt[m] = 0;
    }
    for (uint32_t j = wlo + sub; j < whi; j += BOUND_SPLIT) {
        const float d = dist2(q, cand4[j]);
        const uint32_t notself = (j != qi) ? 1u : 0u;
#pragma unroll
        for (int m = 0; m < LEVELS; ++m) cnt[m] += (d <= th[m]) ? notself : 0u;
    }
    float best = tau;
#pragma unroll
    for (int m = 0; m < LEVELS; ++m) {
#pragma unroll
        for (int o = 1; o < BOUND_SPLIT; o <<= 1) cnt[m] += (uint32_t)__shfl_xor((int)cnt[m], o, 64);
        if (cnt[m] >= (uint32_t)k) best = th[m];
    }
    return run ? best : -1.0f;
}

// Points [lo, lo + count) of the P1 order, staged in LDS.
struct StagedPts {
    const float4* s;
    uint32_t lo;
    __device__ float4 operator[](uint32_t j) const { return s[j - lo]; }
};

// BOUND_SPLIT lanes per P1 point: its bound, and, for the first query of each
// tile, the tile's work items (one per candidate chunk) at the queue position
// the plan gave the leaf. A block takes BOUND_Q consecutive queries; every
// window lies within BOUND_MARGIN of its query, so the block stages those
// points.
template <int LEVELS>
__global__ __launch_bounds__(BOUND_Q * BOUND_SPLIT) void knn_bound_kernel(Plan P, const float4* __restrict__ cand4,
                                                                         int k) {
    __shared__ float4 s_pts[BOUND_Q + 2 * BOUND_MARGIN + 1];
    const uint32_t np1 = P.ctr->n_p1;
    const uint32_t sub = threadIdx.x % BOUND_SPLIT, ql = threadIdx.x / BOUND_SPLIT;
    for (uint32_t q_first = blockIdx.x * BOUND_Q; q_first < np1; q_first += gridDim.x * BOUND_Q) {
        const uint32_t lo = q_first > (uint32_t)BOUND_MARGIN ? q_first - (uint32_t)BOUND_MARGIN : 0u;
        const uint32_t hi = min(np1, q_first + BOUND_Q + (uint32_t)BOUND_MARGIN + 1u);
        for (uint32_t j = lo + threadIdx.x; j < hi; j += blockDim.x) s_pts[j - lo] = cand4[j];
        __syncthreads();
        {
            // the boxes of the culling groups among this block's queries (q_first
            // is a multiple of KNN_GRP), one wave per group
            const uint32_t wv = threadIdx.x / 64u, ln = threadIdx.x % 64u;
            const uint32_t g0 = q_first + wv * (uint32_t)KNN_GRP;
            if (wv < (uint32_t)(BOUND_Q / KNN_GRP) && g0 < np1) {
                const uint32_t p = g0 + ln;
                const bool ok = p < np1;
                const float4 c = ok ? s_pts[p - lo] : make_float4(0.f, 0.f, 0.f, 0.f);
                const float lx = wave_min(ok ? c.x : INFINITY, ln), ly = wave_min(ok ? c.y : INFINITY, ln),
                            lz = wave_min(ok ? c.z : INFINITY, ln);
                const float hx = wave_max(ok ? c.x : -INFINITY, ln), hy = wave_max(ok ? c.y : -INFINITY, ln),
                            hz = wave_max(ok ? c.z : -INFINITY, ln);
                if (ln == 0u)
                    P.gbox[g0 / (uint32_t)KNN_GRP] = GroupBox{make_float4(lx, ly, lz, 0.f), make_float4(hx, hy, hz, 0.f)};
            }
        }
        const uint32_t qi = q_first + ql;
        const bool live = qi < np1;
        uint32_t t = 0, qb = 0, qe = 0, rb = 0, re = 0;
        if (live) {
            t = P.cand_leaf[qi];
            qb = P.p1pos[P.leaf_begin[t]];
            qe = P.p1pos[P.leaf_begin[t + 1]];
            // the window lives in the merged candidate range holding the query,
            // which may reach past a small leaf (every point of it is a candidate)
            rb = qb;
            re = qe;
            const uint32_t nr = P.leaf_nr[t];
            for (uint32_t r = 0; r < nr; ++r) {
                const uint2 R = P.leaf_ranges[(size_t)t * HALO + r];
                if (R.x <= qi && qi < R.y) {
                    rb = R.x;
                    re = R.y;
                    break;
                }
            }
        }
        const float b = query_bound<LEVELS>(StagedPts{s_pts, lo}, rb, re, qi, k, sub, live);
        if (live && sub == 0u) {
            P.tau_c[qi] = b;
            if ((qi - qb) % (uint32_t)KNN_TQ == 0u) {
                const uint32_t nch = P.leaf_nch[t];
                const uint32_t grp = P.leaf_item[t] + ((qi - qb) / (uint32_t)KNN_TQ) * nch;
                const uint32_t q1 = min(qe, qi + (uint32_t)KNN_TQ);
                for (uint32_t c = 0; c < nch; ++c) P.items[grp + c] = KnnItem{t, qi, q1, c, grp, 0u};
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- kNN

__device__ __forceinline__ void write_final(const Plan& P, uint32_t qi, uint32_t k, uint32_t lane,
                                            unsigned long long v) {
    const bool ok = lane < k && real_entry(v);
    const float d = ok ? __uint_as_float((uint32_t)(v >> 32)) : INFINITY;
    const float d1 = __shfl(d, k >= 2u ? (int)k - 2 : 0, 64);
    if (lane < k) {
        P.nbr[(size_t)qi * k + lane] = ok ? (uint32_t)v : NONE32;
        P.nbr_d2[(size_t)qi * k + lane] = d;
        // the k-th entry and the (k-1)-th distance again, densely, for the density
        if (lane == k - 1) P.krec[qi] = make_uint4(ok ? (uint32_t)v : NONE32, __float_as_uint(d1), __float_as_uint(d), 0u);
    }
}

// Distance bound of a list whose k-th key is v: +inf while the list holds
// fewer than k keys.
__device__ __forceinline__ float bound_of(uint32_t hi) {
    return hi == 0x7FFFFFFFu ? INFINITY : __uint_as_float(hi);
}

// Coordinates of query j of a tile (lane j holds them).
__device__ __forceinline__ float4 query_of(float4 qv, uint32_t j) {
    return make_float4(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(qv.x), (int)j)),
                       __int_as_float(__builtin_amdgcn_readlane(__float_as_int(qv.y), (int)j)),
                       __int_as_float(__builtin_amdgcn_readlane(__float_as_int(qv.z), (int)j)), 0.f);
}

// Pending buffers hold either the keys themselves (POS = false) or the
// candidates' P1 positions (POS = true, half the LDS: more waves per CU, one
// gather per merge). A position's key is rebuilt with the same fp32
// expression as in the hot loop, so it is bit-identical to the one that
// passed the test.
template <bool POS>
struct Pending {
    using T = unsigned long long;
};
template <>
struct Pending<true> {
    using T = uint32_t;
};

template <bool POS>
__device__ __forceinline__ unsigned long long pending_key(const float4* __restrict__ cand4,
                                                          const typename Pending<POS>::T* __restrict__ pend,
                                                          uint32_t e, float4 q) {
    if constexpr (POS) {
        const float4 c = cand4[pend[e]];
        return make_key(dist2(q, c), __float_as_uint(c.w));
    } else {
        return pend[e];
    }
}

// Merge query j's pending candidates into its list, dropping the query's own
// key (the hot loop does not test for it); returns the new distance bound.
template <bool POS>
__device__ __forceinline__ float flush(unsigned long long* __restrict__ lst,
                                       const typename Pending<POS>::T* __restrict__ pend, uint32_t cnt,
                                       uint32_t lane, uint32_t k, unsigned long long selfkey,
                                       const float4* __restrict__ cand4, float4 q) {
    wave_lds_fence();
    unsigned long long v = lane < cnt ? pending_key<POS>(cand4, pend, lane, q) : KEY_EMPTY;
    if (v == selfkey) v = KEY_EMPTY;
    const unsigned long long L = lane < k ? lst[lane] : KEY_EMPTY;
    v = sort64_desc(v, lane);
    v = merge64_asc(L < v ? L : v, lane);
    if (lane < k) lst[lane] = v;
    wave_lds_fence();
    return bound_of((uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)k - 1));
}

// k <= 32: the lists of two queries, one per 32-lane half (`two` = false:
// only the lower half's query). Each half merges at most 32 pending keys.
// Returns the new bounds of both through b0 / b1.
template <bool POS>
__device__ __forceinline__ void flush_half(unsigned long long* __restrict__ lst0,
                                           const typename Pending<POS>::T* __restrict__ pend0,
                                           uint32_t cnt0, unsigned long long self0, float4 q0,
                                           unsigned long long* __restrict__ lst1,
                                           const typename Pending<POS>::T* __restrict__ pend1,
                                           uint32_t cnt1, unsigned long long self1, float4 q1, bool two,
                                           uint32_t lane, uint32_t k, const float4* __restrict__ cand4, float* b0,
                                           float* b1) {
    wave_lds_fence();
    const bool up = lane >= 32u;
    const uint32_t h = lane & 31u;
    const bool act = !up || two;
    unsigned long long* const lst = up ? lst1 : lst0;
    const typename Pending<POS>::T* const pend = up ? pend1 : pend0;
    const uint32_t cnt = up ? cnt1 : cnt0;
    unsigned long long v = act && h < cnt ? pending_key<POS>(cand4, pend, h, up ? q1 : q0) : KEY_EMPTY;
    if (v == (up ? self1 : self0)) v = KEY_EMPTY;
    const unsigned long long L = act && h < k ? lst[h] : KEY_EMPTY;
    v = sort32x2_desc(v, lane);
    v = merge32x2_asc(L < v ? L : v, lane);
    if (act && h < k) lst[h] = v;
    wave_lds_fence();
    const uint32_t hi = (uint32_t)(v >> 32);
    *b0 = bound_of((uint32_t)__builtin_amdgcn_readlane((int)hi, (int)k - 1));
    *b1 = bound_of((uint32_t)__builtin_amdgcn_readlane((int)hi, 32 + (int)k - 1));
}

// One wave per block. Dynamic LDS: per query, the list (k keys) and the
// pending buffer (PEND keys or candidate positions).
template <bool POS>
__global__ __launch_bounds__(64) void knn_kernel(Plan P, const float4* __restrict__ cand4, int kk) {
    using PT = typename Pending<POS>::T;
    extern __shared__ unsigned long long s_dyn[];
    const uint32_t lane = threadIdx.x;
    const uint32_t k = (uint32_t)kk;
    const bool half = k <= 32u;
    unsigned long long* const s_list = s_dyn;                    // [QPW][k]
    PT* const s_pend = (PT*)(s_dyn + (size_t)QPW * k);  // [QPW][PEND]
    const uint32_t n_items = P.ctr->n_items;
    // Work queue: every wave starts on item blockIdx.x without an atomic;
    // the rest are claimed from KNN_STREAMS interleaved streams (item i in
    // stream i % KNN_STREAMS, cursor per stream past the items handed out
    // statically), own stream first, then the others. One device-scope
    // cursor for all would serialise every claim on one address.
    const uint32_t G = gridDim.x;
    const uint32_t s0 = blockIdx.x % KNN_STREAMS;
    uint32_t it = blockIdx.x;
    uint32_t sv = 0;  // streams visited after the own one
    for (;;) {
        while (it >= n_items && sv < KNN_STREAMS) {
            const uint32_t s = (s0 + sv) % KNN_STREAMS;
            uint32_t got = 0;
            if (lane == 0) got = atomicAdd(&P.ctr->knn_q[s][0], 1u);
            got = __builtin_amdgcn_readfirstlane(__shfl(got, 0, 64));
            const uint32_t base = G > s ? (G - s + KNN_STREAMS - 1) / KNN_STREAMS : 0u;  // static items of s
            it = (base + got) * KNN_STREAMS + s;
            if (it >= n_items) ++sv;
        }
        if (it >= n_items) break;
        const KnnItem w = P.items[it];
        const uint32_t t = w.leaf;
        const uint32_t nr = P.leaf_nr[t];
        const uint32_t ncand = P.leaf_ncand[t], nch = P.leaf_nch[t], cc = P.leaf_cc[t];
        const uint32_t qb = P.p1pos[P.leaf_begin[t]];
        const uint32_t qn = w.q1 - w.q0;

        // The leaf's candidate ranges, concatenated: lane r holds where range
        // r starts in that order (cpre; past the end for lanes >= nr) and the
        // offset from there to its P1 index (coff). The range of a position L
        // is the number of lanes 1..nr-1 with cpre <= L.
        uint32_t len = 0, rbeg = 0;
        if (lane < nr) {
            const uint2 R = P.leaf_ranges[(size_t)t * HALO + lane];
            rbeg = R.x;
            len = R.y - R.x;
        }
        const uint32_t cpre = wave_incl_scan(len) - len + (lane < nr ? 0u : ncand);
        const uint32_t coff = rbeg - cpre;
        auto range_of = [&](uint32_t L) -> uint32_t {
            return (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(lane >= 1u && lane < nr && cpre <= L));
        };

        // lists start as k tau placeholders (or empty); lane j holds query
        // j's coordinates, its distance bound (`worst`: candidates with d2 <=
        // worst may enter) and its pending count
        float worst = lane < qn ? INFINITY : -1.0f;
        uint32_t pcnt = 0;
        float4 qv = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lane < qn) {
            const float tb = P.tau_c[w.q0 + lane];
            if (tb >= 0.0f) worst = tb;
            qv = cand4[w.q0 + lane];
        }
        for (uint32_t j = 0; j < qn; ++j) {
            const float tb = P.tau_c[w.q0 + j];
            if (lane < k) s_list[j * k + lane] = tb >= 0.0f ? make_key(tb, NONE32) : KEY_EMPTY;
        }
        wave_lds_fence();

        const uint32_t c_lo = w.chunk * cc;
        const uint32_t c_hi = min(ncand, c_lo + cc);
        float4 cn[CPL];
        uint32_t cni[CPL];  // their P1 indices
        // candidates [pos, pos + CBLK) of the concatenated order into cn
        auto load_block = [&](uint32_t pos) {
            const uint32_t last = min(c_hi, pos + (uint32_t)CBLK) - 1u;
            const uint32_t ra = range_of(pos), rb = range_of(last);
            const uint32_t off0 = (uint32_t)__builtin_amdgcn_readlane((int)coff, (int)ra);
#pragma unroll
            for (int g = 0; g < CPL; ++g) {
                const uint32_t Lg = pos + (uint32_t)g * 64u + lane;
                uint32_t off = off0;
                for (uint32_t r = ra + 1u; r <= rb; ++r)
                    if ((uint32_t)__builtin_amdgcn_readlane((int)cpre, (int)r) <= Lg)
                        off = (uint32_t)__builtin_amdgcn_readlane((int)coff, (int)r);
                if (Lg < c_hi) {
                    cn[g] = cand4[off + Lg];
                    cni[g] = off + Lg;
                } else {
                    // NaN coordinates: d2 <= bound never holds
                    const float nan = __uint_as_float(0x7FC00000u);
                    cn[g] = make_float4(nan, nan, nan, __uint_as_float(NONE32));
                    cni[g] = NONE32;
                }
            }
        };
        // Blocks nearest to the tile in Morton order first, so that the bounds
        // tighten early: start at the block holding the tile's position in the
        // concatenated order (or the chunk end nearest to it), then alternate
        // outwards.
        const uint32_t ro = (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(lane >= 1u && lane < nr && rbeg <= w.q0));
        const uint32_t p_t = (uint32_t)__builtin_amdgcn_readlane((int)cpre, (int)ro) +
                             (w.q0 - (uint32_t)__builtin_amdgcn_readlane((int)rbeg, (int)ro));
        const int nblk = c_lo < c_hi ? (int)((c_hi - c_lo + CBLK - 1) / CBLK) : 0;
        const int b_start = p_t < c_lo ? 0 : min((int)((p_t - c_lo) / CBLK), nblk - 1);
        int nx_hi = b_start + 1, nx_lo = b_start - 1;
        bool up = true;
        auto next_block = [&]() -> int {
            if (up && nx_hi < nblk) {
                up = false;
                return nx_hi++;
            }
            if (nx_lo >= 0) {
                up = true;
                return nx_lo--;
            }
            if (nx_hi < nblk) return nx_hi++;
            return -1;
        };
        if (nblk > 0) load_block(c_lo + (uint32_t)b_start * CBLK);
        for (int b = nblk > 0 ? b_start : -1; b >= 0;) {
            float4 c[CPL];
            uint32_t ci[CPL];
#pragma unroll
            for (int g = 0; g < CPL; ++g) {
                c[g] = cn[g];
                ci[g] = cni[g];
            }
            const int b_next = next_block();
            if (b_next >= 0) load_block(c_lo + (uint32_t)b_next * CBLK);
            b = b_next;
            // append query j's passing candidates (masks m) to its pending
            // buffer, merging the buffer into the list when it would overflow
            auto append = [&](uint32_t j, float wj, unsigned long long (&m)[CPL], const float (&d)[CPL], float4 q) {
                uint32_t cnt = (uint32_t)__builtin_amdgcn_readlane((int)pcnt, (int)j);
                const unsigned long long selfkey =
                    (unsigned long long)(uint32_t)__builtin_amdgcn_readlane(__float_as_int(qv.w), (int)j);
                PT* const pend = s_pend + (size_t)j * PEND;
                unsigned long long* const lst = s_list + (size_t)j * k;
#pragma unroll
                for (int g = 0; g < CPL; ++g) {
                    if (m[g] == 0ull) continue;
                    uint32_t pc = (uint32_t)__popcll(m[g]);
                    if (cnt + pc > (uint32_t)PEND) {
                        wj = fminf(wj, flush<POS>(lst, pend, cnt, lane, k, selfkey, cand4, q));
                        cnt = 0;
#pragma unroll
                        for (int h = g; h < CPL; ++h) m[h] = __builtin_amdgcn_ballot_w64(d[h] <= wj);
                        pc = (uint32_t)__popcll(m[g]);
                        if (pc == 0u) continue;
                    }
                    const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(m[g] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m[g], 0u));
                    if ((m[g] >> lane) & 1ull) {
                        if constexpr (POS)
                            pend[cnt + rank] = ci[g];
                        else
                            pend[cnt + rank] = make_key(d[g], __float_as_uint(c[g].w));
                    }
                    cnt += pc;
                }
                if (lane == j) {
                    pcnt = cnt;
                    worst = wj;
                }
            };
            // Cull by the block's bounding box: with lo <= c <= hi per axis,
            // fl(lo - q) <= fl(c - q) (and likewise above hi), and rounded
            // squares and sums are monotone, so the box distance computed in
            // the same order as dist2 is <= the d2 of every candidate in the
            // block. A query whose box distance exceeds its bound skips the
            // block; the result is unchanged. (fminf/fmaxf skip the NaN
            // padding of a ragged block.)
            float lx = c[0].x, ly = c[0].y, lz = c[0].z, hx = c[0].x, hy = c[0].y, hz = c[0].z;
#pragma unroll
            for (int g = 1; g < CPL; ++g) {
                lx = fminf(lx, c[g].x); ly = fminf(ly, c[g].y); lz = fminf(lz, c[g].z);
                hx = fmaxf(hx, c[g].x); hy = fmaxf(hy, c[g].y); hz = fmaxf(hz, c[g].z);
            }
            lx = wave_min(lx, lane); ly = wave_min(ly, lane); lz = wave_min(lz, lane);
            hx = wave_max(hx, lane); hy = wave_max(hy, lane); hz = wave_max(hz, lane);
            const float gx = fmaxf(fmaxf(lx - qv.x, qv.x - hx), 0.0f);
            const float gy = fmaxf(fmaxf(ly - qv.y, qv.y - hy), 0.0f);
            const float gz = fmaxf(fmaxf(lz - qv.z, qv.z - hz), 0.0f);
            const float bd = (gx * gx + gy * gy) + gz * gz;
            unsigned long long qm = __builtin_amdgcn_ballot_w64(lane < qn && !(bd > worst));
            while (qm != 0ull) {
                const uint32_t j = (uint32_t)__ffsll((long long)qm) - 1u;
                qm &= qm - 1ull;
                const float4 q = query_of(qv, j);
                float wj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(worst), (int)j));
                float d[CPL];
                unsigned long long m[CPL];
                unsigned long long any = 0ull;
                uint32_t tot = 0;
#pragma unroll
                for (int g = 0; g < CPL; ++g) {
                    d[g] = dist2(q, c[g]);
                    m[g] = __builtin_amdgcn_ballot_w64(d[g] <= wj);
                    any |= m[g];
                    tot += (uint32_t)__popcll(m[g]);
                }
                // A block that would overflow the pending buffer first lowers
                // the bound: if at least k + 1 of its candidates (one may be
                // the query itself) lie within wj * 2^(-1/4), the k-th
                // distance cannot exceed that, so nothing needed is lost.
                if (tot > (uint32_t)PEND - (uint32_t)__builtin_amdgcn_readlane((int)pcnt, (int)j) &&
                    tot > k + 1u && wj < INFINITY) {
                    for (int i = 0; i < 12; ++i) {
                        const float t2 = wj * 0.84089642f;
                        uint32_t c2 = 0;
#pragma unroll
                        for (int g = 0; g < CPL; ++g)
                            c2 += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(d[g] <= t2));
                        if (c2 < k + 1u) break;
                        wj = t2;
                    }
                    any = 0ull;
#pragma unroll
                    for (int g = 0; g < CPL; ++g) {
                        m[g] = __builtin_amdgcn_ballot_w64(d[g] <= wj);
                        any |= m[g];
                    }
                    if (lane == j) worst = wj;
                }
                if (any != 0ull) append(j, wj, m, d, q);
            }
        }
        // drain the pending buffers: when k <= 32, two queries per merge if
        // both hold at most 32 pending keys
        if (half) {
            for (uint32_t j = 0; j < qn; j += 2u) {
                const uint32_t j1 = j + 1u;
                const bool two = j1 < qn;
                const uint32_t c0 = (uint32_t)__builtin_amdgcn_readlane((int)pcnt, (int)j);
                const uint32_t c1 = two ? (uint32_t)__builtin_amdgcn_readlane((int)pcnt, (int)j1) : 0u;
                if ((c0 | c1) == 0u) continue;
                const unsigned long long s0 =
                    (unsigned long long)(uint32_t)__builtin_amdgcn_readlane(__float_as_int(qv.w), (int)j);
                const unsigned long long s1 =
                    two ? (unsigned long long)(uint32_t)__builtin_amdgcn_readlane(__float_as_int(qv.w), (int)j1) : 0ull;
                unsigned long long* const l0 = s_list + (size_t)j * k;
                PT* const p0 = s_pend + (size_t)j * PEND;
                const float4 q0 = query_of(qv, j);
                const float4 q1 = two ? query_of(qv, j1) : q0;
                if (c0 <= (uint32_t)PEND_HALF && c1 <= (uint32_t)PEND_HALF) {
                    float b0, b1;
                    // without a second query the upper half touches no memory
                    flush_half<POS>(l0, p0, c0, s0, q0, l0 + k, p0 + PEND, c1, s1, q1, two, lane, k, cand4, &b0,
                                    &b1);
                } else {
                    if (c0) (void)flush<POS>(l0, p0, c0, lane, k, s0, cand4, q0);
                    if (c1) (void)flush<POS>(l0 + k, p0 + PEND, c1, lane, k, s1, cand4, q1);
                }
            }
        } else {
            for (uint32_t j = 0; j < qn; ++j) {
                const uint32_t cnt = (uint32_t)__builtin_amdgcn_readlane((int)pcnt, (int)j);
                const unsigned long long selfkey =
                    (unsigned long long)(uint32_t)__builtin_amdgcn_readlane(__float_as_int(qv.w), (int)j);
                if (cnt)
                    (void)flush<POS>(s_list + (size_t)j * k, s_pend + (size_t)j * PEND, cnt, lane, k, selfkey,
                                     cand4, query_of(qv, j));
            }
        }

        if (nch > 1) {
            // partial lists [query][chunk][r]: one coalesced row per list,
            // merged by knn_merge_kernel
            unsigned long long* base = (unsigned long long*)P.plist + (size_t)P.leaf_plist[t] * k;
            for (uint32_t j = 0; j < qn; ++j)
                if (lane < k) base[((size_t)(w.q0 + j - qb) * nch + w.chunk) * k + lane] = s_list[j * k + lane];
        } else {
            for (uint32_t j = 0; j < qn; ++j) {
                const unsigned long long v = lane < k ? s_list[j * k + lane] : KEY_EMPTY;
                write_final(P, w.q0 + j, k, lane, v);
            }
        }
        wave_lds_fence();
        it = n_items;  // claim the next one
    }
}

// ---------------------------------------------------------------- kNN by culling groups
//
// The candidates of an item are visited in aligned groups of KNN_GRP P1
// positions (one per lane), whose bounding boxes the bound kernel wrote. A
// group is loaded only if the box passes for at least one query of the
// tile: a round box-tests GPT groups against the Q queries at once (lane
// L: query L % Q, group L / Q), with the same fp32 operations as dist2, so a
// skipped group holds no candidate with d2 <= the query's bound. Positions of
// a group outside the range's part in this chunk are not candidates; they
// are given NaN coordinates (d2 <= bound never holds). Groups of the range
// holding the tile come first, from the tile's group outwards, then the
// other ranges in order.
template <bool POS, int Q>
__global__ __launch_bounds__(64) void knn_group_kernel(Plan P, const float4* __restrict__ cand4, int kk) {
    using PT = typename Pending<POS>::T;
    constexpr int GPT = 64 / Q;  // groups per box-test round
    static_assert(Q * GPT == 64 && Q <= 64, "tile shape");
    extern __shared__ unsigned long long s_dyn[];
    const uint32_t lane = threadIdx.x;
    const uint32_t k = (uint32_t)kk;
    const bool half = k <= 32u;
    unsigned long long* const s_list = s_dyn;           // [Q][k]
    PT* const s_pend = (PT*)(s_dyn + (size_t)Q * k);    // [Q][PEND]
    const uint32_t jl = lane % (uint32_t)Q;             // this lane's query in box tests
    const uint32_t ul = lane / (uint32_t)Q;             // this lane's group slot in box tests
    const uint32_t n_items = P.ctr->n_items;
    const uint32_t G = gridDim.x;
    const uint32_t s0 = blockIdx.x % KNN_STREAMS;
    uint32_t it = blockIdx.x;
    uint32_t sv = 0;
    for (;;) {
        while (it >= n_items && sv < KNN_STREAMS) {
            const uint32_t s = (s0 + sv) % KNN_STREAMS;
            uint32_t got = 0;
            if (lane == 0) got = atomicAdd(&P.ctr->knn_q[s][0], 1u);
            got = __builtin_amdgcn_readfirstlane(__shfl(got, 0, 64));
            const uint32_t base = G > s ? (G - s + KNN_STREAMS - 1) / KNN_STREAMS : 0u;
            it = (base + got) * KNN_STREAMS + s;
            if (it >= n_items) ++sv;
        }
        if (it >= n_items) break;
        const KnnItem w = P.items[it];
        const uint32_t t = w.leaf;
        const uint32_t nr = P.leaf_nr[t];
        const uint32_t ncand = P.leaf_ncand[t], nch = P.leaf_nch[t], cc = P.leaf_cc[t];
        const uint32_t qb = P.p1pos[P.leaf_begin[t]];
        const uint32_t qn = w.q1 - w.q0;

        // lane r < nr: range r, its part [sa, sb) of P1 positions inside this
        // chunk (the chunk is [c_lo, c_hi) of the ranges' concatenated order)
        // and the aligned groups [g0, g0 + gn) overlapping that part
        uint32_t len = 0, rbeg = 0;
        if (lane < nr) {
            const uint2 R = P.leaf_ranges[(size_t)t * HALO + lane];
            rbeg = R.x;
            len = R.y - R.x;
        }
        const uint32_t cpre = wave_incl_scan(len) - len;
        const uint32_t c_lo = w.chunk * cc;
        const uint32_t c_hi = min(ncand, c_lo + cc);
        uint32_t sa = 0, sb = 0;
        if (lane < nr) {
            const uint32_t a = max(cpre, c_lo), b = min(cpre + len, c_hi);
            if (a < b) {
                sa = rbeg + (a - cpre);
                sb = rbeg + (b - cpre);
            }
        }
        const uint32_t g0 = sa / (uint32_t)KNN_GRP;
        const uint32_t gn = sb > sa ? (sb - 1u) / (uint32_t)KNN_GRP - g0 + 1u : 0u;
        // the range holding the tile's queries comes first
        const uint32_t nro = (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(lane < nr && rbeg <= w.q0));
        const uint32_t ro = nro ? nro - 1u : 0u;  // (a leaf with queries always has its own range)
        const uint32_t g0o = (uint32_t)__builtin_amdgcn_readlane((int)g0, (int)ro);
        const uint32_t gno = (uint32_t)__builtin_amdgcn_readlane((int)gn, (int)ro);
        const uint32_t gt = gno ? min(max(w.q0 / (uint32_t)KNN_GRP, g0o), g0o + gno - 1u) : 0u;
        const uint32_t n_up = gno ? g0o + gno - 1u - gt : 0u, n_dn = gno ? gt - g0o : 0u;
        const uint32_t n_alt = min(n_up, n_dn);
        const uint32_t u2n = (lane < nr && lane != ro) ? gn : 0u;
        const uint32_t u2pre = wave_incl_scan(u2n) - u2n;
        const uint32_t n_units = gno + (uint32_t)__builtin_amdgcn_readlane((int)(u2pre + u2n), 63);
        // unit u -> (range, group): own range outwards, then the others
        auto unit = [&](uint32_t u, uint32_t* r, uint32_t* g) {
            if (u < gno) {
                *r = ro;
                if (u == 0u) {
                    *g = gt;
                } else if (u <= 2u * n_alt) {
                    const uint32_t d = (u + 1u) >> 1;
                    *g = (u & 1u) ? gt + d : gt - d;
                } else {
                    const uint32_t d = u - n_alt;
                    *g = n_up > n_dn ? gt + d : gt - d;
                }
            } else {
                const uint32_t v = u - gno;
                const uint64_t mk = __builtin_amdgcn_ballot_w64(u2n > 0u && u2pre <= v);
                const uint32_t rr = 63u - (uint32_t)__clzll((long long)mk);
                *r = rr;
                *g = (uint32_t)__builtin_amdgcn_readlane((int)g0, (int)rr) + v -
                     (uint32_t)__builtin_amdgcn_readlane((int)u2pre, (int)rr);
            }
        };

        // lists start as k tau placeholders (or empty). Lane L holds query
        // L % Q's coordinates and bound (`worst`: candidates with d2 <= worst
        // may enter); lane j < Q holds query j's pending count.
        const bool qok = jl < qn;
        float worst = -1.0f;
        float4 qv = make_float4(0.f, 0.f, 0.f, 0.f);
        if (qok) {
            const float tb = P.tau_c[w.q0 + jl];
            worst = tb >= 0.0f ? tb : INFINITY;
            qv = cand4[w.q0 + jl];
        }
        uint32_t pcnt = 0;
        for (uint32_t j = 0; j < qn; ++j) {
            const float tb = P.tau_c[w.q0 + j];
            if (lane < k) s_list[j * k + lane] = tb >= 0.0f ? make_key(tb, NONE32) : KEY_EMPTY;
        }
        wave_lds_fence();

        for (uint32_t u0 = 0; u0 < n_units; u0 += (uint32_t)GPT) {
            uint32_t gs[GPT], ra[GPT], rb[GPT];
#pragma unroll
            for (int i = 0; i < GPT; ++i) {
                gs[i] = NONE32;
                ra[i] = rb[i] = 0u;
                if (u0 + (uint32_t)i < n_units) {
                    uint32_t r, g;
                    unit(u0 + (uint32_t)i, &r, &g);
                    gs[i] = g;
                    ra[i] = (uint32_t)__builtin_amdgcn_readlane((int)sa, (int)r);
                    rb[i] = (uint32_t)__builtin_amdgcn_readlane((int)sb, (int)r);
                }
            }
            // box test of (query jl, group slot ul)
            uint32_t gmine = gs[0];
#pragma unroll
            for (int i = 1; i < GPT; ++i)
                if (ul == (uint32_t)i) gmine = gs[i];
            bool need = false;
            if (qok && gmine != NONE32) {
                const GroupBox B = P.gbox[gmine];
                const float gx = fmaxf(fmaxf(B.lo.x - qv.x, qv.x - B.hi.x), 0.0f);
                const float gy = fmaxf(fmaxf(B.lo.y - qv.y, qv.y - B.hi.y), 0.0f);
                const float gz = fmaxf(fmaxf(B.lo.z - qv.z, qv.z - B.hi.z), 0.0f);
                need = !((gx * gx + gy * gy) + gz * gz > worst);
            }
            const unsigned long long nm = __builtin_amdgcn_ballot_w64(need);
            if (nm == 0ull) continue;
            // load the groups some query needs, then test their candidates
            float4 c[GPT];
            uint32_t cp[GPT];
#pragma unroll
            for (int i = 0; i < GPT; ++i) {
                cp[i] = NONE32;
                if ((nm >> (i * Q)) & (Q == 64 ? ~0ull : ((1ull << Q) - 1ull))) {
                    const uint32_t p = gs[i] * (uint32_t)KNN_GRP + lane;
                    if (p >= ra[i] && p < rb[i]) {
                        c[i] = cand4[p];
                        cp[i] = p;
                    } else {
                        const float nan = __uint_as_float(0x7FC00000u);
                        c[i] = make_float4(nan, nan, nan, __uint_as_float(NONE32));
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < GPT; ++i) {
                unsigned long long qm = (nm >> (i * Q)) & (Q == 64 ? ~0ull : ((1ull << Q) - 1ull));
                while (qm != 0ull) {
                    const uint32_t j = (uint32_t)__ffsll((long long)qm) - 1u;
                    qm &= qm - 1ull;
                    const float4 q = query_of(qv, j);
                    float wj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(worst), (int)j));
                    const float d = dist2(q, c[i]);
                    unsigned long long m = __builtin_amdgcn_ballot_w64(d <= wj);
                    if (m == 0ull) continue;
                    uint32_t pc = (uint32_t)__popcll(m);
                    // a group holding more than k + 1 passing candidates (one may
                    // be the query) first lowers the bound: if k + 1 of them lie
                    // within wj * 2^(-1/4), the k-th distance cannot exceed it
                    if (pc > k + 1u && wj < INFINITY) {
                        for (int r = 0; r < 12; ++r) {
                            const float t2 = wj * 0.84089642f;
                            if ((uint32_t)__popcll(__builtin_amdgcn_ballot_w64(d <= t2)) < k + 1u) break;
                            wj = t2;
                        }
                        m = __builtin_amdgcn_ballot_w64(d <= wj);
                        pc = (uint32_t)__popcll(m);
                    }
                    uint32_t cnt = (uint32_t)__builtin_amdgcn_readlane((int)pcnt, (int)j);
                    PT* const pend = s_pend + (size_t)j * PEND;
                    if (cnt + pc > (uint32_t)PEND) {
                        const unsigned long long selfkey =
                            (unsigned long long)(uint32_t)__builtin_amdgcn_readlane(__float_as_int(qv.w), (int)j);
                        wj = fminf(wj, flush<POS>(s_list + (size_t)j * k, pend, cnt, lane, k, selfkey, cand4, q));
                        cnt = 0;
                        m = __builtin_amdgcn_ballot_w64(d <= wj);
                        pc = (uint32_t)__popcll(m);
                    }
                    if (pc) {
                        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                        if ((m >> lane) & 1ull) {
                            if constexpr (POS)
                                pend[cnt + rank] = cp[i];
                            else
                                pend[cnt + rank] = make_key(d, __float_as_uint(c[i].w));
                        }
                        cnt += pc;
                    }
                    if (lane == j) pcnt = cnt;
                    if (jl == j) worst = wj;
                }
            }
        }
        // drain the pending buffers: when k <= 32, two queries per merge if
        // both hold at most 32 pending keys
        if (half) {
            for (uint32_t j = 0; j < qn; j += 2u) {
                const uint32_t j1 = j + 1u;
                const bool two = j1 < qn;
                const uint32_t c0 = (uint32_t)__builtin_amdgcn_readlane((int)pcnt, (int)j);
                const uint32_t c1 = two ? (uint32_t)__builtin_amdgcn_readlane((int)pcnt, (int)j1) : 0u;
                if ((c0 | c1) == 0u) continue;
                const unsigned long long sk0 =
                    (unsigned long long)(uint32_t)__builtin_amdgcn_readlane(__float_as_int(qv.w), (int)j);
                const unsigned long long sk1 =
                    two ? (unsigned long long)(uint32_t)__builtin_amdgcn_readlane(__float_as_int(qv.w), (int)j1) : 0ull;
                unsigned long long* const l0 = s_list + (size_t)j * k;
                PT* const p0 = s_pend + (size_t)j * PEND;
                const float4 q0 = query_of(qv, j);
                const float4 q1 = two ? query_of(qv, j1) : q0;
                if (c0 <= (uint32_t)PEND_HALF && c1 <= (uint32_t)PEND_HALF) {
                    float b0, b1;
                    flush_half<POS>(l0, p0, c0, sk0, q0, l0 + k, p0 + PEND, c1, sk1, q1, two, lane, k, cand4, &b0,
                                    &b1);
                } else {
                    if (c0) (void)flush<POS>(l0, p0, c0, lane, k, sk0, cand4, q0);
                    if (c1) (void)flush<POS>(l0 + k, p0 + PEND, c1, lane, k, sk1, cand4, q1);
                }
            }
        } else {
            for (uint32_t j = 0; j < qn; ++j) {
                const uint32_t cnt = (uint32_t)__builtin_amdgcn_readlane((int)pcnt, (int)j);
                const unsigned long long selfkey =
                    (unsigned long long)(uint32_t)__builtin_amdgcn_readlane(__float_as_int(qv.w), (int)j);
                if (cnt)
                    (void)flush<POS>(s_list + (size_t)j * k, s_pend + (size_t)j * PEND, cnt, lane, k, selfkey,
                                     cand4, query_of(qv, j));
            }
        }

        if (nch > 1) {
            unsigned long long* base = (unsigned long long*)P.plist + (size_t)P.leaf_plist[t] * k;
            for (uint32_t j = 0; j < qn; ++j)
                if (lane < k) base[((size_t)(w.q0 + j - qb) * nch + w.chunk) * k + lane] = s_list[j * k + lane];
        } else {
            for (uint32_t j = 0; j < qn; ++j) {
                const unsigned long long v = lane < k ? s_list[j * k + lane] : KEY_EMPTY;
                write_final(P, w.q0 + j, k, lane, v);
            }
        }
        wave_lds_fence();
        it = n_items;
    }
}

// ---------------------------------------------------------------- chunk merge
//
// MERGE_SPLIT waves per query tile of a chunked leaf (each takes a share of
// the tile's queries, which shortens the longest chain of merges), after the kNN kernel (the kernel
// boundary makes every partial list visible). B_j, the smallest k-th key over
// the chunks of query j, bounds its merged k-th key, so a list whose first key
// exceeds B_j contributes nothing. The first and k-th keys of all lists of the
// tile are fetched together and staged in LDS; the contributing lists are then
// fetched eight at a time, over all queries of the tile, and merged into the
// query's list with the exchange steps of the kNN kernel.
constexpr int MERGE_SPLIT = 4;

__global__ __launch_bounds__(64) void knn_merge_kernel(Plan P, int kk) {
    __shared__ unsigned long long s_fk[QPW * KNN_NCH_MAX * 2];
    __shared__ unsigned long long s_lst[QPW * 64];
    const uint32_t lane = threadIdx.x;
    const uint32_t k = (uint32_t)kk;
    const uint32_t nci = P.ctr->n_chunked_items;
    for (uint32_t u = blockIdx.x; u < nci * MERGE_SPLIT; u += gridDim.x) {
        const uint32_t it = u / MERGE_SPLIT, part = u % MERGE_SPLIT;
        const KnnItem w = P.items[it];
        if (w.chunk != 0u) continue;
        // this wave's share of the tile's queries
        const uint32_t q0 = w.q0 + part * (uint32_t)(KNN_TQ / MERGE_SPLIT);
        if (q0 >= w.q1) continue;
        const uint32_t q1 = min(w.q1, q0 + (uint32_t)(KNN_TQ / MERGE_SPLIT));
        const uint32_t t = w.leaf;
        const uint32_t nch = P.leaf_nch[t];
        const uint32_t qb = P.p1pos[P.leaf_begin[t]];
        const uint32_t qn = q1 - q0;
        const unsigned long long* base = (const unsigned long long*)P.plist + (size_t)P.leaf_plist[t] * k;
        const uint32_t tot = qn * nch;
        for (uint32_t e0 = 0; e0 < tot; e0 += 256u) {
            unsigned long long f[4], kt[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint32_t e = e0 + (uint32_t)b * 64u + lane;
                if (e < tot) {
                    const uint32_t j = e / nch, c = e - j * nch;
                    const unsigned long long* l = base + ((size_t)(q0 + j - qb) * nch + c) * k;
                    f[b] = l[0];
                    kt[b] = l[k - 1];
                }
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint32_t e = e0 + (uint32_t)b * 64u + lane;
                if (e < tot) {
                    const uint32_t j = e / nch, c = e - j * nch;
                    s_fk[(j * KNN_NCH_MAX + c) * 2u] = f[b];
                    s_fk[(j * KNN_NCH_MAX + c) * 2u + 1u] = kt[b];
                }
            }
        }
        for (uint32_t j = 0; j < qn; ++j) s_lst[j * 64u + lane] = KEY_EMPTY;
        wave_lds_fence();
        uint32_t cm = 0;  // lane j: contributing chunks of query j
        if (lane < qn) {
            unsigned long long B = KEY_EMPTY;
            for (uint32_t c = 0; c < nch; ++c) {
                const unsigned long long v = s_fk[(lane * KNN_NCH_MAX + c) * 2u + 1u];
                B = v < B ? v : B;
            }
            for (uint32_t c = 0; c < nch; ++c) {
                const unsigned long long v = s_fk[(lane * KNN_NCH_MAX + c) * 2u];
                if (real_entry(v) && v <= B) cm |= 1u << c;
            }
        }
        // flattened (query, chunk) pairs: pair p belongs to the last query j
        // with excl_j <= p among the queries that have pairs
        const uint32_t pc = (uint32_t)__popc(cm);
        const uint32_t incl = wave_incl_scan(pc);
        const uint32_t excl = incl - pc;
        const uint32_t T = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        for (uint32_t p0 = 0; p0 < T; p0 += 8u) {
            unsigned long long pv[8];
            uint32_t pj[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const uint32_t p = p0 + (uint32_t)b;
                pv[b] = KEY_EMPTY;
                pj[b] = NONE32;
                if (p < T) {
                    const unsigned long long mk = __builtin_amdgcn_ballot_w64(pc > 0u && excl <= p);
                    const uint32_t j = 63u - (uint32_t)__clzll((long long)mk);
                    uint32_t bits = (uint32_t)__builtin_amdgcn_readlane((int)cm, (int)j);
                    for (uint32_t r = p - (uint32_t)__builtin_amdgcn_readlane((int)excl, (int)j); r > 0u; --r)
                        bits &= bits - 1u;
                    const uint32_t c = (uint32_t)__ffs((int)bits) - 1u;
                    if (lane < k) pv[b] = base[((size_t)(q0 + j - qb) * nch + c) * k + lane];
                    pj[b] = j;
                }
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                if (pj[b] == NONE32) continue;
                unsigned long long* const lst = s_lst + pj[b] * 64u;
                const unsigned long long L = lane < k ? lst[lane] : KEY_EMPTY;
                const unsigned long long rv = shfl64(pv[b], 63 - (int)lane);  // descending
                const unsigned long long v = merge64_asc(L < rv ? L : rv, lane);
                if (lane < k) lst[lane] = v;
                wave_lds_fence();
            }
        }
        for (uint32_t j = 0; j < qn; ++j) {
            const unsigned long long v = lane < k ? s_lst[j * 64u + lane] : KEY_EMPTY;
            write_final(P, q0 + j, k, lane, v);
        }
        wave_lds_fence();
    }
}

void launch_knn_bound(const Plan& P, int k, int num_cus, hipStream_t st) {
    (void)num_cus;
    unsigned blocks = (P.n + BOUND_Q - 1) / BOUND_Q;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(P.n > BOUND_COARSE_MIN_N ? knn_bound_kernel<5> : knn_bound_kernel<10>, dim3(blocks),
                       dim3(BOUND_Q * BOUND_SPLIT), 0, st, P, (const float4*)P.cand4, k);
}

size_t knn_lds_bytes(int k, bool pos) {
    return (size_t)QPW * ((size_t)k * sizeof(unsigned long long) +
                          (size_t)PEND * (pos ? sizeof(uint32_t) : sizeof(unsigned long long)));
}

void launch_knn(const Plan& P, int k, int num_cus, hipStream_t st) {
    const unsigned blocks = (unsigned)(num_cus > 0 ? num_cus : 256) * 16u;
    // Large batches run long enough for occupancy to pay (positions); a single
    // frame's run is set by its longest items, where a gather per merge costs
    // more (keys).
    if (P.n > KNN_POS_MIN_N)
        hipLaunchKernelGGL((knn_group_kernel<true, QPW>), dim3(blocks), dim3(64), knn_lds_bytes(k, true), st, P,
                           (const float4*)P.cand4, k);
    else
        hipLaunchKernelGGL((knn_group_kernel<false, QPW>), dim3(blocks), dim3(64), knn_lds_bytes(k, false), st, P,
                           (const float4*)P.cand4, k);
}

void launch_knn_merge(const Plan& P, int k, int num_cus, hipStream_t st) {
    const unsigned blocks = (unsigned)(num_cus > 0 ? num_cus : 256) * 8u;
    hipLaunchKernelGGL(knn_merge_kernel, dim3(blocks), dim3(64), 0, st, P, k);
}

}  // namespace gdn
