// Leaf-local brute-force kNN with halo candidates (Sec. 3: N_K(i), d_ij and
// r_K,i on the voxel-filtered set P1).
//
// Work item = (leaf, a tile of 8 queries (16 above 2^20 points), candidate
// chunk), one wave each. The candidates are the P1 positions of the leaf's
// merged halo ranges; they are visited in aligned groups of 64 positions (one
// per lane), whose bounding boxes the bound kernel writes. Up to 64 groups at
// a time are box-tested against every query of the tile (a query mask per
// group) and ordered nearest-first; the needed groups are then taken four at
// a time into registers, and each query that needs any of them computes its
// squared distances to their 64 candidates, in fp32 as (dx*dx + dy*dy) + dz*dz
// without contraction, so the neighbour sets are exact. A skipped group holds
// no candidate within the query's bound (the box distance uses the same
// rounded operations, which are monotone), so skipping never changes a result.
//
// Each query keeps, in LDS, its k best (d2, original index) keys (d2 bits <<
// 32 | index), sorted, and a pending buffer of up to 64 candidates (the keys,
// or their P1 positions above 1M points, which halves the LDS a wave needs; a
// key is then rebuilt from the position with the same fp32 expression). A
// candidate passes with one compare against the query's bound; the passing
// ones are appended (ballot + lane rank). A full buffer, and the buffer at
// the end of the item, is merged into the list: the pending keys are sorted
// descending across the wave, the elementwise minimum with the ascending list
// holds the 64 smallest keys of both as a bitonic sequence, and six more
// exchange steps sort it; a list never merged into takes its pending keys
// sorted ascending. The sorts run on 32-bit keys (the top 26 bits of d2 and
// the lane) and fall back to the 64-bit keys when two of them could tie.
// When k <= 32, buffers holding at most 32 keys at the end of an item are
// merged on 32-lane halves, two queries at once.
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
constexpr int PEND = 64;     // pending keys per query
constexpr int PEND_HALF = 32;  // pending keys a half-wave merge takes (k <= 32)
constexpr uint32_t KNN_POS_MIN_N = 1u << 20;  // above: pending buffers of positions
constexpr int KNN_NB = 4;      // needed groups held in registers at a time

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
// Threshold ladder tau * 2^-m, m = 1..BOUND_RUNGS, then BOUND_BISECT geometric
// bisection steps (down to a factor 2^(1/32) between thresholds tried).
constexpr int BOUND_RUNGS = 5;
constexpr int BOUND_BISECT = 5;
constexpr int BOUND_Q = 128;       // queries per block (BOUND_Q * BOUND_SPLIT threads)
static_assert(BOUND_Q % KNN_GRP == 0, "a bound block covers whole culling groups");

// tau: the largest d2 to the k points next to the query in Morton order inside
// [qb, qe), a run of candidates holding the query; then, over the run's points
// within BOUND_MARGIN positions, count those under each rung of the ladder
// (BOUND_RUNGS rungs, each half the previous) and keep the smallest threshold
// still holding k; finally bisect (geometrically, BOUND_BISECT steps) between that
// rung and the next one down, keeping the smaller threshold whenever it still
// holds k. Every threshold kept holds k of the query's own candidates, so it
// is >= its k-th distance. -1 when the run has <= k points.
// The BOUND_SPLIT lanes of a query each take every BOUND_SPLIT-th point and
// combine their maxima and counts (exact, so tau does not depend on the
// split); every lane of the wave calls this, `run` false for idle ones.
constexpr int BOUND_WPL = (2 * BOUND_MARGIN + 1 + BOUND_SPLIT - 1) / BOUND_SPLIT;  // window points per lane
template <class Pts>
__device__ float query_bound(Pts cand4, uint32_t qb, uint32_t qe, uint32_t qi, int k, uint32_t sub, bool live) {
    constexpr int LEVELS = BOUND_RUNGS;
    constexpr float STEP = 0.5f;
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
    static_assert(BOUND_SPLIT == 8, "the lane groups are DPP rows of 8");
    const uint32_t lane = threadIdx.x & 63u;
    // sum / max over the BOUND_SPLIT lanes of a query (lanes ^ 1, 2, 4), by DPP
    auto sum8 = [&](uint32_t c) -> uint32_t {
        c += xor_lane<1>(c, lane);
        c += xor_lane<2>(c, lane);
        return c + xor_lane<4>(c, lane);
    };
    float tau = 0.0f;
    for (uint32_t j = s0 + sub; j < s1; j += BOUND_SPLIT)
        if (j != qi) tau = fmaxf(tau, dist2(q, cand4[j]));
    tau = fmaxf(tau, xor_f32<1>(tau, lane));
    tau = fmaxf(tau, xor_f32<2>(tau, lane));
    tau = fmaxf(tau, xor_f32<4>(tau, lane));
    // this lane's window distances (the query itself and absent points: +inf)
    float dw[BOUND_WPL];
#pragma unroll
    for (int i = 0; i < BOUND_WPL; ++i) {
        const uint32_t j = wlo + sub + (uint32_t)i * BOUND_SPLIT;
        dw[i] = (j < whi && j != qi) ? dist2(q, cand4[j]) : INFINITY;
    }
    auto count_le = [&](float t) -> uint32_t {
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < BOUND_WPL; ++i) c += (dw[i] <= t) ? 1u : 0u;
        return sum8(c);
    };
    // the rungs' counts are independent: all of them first, then the choice
    float th[LEVELS];
    uint32_t cnt[LEVELS];
    float f = tau;
#pragma unroll
    for (int m = 0; m < LEVELS; ++m) {
        f = f * STEP;
        th[m] = f;
        cnt[m] = 0;
#pragma unroll
        for (int i = 0; i < BOUND_WPL; ++i) cnt[m] += (dw[i] <= f) ? 1u : 0u;
    }
    float best = tau;
#pragma unroll
    for (int m = 0; m < LEVELS; ++m)
        if (sum8(cnt[m]) >= (uint32_t)k) best = th[m];
    float r = STEP;
#pragma unroll
    for (int b = 0; b < BOUND_BISECT; ++b) {
        r = sqrtf(r);
        const float mid = best * r;
        if (count_le(mid) >= (uint32_t)k) best = mid;
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
            const uint2 R = P.leaf_own[t];
            rb = R.x;
            re = R.y;
        }
        const float b = query_bound(StagedPts{s_pts, lo}, rb, re, qi, k, sub, live);
        if (live && sub == 0u) {
            P.tau_c[qi] = b;
            if ((qi - qb) % P.tq == 0u) {
                const uint32_t nch = P.leaf_nch[t];
                const uint32_t grp = P.leaf_item[t] + ((qi - qb) / P.tq) * nch;
                const uint32_t q1 = min(qe, qi + P.tq);
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
        // the list is ordered by (d2, original index); the neighbour is stored
        // by its P1 position, where everything read about it later sits in
        // Morton order
        const uint32_t pj = ok ? P.inv_p1[(uint32_t)v] : NONE32;
        P.nbr[(size_t)qi * k + lane] = pj;
        P.nbr_d2[(size_t)qi * k + lane] = d;
        // the k-th entry and the (k-1)-th distance again, densely, for the density
        if (lane == k - 1) P.krec[qi] = make_uint4(pj, __float_as_uint(d1), __float_as_uint(d), 0u);
    }
}

// s_waitcnt operand: vector-memory count 0, export and LDS counts left at
// their maxima (gfx9 field layout).
constexpr int VMCNT0 = (7 << 4) | (15 << 8);

// The final lists of a tile's qn queries (in LDS, k keys each), eight
// queries at a time: their position lookups are issued before any store, so
// the tile waits for a round trip per eight queries instead of per query.
__device__ __forceinline__ void write_tile(const Plan& P, const unsigned long long* s_list, uint32_t q0, uint32_t qn,
                                           uint32_t k, uint32_t lane) {
    constexpr int B = 8;
    for (uint32_t j0 = 0; j0 < qn; j0 += (uint32_t)B) {
        unsigned long long v[B];
        uint32_t pj[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            v[j] = (j0 + (uint32_t)j < qn && lane < k) ? s_list[(j0 + (uint32_t)j) * k + lane] : KEY_EMPTY;
            pj[j] = NONE32;
        }
#pragma unroll
        for (int j = 0; j < B; ++j)
            if (lane < k && real_entry(v[j])) pj[j] = P.inv_p1[(uint32_t)v[j]];
        // one wait for all lookups: left to itself the compiler waits for the
        // whole vector-memory counter before each query's stores (the lookups
        // sit in branches), which on this chip also waits for the previous
        // query's stores to be written
        __builtin_amdgcn_s_waitcnt(VMCNT0);
#pragma unroll
        for (int j = 0; j < B; ++j) {
            if (j0 + (uint32_t)j >= qn) break;
            const uint32_t qi = q0 + j0 + (uint32_t)j;
            const bool ok = lane < k && real_entry(v[j]);
            const float d = ok ? __uint_as_float((uint32_t)(v[j] >> 32)) : INFINITY;
            const float d1 = __shfl(d, k >= 2u ? (int)k - 2 : 0, 64);
            if (lane < k) {
                P.nbr[(size_t)qi * k + lane] = pj[j];
                P.nbr_d2[(size_t)qi * k + lane] = d;
                if (lane == k - 1) P.krec[qi] = make_uint4(pj[j], __float_as_uint(d1), __float_as_uint(d), 0u);
            }
        }
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

// The 64 keys of the wave (one per lane, empty = KEY_EMPTY) in ascending
// order, as the 64-bit (d2, index) keys order them, lanes 0..k-1 exact. They
// are first sorted on 32 bits: the top 26 bits of the d2 field (a relative
// step of 2^-17) and the source lane, and each lane then fetches its key from
// that lane. That order is the exact one for the first k positions unless two
// real keys among the first k + 1 agree on those 26 bits; then the 64-bit
// network runs instead.
__device__ __forceinline__ unsigned long long sort_keys_asc(unsigned long long v, uint32_t lane, uint32_t k) {
    constexpr uint32_t EMPTY_TOP = (uint32_t)(KEY_EMPTY >> 32) >> 6;
    const uint32_t s = sort64_u32<true>(((uint32_t)(v >> 32) & ~63u) | lane, lane);
    const uint32_t p = (uint32_t)__shfl_up((int)s, 1u, 64);
    const bool near = lane >= 1u && lane <= k && (s >> 6) == (p >> 6) && (s >> 6) != EMPTY_TOP;
    if (__builtin_amdgcn_ballot_w64(near) == 0ull) return shfl64(v, (int)(s & 63u));
    return ~sort64_desc(~v, lane);
}

// The 64 keys in exact descending order, by the same 32-bit sort (its
// order is exact unless two real keys agree on the top 26 bits of d2; then
// the 64-bit network).
__device__ __forceinline__ unsigned long long sort_keys_desc(unsigned long long v, uint32_t lane) {
    constexpr uint32_t EMPTY_TOP = (uint32_t)(KEY_EMPTY >> 32) >> 6;
    const uint32_t s = sort64_u32<false>(((uint32_t)(v >> 32) & ~63u) | lane, lane);
    const uint32_t p = (uint32_t)__shfl_up((int)s, 1u, 64);
    const bool near = lane >= 1u && (s >> 6) == (p >> 6) && (s >> 6) != EMPTY_TOP;
    if (__builtin_amdgcn_ballot_w64(near) == 0ull) return shfl64(v, (int)(s & 63u));
    return sort64_desc(v, lane);
}

// Merge query j's pending candidates into its list, dropping the query's own
// key (the hot loop does not test for it); returns the new distance bound.
// `fresh`: the list still holds only its placeholders (tau, 0xFFFFFFFF),
// which exceed every pending key (pending keys have d2 <= tau and a real
// index): the result is then the pending keys sorted ascending (a descending
// sort of their complements), with empty keys after them, and the list is
// not read.
template <bool POS>
__device__ __forceinline__ float flush(unsigned long long* __restrict__ lst,
                                       const typename Pending<POS>::T* __restrict__ pend, uint32_t cnt,
                                       uint32_t lane, uint32_t k, unsigned long long selfkey,
                                       const float4* __restrict__ cand4, float4 q, bool fresh = false) {
    wave_lds_fence();
    unsigned long long v = lane < cnt ? pending_key<POS>(cand4, pend, lane, q) : KEY_EMPTY;
    if (v == selfkey) v = KEY_EMPTY;
    if (fresh) {
        v = sort_keys_asc(v, lane, k);
    } else {
        const unsigned long long L = lane < k ? lst[lane] : KEY_EMPTY;
        // (the 32-bit form costs large inputs a wave per SIMD in registers)
        v = POS ? sort64_desc(v, lane) : sort_keys_desc(v, lane);
        v = merge64_asc(L < v ? L : v, lane);
    }
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
                                           float* b1, bool fresh = false) {
    wave_lds_fence();
    const bool up = lane >= 32u;
    const uint32_t h = lane & 31u;
    const bool act = !up || two;
    unsigned long long* const lst = up ? lst1 : lst0;
    const typename Pending<POS>::T* const pend = up ? pend1 : pend0;
    const uint32_t cnt = up ? cnt1 : cnt0;
    unsigned long long v = act && h < cnt ? pending_key<POS>(cand4, pend, h, up ? q1 : q0) : KEY_EMPTY;
    if (v == (up ? self1 : self0)) v = KEY_EMPTY;
    if (fresh) {  // both lists hold only placeholders (see flush)
        v = ~sort32x2_desc(~v, lane);
    } else {
        const unsigned long long L = act && h < k ? lst[h] : KEY_EMPTY;
        v = sort32x2_desc(v, lane);
        v = merge32x2_asc(L < v ? L : v, lane);
    }
    if (act && h < k) lst[h] = v;
    wave_lds_fence();
    const uint32_t hi = (uint32_t)(v >> 32);
    *b0 = bound_of((uint32_t)__builtin_amdgcn_readlane((int)hi, (int)k - 1));
    *b1 = bound_of((uint32_t)__builtin_amdgcn_readlane((int)hi, 32 + (int)k - 1));
}

// ---------------------------------------------------------------- kNN by culling groups
//
// The candidates of an item are visited in aligned groups of KNN_GRP P1
// positions (one per lane), whose bounding boxes the bound kernel wrote. Up
// to 64 groups at a time are mapped onto the lanes (their boxes loaded in one
// coalesced load) and box-tested against every query of the tile, with the
// same fp32 operations as dist2: a query skips a group whose box distance
// exceeds its bound, so the group holds no candidate with d2 <= that bound.
// Lane u then holds group u's mask of the queries that need it; a group is
// loaded only if some query needs it, four at a time (with PREFETCH the next
// four are fetched while these are evaluated). Positions of a group outside
// the range's part in this chunk are not candidates: they get NaN coordinates
// (d2 <= bound never holds). Groups of the range holding the tile come first,
// from the tile's group outwards, then the other ranges in order.
// PREFETCH (single frames): the extra registers drop the kernel to 4 waves
// per SIMD, which is what their grid launches anyway; large inputs run 5
// waves per SIMD and lose more to the lower occupancy than they gain.
template <bool POS, int Q, bool PREFETCH = !POS>
__global__ __launch_bounds__(64) void knn_group_kernel(Plan P, const float4* __restrict__ cand4, int kk) {
    using PT = typename Pending<POS>::T;
    static_assert(Q <= 32, "tile shape (a query mask per group fits 32 bits)");
    extern __shared__ unsigned long long s_dyn[];
    const uint32_t lane = threadIdx.x;
    const uint32_t k = (uint32_t)kk;
    const bool half = k <= 32u;
    unsigned long long* const s_list = s_dyn;           // [Q][k]
    PT* const s_pend = (PT*)(s_dyn + (size_t)Q * k);    // [Q][PEND]
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

        // lists start as k tau placeholders (or empty); lane j < qn holds query
        // j's coordinates, bound (`worst`: candidates with d2 <= worst may
        // enter) and pending count
        float worst = -1.0f;
        float4 qv = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lane < qn) {
            const float tb = P.tau_c[w.q0 + lane];
            worst = tb >= 0.0f ? tb : INFINITY;
            qv = cand4[w.q0 + lane];
        }
        uint32_t pcnt = 0;
        for (uint32_t j = 0; j < qn; ++j) {
            const float tb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(worst), (int)j));
            if (lane < k) s_list[j * k + lane] = tb < INFINITY ? make_key(tb, NONE32) : KEY_EMPTY;
        }
        wave_lds_fence();

        unsigned long long merged = 0;  // bit j: query j's list has been merged into during this item
        for (uint32_t ub = 0; ub < n_units; ub += 64u) {
            // lane u: unit ub + u -> its range's part [ua, ue) and group ug
            const uint32_t u = ub + lane;
            uint32_t ug = 0, ua = 0, ue = 0;
            const bool uok = u < n_units;
            {
                uint32_t r = ro;
                if (u < gno) {
                    if (u == 0u) ug = gt;
                    else if (u <= 2u * n_alt) ug = (u & 1u) ? gt + ((u + 1u) >> 1) : gt - ((u + 1u) >> 1);
                    else ug = n_up > n_dn ? gt + (u - n_alt) : gt - (u - n_alt);
                } else {
                    const uint32_t v = u - gno;
                    uint32_t vg = 0;
                    for (uint32_t q = 0; q < nr; ++q) {
                        const uint32_t pn = (uint32_t)__builtin_amdgcn_readlane((int)u2n, (int)q);
                        const uint32_t pp = (uint32_t)__builtin_amdgcn_readlane((int)u2pre, (int)q);
                        if (pn > 0u && pp <= v) {
                            r = q;
                            vg = (uint32_t)__builtin_amdgcn_readlane((int)g0, (int)q) + (v - pp);
                        }
                    }
                    ug = vg;
                }
                ua = (uint32_t)__shfl((int)sa, (int)r, 64);
                ue = (uint32_t)__shfl((int)sb, (int)r, 64);
            }
            // lane u: its group's box, the smallest box distance to a query of
            // the tile and the queries that need the group (bit j: the box
            // distance to query j does not exceed its bound)
            uint32_t qmask = 0;
            float bmin = INFINITY;
            if (uok) {
                const GroupBox B = P.gbox[ug];
                for (uint32_t j = 0; j < qn; ++j) {
                    const float4 q = query_of(qv, j);
                    const float wj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(worst), (int)j));
                    const float gx = fmaxf(fmaxf(B.lo.x - q.x, q.x - B.hi.x), 0.0f);
                    const float gy = fmaxf(fmaxf(B.lo.y - q.y, q.y - B.hi.y), 0.0f);
                    const float gz = fmaxf(fmaxf(B.lo.z - q.z, q.z - B.hi.z), 0.0f);
                    const float bd = (gx * gx + gy * gy) + gz * gz;
                    bmin = fminf(bmin, bd);
                    if (!(bd > wj)) qmask |= 1u << j;
                }
            }
            const uint32_t nn = (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(qmask != 0u));
            if (nn == 0u) continue;
            // needed groups nearest first (by the top 26 bits of the box
            // distance, a visiting order only): sorted descending over the
            // lanes, so the i-th nearest sits in lane 63 - i
            const uint32_t sk =
                sort64_u32<false>(qmask ? ((__float_as_uint(bmin) & ~63u) | (63u - lane)) : 0xFFFFFFFFu, lane);
            // the KNN_NB needed groups from the i-th on: candidates in
            // registers (NaN outside the range part), group base and query
            // mask uniform
            auto load_batch = [&](uint32_t i, float4 (&c)[KNN_NB], uint32_t (&gb)[KNN_NB], uint32_t (&mk)[KNN_NB]) {
#pragma unroll
                for (int b = 0; b < KNN_NB; ++b) {
                    const float nan = __uint_as_float(0x7FC00000u);
                    c[b] = make_float4(nan, nan, nan, __uint_as_float(NONE32));
                    gb[b] = 0u;
                    mk[b] = 0u;
                    if (i + (uint32_t)b < nn) {
                        const uint32_t uu =
                            63u - ((uint32_t)__builtin_amdgcn_readlane((int)sk, 63 - (int)(i + (uint32_t)b)) & 63u);
                        const uint32_t gg = (uint32_t)__builtin_amdgcn_readlane((int)ug, (int)uu);
                        const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)ua, (int)uu);
                        const uint32_t e = (uint32_t)__builtin_amdgcn_readlane((int)ue, (int)uu);
                        mk[b] = (uint32_t)__builtin_amdgcn_readlane((int)qmask, (int)uu);
                        gb[b] = gg * (uint32_t)KNN_GRP;
                        const uint32_t p = gb[b] + lane;
                        if (p >= a && p < e) c[b] = cand4[p];
                    }
                }
            };
            float4 c[KNN_NB];
            uint32_t gb[KNN_NB], mk[KNN_NB];
            load_batch(0u, c, gb, mk);
            for (uint32_t i0 = 0; i0 < nn; i0 += (uint32_t)KNN_NB) {
                // PREFETCH: the next batch's candidates are loaded while this
                // one is evaluated (a long item needs many batches in turn)
                float4 cn[KNN_NB];
                uint32_t gbn[KNN_NB], mkn[KNN_NB];
                if constexpr (PREFETCH) {
                    if (i0 + (uint32_t)KNN_NB < nn) load_batch(i0 + (uint32_t)KNN_NB, cn, gbn, mkn);
                }
                uint32_t qany = 0;
#pragma unroll
                for (int b = 0; b < KNN_NB; ++b) qany |= mk[b];
                // each query that needs any of them, against those it needs:
                // the passing candidates of all of them at the query's bound;
                // appended at once unless the buffer would overflow or a group
                // holds more than k + 1 passing candidates
                while (qany != 0u) {
                    const uint32_t j = (uint32_t)__ffs(qany) - 1u;
                    qany &= qany - 1u;
                    const float4 q = query_of(qv, j);
                    float wj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(worst), (int)j));
                    float d[KNN_NB];
                    unsigned long long m[KNN_NB];
                    uint32_t tot = 0;
                    bool slow = false;
#pragma unroll
                    for (int b = 0; b < KNN_NB; ++b) {
                        d[b] = INFINITY;
                        m[b] = 0ull;
                        if ((mk[b] >> j) & 1u) {
                            d[b] = dist2(q, c[b]);
                            m[b] = __builtin_amdgcn_ballot_w64(d[b] <= wj);
                            const uint32_t pc = (uint32_t)__popcll(m[b]);
                            tot += pc;
                            slow = slow || (pc > k + 1u && wj < INFINITY);
                        }
                    }
                    if (tot == 0u) continue;
                    uint32_t cnt = (uint32_t)__builtin_amdgcn_readlane((int)pcnt, (int)j);
                    PT* const pend = s_pend + (size_t)j * PEND;
                    if (!slow && cnt + tot <= (uint32_t)PEND) {
#pragma unroll
                        for (int b = 0; b < KNN_NB; ++b) {
                            if (m[b] == 0ull) continue;
                            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(m[b] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m[b], 0u));
                            if (d[b] <= wj) {  // this lane's bit of m[b]
                                if constexpr (POS)
                                    pend[cnt + rank] = gb[b] + lane;
                                else
                                    pend[cnt + rank] = make_key(d[b], __float_as_uint(c[b].w));
                            }
                            cnt += (uint32_t)__popcll(m[b]);
                        }
                    } else {
                        // one group at a time: a group holding more than k + 1
                        // passing candidates (one may be the query) first lowers
                        // the bound (if k + 1 of them lie within wj * 2^(-1/4),
                        // the k-th distance cannot exceed it); a full buffer is
                        // merged into the list, which lowers the bound too
                        const unsigned long long selfkey =
                            (unsigned long long)(uint32_t)__builtin_amdgcn_readlane(__float_as_int(qv.w), (int)j);
                        bool mj = false;
#pragma nounroll
                        for (int b = 0; b < KNN_NB; ++b) {
                            float db = d[0];
                            uint32_t gbb = gb[0];
                            float cw = c[0].w;
#pragma unroll
                            for (int x = 1; x < KNN_NB; ++x)
                                if (b == x) {
                                    db = d[x];
                                    gbb = gb[x];
                                    cw = c[x].w;
                                }
                            unsigned long long mm = __builtin_amdgcn_ballot_w64(db <= wj);
                            if (mm == 0ull) continue;
                            uint32_t pc = (uint32_t)__popcll(mm);
                            if (pc > k + 1u && wj < INFINITY) {
                                for (int r = 0; r < 12; ++r) {
                                    const float t2 = wj * 0.84089642f;
                                    if ((uint32_t)__popcll(__builtin_amdgcn_ballot_w64(db <= t2)) < k + 1u) break;
                                    wj = t2;
                                }
                                mm = __builtin_amdgcn_ballot_w64(db <= wj);
                                pc = (uint32_t)__popcll(mm);
                            }
                            if (cnt + pc > (uint32_t)PEND) {
                                wj = fminf(wj, flush<POS>(s_list + (size_t)j * k, pend, cnt, lane, k, selfkey, cand4, q));
                                mj = true;
                                cnt = 0;
                                mm = __builtin_amdgcn_ballot_w64(db <= wj);
                                pc = (uint32_t)__popcll(mm);
                            }
                            if (pc) {
                                const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                                    (uint32_t)(mm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mm, 0u));
                                if (db <= wj) {  // this lane's bit of mm
                                    if constexpr (POS)
                                        pend[cnt + rank] = gbb + lane;
                                    else
                                        pend[cnt + rank] = make_key(db, __float_as_uint(cw));
                                }
                                cnt += pc;
                            }
                        }
                        if (lane == j) worst = wj;
                        if (mj) merged |= 1ull << j;
                    }
                    if (lane == j) pcnt = cnt;
                }
                if (i0 + (uint32_t)KNN_NB < nn) {
                    if constexpr (PREFETCH) {
#pragma unroll
                        for (int b = 0; b < KNN_NB; ++b) {
                            c[b] = cn[b];
                            gb[b] = gbn[b];
                            mk[b] = mkn[b];
                        }
                    } else {
                        load_batch(i0 + (uint32_t)KNN_NB, c, gb, mk);
                    }
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
                const bool f0 = ((merged >> j) & 1ull) == 0ull;
                const bool f1 = !two || ((merged >> j1) & 1ull) == 0ull;
                if (c0 <= (uint32_t)PEND_HALF && c1 <= (uint32_t)PEND_HALF) {
                    float b0, b1;
                    flush_half<POS>(l0, p0, c0, sk0, q0, l0 + k, p0 + PEND, c1, sk1, q1, two, lane, k, cand4, &b0,
                                    &b1, f0 && f1);
                } else {
                    if (c0) (void)flush<POS>(l0, p0, c0, lane, k, sk0, cand4, q0, f0);
                    if (c1) (void)flush<POS>(l0 + k, p0 + PEND, c1, lane, k, sk1, cand4, q1, f1);
                }
            }
        } else {
            for (uint32_t j = 0; j < qn; ++j) {
                const uint32_t cnt = (uint32_t)__builtin_amdgcn_readlane((int)pcnt, (int)j);
                const unsigned long long selfkey =
                    (unsigned long long)(uint32_t)__builtin_amdgcn_readlane(__float_as_int(qv.w), (int)j);
                if (cnt)
                    (void)flush<POS>(s_list + (size_t)j * k, s_pend + (size_t)j * PEND, cnt, lane, k, selfkey,
                                     cand4, query_of(qv, j), ((merged >> j) & 1ull) == 0ull);
            }
        }

        if (nch > 1) {
            unsigned long long* base = (unsigned long long*)P.plist + (size_t)P.leaf_plist[t] * k;
            for (uint32_t j = 0; j < qn; ++j)
                if (lane < k) base[((size_t)(w.q0 + j - qb) * nch + w.chunk) * k + lane] = s_list[j * k + lane];
        } else {
            write_tile(P, s_list, w.q0, qn, k, lane);
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
        const uint32_t q0 = w.q0 + part * (P.tq / (uint32_t)MERGE_SPLIT);
        if (q0 >= w.q1) continue;
        const uint32_t q1 = min(w.q1, q0 + P.tq / (uint32_t)MERGE_SPLIT);
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
    hipLaunchKernelGGL(knn_bound_kernel, dim3(blocks),
                       dim3(BOUND_Q * BOUND_SPLIT), 0, st, P, (const float4*)P.cand4, k);
}

size_t knn_lds_bytes(uint32_t q, int k, bool pos) {
    return (size_t)q * ((size_t)k * sizeof(unsigned long long) +
                        (size_t)PEND * (pos ? sizeof(uint32_t) : sizeof(unsigned long long)));
}

void launch_knn(const Plan& P, int k, int num_cus, hipStream_t st) {
    const unsigned blocks = (unsigned)(num_cus > 0 ? num_cus : 256) * (P.n > KNN_POS_MIN_N ? 20u : 16u);
    // Large batches run long enough for occupancy to pay (positions); a single
    // frame's run is set by its longest items, where a gather per merge costs
    // more (keys).
    // The plan's tile size goes with the pending-buffer kind: tiles of
    // KNN_TQ_SMALL queries exactly for the inputs that keep keys.
    static_assert(KNN_TQ_SMALL_MAX_N == KNN_POS_MIN_N, "tile size and buffer kind switch together");
    if (P.n > KNN_POS_MIN_N)
        hipLaunchKernelGGL((knn_group_kernel<true, KNN_TQ>), dim3(blocks), dim3(64), knn_lds_bytes(KNN_TQ, k, true),
                           st, P, (const float4*)P.cand4, k);
    else
        hipLaunchKernelGGL((knn_group_kernel<false, KNN_TQ_SMALL>), dim3(blocks), dim3(64),
                           knn_lds_bytes(KNN_TQ_SMALL, k, false), st, P, (const float4*)P.cand4, k);
}

void launch_knn_merge(const Plan& P, int k, int num_cus, hipStream_t st) {
    const unsigned blocks = (unsigned)(num_cus > 0 ? num_cus : 256) * 8u;
    hipLaunchKernelGGL(knn_merge_kernel, dim3(blocks), dim3(64), 0, st, P, k);
}

}  // namespace gdn
