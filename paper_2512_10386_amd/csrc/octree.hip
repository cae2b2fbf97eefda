// Octree partition (Sec. 3), per-leaf adaptive voxel filter (Eq. 10-12),
// compaction of P1, the 27-cell halo candidate ranges of each leaf and the
// kNN work plan.
#include "kernels.hpp"
#include "scan.hpp"
#include "wave.hpp"

namespace gdn {

// Number of leading octal digits two 63-bit Morton keys share (21 if equal).
__device__ __forceinline__ int common_digits(uint64_t a, uint64_t b) {
    if (a == b) return MORTON_BITS;
    return (__clzll((long long)(a ^ b)) - 1) / 3;
}

// ---------------------------------------------------------------- leaves
//
// Leaves are the non-empty nodes reached by splitting every node that holds
// more than leaf_cap points above the depth limit. In the sorted key order a
// leaf boundary falls between positions j-1 and j exactly when the deepest
// cell holding both (level l = their common digits) is split, i.e. l < dmax
// and that cell holds more than leaf_cap points. The cell count is tested
// with one windowed binary search (window leaf_cap + 1).

// Frame of sorted position j (frames keep their input ranges after the sort).
__device__ __forceinline__ uint32_t frame_of_sorted(const Plan& P, uint32_t j) {
    return P.nf > 1 ? frame_of(P.foff, P.nf, j) : 0u;
}

// Boundary test of sorted position j inside its frame [fs, fe): the frame's
// first point starts a leaf; otherwise the rule above with the frame's depth
// limit and the search window clipped to the frame.
// Positions that share a level-10 cell lie in one leaf unless the cell is
// deep (more than leaf_cap points: it was re-sorted on the whole key, and the
// test below applies inside it).
__device__ uint32_t leaf_boundary(const uint64_t* keys, uint32_t j, uint32_t fs, uint32_t fe, int dmax, bool deep,
                                  uint32_t cap) {
    if (j == fs) return 1u;
    const uint64_t a = keys[j - 1], b = keys[j];
    const int l = common_digits(a, b);
    if (l >= dmax || (l >= SORT_SHORT_LEVEL && !deep)) return 0u;
    const int sh = 3 * (MORTON_BITS - l);
    const uint64_t P = b >> sh;
    uint32_t lo = (j - 1 - fs > cap) ? j - 1 - cap : fs;
    uint32_t hi = j - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if ((keys[mid] >> sh) < P) lo = mid + 1;
        else hi = mid;
    }
    const uint64_t probe = (uint64_t)lo + cap;
    return (probe < fe && (keys[probe] >> sh) == P) ? 1u : 0u;
}

struct BoundaryEmit {
    uint32_t* leaf_of;
    uint32_t* leaf_begin;
    __device__ void operator()(uint32_t j, uint32_t ex, uint32_t f) const {
        leaf_of[j] = ex + f - 1u;
        if (f) leaf_begin[ex] = j;
    }
};

struct BoundaryFin {
    Counters* c;
    uint32_t* leaf_begin;
    uint32_t n;
    __device__ void operator()(uint32_t total) const {
        c->n_leaves = total;
        leaf_begin[total] = n;
    }
};

// Level and prefix of leaf t = [s, e) of frame [fs, fe): with m = the larger
// of the common digits across its two borders, the leaf is the level-(m+1)
// cell unless it is an over-full cell at the depth limit. (The halo kernel
// derives them as it starts on the leaf.)
__device__ __forceinline__ int leaf_level_of(const Plan& P, uint32_t s, uint32_t e, uint32_t fs, uint32_t fe,
                                             int dmax, uint32_t cap) {
    int m = -1;
    if (s > fs) m = common_digits(P.keys_a[s - 1], P.keys_a[s]);
    if (e < fe) m = max(m, common_digits(P.keys_a[e - 1], P.keys_a[e]));
    int level = (e - s <= cap) ? m + 1 : dmax;
    return level < 0 ? 0 : (level > MORTON_BITS ? MORTON_BITS : level);
}

// The boundary tests run one thread per position (each is a chain of
// dependent loads); the scan then only reads the flags. The same pass
// gathers the points' coordinates into sorted order (pos4: x, y, z and the
// original index's bits); each XCD takes one eighth of the positions, so a
// frame's coordinates are fetched into one XCD's L2.
// LDS: the batch's frame offsets are staged in LDS (fewer than SORT_FOFF_LDS
// frames); a compile-time choice, so that the offsets are read with LDS or
// with global instructions rather than generic ones through a pointer that
// may be either.
template <bool LDS>
__global__ __launch_bounds__(256) void boundary_flag_kernel(Plan P, uint32_t cap, const float* __restrict__ xyz) {
    // batches of fewer than SORT_FOFF_LDS frames search the offsets in LDS
    __shared__ uint32_t s_foff[SORT_FOFF_LDS];
    constexpr bool lds = LDS;
    if (lds) {
        for (uint32_t i = threadIdx.x; i <= P.nf; i += blockDim.x) s_foff[i] = P.foff[i];
        __syncthreads();
    }
    const XcdPart R = xcd_part(P.n);
    for (uint32_t j = R.first; j < R.end; j += R.step) {
        const uint32_t i = P.idx_a[j];
        P.pos4[j] = make_float4(xyz[3 * (size_t)i], xyz[3 * (size_t)i + 1], xyz[3 * (size_t)i + 2], __uint_as_float(i));
        uint32_t f, fs, fe;
        if (lds) {
            f = frame_of(s_foff, P.nf, j);
            fs = s_foff[f];
            fe = s_foff[f + 1];
        } else {
            f = frame_of_sorted(P, j);
            fs = P.foff[f];
            fe = P.foff[f + 1];
        }
        P.bflag[j] = (uint8_t)leaf_boundary(P.keys_a, j, fs, fe, P.fc[f].dmax, P.deepf[j] != 0u, cap);
    }
}

struct FlagGet {
    const uint8_t* f;
    __device__ uint32_t operator()(uint32_t j) const { return f[j]; }
};

void launch_leaves(const Plan& P, const Params& prm, const float* xyz, hipStream_t st) {
    unsigned blocks = (P.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    const bool lds = P.nf > 1u && P.nf < SORT_FOFF_LDS;
    hipLaunchKernelGGL(lds ? boundary_flag_kernel<true> : boundary_flag_kernel<false>, dim3(xcd_grid(blocks)), dim3(256),
                       0, st, P, (uint32_t)prm.leaf_cap,
                       xyz);
    BoundaryEmit e{P.leaf_of, P.leaf_begin};
    BoundaryFin f{P.ctr, P.leaf_begin, P.n};
    launch_scan(FlagGet{P.bflag}, e, f, nullptr, P.n, P.scan_status, &P.ctr->status, st);
}

// ---------------------------------------------------------------- voxel filter
//
// One workgroup per leaf: tight fp32 bbox of the leaf's points, V_t (Eq. 10),
// h = beta * (V_t / N_t)^(1/3) rounded to fp32 (Eq. 11), voxel index
// floor((x - min) / h) per axis in FP64, occupancy n(voxel(p)) by an
// LDS-private hash (a per-leaf global region for leaves too big for LDS), and
// P1 = occupancy >= n_v (Eq. 12).

__device__ __forceinline__ uint32_t vox_hash(uint64_t k) {
    return (uint32_t)((k * 0x9E3779B97F4A7C15ull) >> 32);
}

__device__ __forceinline__ uint64_t vox_key(float4 p, float mx_, float my_, float mz_, double h) {
    double v[3] = {floor(((double)p.x - (double)mx_) / h), floor(((double)p.y - (double)my_) / h),
                   floor(((double)p.z - (double)mz_) / h)};
    uint64_t k = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double f = v[a];
        if (!(f >= 0.0)) f = 0.0;
        if (f > (double)QMAX) f = (double)QMAX;
        k |= (uint64_t)f << (21 * a);
    }
    return k;
}

// Leaf voxel size (Eq. 10, 11) from its fp32 bbox: h = beta * cbrt(V / nt)
// rounded to fp32, 0 for a flat or degenerate leaf.
__device__ __forceinline__ float leaf_voxel_size(const float* lo, const float* hi, uint32_t nt, double beta) {
    double H[3];
    for (int a = 0; a < 3; ++a) H[a] = (double)hi[a] - (double)lo[a];
    const double V = (H[0] * H[1]) * H[2];
    float h32 = (float)(beta * cbrt(V / (double)nt));
    if (!(h32 > 0.0f) || !isfinite(h32)) h32 = 0.0f;
    return h32;
}

// Small leaves (at most VOX_WAVE_MAX points) of large batches: one wave per
// leaf with its own LDS table, no block barriers; every lane computes the
// leaf's h (uniform) instead of one thread behind two barriers. Same
// expressions and hash as voxel_kernel, so the counts are identical.
constexpr uint32_t VOX_WAVE_MAX = 256;
constexpr uint32_t VOX_WAVE_SLOTS = 2 * VOX_WAVE_MAX;
constexpr uint32_t VOX_WAVE_MIN_N = 1u << 20;

__global__ __launch_bounds__(256) void voxel_wave_kernel(Plan P, double beta, uint32_t nv) {
    __shared__ unsigned long long s_key[4][VOX_WAVE_SLOTS];
    __shared__ uint32_t s_cnt[4][VOX_WAVE_SLOTS];
    constexpr unsigned long long EMPTY = ~0ull;
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    const uint32_t nl = P.ctr->n_leaves;
    unsigned long long* tk = s_key[w];
    uint32_t* tc = s_cnt[w];
    for (uint32_t t = wid; t < nl; t += nw) {
        const uint32_t b = P.leaf_begin[t], e = P.leaf_begin[t + 1], nt = e - b;
        if (nt > VOX_WAVE_MAX) continue;
        float4 p[VOX_WAVE_MAX / 64];
        float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
        for (uint32_t r = 0; r < VOX_WAVE_MAX / 64; ++r) {
            const uint32_t s = b + r * 64u + lane;
            if (s < e) {
                p[r] = P.pos4[s];
                mn[0] = fminf(mn[0], p[r].x); mx[0] = fmaxf(mx[0], p[r].x);
                mn[1] = fminf(mn[1], p[r].y); mx[1] = fmaxf(mx[1], p[r].y);
                mn[2] = fminf(mn[2], p[r].z); mx[2] = fmaxf(mx[2], p[r].z);
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                mn[a] = fminf(mn[a], __shfl_xor(mn[a], o, 64));
                mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], o, 64));
            }
        const float h32 = leaf_voxel_size(mn, mx, nt, beta);
        if (lane == 0u) P.leaf_h[t] = h32;
        if (h32 == 0.0f) {
            for (uint32_t s = b + lane; s < e; s += 64u) {
                P.occ[s] = nt;
                P.p1[s] = nt >= nv;
            }
            continue;
        }
        const double h = (double)h32;
        uint32_t slots = 64u;
        while (slots < 2u * nt) slots <<= 1;
        for (uint32_t i = lane; i < slots; i += 64u) {
            tk[i] = EMPTY;
            tc[i] = 0u;
        }
        wave_lds_fence();
        unsigned long long key[VOX_WAVE_MAX / 64];
#pragma unroll
        for (uint32_t r = 0; r < VOX_WAVE_MAX / 64; ++r) {
            const uint32_t s = b + r * 64u + lane;
            if (s < e) {
                key[r] = vox_key(p[r], mn[0], mn[1], mn[2], h);
                uint32_t slot = vox_hash(key[r]) & (slots - 1u);
                for (uint32_t probe = 0; probe < slots; ++probe) {
                    const unsigned long long prev = atomicCAS(&tk[slot], EMPTY, key[r]);
                    if (prev == EMPTY || prev == key[r]) {
                        atomicAdd(&tc[slot], 1u);
                        break;
                    }
                    slot = (slot + 1 == slots) ? 0u : slot + 1;
                }
            }
        }
        wave_lds_fence();
#pragma unroll
        for (uint32_t r = 0; r < VOX_WAVE_MAX / 64; ++r) {
            const uint32_t s = b + r * 64u + lane;
            if (s < e) {
                uint32_t slot = vox_hash(key[r]) & (slots - 1u);
                uint32_t c = 0;
                for (uint32_t probe = 0; probe < slots; ++probe) {
                    if (tk[slot] == key[r]) {
                        c = tc[slot];
                        break;
                    }
                    slot = (slot + 1 == slots) ? 0u : slot + 1;
                }
                P.occ[s] = c;
                P.p1[s] = c >= nv;
            }
        }
        wave_lds_fence();
    }
}

// SLOTS: LDS hash capacity, picked from the leaf cap so that small-leaf
// octrees keep many workgroups per CU; leaves above SLOTS/2 points (only
// over-full leaves at the depth limit, or caps above 2048) use the global
// per-leaf region.
template <int SLOTS>
__global__ __launch_bounds__(VOX_BLOCK) void voxel_kernel(Plan P, double beta, uint32_t nv, bool skip_small) {
    __shared__ unsigned long long s_key[SLOTS];
    __shared__ uint32_t s_cnt[SLOTS];
    __shared__ float s_red[6][VOX_BLOCK / 64];
    __shared__ float s_mn[3];
    __shared__ float s_h;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t nl = P.ctr->n_leaves;
    constexpr unsigned long long EMPTY = ~0ull;
    for (uint32_t t = blockIdx.x; t < nl; t += gridDim.x) {
        const uint32_t b = P.leaf_begin[t], e = P.leaf_begin[t + 1], nt = e - b;
        if (skip_small && nt <= VOX_WAVE_MAX) continue;  // voxel_wave_kernel
        float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (uint32_t s = b + tid; s < e; s += VOX_BLOCK) {
            float4 p = P.pos4[s];
            mn[0] = fminf(mn[0], p.x); mx[0] = fmaxf(mx[0], p.x);
            mn[1] = fminf(mn[1], p.y); mx[1] = fmaxf(mx[1], p.y);
            mn[2] = fminf(mn[2], p.z); mx[2] = fmaxf(mx[2], p.z);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                mn[a] = fminf(mn[a], __shfl_xor(mn[a], o, 64));
                mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], o, 64));
            }
        if (lane == 0)
            for (int a = 0; a < 3; ++a) { s_red[a][wave] = mn[a]; s_red[3 + a][wave] = mx[a]; }
        __syncthreads();
        if (tid == 0) {
            float lo[3], hi[3];
            for (int a = 0; a < 3; ++a) {
                lo[a] = s_red[a][0];
                hi[a] = s_red[3 + a][0];
                for (int w = 1; w < VOX_BLOCK / 64; ++w) {
                    lo[a] = fminf(lo[a], s_red[a][w]);
                    hi[a] = fmaxf(hi[a], s_red[3 + a][w]);
                }
                s_mn[a] = lo[a];
            }
            const float h32 = leaf_voxel_size(lo, hi, nt, beta);
            s_h = h32;
            P.leaf_h[t] = h32;
        }
        __syncthreads();
        const float h32 = s_h;
        if (h32 == 0.0f) {
            for (uint32_t s = b + tid; s < e; s += VOX_BLOCK) {
                P.occ[s] = nt;
                P.p1[s] = nt >= nv;
            }
        } else {
            const double h = (double)h32;
            const float m0 = s_mn[0], m1 = s_mn[1], m2 = s_mn[2];
            // LDS table sized to the leaf: a power of two >= 2 nt (>= 64)
            const bool lds = nt <= SLOTS / 2;
            uint32_t slots = 2u * nt;
            if (lds) {
                uint32_t p2 = 64u;
                while (p2 < slots) p2 <<= 1;
                slots = p2;
            }
            unsigned long long* tk = lds ? s_key : (unsigned long long*)(P.vox_keys + 2 * (size_t)b);
            uint32_t* tc = lds ? s_cnt : P.vox_cnt + 2 * (size_t)b;
            for (uint32_t i = tid; i < slots; i += VOX_BLOCK) { tk[i] = EMPTY; tc[i] = 0u; }
            __syncthreads();
            for (uint32_t s = b + tid; s < e; s += VOX_BLOCK) {
                const unsigned long long k = vox_key(P.pos4[s], m0, m1, m2, h);
                uint32_t slot = lds ? (vox_hash(k) & (slots - 1u)) : vox_hash(k) % slots;
                for (uint32_t probe = 0; probe < slots; ++probe) {
                    unsigned long long prev = atomicCAS(&tk[slot], EMPTY, k);
                    if (prev == EMPTY || prev == k) {
                        atomicAdd(&tc[slot], 1u);
                        break;
                    }
                    slot = (slot + 1 == slots) ? 0u : slot + 1;
                }
            }
            __syncthreads();
            for (uint32_t s = b + tid; s < e; s += VOX_BLOCK) {
                const unsigned long long k = vox_key(P.pos4[s], m0, m1, m2, h);
                uint32_t slot = lds ? (vox_hash(k) & (slots - 1u)) : vox_hash(k) % slots;
                uint32_t c = 0;
                for (uint32_t probe = 0; probe < slots; ++probe) {
                    if (tk[slot] == k) { c = tc[slot]; break; }
                    slot = (slot + 1 == slots) ? 0u : slot + 1;
                }
                P.occ[s] = c;
                P.p1[s] = c >= nv;
            }
        }
        __syncthreads();
    }
}

void launch_voxel(const Plan& P, const Params& prm, hipStream_t st) {
    // the wave path pays off for the many small leaves of large batches
    const bool small = P.n > VOX_WAVE_MIN_N;
    if (small) {
        unsigned wb = (P.n / 128 + 3) / 4;
        if (wb > 8192) wb = 8192;
        hipLaunchKernelGGL(voxel_wave_kernel, dim3(wb), dim3(256), 0, st, P, prm.beta, (uint32_t)prm.min_vox_count);
    }
    unsigned blocks = P.n / 128;
    if (blocks > (small ? 2048u : 16384u)) blocks = small ? 2048u : 16384u;  // small: only the big leaves remain
    if (blocks == 0) blocks = 1;
    if (prm.leaf_cap <= 256)
        hipLaunchKernelGGL(voxel_kernel<512>, dim3(blocks), dim3(VOX_BLOCK), 0, st, P, prm.beta,
                           (uint32_t)prm.min_vox_count, small);
    else
        hipLaunchKernelGGL(voxel_kernel<VOX_LDS_SLOTS>, dim3(blocks), dim3(VOX_BLOCK), 0, st, P, prm.beta,
                           (uint32_t)prm.min_vox_count, small);
}

// ---------------------------------------------------------------- P1 compaction

struct P1Get {
    const uint8_t* p1;
    __device__ uint32_t operator()(uint32_t s) const { return p1[s]; }
};
struct P1Emit {
    uint32_t* p1pos;
    const float4* pos4;
    const uint32_t* leaf_of;
    float4* cand4;
    uint32_t* cand_leaf;
    uint32_t* inv_p1;
    struct Pre {
        float4 c;
        uint32_t leaf;
    };
    __device__ Pre pre(uint32_t s) const { return Pre{pos4[s], leaf_of[s]}; }
    __device__ void operator()(uint32_t s, uint32_t ex, uint32_t f, const Pre& r) const {
        p1pos[s] = ex;
        if (f) {
            cand4[ex] = r.c;
            cand_leaf[ex] = r.leaf;
            inv_p1[__float_as_uint(r.c.w)] = ex;
        }
    }
};
struct P1Fin {
    Counters* c;
    uint32_t* p1pos;
    uint32_t n;
    __device__ void operator()(uint32_t total) const {
        c->n_p1 = total;
        p1pos[n] = total;
    }
};

void launch_p1_compact(const Plan& P, hipStream_t st) {
    launch_scan(P1Get{P.p1}, P1Emit{P.p1pos, P.pos4, P.leaf_of, P.cand4, P.cand_leaf, P.inv_p1},
                P1Fin{P.ctr, P.p1pos, P.n}, nullptr, P.n, P.scan_status + P.scan_tiles,
                &P.ctr->status, st);
}

// ---------------------------------------------------------------- halo ranges
//
// Candidates of leaf t at level d: the P1 points of the 3x3x3 block of
// level-d cells around the leaf's cell (clipped to the root cube). Each cell
// is one contiguous Morton key range: two binary searches give its sorted
// positions, the P1 prefix sums its compacted range. Ranges are sorted and
// joined where contiguous.

// Both ends of a key range, the two binary searches interleaved so that their
// loads overlap.
__device__ __forceinline__ void lower_bound2_u64(const uint64_t* a, uint32_t n, uint64_t x0, uint64_t x1,
                                                 uint32_t* r0, uint32_t* r1) {
    uint32_t lo0 = 0, hi0 = n, lo1 = 0, hi1 = n;
    while (lo0 < hi0 || lo1 < hi1) {
        const uint32_t m0 = (lo0 + hi0) >> 1, m1 = (lo1 + hi1) >> 1;
        const uint64_t v0 = lo0 < hi0 ? a[m0] : 0ull;
        const uint64_t v1 = lo1 < hi1 ? a[m1] : 0ull;
        if (lo0 < hi0) {
            if (v0 < x0) lo0 = m0 + 1;
            else hi0 = m0;
        }
        if (lo1 < hi1) {
            if (v1 < x1) lo1 = m1 + 1;
            else hi1 = m1;
        }
    }
    *r0 = lo0;
    *r1 = lo1;
}

constexpr int HALO_LEAVES = 8;  // leaves per 256-thread block (32 threads each, 27 used)

// Per leaf, 27 threads find the key ranges of the 27 same-level cells around
// it (clipped to the grid and to the frame), then the non-empty ranges are
// sorted by rank counting and runs of touching ranges merged with ballots;
// the result is the leaf's candidate ranges in P1 order.
template <bool LDS>
__global__ __launch_bounds__(256) void halo_kernel(Plan P, uint32_t cap) {
    __shared__ uint2 s_r[HALO_LEAVES][32];
    __shared__ uint2 s_s[HALO_LEAVES][32];
    const int tid = threadIdx.x, grp = tid >> 5, g = tid & 31;
    const uint32_t lane = (uint32_t)tid & 63u;
    const uint32_t nl = P.ctr->n_leaves;
    // this thread's half of the wave
    const unsigned long long half = (lane & 32u) ? 0xFFFFFFFF00000000ull : 0x00000000FFFFFFFFull;
    const unsigned long long below = lane == 0u ? 0ull : (~0ull >> (64u - lane));
    __shared__ uint32_t s_foff[SORT_FOFF_LDS];  // batches of fewer frames search the offsets here
    constexpr bool lds = LDS;
    if (lds)
        for (uint32_t i = threadIdx.x; i <= P.nf; i += blockDim.x) s_foff[i] = P.foff[i];
    __syncthreads();
    for (uint32_t base = blockIdx.x * HALO_LEAVES; base < nl; base += gridDim.x * HALO_LEAVES) {
        const uint32_t t = base + grp;
        const bool live = t < nl;
        uint2 r = make_uint2(0u, 0u);
        if (live && g < HALO) {
            const uint32_t lb = P.leaf_begin[t], le = P.leaf_begin[t + 1];
            uint32_t f, fs, fe;
            if (lds) {
                f = frame_of(s_foff, P.nf, lb);
                fs = s_foff[f];
                fe = s_foff[f + 1];
            } else {
                f = frame_of_sorted(P, lb);
                fs = P.foff[f];
                fe = P.foff[f + 1];
            }
            const int d = leaf_level_of(P, lb, le, fs, fe, P.fc[f].dmax, cap);
            const uint64_t pre = P.keys_a[lb] >> (3 * (MORTON_BITS - d));
            if (g == 0) {
                P.leaf_level[t] = (uint32_t)d;
                P.leaf_prefix[t] = pre;
            }
            const int64_t cx = compact3(pre), cy = compact3(pre >> 1), cz = compact3(pre >> 2);
            const int64_t nx = cx + (g % 3) - 1, ny = cy + (g / 3) % 3 - 1, nz = cz + g / 9 - 1;
            const int64_t side = (int64_t)1 << d;
            if (nx >= 0 && ny >= 0 && nz >= 0 && nx < side && ny < side && nz < side) {
                const int sh = 3 * (MORTON_BITS - d);
                const uint64_t klo = morton3((uint32_t)nx, (uint32_t)ny, (uint32_t)nz) << sh;
                const uint64_t khi = klo + (1ull << sh);
                uint32_t lo, hi;
                lower_bound2_u64(P.keys_a + fs, fe - fs, klo, khi, &lo, &hi);
                r = make_uint2(P.p1pos[fs + lo], P.p1pos[fs + hi]);
            }
        }
        const bool ne = r.y > r.x;  // distinct cells: non-empty ranges have distinct starts
        s_r[grp][g] = r;
        __syncthreads();
        uint32_t rank = 0;
        if (ne)
            for (int i = 0; i < HALO; ++i) {
                const uint2 o = s_r[grp][i];
                rank += (o.y > o.x && o.x < r.x) ? 1u : 0u;
            }
        if (ne) s_s[grp][rank] = r;
        const uint32_t m = (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(ne) & half);
        __syncthreads();
        // runs of touching ranges: a run starts where the previous range ends elsewhere
        uint2 cur = make_uint2(0u, 0u);
        bool st = false;
        if ((uint32_t)g < m) {
            cur = s_s[grp][g];
            st = g == 0 || s_s[grp][g - 1].y != cur.x;
        }
        const unsigned long long sm = __builtin_amdgcn_ballot_w64(st) & half;
        if (live && st) {
            const unsigned long long later = sm & ~(below | (1ull << lane));
            const uint32_t nxt = later ? (uint32_t)__ffsll((long long)later) - 1u - (lane & 32u) : m;
            const uint32_t o = (uint32_t)__popcll(sm & below);
            const uint2 run = make_uint2(cur.x, s_s[grp][nxt - 1u].y);
            P.leaf_ranges[(size_t)t * HALO + o] = run;
            // the run holding the leaf's own cell (block position 13) holds its queries
            const uint2 own = s_r[grp][13];
            if (own.y > own.x && run.x <= own.x && own.x < run.y) P.leaf_own[t] = run;
        }
        uint32_t len = (uint32_t)g < m ? cur.y - cur.x : 0u;
        for (int o = 16; o > 0; o >>= 1) len += (uint32_t)__shfl_xor((int)len, o, 32);
        if (live && g == 0) {
            P.leaf_nr[t] = (uint32_t)__popcll(sm);
            P.leaf_ncand[t] = len;
        }
        __syncthreads();
    }
}

void launch_halo(const Plan& P, const Params& prm, hipStream_t st) {
    unsigned blocks = (P.n + HALO_LEAVES - 1) / HALO_LEAVES;
    if (blocks > 2048) blocks = 2048;
    if (blocks == 0) blocks = 1;
    const bool lds = P.nf > 1u && P.nf < SORT_FOFF_LDS;
    hipLaunchKernelGGL(lds ? halo_kernel<true> : halo_kernel<false>, dim3(blocks), dim3(256), 0, st, P,
                       (uint32_t)prm.leaf_cap);
}

// ---------------------------------------------------------------- kNN plan
//
// One workgroup. Work items are (leaf, tile of up to KNN_TQ queries,
// candidate chunk). Leaves whose candidate set exceeds the chunk length are
// split into chunks whose partial top-k lists knn_merge_kernel combines; the
// chunk length doubles until the partial lists and items fit their
// workspace. This kernel fixes, per leaf, the chunking and the index of its
// first item. Items of chunked leaves (the heaviest) come first in the
// queue; the other leaves follow in PLAN_CLASSES classes by candidates per
// query, largest first, each class in leaf order. An item's run time grows
// with that ratio (a leaf of few, isolated points next to dense cells has
// far k-th neighbours, so its queries test many candidate groups), and
// starting such items first keeps them out of the kernel's tail. The items
// themselves are written by the bound kernel, one tile per thread.

constexpr int PLAN_BLOCK = 1024;
constexpr int PLAN_R = 2;        // leaves per thread whose sizes stay in registers (more are re-read)
constexpr int PLAN_CLASSES = 4;

__device__ __forceinline__ uint32_t plan_class(uint32_t n1, uint32_t nc) {
    const uint32_t q = n1 > 0 ? n1 : 1u;
    return nc >= 128u * q ? 0u : nc >= 32u * q ? 1u : nc >= 8u * q ? 2u : 3u;
}

// Block exclusive scans of N values per thread at once (one set of
// barriers); smem needs N * (blockDim / 64 + 1) words.
template <int N>
__device__ __forceinline__ void block_excl_scan_n(const uint32_t (&v)[N], uint32_t (&ex)[N], uint32_t (&tot)[N],
                                                  uint32_t* smem) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t inc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) inc[i] = wave_incl_scan(v[i]);
    if (lane == 63) {
#pragma unroll
        for (int i = 0; i < N; ++i) smem[i * (nw + 1) + wave] = inc[i];
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)N) {
        uint32_t* row = smem + threadIdx.x * (nw + 1);
        uint32_t run = 0;
        for (int w = 0; w < nw; ++w) {
            const uint32_t t = row[w];
            row[w] = run;
            run += t;
        }
        row[nw] = run;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        ex[i] = smem[i * (nw + 1) + wave] + inc[i] - v[i];
        tot[i] = smem[i * (nw + 1) + nw];
    }
    __syncthreads();
}

__global__ __launch_bounds__(PLAN_BLOCK) void knn_plan_kernel(Plan P, int chunk0) {
    constexpr int NS = 2 + PLAN_CLASSES;  // partial lists, chunked items, items per class
    __shared__ unsigned long long s_red[PLAN_BLOCK / 64][3];
    __shared__ uint32_t s_scan[NS * (PLAN_BLOCK / 64 + 1)];
    __shared__ uint32_t s_cc, s_done, s_carry[NS], s_base[NS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t nl = P.ctr->n_leaves;
    // this thread's leaves t = tid + r * PLAN_BLOCK: P1 points and candidates
    uint32_t c_n1[PLAN_R], c_nc[PLAN_R];
#pragma unroll
    for (int r = 0; r < PLAN_R; ++r) {
        const uint32_t t = (uint32_t)tid + (uint32_t)r * PLAN_BLOCK;
        c_n1[r] = 0;
        c_nc[r] = 0;
        if (t < nl) {
            c_n1[r] = P.p1pos[P.leaf_begin[t + 1]] - P.p1pos[P.leaf_begin[t]];
            c_nc[r] = P.leaf_ncand[t];
        }
    }
    auto for_leaves = [&](auto&& f) {
#pragma unroll
        for (int r = 0; r < PLAN_R; ++r) {
            const uint32_t t = (uint32_t)tid + (uint32_t)r * PLAN_BLOCK;
            if (t < nl) f(t, c_n1[r], c_nc[r]);
        }
        for (uint32_t t = (uint32_t)tid + (uint32_t)PLAN_R * PLAN_BLOCK; t < nl; t += PLAN_BLOCK)
            f(t, P.p1pos[P.leaf_begin[t + 1]] - P.p1pos[P.leaf_begin[t]], P.leaf_ncand[t]);
    };
    auto nch_of = [](uint32_t n1, uint32_t nc, uint32_t cc) -> uint32_t {
        if (n1 == 0) return 1u;
        uint32_t nch = (nc + cc - 1) / cc;
        if (nch < 1) nch = 1;
        if (nch > KNN_NCH_MAX) nch = KNN_NCH_MAX;
        return nch;
    };
    if (tid == 0) { s_cc = (uint32_t)chunk0; s_done = 0; }
    __syncthreads();
    for (int iter = 0; iter < 40; ++iter) {
        const uint32_t cc = s_cc;
        unsigned long long lists = 0, items = 0, pairs = 0;
        for_leaves([&](uint32_t, uint32_t n1, uint32_t nc) {
            if (n1 == 0) return;
            const uint32_t nch = nch_of(n1, nc, cc);
            if (nch > 1) lists += (unsigned long long)n1 * nch;
            items += (unsigned long long)((n1 + P.tq - 1) / P.tq) * nch;
            pairs += (unsigned long long)n1 * (nc - 1);
        });
        for (int o = 32; o > 0; o >>= 1) {
            lists += __shfl_xor(lists, o, 64);
            items += __shfl_xor(items, o, 64);
            pairs += __shfl_xor(pairs, o, 64);
        }
        if (lane == 0) { s_red[wave][0] = lists; s_red[wave][1] = items; s_red[wave][2] = pairs; }
        __syncthreads();
        if (tid == 0) {
            unsigned long long L = 0, I = 0, W = 0;
            for (int w = 0; w < PLAN_BLOCK / 64; ++w) { L += s_red[w][0]; I += s_red[w][1]; W += s_red[w][2]; }
            if ((L <= P.plist_max && I <= P.items_max) || cc >= 0x40000000u) {
                s_done = 1;
                P.ctr->pairs = W;
            } else {
                s_cc = cc * 2;
            }
        }
        __syncthreads();
        if (s_done) break;
    }
    const uint32_t cc = s_cc;
    // per leaf: its partial lists, its items (chunked, or in its class)
    auto counts = [&](uint32_t n1, uint32_t nc, uint32_t (&v)[NS], uint32_t& nch) {
        nch = nch_of(n1, nc, cc);
#pragma unroll
        for (int i = 0; i < NS; ++i) v[i] = 0;
        const uint32_t ni = n1 ? ((n1 + P.tq - 1) / P.tq) * nch : 0u;
        if (nch > 1) {
            v[0] = n1 * nch;
            v[1] = ni;
        } else {
            v[2 + plan_class(n1, nc)] = ni;
        }
    };
    if (nl <= (uint32_t)PLAN_BLOCK) {
        // one round: the scan gives every thread the class totals too
        uint32_t v[NS], nch = 1;
        if ((uint32_t)tid < nl) counts(c_n1[0], c_nc[0], v, nch);
        else {
#pragma unroll
            for (int i = 0; i < NS; ++i) v[i] = 0;
        }
        uint32_t ex[NS], tot[NS], base[NS];
        block_excl_scan_n<NS>(v, ex, tot, s_scan);
        base[0] = 0;
        base[1] = 0;
        uint32_t acc = tot[1];  // chunked items first
#pragma unroll
        for (int i = 2; i < NS; ++i) { base[i] = acc; acc += tot[i]; }
        if ((uint32_t)tid < nl) {
            const uint32_t t = (uint32_t)tid, n1 = c_n1[0], nc = c_nc[0];
            P.leaf_nch[t] = nch;
            P.leaf_cc[t] = (nc + nch - 1) / nch;
            P.leaf_plist[t] = ex[0];
            const uint32_t q = nch > 1 ? 1u : 2u + plan_class(n1, nc);
            P.leaf_item[t] = base[q] + ex[q];
        }
        if (tid == 0) {
            P.ctr->n_items = acc;
            P.ctr->n_chunked_items = tot[1];
        }
        return;
    }
    // totals: the queue offset of each class
    {
        uint32_t tot[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) tot[i] = 0;
        for_leaves([&](uint32_t, uint32_t n1, uint32_t nc) {
            uint32_t v[NS], nch;
            counts(n1, nc, v, nch);
#pragma unroll
            for (int i = 0; i < NS; ++i) tot[i] += v[i];
        });
        uint32_t ex[NS], all[NS];
        block_excl_scan_n<NS>(tot, ex, all, s_scan);
        if (tid == 0) {
            uint32_t acc = all[1];  // chunked items first
            s_base[0] = 0;
            s_base[1] = 0;
            for (int i = 2; i < NS; ++i) { s_base[i] = acc; acc += all[i]; }
            for (int i = 0; i < NS; ++i) s_carry[i] = 0;
            P.ctr->n_items = acc;
            P.ctr->n_chunked_items = all[1];
        }
        __syncthreads();
    }
    // offsets, one round of PLAN_BLOCK leaves at a time
    auto round = [&](uint32_t t, uint32_t n1, uint32_t nc) {
        uint32_t v[NS], nch = 1;
        if (t < nl) counts(n1, nc, v, nch);
        else {
#pragma unroll
            for (int i = 0; i < NS; ++i) v[i] = 0;
        }
        uint32_t ex[NS], tot[NS];
        block_excl_scan_n<NS>(v, ex, tot, s_scan);
        if (t < nl) {
            P.leaf_nch[t] = nch;
            P.leaf_cc[t] = (nc + nch - 1) / nch;
            P.leaf_plist[t] = s_carry[0] + ex[0];
            const uint32_t q = nch > 1 ? 1u : 2u + plan_class(n1, nc);
            P.leaf_item[t] = s_base[q] + s_carry[q] + ex[q];
        }
        __syncthreads();
        if (tid < NS) s_carry[tid] += tot[tid];
        __syncthreads();
    };
#pragma unroll
    for (int r = 0; r < PLAN_R; ++r) {
        const uint32_t t0 = (uint32_t)r * PLAN_BLOCK;
        if (t0 < nl) round(t0 + (uint32_t)tid, c_n1[r], c_nc[r]);
    }
    for (uint32_t t0 = (uint32_t)PLAN_R * PLAN_BLOCK; t0 < nl; t0 += PLAN_BLOCK) {
        const uint32_t t = t0 + (uint32_t)tid;
        uint32_t n1 = 0, nc = 0;
        if (t < nl) {
            n1 = P.p1pos[P.leaf_begin[t + 1]] - P.p1pos[P.leaf_begin[t]];
            nc = P.leaf_ncand[t];
        }
        round(t, n1, nc);
    }
}

// Parallel plan for large batches (the single workgroup above would walk
// every leaf several times): one pass counts partial lists, items and
// chunked items per leaf for each candidate chunk length chunk0 << l, a
// single thread picks the first length that fits (else no chunking), and
// three look-back scans over the leaves give the partial-list offsets and
// the queue offsets of chunked and unchunked leaves.

__device__ __forceinline__ uint32_t plan_nch(uint32_t n1, uint32_t nc, uint32_t cc) {
    if (n1 == 0) return 1u;
    uint32_t nch = (nc + cc - 1) / cc;
    if (nch < 1) nch = 1;
    if (nch > KNN_NCH_MAX) nch = KNN_NCH_MAX;
    return nch;
}

__global__ __launch_bounds__(256) void plan_count_kernel(Plan P, uint32_t chunk0) {
    __shared__ unsigned long long s_acc[PLAN_LEVELS * 3 + 1];
    for (int i = threadIdx.x; i < PLAN_LEVELS * 3 + 1; i += blockDim.x) s_acc[i] = 0ull;
    __syncthreads();
    const uint32_t nl = P.ctr->n_leaves;
    unsigned long long acc[PLAN_LEVELS * 3 + 1];
#pragma unroll
    for (int i = 0; i < PLAN_LEVELS * 3 + 1; ++i) acc[i] = 0ull;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nl; t += gridDim.x * blockDim.x) {
        const uint32_t n1 = P.p1pos[P.leaf_begin[t + 1]] - P.p1pos[P.leaf_begin[t]], nc = P.leaf_ncand[t];
        if (n1 == 0) continue;
        const unsigned long long tiles = (n1 + P.tq - 1) / P.tq;
#pragma unroll
        for (int l = 0; l < PLAN_LEVELS; ++l) {
            const uint32_t cc = chunk0 << l;
            const uint32_t nch = plan_nch(n1, nc, cc);
            if (nch > 1) {
                acc[3 * l] += (unsigned long long)n1 * nch;
                acc[3 * l + 2] += tiles * nch;
            }
            acc[3 * l + 1] += tiles * nch;
        }
        acc[PLAN_LEVELS * 3] += (unsigned long long)n1 * (nc - 1);
    }
#pragma unroll
    for (int i = 0; i < PLAN_LEVELS * 3 + 1; ++i) {
        unsigned long long v = acc[i];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0 && v) atomicAdd(&s_acc[i], v);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < PLAN_LEVELS * 3 + 1; i += blockDim.x) {
        if (s_acc[i]) {
            if (i < PLAN_LEVELS * 3) atomicAdd(&P.ctr->plan_acc[i / 3][i % 3], s_acc[i]);
            else atomicAdd(&P.ctr->plan_pairs, s_acc[i]);
        }
    }
}

__global__ void plan_pick_kernel(Plan P, uint32_t chunk0) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    Counters* c = P.ctr;
    uint32_t cc = 0x40000000u, chunked = 0;
    unsigned long long items = 0;
    for (int l = 0; l < PLAN_LEVELS; ++l) {
        if (c->plan_acc[l][0] <= P.plist_max && c->plan_acc[l][1] <= P.items_max) {
            cc = chunk0 << l;
            items = c->plan_acc[l][1];
            chunked = (uint32_t)c->plan_acc[l][2];
            break;
        }
    }
    if (cc == 0x40000000u) items = 0;  // no chunking: items counted by the scan below
    c->plan_cc = cc;
    c->n_chunked_items = chunked;
    c->n_items = (uint32_t)items;
    c->pairs = c->plan_pairs;
}

struct PlanLeaf {
    const Plan* P;
    __device__ void get(uint32_t t, uint32_t* n1, uint32_t* nc, uint32_t* nch) const {
        *n1 = P->p1pos[P->leaf_begin[t + 1]] - P->p1pos[P->leaf_begin[t]];
        *nc = P->leaf_ncand[t];
        *nch = plan_nch(*n1, *nc, P->ctr->plan_cc);
    }
};
struct ListsGet {
    Plan P;
    __device__ uint32_t operator()(uint32_t t) const {
        uint32_t n1, nc, nch;
        PlanLeaf{&P}.get(t, &n1, &nc, &nch);
        return nch > 1 ? n1 * nch : 0u;
    }
};
struct ListsEmit {
    Plan P;
    __device__ void operator()(uint32_t t, uint32_t ex, uint32_t) const {
        uint32_t n1, nc, nch;
        PlanLeaf{&P}.get(t, &n1, &nc, &nch);
        P.leaf_nch[t] = nch;
        P.leaf_cc[t] = (nc + nch - 1) / nch;
        P.leaf_plist[t] = ex;
    }
};
template <bool CHUNKED>
struct ItemsGet {
    Plan P;
    __device__ uint32_t operator()(uint32_t t) const {
        uint32_t n1, nc, nch;
        PlanLeaf{&P}.get(t, &n1, &nc, &nch);
        return ((nch > 1) == CHUNKED && n1) ? ((n1 + P.tq - 1) / P.tq) * nch : 0u;
    }
};
template <bool CHUNKED>
struct ItemsEmit {
    Plan P;
    __device__ void operator()(uint32_t t, uint32_t ex, uint32_t) const {
        uint32_t n1, nc, nch;
        PlanLeaf{&P}.get(t, &n1, &nc, &nch);
        if ((nch > 1) == CHUNKED) P.leaf_item[t] = CHUNKED ? ex : P.ctr->n_chunked_items + ex;
    }
};
struct NoFin {
    __device__ void operator()(uint32_t) const {}
};
struct ItemsFin {
    Counters* c;
    __device__ void operator()(uint32_t total) const { c->n_items = c->n_chunked_items + total; }
};

void launch_knn_plan(const Plan& P, const Params& prm, hipStream_t st) {
    const int chunk0 = prm.knn_chunk > 0 ? prm.knn_chunk : KNN_CC0;
    if (P.n <= (1u << 19)) {
        hipLaunchKernelGGL(knn_plan_kernel, dim3(1), dim3(PLAN_BLOCK), 0, st, P, chunk0);
        return;
    }
    unsigned blocks = (P.n / 8 + 255) / 256;
    if (blocks > 512) blocks = 512;
    hipLaunchKernelGGL(plan_count_kernel, dim3(blocks), dim3(256), 0, st, P, (uint32_t)chunk0);
    hipLaunchKernelGGL(plan_pick_kernel, dim3(1), dim3(64), 0, st, P, (uint32_t)chunk0);
    // scans over the leaves (far fewer than the points that bound them): a
    // small grid that loops over the tiles, not one workgroup per possible tile
    const uint32_t* nl = &P.ctr->n_leaves;
    constexpr uint32_t LEAF_SCAN_BLOCKS = 64;
    launch_scan(ListsGet{P}, ListsEmit{P}, NoFin{}, nl, P.n, P.scan_status + 3 * (size_t)P.scan_tiles,
                &P.ctr->status, st, LEAF_SCAN_BLOCKS);
    launch_scan(ItemsGet<true>{P}, ItemsEmit<true>{P}, NoFin{}, nl, P.n, P.scan_status + 4 * (size_t)P.scan_tiles,
                &P.ctr->status, st, LEAF_SCAN_BLOCKS);
    launch_scan(ItemsGet<false>{P}, ItemsEmit<false>{P}, ItemsFin{P.ctr}, nl, P.n,
                P.scan_status + 5 * (size_t)P.scan_tiles, &P.ctr->status, st, LEAF_SCAN_BLOCKS);
}

}  // namespace gdn
