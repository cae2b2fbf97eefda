// Frame-level passes: zero-fill of the workspace control block, the frame
// bounding box (the octree root cube, Sec. 3 with Eq. 2), 63-bit Morton keys,
// the stable LSD radix sort of (key, original index) on the digits the octree
// needs, and the whole-key re-sort of deep level-10 cells.
#include "kernels.hpp"

namespace gdn {

// ---------------------------------------------------------------- zero fill

__global__ void zero_kernel(uint4* p, size_t n16, uint32_t* foff, uint32_t n, uint32_t one_frame) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
    if (one_frame && blockIdx.x == 0 && threadIdx.x == 0) {
        foff[0] = 0u;
        foff[1] = n;
    }
}

void launch_zero(const Plan& P, hipStream_t st) {
    size_t n16 = P.zero_bytes / 16;
    unsigned blocks = (unsigned)((n16 + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, st, (uint4*)P.zero_begin, n16, P.foff, P.n,
                       P.nf == 1 ? 1u : 0u);
}

// ---------------------------------------------------------------- frame table
//
// Checked copy of the caller's frame offsets (int64[nf+1]): clamped to [0, n]
// and made non-decreasing (a running maximum), with foff[0] = 0 and
// foff[nf] = n. Any repair sets DEV_BAD_FRAMES; the batch is then processed
// with the repaired table (memory-safe, results unspecified).
__global__ __launch_bounds__(256) void frames_kernel(const int64_t* __restrict__ in, uint32_t nf, uint32_t n,
                                                     uint32_t* foff, Counters* c) {
    __shared__ uint32_t s_max[256];
    constexpr uint32_t PER = (MAX_FRAMES + 1 + 255) / 256;
    const uint32_t t = threadIdx.x, b0 = t * PER;
    uint32_t v[PER];
    uint32_t m = 0, bad = 0;
#pragma unroll
    for (uint32_t i = 0; i < PER; ++i) {
        const uint32_t f = b0 + i;
        uint32_t x = 0;
        if (f <= nf) {
            const int64_t r = in[f];
            x = r < 0 ? 0u : (r > (int64_t)n ? n : (uint32_t)r);
            if (r < 0 || r > (int64_t)n) bad = 1;
            if (f == 0 && r != 0) bad = 1;
            if (f == nf && r != (int64_t)n) bad = 1;
            if (f > 0 && r < in[f - 1]) bad = 1;
        }
        m = x > m ? x : m;
        v[i] = m;  // running max within this thread's entries
    }
    s_max[t] = m;
    __syncthreads();
    if (t == 0) {
        uint32_t run = 0;
        for (int i = 0; i < 256; ++i) {
            const uint32_t x = s_max[i];
            s_max[i] = run;  // max over earlier threads
            run = x > run ? x : run;
        }
    }
    __syncthreads();
    const uint32_t pre = s_max[t];
#pragma unroll
    for (uint32_t i = 0; i < PER; ++i) {
        const uint32_t f = b0 + i;
        if (f <= nf) {
            uint32_t x = v[i] > pre ? v[i] : pre;
            if (f == 0) x = 0u;
            if (f == nf) x = n;
            foff[f] = x;
        }
    }
    if (bad) atomicOr(&c->status, DEV_BAD_FRAMES);
}

void launch_frames(const Plan& P, const int64_t* frame_off, hipStream_t st) {
    hipLaunchKernelGGL(frames_kernel, dim3(1), dim3(256), 0, st, frame_off, P.nf, P.n, P.foff, P.ctr);
}

// ---------------------------------------------------------------- bbox

// Waves take chunks of BBOX_CHUNK consecutive points (coalesced). A chunk
// inside one frame writes its reduced box to bbox_part[chunk] and a second
// kernel folds each frame's chunks (no contended atomics); a chunk across a
// frame border (at most nf - 1 of them) reduces each of its frames over the
// wave and adds them with atomics. With few chunks (`direct`) every chunk
// uses the atomics and there is no fold. Batches also record each point's
// frame.
constexpr uint32_t BBOX_CHUNK = 1024;

__device__ __forceinline__ void bbox_reduce_wave(float* mn, float* mx, uint32_t& bad) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = fminf(mn[a], __shfl_xor(mn[a], o, 64));
            mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], o, 64));
        }
        bad += __shfl_xor(bad, o, 64);
    }
}

// Adds the points [lo, hi) to a lane's box (non-finite points are counted
// in `bad` instead), lane l taking points lo + l, lo + l + 64, ... in that
// order; BBOX_U loads per lane are issued before any is used (a lane past hi
// reads the last point and drops it). With fid, also records frame f of each
// point.
constexpr int BBOX_U = 8;
__device__ __forceinline__ void bbox_add_range(const float* __restrict__ xyz, uint32_t lo, uint32_t hi,
                                               uint32_t lane, float* mn, float* mx, uint32_t& bad, uint32_t* fid,
                                               uint32_t f) {
    for (uint32_t i0 = lo + lane; i0 < hi; i0 += 64u * BBOX_U) {
        float x[BBOX_U], y[BBOX_U], z[BBOX_U];
#pragma unroll
        for (int u = 0; u < BBOX_U; ++u) {
            const size_t j = min(i0 + 64u * (uint32_t)u, hi - 1u);
            x[u] = xyz[3 * j];
            y[u] = xyz[3 * j + 1];
            z[u] = xyz[3 * j + 2];
        }
#pragma unroll
        for (int u = 0; u < BBOX_U; ++u) {
            const uint32_t i = i0 + 64u * (uint32_t)u;
            const bool in = i < hi;
            const bool fin = isfinite(x[u]) && isfinite(y[u]) && isfinite(z[u]);
            const bool ok = in && fin;
            mn[0] = fminf(mn[0], ok ? x[u] : INFINITY); mx[0] = fmaxf(mx[0], ok ? x[u] : -INFINITY);
            mn[1] = fminf(mn[1], ok ? y[u] : INFINITY); mx[1] = fmaxf(mx[1], ok ? y[u] : -INFINITY);
            mn[2] = fminf(mn[2], ok ? z[u] : INFINITY); mx[2] = fmaxf(mx[2], ok ? z[u] : -INFINITY);
            bad += (in && !fin) ? 1u : 0u;
            if (fid && in) fid[i] = f;
        }
    }
}

__global__ __launch_bounds__(256) void bbox_kernel(const float* __restrict__ xyz, Plan P, bool direct,
                                                   uint32_t chunk) {
    __shared__ uint32_t s_foff[MAX_FRAMES + 1];
    const uint32_t n = P.n, nf = P.nf;
    if (nf > 1) {
        for (uint32_t f = threadIdx.x; f <= nf; f += blockDim.x) s_foff[f] = P.foff[f];
        __syncthreads();
    }
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    const uint32_t nchunks = (n + chunk - 1) / chunk;
    for (uint32_t c = wid; c < nchunks; c += nw) {
        const uint32_t base = c * chunk, end = min(n, base + chunk);
        const uint32_t f0 = nf > 1 ? frame_of(s_foff, nf, base) : 0u;
        const uint32_t f1 = nf > 1 ? frame_of(s_foff, nf, end - 1u) : 0u;
        for (uint32_t f = f0; f <= f1; ++f) {
            const uint32_t lo = f == f0 ? base : max(base, s_foff[f]);
            const uint32_t hi = f == f1 ? end : min(end, s_foff[f + 1]);
            float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
            uint32_t bad = 0;
            bbox_add_range(xyz, lo, hi, lane, mn, mx, bad, nf > 1 ? P.fid : nullptr, f);
            bbox_reduce_wave(mn, mx, bad);
            if (f0 == f1 && !direct) {
                // whole chunk in one frame: ordered-uint max of -min / max, bad count
                uint32_t* part = P.bbox_part + 8 * (size_t)c;
                if (lane < 3u) {
                    part[lane] = mn[lane] <= mx[lane] ? ~f32_ordered(mn[lane]) : 0u;
                    part[3 + lane] = mn[lane] <= mx[lane] ? f32_ordered(mx[lane]) : 0u;
                }
                if (lane == 3u) part[6] = bad;
            } else {
                FrameStat* fs = P.fstat + f;
                if (lane < 3u && mn[lane] <= mx[lane]) {
                    atomicMax(&fs->bbox_nmin[lane], ~f32_ordered(mn[lane]));
                    atomicMax(&fs->bbox_max[lane], f32_ordered(mx[lane]));
                }
                if (lane == 3u && bad) {
                    atomicAdd(&fs->nonfinite, bad);
                    atomicOr(&P.ctr->status, DEV_NONFINITE);
                }
            }
        }
    }
}

// A single frame with few points: each wave reduces its 512-point chunks and
// the block combines its four waves; each block writes its box (ordered-uint
// max of -min and max) and non-finite count to bbox_part[block], which the
// Morton kernel folds (no atomics, so the accumulators need no clearing). On a
// plain call the blocks also clear the workspace's zeroed block (counters,
// histograms, look-back status words: nothing here uses them) and write the
// one-frame offset table, in place of a separate fill launch.
__global__ __launch_bounds__(256) void bbox_one_kernel(const float* __restrict__ xyz, Plan P, uint32_t chunk,
                                                       bool clear) {
    __shared__ float s_mn[4][3], s_mx[4][3];
    __shared__ uint32_t s_bad[4];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    const uint32_t n = P.n, nchunks = (n + chunk - 1) / chunk;
    if (clear) {
        uint4* z = (uint4*)P.zero_begin;
        const size_t n16 = P.zero_bytes / 16;
        for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
            z[i] = make_uint4(0u, 0u, 0u, 0u);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            P.foff[0] = 0u;
            P.foff[1] = n;
        }
    }
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    uint32_t bad = 0;
    for (uint32_t c = wid; c < nchunks; c += nw)
        bbox_add_range(xyz, c * chunk, min(n, (c + 1u) * chunk), lane, mn, mx, bad, nullptr, 0u);
    bbox_reduce_wave(mn, mx, bad);
    if (lane == 0u) {
        for (int a = 0; a < 3; ++a) {
            s_mn[wave][a] = mn[a];
            s_mx[wave][a] = mx[a];
        }
        s_bad[wave] = bad;
    }
    __syncthreads();
    uint32_t* part = P.bbox_part + 8 * (size_t)blockIdx.x;
    if (threadIdx.x < 3u) {
        const uint32_t a = threadIdx.x;
        float lo = s_mn[0][a], hi = s_mx[0][a];
        for (int w = 1; w < 4; ++w) {
            lo = fminf(lo, s_mn[w][a]);
            hi = fmaxf(hi, s_mx[w][a]);
        }
        part[a] = lo <= hi ? ~f32_ordered(lo) : 0u;
        part[3 + a] = lo <= hi ? f32_ordered(hi) : 0u;
    }
    if (threadIdx.x == 3u) part[6] = s_bad[0] + s_bad[1] + s_bad[2] + s_bad[3];
}

// One wave per frame: fold the frame's whole chunks into its accumulators.
__global__ __launch_bounds__(256) void bbox_fold_kernel(Plan P) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t f = wid; f < P.nf; f += nw) {
        const uint32_t fs = P.foff[f], fe = P.foff[f + 1];
        const uint32_t c0 = (fs + BBOX_CHUNK - 1) / BBOX_CHUNK;
        const uint32_t c1 = fe == P.n ? (fe + BBOX_CHUNK - 1) / BBOX_CHUNK : fe / BBOX_CHUNK;
        uint32_t v[7] = {0u, 0u, 0u, 0u, 0u, 0u, 0u};
        for (uint32_t c = c0 + lane; c < c1; c += 64u) {
            const uint32_t* part = P.bbox_part + 8 * (size_t)c;
#pragma unroll
            for (int a = 0; a < 6; ++a) v[a] = max(v[a], part[a]);
            v[6] += part[6];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
            for (int a = 0; a < 6; ++a) v[a] = max(v[a], (uint32_t)__shfl_xor((int)v[a], o, 64));
            v[6] += (uint32_t)__shfl_xor((int)v[6], o, 64);
        }
        FrameStat* st = P.fstat + f;
        if (lane < 3u) {
            if (v[lane]) atomicMax(&st->bbox_nmin[lane], v[lane]);
            if (v[3 + lane]) atomicMax(&st->bbox_max[lane], v[3 + lane]);
        }
        if (lane == 3u && v[6]) atomicAdd(&st->nonfinite, v[6]);
        if (lane == 4u && (v[6] || st->nonfinite)) atomicOr(&P.ctr->status, DEV_NONFINITE);
    }
}

// Few points: 512-point chunks (one wave each, enough waves to cover the
// load latency); otherwise BBOX_CHUNK chunks and the fold.
static bool bbox_direct(const Plan& P) { return P.n <= (1u << 20); }
static unsigned bbox_blocks(const Plan& P) {
    const uint32_t chunk = bbox_direct(P) ? 512u : BBOX_CHUNK;
    const uint32_t nchunks = (P.n + chunk - 1) / chunk;
    unsigned blocks = (nchunks + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    return blocks ? blocks : 1u;
}
bool bbox_one_frame(const Plan& P) { return bbox_direct(P) && P.nf == 1; }

void launch_bbox(const Plan& P, const float* xyz, hipStream_t st, bool clear) {
    const bool direct = bbox_direct(P);
    const uint32_t chunk = direct ? 512u : BBOX_CHUNK;
    const unsigned blocks = bbox_blocks(P);
    if (bbox_one_frame(P)) {
        hipLaunchKernelGGL(bbox_one_kernel, dim3(blocks), dim3(256), 0, st, xyz, P, chunk, clear);
        return;
    }
    hipLaunchKernelGGL(bbox_kernel, dim3(blocks), dim3(256), 0, st, xyz, P, direct, chunk);
    if (direct) return;
    unsigned fb = (P.nf + 3) / 4;
    if (fb > 1024) fb = 1024;
    hipLaunchKernelGGL(bbox_fold_kernel, dim3(fb), dim3(256), 0, st, P);
}

// ---------------------------------------------------------------- Morton keys

// Root cube: side S = largest bbox extent at the bbox minimum; depth limit from
// the minimum leaf side. Same FP64 expressions for every consumer.
__device__ void frame_consts(const FrameStat* c, double min_leaf_side, FrameConst* f) {
    double S = 0.0;
    for (int a = 0; a < 3; ++a) {
        float lo = f32_from_ordered(~c->bbox_nmin[a]);
        float hi = f32_from_ordered(c->bbox_max[a]);
        f->lo[a] = lo;
        double H = (double)hi - (double)lo;
        if (H > S) S = H;
    }
    if (!(S > 0.0) || !(S < INFINITY)) S = 1.0;
    f->S = S;
    f->scale = 2097152.0 / S;
    int d = MORTON_BITS;
    if (min_leaf_side > 0.0) {
        d = 0;
        while (d < MORTON_BITS && ldexp(S, -(d + 1)) >= min_leaf_side) ++d;
    }
    f->dmax = d;
}

__device__ __forceinline__ uint32_t quantise(float x, float lo, double scale) {
    double q = floor(((double)x - (double)lo) * scale);
    if (!(q >= 0.0)) q = 0.0;
    if (q > (double)QMAX) q = (double)QMAX;
    return (uint32_t)q;
}

// Frame constants of every frame of a batch (one thread per frame).
__global__ __launch_bounds__(256) void frame_const_kernel(Plan P, double min_leaf_side) {
    for (uint32_t f = threadIdx.x; f < P.nf; f += blockDim.x) frame_consts(P.fstat + f, min_leaf_side, P.fc + f);
}

// Keys (quantised with the point's own frame constants), the identity
// payload and the digit histograms of the sort: key digits 4..7, then the
// frame id digits of a batch. A single frame computes its constants per block.
constexpr uint32_t MORTON_U = 8;
// nparts > 0: a single frame whose box is in nparts per-block records of
// bbox_one_kernel, folded here by every block (block 0 also stores the
// frame's statistics and constants and flags non-finite input).
__global__ __launch_bounds__(256) void morton_kernel(const float* __restrict__ xyz, Plan P, double min_leaf_side,
                                                     uint32_t nparts) {
    __shared__ FrameConst s_fc;
    __shared__ FrameStat s_stat;
    __shared__ uint32_t s_hist[SORT_PASSES_MAX][256];
    const uint32_t n = P.n, nf = P.nf, nh = P.sort_passes;
    for (uint32_t i = threadIdx.x; i < nh * 256u; i += blockDim.x) (&s_hist[0][0])[i] = 0u;
    if (nf == 1 && nparts > 0 && threadIdx.x < 64u) {
        const uint32_t lane = threadIdx.x;
        uint32_t v[7] = {0u, 0u, 0u, 0u, 0u, 0u, 0u};
        for (uint32_t c = lane; c < nparts; c += 64u) {
            const uint32_t* part = P.bbox_part + 8 * (size_t)c;
#pragma unroll
            for (int a = 0; a < 6; ++a) v[a] = max(v[a], part[a]);
            v[6] += part[6];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
            for (int a = 0; a < 6; ++a) v[a] = max(v[a], (uint32_t)__shfl_xor((int)v[a], o, 64));
            v[6] += (uint32_t)__shfl_xor((int)v[6], o, 64);
        }
        if (lane == 0) {
            for (int a = 0; a < 3; ++a) {
                s_stat.bbox_nmin[a] = v[a];
                s_stat.bbox_max[a] = v[3 + a];
            }
            s_stat.nonfinite = v[6];
            s_stat.pad = 0u;
            frame_consts(&s_stat, min_leaf_side, &s_fc);
            if (blockIdx.x == 0) {
                *P.fstat = s_stat;
                *P.fc = s_fc;
                if (v[6]) atomicOr(&P.ctr->status, DEV_NONFINITE);
            }
        }
    } else if (nf == 1 && threadIdx.x == 0) {
        frame_consts(P.fstat, min_leaf_side, &s_fc);
        if (blockIdx.x == 0) *P.fc = s_fc;
    }
    __syncthreads();
    // MORTON_U points per thread at a time, their loads (and a batch's frame
    // constants) issued before any is used (a point past n reads the last
    // one and is dropped)
    const uint32_t stride = gridDim.x * blockDim.x;
    const float c0 = s_fc.lo[0], c1 = s_fc.lo[1], c2 = s_fc.lo[2];
    const double csc = s_fc.scale;
    for (uint32_t i0 = blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += MORTON_U * stride) {
        float x[MORTON_U], y[MORTON_U], z[MORTON_U];
        uint32_t f[MORTON_U];
#pragma unroll
        for (int u = 0; u < MORTON_U; ++u) {
            const uint32_t j = min(i0 + (uint32_t)u * stride, n - 1u);
            x[u] = xyz[3 * (size_t)j];
            y[u] = xyz[3 * (size_t)j + 1];
            z[u] = xyz[3 * (size_t)j + 2];
            f[u] = nf > 1 ? P.fid[j] : 0u;
        }
        float l0[MORTON_U], l1[MORTON_U], l2[MORTON_U];
        double sc[MORTON_U];
#pragma unroll
        for (int u = 0; u < MORTON_U; ++u) {
            if (nf > 1) {
                const FrameConst& fc = P.fc[f[u]];
                l0[u] = fc.lo[0];
                l1[u] = fc.lo[1];
                l2[u] = fc.lo[2];
                sc[u] = fc.scale;
            } else {
                l0[u] = c0;
                l1[u] = c1;
                l2[u] = c2;
                sc[u] = csc;
            }
        }
        // (an empty statement taking the loaded values keeps the compiler from
        // moving each load into the branch of its point)
#pragma unroll
        for (int u = 0; u < MORTON_U; ++u) asm volatile("" ::"v"(x[u]), "v"(y[u]), "v"(z[u]), "v"(f[u]));
#pragma unroll
        for (int u = 0; u < MORTON_U; ++u) {
            const uint32_t i = i0 + (uint32_t)u * stride;
            if (i >= n) break;
            const uint32_t qx = quantise(x[u], l0[u], sc[u]);
            const uint32_t qy = quantise(y[u], l1[u], sc[u]);
            const uint32_t qz = quantise(z[u], l2[u], sc[u]);
            const uint64_t key = morton3(qx, qy, qz);
            P.keys_src[i] = key;
            P.idx_src[i] = i;
#pragma unroll
            for (int p = SORT_SHORT_FIRST; p < SORT_PASSES; ++p)
                atomicAdd(&s_hist[p][(key >> (8 * p)) & 255u], 1u);
            for (uint32_t p = SORT_PASSES; p < nh; ++p)
                atomicAdd(&s_hist[p][(f[u] >> (8 * (p - SORT_PASSES))) & 255u], 1u);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nh * 256u; i += blockDim.x) {
        uint32_t v = (&s_hist[0][0])[i];
        if (v) atomicAdd(&P.sort_hist[i], v);
    }
}

void launch_morton(const Plan& P, const Params& prm, const float* xyz, hipStream_t st) {
    if (P.nf > 1) hipLaunchKernelGGL(frame_const_kernel, dim3(1), dim3(256), 0, st, P, prm.min_leaf_side);
    unsigned blocks = (P.n + 2047) / 2048;
    if (blocks > 512) blocks = 512;
    const uint32_t nparts = bbox_one_frame(P) ? bbox_blocks(P) : 0u;
    hipLaunchKernelGGL(morton_kernel, dim3(blocks), dim3(256), 0, st, xyz, P, prm.min_leaf_side, nparts);
}

// ---------------------------------------------------------------- radix sort

// One stable LSD pass over digit `pass` (8 bits) in the onesweep style: local
// ranks by wave-level digit matching, digit offsets of earlier tiles by
// decoupled look-back (bounded waits), global digit bases from the histogram.
// Passes past the key's 8 take the digit from the frame of the payload (the
// original index, found in the frame offsets), so a batch ends sorted by
// (frame, key bits 32..62, index); only passes from SORT_SHORT_FIRST on are
// launched.
template <int ITEMS>
__global__ __launch_bounds__(SORT_BLOCK) void radix_pass_kernel(const uint64_t* __restrict__ kin,
                                                                const uint32_t* __restrict__ vin,
                                                                uint64_t* __restrict__ kout,
                                                                uint32_t* __restrict__ vout, uint32_t n,
                                                                int pass, const uint32_t* __restrict__ hist,
                                                                uint32_t* status, uint32_t* dev_status,
                                                                const uint32_t* __restrict__ foff,
                                                                uint32_t nf) {
    __shared__ uint32_t s_w[SORT_BLOCK / 64][256];
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_scan[SORT_BLOCK / 64 + 1];
    __shared__ uint32_t s_foff[SORT_FOFF_LDS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int shift = 8 * pass;
    // this digit's total over the pass, needed only after the ranking: read first
    const uint32_t hv = hist[tid];
    // frame passes of batches with few frames search the offsets in LDS
    const bool foff_lds = pass >= SORT_PASSES && nf < SORT_FOFF_LDS;
    if (foff_lds)
        for (uint32_t i = tid; i <= nf; i += SORT_BLOCK) s_foff[i] = foff[i];
    for (int i = tid; i < (SORT_BLOCK / 64) * 256; i += SORT_BLOCK) (&s_w[0][0])[i] = 0u;

    uint64_t key[ITEMS];
    uint32_t val[ITEMS], dig[ITEMS], rank[ITEMS];
    auto load_tile = [&](uint32_t tl) {
        const uint32_t tb = tl * (SORT_BLOCK * ITEMS) + wave * (64 * ITEMS);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t pos = tb + i * 64 + lane;
            const bool ok = pos < n;
            key[i] = ok ? kin[pos] : 0ull;
            val[i] = ok ? vin[pos] : 0u;
        }
    };
    // Tile = workgroup index. Each XCD starts its workgroups in index order,
    // so every tile a look-back waits on has been started and only waits on
    // lower tiles in turn; the waits are bounded anyway (SPIN_LIMIT, then a
    // status bit). A tile counter taken with an atomic cost a round trip
    // before the loads, and on large inputs, where the workgroups that start
    // together race for it, a second load of the tile.
    load_tile(blockIdx.x);
    __syncthreads();
    const uint32_t tile = blockIdx.x;
    const uint32_t tbase = tile * (SORT_BLOCK * ITEMS) + wave * (64 * ITEMS);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        uint32_t pos = tbase + i * 64 + lane;
        bool ok = pos < n;
        uint32_t d;
        if (pass < SORT_PASSES) {
            d = (uint32_t)((key[i] >> shift) & 255u);
        } else {
            const uint32_t v = ok ? val[i] : 0u;
            const uint32_t f = foff_lds ? frame_of(s_foff, nf, v) : frame_of(foff, nf, v);
            d = (f >> (8 * (pass - SORT_PASSES))) & 255u;
        }
        dig[i] = ok ? d : 256u;
    }
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t d = dig[i];
        const bool ok = d < 256u;
        uint64_t m = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        uint32_t before = __popcll(m & lt_mask);
        uint32_t cnt = __popcll(m);
        uint32_t wb = ok ? s_w[wave][d & 255u] : 0u;
        rank[i] = wb + before;
        bool leader = ok && ((m >> lane) == 1ull);
        if (leader) s_w[wave][d] = wb + cnt;
    }
    __syncthreads();

    // per digit: offsets of the waves of this tile, tile total
    uint32_t tcnt = 0;
    {
        const int d = tid;
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < SORT_BLOCK / 64; ++w) {
            uint32_t c = s_w[w][d];
            s_w[w][d] = run;
            run += c;
        }
        tcnt = run;
    }
    // look-back over earlier tiles, digit by digit
    uint32_t* st = status + (size_t)tile * 256 + tid;
    uint32_t excl = 0;
    st_relaxed_agent(st, (tile == 0 ? LB_FLAG_PRE : LB_FLAG_AGG) | tcnt);
    // global base of each digit (while the earlier tiles publish theirs)
    uint32_t total;
    const uint32_t gex = block_excl_scan(hv, s_scan, &total);
    if (tile != 0) {
        // LB_WINDOW predecessors per round trip; consume ready words nearest
        // first until an inclusive prefix, stop at the first one not ready
        int j = (int)tile - 1;
        uint32_t spins = 0;
        while (j >= 0) {
            uint32_t w[LB_WINDOW];
#pragma unroll
            for (int b = 0; b < LB_WINDOW; ++b)
                w[b] = j - b >= 0 ? ld_relaxed_agent(status + (size_t)(j - b) * 256 + tid) : 0u;
            int used = 0;
            bool stop = false, pre = false;
#pragma unroll
            for (int b = 0; b < LB_WINDOW; ++b) {
                if (!stop) {
                    if (j - b < 0 || (w[b] & ~LB_VALUE) == 0u) {
                        stop = true;
                    } else {
                        excl += w[b] & LB_VALUE;
                        ++used;
                        if (w[b] & LB_FLAG_PRE) pre = stop = true;
                    }
                }
            }
            if (pre) break;
            j -= used;
            if (used == 0) {
                if (++spins > SPIN_LIMIT) {
                    atomicOr(dev_status, DEV_WAIT_LIMIT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        st_relaxed_agent(st, LB_FLAG_PRE | ((excl + tcnt) & LB_VALUE));
    }
    s_base[tid] = gex + excl;
    if constexpr (ITEMS >= 16) {
        // Large tiles: stage the tile in LDS in digit order, then write each
        // digit's run with consecutive threads (coalesced) instead of
        // scattering from registers.
        __shared__ uint64_t s_k[SORT_BLOCK * ITEMS];
        __shared__ uint32_t s_v[SORT_BLOCK * ITEMS];
        __shared__ uint8_t s_dg[SORT_BLOCK * ITEMS];  // frame digits, found once per element
        __shared__ uint32_t s_toff[256];
        uint32_t ttot;
        const uint32_t tex = block_excl_scan(tcnt, s_scan, &ttot);
        s_toff[tid] = tex;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t d = dig[i];
            if (d < 256u) {
                const uint32_t lp = s_toff[d] + s_w[wave][d] + rank[i];
                s_k[lp] = key[i];
                s_v[lp] = val[i];
                if (pass >= SORT_PASSES) s_dg[lp] = (uint8_t)d;
            }
        }
        __syncthreads();
        for (uint32_t p = tid; p < ttot; p += SORT_BLOCK) {
            const uint64_t kk = s_k[p];
            const uint32_t vv = s_v[p];
            const uint32_t d = pass < SORT_PASSES ? (uint32_t)((kk >> shift) & 255u) : (uint32_t)s_dg[p];
            const uint32_t o = s_base[d] + (p - s_toff[d]);
            if (o < n) {  // always true unless a look-back wait expired
                kout[o] = kk;
                vout[o] = vv;
            }
        }
    } else {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t d = dig[i];
            if (d < 256u) {
                const uint32_t o = s_base[d] + s_w[wave][d] + rank[i];
                if (o < n) {  // always true unless a look-back wait expired
                    kout[o] = key[i];
                    vout[o] = val[i];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- deep cells

constexpr int CELL_SHIFT = 3 * (MORTON_BITS - SORT_SHORT_LEVEL);  // level-10 prefix = key >> 33
constexpr int SEG_BLOCK = 256;
constexpr int SEG_PASSES = 6;  // key bits 0..47; bits 33..62 are the cell's own, and 6 passes end in keys_a

// Stable LSD radix sort of the keys and payloads of one level-10 cell [a, b)
// over key bits 0..47 (the cell's points share bits 33..62), by the whole
// block, tile by tile in order through keys_b / idx_b (scratch after the main
// sort): the cell's (original index) order becomes (key, index) order. A deep
// cell's positions are then flagged for the boundary test; a cell re-sorted
// only because it borders a deep one has its mark cleared.
__device__ void sort_cell(const Plan& P, uint32_t a, uint32_t b, bool deep, uint32_t* s_base,
                          uint32_t (*s_w)[256], uint32_t* s_scan) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int pass = 0; pass < SEG_PASSES; ++pass) {
        const int shift = 8 * pass;
        const uint64_t* ks = (pass & 1) ? P.keys_b : P.keys_a;
        const uint32_t* vs = (pass & 1) ? P.idx_b : P.idx_a;
        uint64_t* kd = (pass & 1) ? P.keys_a : P.keys_b;
        uint32_t* vd = (pass & 1) ? P.idx_a : P.idx_b;
        s_base[tid] = 0u;
        __syncthreads();
        for (uint32_t i = a + tid; i < b; i += SEG_BLOCK) atomicAdd(&s_base[(uint32_t)(ks[i] >> shift) & 255u], 1u);
        __syncthreads();
        uint32_t tot;
        const uint32_t ex = block_excl_scan(s_base[tid], s_scan, &tot);
        s_base[tid] = a + ex;
        for (uint32_t t0 = a; t0 < b; t0 += SEG_BLOCK) {
            for (int w = 0; w < SEG_BLOCK / 64; ++w) s_w[w][tid] = 0u;
            __syncthreads();
            const uint32_t i = t0 + tid;
            const bool ok = i < b;
            const uint64_t k = ok ? ks[i] : 0ull;
            const uint32_t v = ok ? vs[i] : 0u;
            const uint32_t d = ok ? (uint32_t)(k >> shift) & 255u : 256u;
            // lanes of this wave with the same digit
            uint64_t m = __ballot(ok);
#pragma unroll
            for (int bt = 0; bt < 8; ++bt) {
                const bool bit = (d >> bt) & 1u;
                const uint64_t bb = __ballot(bit);
                m &= bit ? bb : ~bb;
            }
            const uint32_t before = (uint32_t)__popcll(m & lt_mask);
            if (ok && (m >> lane) == 1ull) s_w[wave][d] = (uint32_t)__popcll(m);
            __syncthreads();
            uint32_t run = 0;
            for (int w = 0; w < SEG_BLOCK / 64; ++w) {
                const uint32_t c = s_w[w][tid];
                s_w[w][tid] = run;
                run += c;
            }
            __syncthreads();
            if (ok) {
                const uint32_t o = s_base[d] + s_w[wave][d] + before;
                if (o < b) {  // always true
                    kd[o] = k;
                    vd[o] = v;
                }
            }
            __syncthreads();
            s_base[tid] += run;
        }
        __syncthreads();  // the pass's writes are complete before the next reads them
    }
    if (deep) {
        for (uint32_t i = a + tid; i < b; i += SEG_BLOCK) P.deepf[i] = 1u;
    } else if (tid == 0) {
        P.deepf[a] = 0u;
    }
    __syncthreads();
}

// Frame of sorted position s and its range [fs, fe).
__device__ __forceinline__ uint32_t frame_range(const Plan& P, const uint32_t* s_foff, bool lds, uint32_t s,
                                                uint32_t* fs, uint32_t* fe) {
    uint32_t f = 0u;
    if (lds) {
        f = frame_of(s_foff, P.nf, s);
        *fs = s_foff[f];
        *fe = s_foff[f + 1];
    } else {
        if (P.nf > 1u) f = frame_of(P.foff, P.nf, s);
        *fs = P.foff[f];
        *fe = P.foff[f + 1];
    }
    return f;
}

// First position in [lo, hi) whose level-10 cell prefix is >= c (the keys
// are in cell order everywhere).
__device__ __forceinline__ uint32_t cell_lower_bound(const uint64_t* keys, uint32_t lo, uint32_t hi, uint64_t c) {
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((keys[mid] >> CELL_SHIFT) < c) lo = mid + 1u;
        else hi = mid;
    }
    return lo;
}

// A level-10 cell splits when it holds more than `cap` points and lies above
// its frame's depth limit ("deep"). Its leaves lie below level 10, and so do
// the halo cells around them, which reach into the 26 level-10 cells next to
// it: every one of those needs its points in whole-key order too, so that a
// deeper cell is one contiguous key range. One thread per sorted position: a
// position that starts a deep cell marks (deepf = 2) the start of that cell
// and of each non-empty neighbouring cell in its frame. The marks are plain
// stores of one value, so cells marked twice need no atomics.
// LDS: the frame offsets are staged in LDS (batches of fewer than
// SORT_FOFF_LDS frames), fixed at compile time so that they are read with LDS
// or global instructions, not generic ones.
template <bool LDS>
__global__ __launch_bounds__(SEG_BLOCK) void deep_mark_kernel(Plan P, uint32_t cap) {
    __shared__ uint32_t s_foff[SORT_FOFF_LDS];  // batches of fewer frames search the offsets here
    constexpr bool lds = LDS;
    if (lds)
        for (uint32_t i = threadIdx.x; i <= P.nf; i += blockDim.x) s_foff[i] = P.foff[i];
    __syncthreads();
    for (uint32_t s = blockIdx.x * SEG_BLOCK + threadIdx.x; s < P.n; s += gridDim.x * SEG_BLOCK) {
        uint32_t fs, fe;
        const uint32_t f = frame_range(P, s_foff, lds, s, &fs, &fe);
        const uint64_t c = P.keys_a[s] >> CELL_SHIFT;
        const bool start = P.fc[f].dmax > SORT_SHORT_LEVEL && (s == fs || (P.keys_a[s - 1] >> CELL_SHIFT) != c) &&
                           (uint64_t)s + cap < fe && (P.keys_a[s + cap] >> CELL_SHIFT) == c;
        if (!start) continue;
        P.deepf[s] = 2u;
        const int32_t cx = (int32_t)compact3(c), cy = (int32_t)compact3(c >> 1), cz = (int32_t)compact3(c >> 2);
        const int32_t side = 1 << SORT_SHORT_LEVEL;
        for (int g = 0; g < 27; ++g) {
            const int32_t nx = cx + g % 3 - 1, ny = cy + (g / 3) % 3 - 1, nz = cz + g / 9 - 1;
            if (g == 13 || nx < 0 || ny < 0 || nz < 0 || nx >= side || ny >= side || nz >= side) continue;
            const uint64_t nc = morton3((uint32_t)nx, (uint32_t)ny, (uint32_t)nz);
            const uint32_t q = cell_lower_bound(P.keys_a, fs, fe, nc);
            if (q < fe && (P.keys_a[q] >> CELL_SHIFT) == nc) P.deepf[q] = 2u;
        }
    }
}

// One thread per sorted position: a marked position starts a cell to re-sort;
// it finds the cell's end, and the block then sorts the cells that start
// among its positions (deep ones flagged, the others unmarked). Blocks that
// read keys of a cell another block is sorting compare cell prefixes only,
// which the sort does not change; a mark is only read by the thread of its
// own position, and only that cell's block rewrites it.
template <bool LDS>
__global__ __launch_bounds__(SEG_BLOCK) void deep_cells_kernel(Plan P, uint32_t cap) {
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_w[SEG_BLOCK / 64][256];
    __shared__ uint32_t s_scan[SEG_BLOCK / 64 + 1];
    __shared__ uint2 s_seg[SEG_BLOCK];
    __shared__ uint8_t s_deep[SEG_BLOCK];
    __shared__ uint32_t s_nseg;
    __shared__ uint32_t s_foff[SORT_FOFF_LDS];  // batches of fewer frames search the offsets here
    constexpr bool lds = LDS;
    if (lds)
        for (uint32_t i = threadIdx.x; i <= P.nf; i += blockDim.x) s_foff[i] = P.foff[i];
    for (uint32_t base = blockIdx.x * SEG_BLOCK; base < P.n; base += gridDim.x * SEG_BLOCK) {
        if (threadIdx.x == 0) s_nseg = 0u;
        __syncthreads();
        const uint32_t s = base + threadIdx.x;
        if (s < P.n && P.deepf[s] == 2u) {
            uint32_t fs, fe;
            const uint32_t f = frame_range(P, s_foff, lds, s, &fs, &fe);
            const uint64_t c = P.keys_a[s] >> CELL_SHIFT;
            const uint32_t e = cell_lower_bound(P.keys_a, s + 1u, fe, c + 1u);
            const uint32_t slot = atomicAdd(&s_nseg, 1u);
            s_seg[slot] = make_uint2(s, e);
            s_deep[slot] = (uint8_t)(P.fc[f].dmax > SORT_SHORT_LEVEL && e - s > cap);
        }
        __syncthreads();
        const uint32_t ns = s_nseg;
        for (uint32_t g = 0; g < ns; ++g) sort_cell(P, s_seg[g].x, s_seg[g].y, s_deep[g] != 0u, s_base, s_w, s_scan);
        __syncthreads();
    }
}

void launch_sort(const Plan& P, const Params& prm, hipStream_t st) {
    // the keys start where the launched passes leave them in keys_a
    const uint64_t* kin = P.keys_src;
    const uint32_t* vin = P.idx_src;
    uint64_t* kout = P.keys_src == P.keys_a ? P.keys_b : P.keys_a;
    uint32_t* vout = P.idx_src == P.idx_a ? P.idx_b : P.idx_a;
    for (uint32_t pass = SORT_SHORT_FIRST; pass < P.sort_passes; ++pass) {
        // small inputs: many small tiles (latency); large: fewer, fuller tiles
        auto kern = P.sort_items == 4 ? radix_pass_kernel<4> : radix_pass_kernel<16>;
        hipLaunchKernelGGL(kern, dim3(P.sort_tiles), dim3(SORT_BLOCK), 0, st, kin, vin, kout, vout,
                           P.n, (int)pass, P.sort_hist + 256 * pass,
                           P.sort_status + (size_t)pass * P.sort_tiles * 256, &P.ctr->status,
                           (const uint32_t*)P.foff, P.nf);
        const uint64_t* tk = kout;
        const uint32_t* tv = vout;
        kout = (uint64_t*)kin;
        vout = (uint32_t*)vin;
        kin = tk;
        vin = tv;
    }
    unsigned blocks = (P.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    const bool lds = P.nf > 1u && P.nf < SORT_FOFF_LDS;
    hipLaunchKernelGGL(lds ? deep_mark_kernel<true> : deep_mark_kernel<false>, dim3(blocks), dim3(SEG_BLOCK), 0, st, P,
                       (uint32_t)prm.leaf_cap);
    hipLaunchKernelGGL(lds ? deep_cells_kernel<true> : deep_cells_kernel<false>, dim3(blocks), dim3(SEG_BLOCK), 0, st,
                       P, (uint32_t)prm.leaf_cap);
}

}  // namespace gdn
