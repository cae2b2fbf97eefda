// Frame-level passes: zero-fill of the workspace control block, the frame
// bounding box (the octree root cube, Sec. 3 with Eq. 2), 63-bit Morton keys,
// the stable LSD radix sort of (key, original index) and the gather of the
// sorted coordinates.
#include "kernels.hpp"

namespace gdn {

// ---------------------------------------------------------------- zero fill

__global__ void zero_kernel(uint4* p, size_t n16) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

void launch_zero(const Plan& P, hipStream_t st) {
    size_t n16 = P.zero_bytes / 16;
    unsigned blocks = (unsigned)((n16 + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, st, (uint4*)P.zero_begin, n16);
}

// ---------------------------------------------------------------- bbox

__global__ __launch_bounds__(256) void bbox_kernel(const float* __restrict__ xyz, uint32_t n, Counters* c) {
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    uint32_t bad = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float x = xyz[3 * (size_t)i], y = xyz[3 * (size_t)i + 1], z = xyz[3 * (size_t)i + 2];
        if (isfinite(x) && isfinite(y) && isfinite(z)) {
            mn[0] = fminf(mn[0], x); mx[0] = fmaxf(mx[0], x);
            mn[1] = fminf(mn[1], y); mx[1] = fmaxf(mx[1], y);
            mn[2] = fminf(mn[2], z); mx[2] = fmaxf(mx[2], z);
        } else {
            ++bad;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = fminf(mn[a], __shfl_xor(mn[a], o, 64));
            mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], o, 64));
        }
        bad += __shfl_xor(bad, o, 64);
    }
    __shared__ float s_mn[3][4], s_mx[3][4];
    __shared__ uint32_t s_bad[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        for (int a = 0; a < 3; ++a) { s_mn[a][wave] = mn[a]; s_mx[a][wave] = mx[a]; }
        s_bad[wave] = bad;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int a = threadIdx.x;
        float m0 = s_mn[a][0], m1 = s_mx[a][0];
        for (int w = 1; w < 4; ++w) { m0 = fminf(m0, s_mn[a][w]); m1 = fmaxf(m1, s_mx[a][w]); }
        if (m0 <= m1) {
            atomicMax(&c->bbox_nmin[a], ~f32_ordered(m0));
            atomicMax(&c->bbox_max[a], f32_ordered(m1));
        }
    }
    if (threadIdx.x == 3) {
        uint32_t b = s_bad[0] + s_bad[1] + s_bad[2] + s_bad[3];
        if (b) {
            atomicAdd(&c->nonfinite, b);
            atomicOr(&c->status, DEV_NONFINITE);
        }
    }
}

void launch_bbox(const Plan& P, const float* xyz, hipStream_t st) {
    unsigned blocks = (P.n + 1023) / 1024;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(bbox_kernel, dim3(blocks), dim3(256), 0, st, xyz, P.n, P.ctr);
}

// ---------------------------------------------------------------- Morton keys

// Root cube: side S = largest bbox extent at the bbox minimum; depth limit from
// the minimum leaf side. Same FP64 expressions for every consumer.
__device__ void frame_consts(const Counters* c, double min_leaf_side, FrameConst* f) {
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

// Keys, the identity payload and the 8 digit histograms of the sort.
__global__ __launch_bounds__(256) void morton_kernel(const float* __restrict__ xyz, uint32_t n, Plan P,
                                                     double min_leaf_side) {
    __shared__ FrameConst s_fc;
    __shared__ uint32_t s_hist[SORT_PASSES][256];
    for (int i = threadIdx.x; i < SORT_PASSES * 256; i += blockDim.x) (&s_hist[0][0])[i] = 0u;
    if (threadIdx.x == 0) {
        frame_consts(P.ctr, min_leaf_side, &s_fc);
        if (blockIdx.x == 0) *P.fc = s_fc;
    }
    __syncthreads();
    const float lx = s_fc.lo[0], ly = s_fc.lo[1], lz = s_fc.lo[2];
    const double scale = s_fc.scale;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        uint32_t qx = quantise(xyz[3 * (size_t)i], lx, scale);
        uint32_t qy = quantise(xyz[3 * (size_t)i + 1], ly, scale);
        uint32_t qz = quantise(xyz[3 * (size_t)i + 2], lz, scale);
        uint64_t key = morton3(qx, qy, qz);
        P.keys_a[i] = key;
        P.idx_a[i] = i;
#pragma unroll
        for (int p = 0; p < SORT_PASSES; ++p) atomicAdd(&s_hist[p][(key >> (8 * p)) & 255u], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < SORT_PASSES * 256; i += blockDim.x) {
        uint32_t v = (&s_hist[0][0])[i];
        if (v) atomicAdd(&P.sort_hist[i], v);
    }
}

void launch_morton(const Plan& P, const Params& prm, const float* xyz, hipStream_t st) {
    unsigned blocks = (P.n + 2047) / 2048;
    if (blocks > 512) blocks = 512;
    hipLaunchKernelGGL(morton_kernel, dim3(blocks), dim3(256), 0, st, xyz, P.n, P, prm.min_leaf_side);
}

// ---------------------------------------------------------------- radix sort

// One stable LSD pass over digit `pass` (8 bits) in the onesweep style: local
// ranks by wave-level digit matching, digit offsets of earlier tiles by
// decoupled look-back (bounded waits), global digit bases from the histogram.
__global__ __launch_bounds__(SORT_BLOCK) void radix_pass_kernel(const uint64_t* __restrict__ kin,
                                                                const uint32_t* __restrict__ vin,
                                                                uint64_t* __restrict__ kout,
                                                                uint32_t* __restrict__ vout, uint32_t n,
                                                                int pass, const uint32_t* __restrict__ hist,
                                                                uint32_t* status, uint32_t* tile_ctr,
                                                                uint32_t* dev_status) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_w[SORT_BLOCK / 64][256];
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_scan[SORT_BLOCK / 64 + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int shift = 8 * pass;
    for (int i = tid; i < (SORT_BLOCK / 64) * 256; i += SORT_BLOCK) (&s_w[0][0])[i] = 0u;
    if (tid == 0) s_tile = atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t tbase = tile * SORT_TILE + wave * (64 * SORT_ITEMS);

    uint64_t key[SORT_ITEMS];
    uint32_t val[SORT_ITEMS], dig[SORT_ITEMS], rank[SORT_ITEMS];
#pragma unroll
    for (int i = 0; i < SORT_ITEMS; ++i) {
        uint32_t pos = tbase + i * 64 + lane;
        bool ok = pos < n;
        key[i] = ok ? kin[pos] : 0ull;
        val[i] = ok ? vin[pos] : 0u;
        dig[i] = ok ? (uint32_t)((key[i] >> shift) & 255u) : 256u;
    }
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int i = 0; i < SORT_ITEMS; ++i) {
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
    if (tile == 0) {
        st_relaxed_agent(st, LB_FLAG_PRE | tcnt);
    } else {
        st_relaxed_agent(st, LB_FLAG_AGG | tcnt);
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
    // global base of each digit
    uint32_t total;
    uint32_t gex = block_excl_scan(hist[tid], s_scan, &total);
    s_base[tid] = gex + excl;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SORT_ITEMS; ++i) {
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

void launch_sort(const Plan& P, hipStream_t st) {
    const uint64_t* kin = P.keys_a;
    const uint32_t* vin = P.idx_a;
    uint64_t* kout = P.keys_b;
    uint32_t* vout = P.idx_b;
    for (int pass = 0; pass < SORT_PASSES; ++pass) {
        hipLaunchKernelGGL(radix_pass_kernel, dim3(P.sort_tiles), dim3(SORT_BLOCK), 0, st, kin, vin, kout, vout,
                           P.n, pass, P.sort_hist + 256 * pass,
                           P.sort_status + (size_t)pass * P.sort_tiles * 256, &P.ctr->sort_tile_ctr[pass],
                           &P.ctr->status);
        const uint64_t* tk = kout;
        const uint32_t* tv = vout;
        kout = (uint64_t*)kin;
        vout = (uint32_t*)vin;
        kin = tk;
        vin = tv;
    }
    // SORT_PASSES is even: the sorted keys end in keys_a / idx_a
}

// ---------------------------------------------------------------- permute

__global__ __launch_bounds__(256) void permute_kernel(const float* __restrict__ xyz, Plan P) {
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < P.n; s += gridDim.x * blockDim.x) {
        uint32_t i = P.idx_a[s];
        P.pos4[s] = make_float4(xyz[3 * (size_t)i], xyz[3 * (size_t)i + 1], xyz[3 * (size_t)i + 2],
                                __uint_as_float(i));
    }
}

void launch_permute(const Plan& P, const float* xyz, hipStream_t st) {
    unsigned blocks = (P.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(permute_kernel, dim3(blocks), dim3(256), 0, st, xyz, P);
}

}  // namespace gdn
