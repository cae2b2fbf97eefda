// Evaluation kernels (include/gdn.h, gdn_nearest / gdn_eval_metrics): exact
// nearest neighbours between two clouds and the quality metrics of a
// denoised cloud, PSNR (Eq. 29) and the Chamfer distance (Eq. 30).
//
// Nearest: brute force, one thread per query point, the reference cloud
// streamed through LDS in tiles; the reference is split into chunks over a
// second grid dimension so that small query sets still fill the chip, and the
// chunks' answers are combined with a 64-bit atomic minimum on the key
// (fp32 d2 bits << 32 | index): d2 >= 0, so the bit order is the value
// order, and equal distances resolve to the smaller index.
#include "kernels.hpp"

namespace gdn {

namespace {

constexpr int NN_BLOCK = 256;
constexpr int NN_TILE = 1024;               // reference points per LDS tile
constexpr unsigned NN_MIN_BLOCKS = 2048;    // split the reference until the grid has this many blocks
constexpr int EV_BLOCK = 256;
constexpr unsigned EV_BLOCKS_MAX = 1024;
constexpr int EV_STRIDE = 8;                // doubles per block partial

__global__ __launch_bounds__(256) void nn_init_kernel(unsigned long long* __restrict__ key, uint32_t na) {
    const unsigned long long none = (unsigned long long)__float_as_uint(INFINITY) << 32;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += gridDim.x * blockDim.x) key[i] = none;
}

__global__ __launch_bounds__(NN_BLOCK) void nn_kernel(const float* __restrict__ a, uint32_t na,
                                                      const float* __restrict__ b, uint32_t nb, uint32_t chunk,
                                                      unsigned long long* __restrict__ key) {
    __shared__ float sx[NN_TILE], sy[NN_TILE], sz[NN_TILE];
    const uint32_t i = blockIdx.x * NN_BLOCK + threadIdx.x;
    const bool live = i < na;
    float ax = 0.f, ay = 0.f, az = 0.f;
    if (live) {
        ax = a[3 * (size_t)i];
        ay = a[3 * (size_t)i + 1];
        az = a[3 * (size_t)i + 2];
    }
    const uint32_t c0 = blockIdx.y * chunk;
    const uint32_t c1 = min(nb, c0 + chunk);
    float best = INFINITY;
    uint32_t bi = 0;
    for (uint32_t t0 = c0; t0 < c1; t0 += NN_TILE) {
        const uint32_t tn = min((uint32_t)NN_TILE, c1 - t0);
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < tn; e += NN_BLOCK) {
            sx[e] = b[3 * (size_t)(t0 + e)];
            sy[e] = b[3 * (size_t)(t0 + e) + 1];
            sz[e] = b[3 * (size_t)(t0 + e) + 2];
        }
        __syncthreads();
        for (uint32_t e = 0; e < tn; ++e) {
            const float dx = sx[e] - ax, dy = sy[e] - ay, dz = sz[e] - az;
            const float d = (dx * dx + dy * dy) + dz * dz;  // compiled without contraction (no FMA)
            if (d < best) {
                best = d;
                bi = t0 + e;
            }
        }
    }
    if (live && best < INFINITY)
        atomicMin(&key[i], ((unsigned long long)__float_as_uint(best) << 32) | bi);
}

__global__ __launch_bounds__(256) void nn_out_kernel(const unsigned long long* __restrict__ key, uint32_t na,
                                                     uint32_t* __restrict__ idx, float* __restrict__ d2) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += gridDim.x * blockDim.x) {
        const unsigned long long k = key[i];
        idx[i] = (uint32_t)k;
        d2[i] = __uint_as_float((uint32_t)(k >> 32));
    }
}

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_min_f(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_max_f(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Per block: sum of the FP64 squared distances from points of a to their
// matched points of b (slot 0), and the fp32 min/max per axis of a (slots
// 1..6, only when `box` is set).
__global__ __launch_bounds__(EV_BLOCK) void ev_sum_kernel(const float* __restrict__ a, uint32_t na,
                                                          const float* __restrict__ b,
                                                          const unsigned long long* __restrict__ key, bool box,
                                                          double* __restrict__ part) {
    __shared__ double s_sum[EV_BLOCK / 64];
    __shared__ float s_lo[EV_BLOCK / 64][3], s_hi[EV_BLOCK / 64][3];
    double s = 0.0;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t i = blockIdx.x * EV_BLOCK + threadIdx.x; i < na; i += gridDim.x * EV_BLOCK) {
        const uint32_t j = (uint32_t)key[i];
        double d = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float ac = a[3 * (size_t)i + c];
            const double e = (double)b[3 * (size_t)j + c] - (double)ac;
            d += e * e;
            lo[c] = fminf(lo[c], ac);
            hi[c] = fmaxf(hi[c], ac);
        }
        s += d;
    }
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    s = wave_sum_d(s);
    for (int c = 0; c < 3; ++c) {
        lo[c] = wave_min_f(lo[c]);
        hi[c] = wave_max_f(hi[c]);
    }
    if (lane == 0) {
        s_sum[w] = s;
        for (int c = 0; c < 3; ++c) {
            s_lo[w][c] = lo[c];
            s_hi[w][c] = hi[c];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < EV_BLOCK / 64; ++q) t += s_sum[q];
        part[(size_t)blockIdx.x * EV_STRIDE] = t;
        if (box) {
            for (int c = 0; c < 3; ++c) {
                float l = s_lo[0][c], h = s_hi[0][c];
                for (int q = 1; q < EV_BLOCK / 64; ++q) {
                    l = fminf(l, s_lo[q][c]);
                    h = fmaxf(h, s_hi[q][c]);
                }
                part[(size_t)blockIdx.x * EV_STRIDE + 1 + c] = (double)l;
                part[(size_t)blockIdx.x * EV_STRIDE + 4 + c] = (double)h;
            }
        }
    }
}

// One wave: MSE (clean -> denoised), mean denoised -> clean, CD, PSNR.
__global__ __launch_bounds__(64) void ev_final_kernel(const double* __restrict__ pc, uint32_t nbc,
                                                      const double* __restrict__ pd, uint32_t nbd, uint32_t nc,
                                                      uint32_t nd, double* __restrict__ out) {
    const uint32_t lane = threadIdx.x;
    double sc = 0.0, sd = 0.0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t q = lane; q < nbc; q += 64u) {
        sc += pc[(size_t)q * EV_STRIDE];
        for (int c = 0; c < 3; ++c) {
            lo[c] = fmin(lo[c], pc[(size_t)q * EV_STRIDE + 1 + c]);
            hi[c] = fmax(hi[c], pc[(size_t)q * EV_STRIDE + 4 + c]);
        }
    }
    for (uint32_t q = lane; q < nbd; q += 64u) sd += pd[(size_t)q * EV_STRIDE];
    sc = wave_sum_d(sc);
    sd = wave_sum_d(sd);
    for (int c = 0; c < 3; ++c) {
        for (int o = 32; o > 0; o >>= 1) {
            lo[c] = fmin(lo[c], __shfl_xor(lo[c], o, 64));
            hi[c] = fmax(hi[c], __shfl_xor(hi[c], o, 64));
        }
    }
    if (lane == 0) {
        double m2 = 0.0;
        for (int c = 0; c < 3; ++c) m2 += (hi[c] - lo[c]) * (hi[c] - lo[c]);
        const double mse = sc / (double)nc;
        out[0] = mse;
        out[1] = sd / (double)nd;
        out[2] = out[0] + out[1];
        out[3] = 10.0 * log10(m2 / mse);
    }
}

unsigned ev_blocks(uint32_t n) {
    unsigned b = (n + EV_BLOCK - 1) / EV_BLOCK;
    if (b > EV_BLOCKS_MAX) b = EV_BLOCKS_MAX;
    return b == 0 ? 1u : b;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t nearest_workspace_bytes(uint32_t na) { return al256((size_t)8 * na); }

void launch_nearest_keys(const float* a, uint32_t na, const float* b, uint32_t nb, unsigned long long* key,
                         hipStream_t st) {
    unsigned ib = (na + 255) / 256;
    if (ib > 4096) ib = 4096;
    hipLaunchKernelGGL(nn_init_kernel, dim3(ib), dim3(256), 0, st, key, na);
    const unsigned qb = (na + NN_BLOCK - 1) / NN_BLOCK;
    const unsigned tiles = (nb + NN_TILE - 1) / NN_TILE;
    unsigned split = (NN_MIN_BLOCKS + qb - 1) / qb;
    if (split > tiles) split = tiles;
    if (split < 1) split = 1;
    const uint32_t chunk = ((nb + split - 1) / split + NN_TILE - 1) / NN_TILE * NN_TILE;
    split = (nb + chunk - 1) / chunk;
    hipLaunchKernelGGL(nn_kernel, dim3(qb, split), dim3(NN_BLOCK), 0, st, a, na, b, nb, chunk, key);
}

void launch_nearest(const float* a, uint32_t na, const float* b, uint32_t nb, void* ws, uint32_t* idx, float* d2,
                    hipStream_t st) {
    unsigned long long* key = (unsigned long long*)ws;
    launch_nearest_keys(a, na, b, nb, key, st);
    unsigned ob = (na + 255) / 256;
    if (ob > 4096) ob = 4096;
    hipLaunchKernelGGL(nn_out_kernel, dim3(ob), dim3(256), 0, st, key, na, idx, d2);
}

size_t eval_workspace_bytes(uint32_t nc, uint32_t nd) {
    return al256((size_t)8 * nc) + al256((size_t)8 * nd) + 2 * al256((size_t)8 * EV_STRIDE * EV_BLOCKS_MAX);
}

void launch_eval(const float* clean, uint32_t nc, const float* den, uint32_t nd, void* ws, double* out,
                 hipStream_t st) {
    char* w = (char*)ws;
    unsigned long long* kc = (unsigned long long*)w;
    w += al256((size_t)8 * nc);
    unsigned long long* kd = (unsigned long long*)w;
    w += al256((size_t)8 * nd);
    double* pc = (double*)w;
    w += al256((size_t)8 * EV_STRIDE * EV_BLOCKS_MAX);
    double* pd = (double*)w;
    launch_nearest_keys(clean, nc, den, nd, kc, st);
    launch_nearest_keys(den, nd, clean, nc, kd, st);
    const unsigned bc = ev_blocks(nc), bd = ev_blocks(nd);
    hipLaunchKernelGGL(ev_sum_kernel, dim3(bc), dim3(EV_BLOCK), 0, st, clean, nc, den, kc, true, pc);
    hipLaunchKernelGGL(ev_sum_kernel, dim3(bd), dim3(EV_BLOCK), 0, st, den, nd, clean, kd, false, pd);
    hipLaunchKernelGGL(ev_final_kernel, dim3(1), dim3(64), 0, st, pc, bc, pd, bd, nc, nd, out);
}

}  // namespace gdn
