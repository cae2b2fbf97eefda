// Score fit (include/gdn.h, gdn_fit_loss_grad): the loss of a relaxed
// threshold on ln F_i and its gradient over alpha, sigma, gamma and tau, on
// the neighbour sets, densities, medians and P2 of the last pipeline pass.
//
// F_i follows Eq. 21 with the kernel of Eq. 20 raised to gamma/2:
//   t_ij = exp(alpha/2 * ln(rho_i rho_j / (rho_med^2 + eps)))     (Eq. 17)
//        * exp(-d_ij^2 / (2 sigma^2 r_K,i^2))                      (Eq. 18, 19)
//        * exp(-gamma/2 * ln(d_ij^2 + eps))                        (Eq. 20)
// and its log-derivatives are, term by term,
//   d/dalpha ln t = ln(ratio) / 2, d/dsigma ln t = d^2 / (sigma^3 r^2),
//   d/dgamma ln t = -ln(d^2 + eps) / 2.
// With y_i = 1 for a clean point, z_i = (ln F_i - tau) / T and
// p_i = sigmoid(z_i), the loss is the mean binary cross-entropy over the P2
// points with 0 < F_i < inf, and dL/dz_i = (p_i - y_i) / count.
//
// One lane per neighbour (as the score kernel); per-block partial sums in a
// fixed order, then one block sums the partials: the result does not depend
// on scheduling.
#include "kernels.hpp"

namespace gdn {

namespace {

constexpr int FIT_PARTS = 6;        // loss, d/dalpha, d/dsigma, d/dgamma, d/dtau, count
constexpr int FIT_STRIDE = 8;       // doubles per block partial
constexpr unsigned FIT_BLOCKS_MAX = 1024;

__device__ __forceinline__ double seg_sum_f(double v, uint32_t kp) {
    for (uint32_t o = kp >> 1; o > 0; o >>= 1) v += __shfl_xor(v, (int)o, 64);
    return v;
}

__device__ __forceinline__ double wave_sum_f(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ln rho of every P1 point, at its P1 position (where the neighbour lists
// point). rho = 0 (fewer than k candidates) gives -inf.
__global__ __launch_bounds__(256) void fit_prep_kernel(Plan P, double* __restrict__ lrho_p) {
    const uint32_t np1 = P.ctr->n_p1;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < np1; q += gridDim.x * blockDim.x)
        lrho_p[q] = log(P.rho_c[q]);
}

__global__ __launch_bounds__(256) void fit_kernel(Plan P, const float* __restrict__ xyz,
                                                  const uint8_t* __restrict__ label,
                                                  const double* __restrict__ lrho_p, int kk, FitArgs a,
                                                  double* __restrict__ part) {
    __shared__ double s_red[4][FIT_PARTS];
    const uint32_t np1 = P.ctr->n_p1;
    const uint32_t k = (uint32_t)kk;
    uint32_t kp = 1;
    while (kp < k) kp <<= 1;
    const uint32_t qpw = 64u / kp;
    const uint32_t lane = threadIdx.x & 63u, seg = lane / kp, r = lane % kp;
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    const double s3 = a.sigma * a.sigma * a.sigma;
    double acc[FIT_PARTS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (uint32_t q0 = wid * qpw; q0 < np1; q0 += nw * qpw) {
        const uint32_t qi = q0 + seg;
        const bool live = qi < np1 && P.p2[qi];
        double t = 0.0, tA = 0.0, tS = 0.0, tG = 0.0;
        uint32_t i = 0;
        if (live) i = __float_as_uint(P.cand4[qi].w);
        if (live && r < k) {
            const uint32_t j = P.nbr[(size_t)qi * k + r];
            if (j < P.n) {
                const double med = P.leaf_rho_med[P.cand_leaf[qi]];
                const double lr = log(P.rho_c[qi]) + lrho_p[j] - log(med * med + a.eps);
                const double r64 = P.r64_c[qi];
                const double r2 = r64 * r64;
                // the neighbour (P1 position j) and the query from their sorted
                // copies of the input coordinates
                const float4 cj = P.cand4[j], ci = P.cand4[qi];
                const double dx = (double)cj.x - (double)ci.x;
                const double dy = (double)cj.y - (double)ci.y;
                const double dz = (double)cj.z - (double)ci.z;
                const double d2 = dx * dx + dy * dy + dz * dz;
                const double lk = log(d2 + a.eps);
                const double w_den = exp(0.5 * a.alpha * lr);
                const double w_dis = d2 == 0.0 ? 1.0 : exp(-d2 / (2.0 * a.sigma * a.sigma * r2));
                const double tt = w_den * w_dis * exp(-0.5 * a.gamma * lk);
                if (tt != 0.0) {
                    t = tt;
                    tA = tt * 0.5 * lr;
                    tS = d2 != 0.0 ? tt * d2 / (s3 * r2) : 0.0;
                    tG = tt * (-0.5 * lk);
                }
            }
        }
        const double F = seg_sum_f(t, kp);
        const double A = seg_sum_f(tA, kp);
        const double S = seg_sum_f(tS, kp);
        const double G = seg_sum_f(tG, kp);
        if (live && r == 0 && F > 0.0 && F < INFINITY) {
            const double y = label[i] ? 0.0 : 1.0;
            const double z = (log(F) - a.tau) / a.T;
            const double p = 1.0 / (1.0 + exp(-z));
            acc[0] += (z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z))) - y * z;
            const double g = (p - y) / a.T;
            acc[1] += g * A / F;
            acc[2] += g * S / F;
            acc[3] += g * G / F;
            acc[4] -= g;
            acc[5] += 1.0;
        }
    }
    const uint32_t wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < FIT_PARTS; ++c) {
        const double v = wave_sum_f(acc[c]);
        if (lane == 0) s_red[wave][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < FIT_PARTS) {
        const uint32_t c = threadIdx.x;
        part[(size_t)blockIdx.x * FIT_STRIDE + c] = ((s_red[0][c] + s_red[1][c]) + s_red[2][c]) + s_red[3][c];
    }
}

// One wave: sums the block partials in a fixed order and normalises by the count.
__global__ __launch_bounds__(64) void fit_final_kernel(const double* __restrict__ part, uint32_t nb,
                                                       double* __restrict__ out) {
    const uint32_t lane = threadIdx.x;
    double tot[FIT_PARTS];
#pragma unroll
    for (int c = 0; c < FIT_PARTS; ++c) {
        double v = 0.0;
        for (uint32_t b = lane; b < nb; b += 64u) v += part[(size_t)b * FIT_STRIDE + c];
        tot[c] = wave_sum_f(v);
    }
    if (lane == 0) {
        const double cnt = tot[5];
        const double d = cnt > 0.0 ? cnt : 1.0;
        for (int c = 0; c < 5; ++c) out[c] = tot[c] / d;
        out[5] = cnt;
    }
}

unsigned fit_blocks(uint32_t n, int k) {
    uint32_t kp = 1;
    while (kp < (uint32_t)k) kp <<= 1;
    const uint64_t waves = ((uint64_t)n * kp + 63) / 64;
    uint64_t b = (waves + 3) / 4;
    if (b > FIT_BLOCKS_MAX) b = FIT_BLOCKS_MAX;
    return b == 0 ? 1u : (unsigned)b;
}

}  // namespace

size_t fit_workspace_bytes(uint32_t n) {
    return (((size_t)8 * n + 255) & ~(size_t)255) + (size_t)FIT_STRIDE * 8 * FIT_BLOCKS_MAX;
}

void launch_fit(const Plan& P, const float* xyz, const uint8_t* label, const FitArgs& a, void* workspace,
                double* out, hipStream_t st) {
    double* lrho_p = (double*)workspace;
    double* part = (double*)((char*)workspace + (((size_t)8 * P.n + 255) & ~(size_t)255));
    unsigned pb = (P.n + 255) / 256;
    if (pb > 4096) pb = 4096;
    if (pb == 0) pb = 1;
    hipLaunchKernelGGL(fit_prep_kernel, dim3(pb), dim3(256), 0, st, P, lrho_p);
    const unsigned nb = fit_blocks(P.n, P.k);
    hipLaunchKernelGGL(fit_kernel, dim3(nb), dim3(256), 0, st, P, xyz, label, lrho_p, P.k, a, part);
    hipLaunchKernelGGL(fit_final_kernel, dim3(1), dim3(64), 0, st, part, nb, out);
}

}  // namespace gdn
