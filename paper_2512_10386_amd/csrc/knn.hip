// Leaf-local brute-force kNN with halo candidates (Sec. 3: N_K(i), d_ij and
// r_K,i on the voxel-filtered set P1).
//
// One lane per query; candidates are staged in LDS tiles and read as
// broadcasts. Squared distances are fp32 (dx*dx + dy*dy) + dz*dz without
// contraction, so the neighbour sets are exact. Each lane keeps its k best
// (d2, original index) pairs as sorted 64-bit keys (d2 bits << 32 | index) in
// registers, updated by a fully unrolled insertion network; a list of KMAX
// slots serves any k <= KMAX by parking KMAX - k sentinel keys (-1) in front.
// Four candidates are tested against the current k-th distance with one
// comparison of their minimum, so the insertion path is only entered when one
// of them can enter the list.
#include <climits>

#include "kernels.hpp"

namespace gdn {

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

template <int KMAX>
__global__ __launch_bounds__(KNN_TQ) void knn_kernel(Plan P, int k) {
    __shared__ float4 s_c[KNN_CT];
    __shared__ uint2 s_r[HALO];
    __shared__ uint32_t s_it;
    const int tid = threadIdx.x;
    const uint32_t n_items = P.ctr->n_items;
    for (;;) {
        if (tid == 0) s_it = atomicAdd(&P.ctr->knn_next, 1u);
        __syncthreads();
        const uint32_t it = s_it;
        if (it >= n_items) break;
        const KnnItem w = P.items[it];
        const uint32_t t = w.leaf;
        const uint32_t nr = P.leaf_nr[t];
        if (tid < HALO) s_r[tid] = (tid < (int)nr) ? P.leaf_ranges[(size_t)t * HALO + tid] : make_uint2(0u, 0u);
        const uint32_t ncand = P.leaf_ncand[t], nch = P.leaf_nch[t], cc = P.leaf_cc[t];
        const uint32_t c_lo = w.chunk * cc;
        const uint32_t c_hi = min(ncand, c_lo + cc);
        const uint32_t qi = w.q0 + tid;
        const bool vq = qi < w.q1;
        const float4 q = vq ? P.cand4[qi] : make_float4(0.f, 0.f, 0.f, 0.f);
        const uint32_t self = __float_as_uint(q.w);
        long long a[KMAX];
#pragma unroll
        for (int r = 0; r < KMAX; ++r) a[r] = (r < KMAX - k) ? -1ll : LLONG_MAX;
        float worst = __uint_as_float(0x7FFFFFFFu);  // NaN until the list is full
        __syncthreads();

        // cursor (range rr, offset off) at logical candidate position c_lo
        uint32_t rr = 0, off = c_lo;
        while (rr < nr && off >= s_r[rr].y - s_r[rr].x) {
            off -= s_r[rr].y - s_r[rr].x;
            ++rr;
        }
        for (uint32_t pos = c_lo; pos < c_hi; pos += KNN_CT) {
            const uint32_t tn = min((uint32_t)KNN_CT, c_hi - pos);
            uint32_t filled = 0;
            while (filled < tn && rr < nr) {
                const uint2 R = s_r[rr];
                const uint32_t len = R.y - R.x;
                const uint32_t piece = min(len - off, tn - filled);
                if (piece == 0) { ++rr; off = 0; continue; }  // never taken: ranges are non-empty
                for (uint32_t u = tid; u < piece; u += KNN_TQ) s_c[filled + u] = P.cand4[R.x + off + u];
                filled += piece;
                off += piece;
                if (off == len) { ++rr; off = 0; }
            }
            __syncthreads();
            uint32_t j = 0;
            for (; j + 4 <= tn; j += 4) {
                const float4 c0 = s_c[j], c1 = s_c[j + 1], c2 = s_c[j + 2], c3 = s_c[j + 3];
                const float d0 = dist2(q, c0), d1 = dist2(q, c1), d2 = dist2(q, c2), d3 = dist2(q, c3);
                const float dm = fminf(fminf(d0, d1), fminf(d2, d3));
                if (vq && !(dm > worst)) {
                    try_insert<KMAX>(a, worst, d0, c0.w, self);
                    try_insert<KMAX>(a, worst, d1, c1.w, self);
                    try_insert<KMAX>(a, worst, d2, c2.w, self);
                    try_insert<KMAX>(a, worst, d3, c3.w, self);
                }
            }
            for (; j < tn; ++j) {
                const float4 c0 = s_c[j];
                const float d0 = dist2(q, c0);
                if (vq && !(d0 > worst)) try_insert<KMAX>(a, worst, d0, c0.w, self);
            }
            __syncthreads();
        }

        if (vq) {
            if (nch == 1) {
                uint32_t* out = P.nbr + (size_t)qi * k;
                float* od = P.nbr_d2 + (size_t)qi * k;
#pragma unroll
                for (int r = 0; r < KMAX; ++r) {
                    if (r >= KMAX - k) {
                        const long long v = a[r];
                        const bool ok = v != LLONG_MAX;
                        out[r - (KMAX - k)] = ok ? (uint32_t)v : 0xFFFFFFFFu;
                        od[r - (KMAX - k)] = ok ? __uint_as_float((uint32_t)((unsigned long long)v >> 32)) : INFINITY;
                    }
                }
                const long long last = a[KMAX - 1];
                P.r2k[qi] = last != LLONG_MAX ? __uint_as_float((uint32_t)((unsigned long long)last >> 32)) : INFINITY;
            } else {
                const uint32_t qb = P.p1pos[P.leaf_begin[t]];
                long long* pl = (long long*)P.plist +
                                ((size_t)P.leaf_plist[t] + (size_t)(qi - qb) * nch + w.chunk) * (size_t)k;
#pragma unroll
                for (int r = 0; r < KMAX; ++r)
                    if (r >= KMAX - k) pl[r - (KMAX - k)] = a[r];
            }
        }
        __syncthreads();
    }
}

// k-way merge of the sorted partial lists of chunked leaves.
__global__ __launch_bounds__(256) void knn_merge_kernel(Plan P, int k) {
    __shared__ uint8_t s_h[256 * KNN_NCH_MAX];
    uint8_t* h = s_h + threadIdx.x * KNN_NCH_MAX;
    const uint32_t np1 = P.ctr->n_p1;
    for (uint32_t qi = blockIdx.x * blockDim.x + threadIdx.x; qi < np1; qi += gridDim.x * blockDim.x) {
        const uint32_t t = P.cand_leaf[qi];
        const uint32_t nch = P.leaf_nch[t];
        if (nch <= 1) continue;
        const uint32_t qb = P.p1pos[P.leaf_begin[t]];
        const long long* pl = (const long long*)P.plist + ((size_t)P.leaf_plist[t] + (size_t)(qi - qb) * nch) * (size_t)k;
        for (uint32_t c = 0; c < nch; ++c) h[c] = 0;
        uint32_t* out = P.nbr + (size_t)qi * k;
        float* od = P.nbr_d2 + (size_t)qi * k;
        long long last = LLONG_MAX;
        for (int r = 0; r < k; ++r) {
            long long best = LLONG_MAX;
            int bc = -1;
            for (uint32_t c = 0; c < nch; ++c) {
                const int hc = h[c];
                if (hc < k) {
                    const long long v = pl[(size_t)c * k + hc];
                    if (v < best) { best = v; bc = (int)c; }
                }
            }
            if (bc >= 0) h[bc] = (uint8_t)(h[bc] + 1);
            const bool ok = best != LLONG_MAX;
            out[r] = ok ? (uint32_t)best : 0xFFFFFFFFu;
            od[r] = ok ? __uint_as_float((uint32_t)((unsigned long long)best >> 32)) : INFINITY;
            last = best;
        }
        P.r2k[qi] = last != LLONG_MAX ? __uint_as_float((uint32_t)((unsigned long long)last >> 32)) : INFINITY;
    }
}

template <int KMAX>
static void launch_knn_t(const Plan& P, int k, int num_cus, hipStream_t st) {
    const unsigned blocks = (unsigned)(num_cus > 0 ? num_cus : 256) * 4u;
    hipLaunchKernelGGL(knn_kernel<KMAX>, dim3(blocks), dim3(KNN_TQ), 0, st, P, k);
}

void launch_knn(const Plan& P, int k, int num_cus, hipStream_t st) {
    if (k <= 8) launch_knn_t<8>(P, k, num_cus, st);
    else if (k <= 16) launch_knn_t<16>(P, k, num_cus, st);
    else if (k <= 32) launch_knn_t<32>(P, k, num_cus, st);
    else launch_knn_t<64>(P, k, num_cus, st);
    unsigned blocks = (P.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(knn_merge_kernel, dim3(blocks), dim3(256), 0, st, P, k);
}

}  // namespace gdn
