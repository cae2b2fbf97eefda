// Copies of the last frame's intermediates, mapped back to original point
// order, for the per-stage parity checks.
#include "gdn.h"
#include "kernels.hpp"

namespace gdn {

__global__ __launch_bounds__(256) void dump_kernel(Plan P, int what, void* dst) {
    const uint32_t n = P.n, k = (uint32_t)P.k;
    const uint32_t nl = P.ctr->n_leaves;
    const uint32_t lim = n > nl ? n : nl;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < lim; s += gridDim.x * blockDim.x) {
        const bool pt = s < n;
        const uint32_t i = pt ? P.idx_a[s] : 0u;
        const bool in1 = pt && P.p1[s];
        const uint32_t qi = in1 ? P.p1pos[s] : 0u;
        switch (what) {
            case GDN_DUMP_KEYS: if (pt) ((uint64_t*)dst)[i] = P.keys_a[s]; break;
            case GDN_DUMP_ORDER: if (pt) ((uint32_t*)dst)[s] = i; break;
            case GDN_DUMP_LEAF_OF: if (pt) ((uint32_t*)dst)[i] = P.leaf_of[s]; break;
            case GDN_DUMP_OCC: if (pt) ((uint32_t*)dst)[i] = P.occ[s]; break;
            case GDN_DUMP_P1: if (pt) ((uint8_t*)dst)[i] = P.p1[s]; break;
            case GDN_DUMP_NBR_IDX:
                if (pt)
                    for (uint32_t r = 0; r < k; ++r)
                    {
                        // neighbours are stored by P1 position: map back to the original index
                        const uint32_t pj = in1 ? P.nbr[(size_t)qi * k + r] : 0xFFFFFFFFu;
                        ((uint32_t*)dst)[(size_t)i * k + r] = pj != 0xFFFFFFFFu ? __float_as_uint(P.cand4[pj].w) : pj;
                    }
                break;
            case GDN_DUMP_NBR_D2:
                if (pt)
                    for (uint32_t r = 0; r < k; ++r)
                        ((float*)dst)[(size_t)i * k + r] = in1 ? P.nbr_d2[(size_t)qi * k + r] : INFINITY;
                break;
            case GDN_DUMP_R2K: if (pt) ((float*)dst)[i] = in1 ? P.r2k[qi] : __uint_as_float(0x7FC00000u); break;
            case GDN_DUMP_RHO: if (pt) ((double*)dst)[i] = in1 ? P.rho_c[qi] : __longlong_as_double(0x7FF8000000000000ll); break;
            case GDN_DUMP_P2: if (pt) ((uint8_t*)dst)[i] = in1 ? P.p2[qi] : 0; break;
            case GDN_DUMP_SCORE64:
                if (pt) ((double*)dst)[i] = (in1 && P.p2[qi]) ? P.score_c[qi] : -1.0;
                break;
            case GDN_DUMP_LEAF_TABLE:
                if (s < nl) {
                    uint32_t* o = (uint32_t*)dst + 4 * (size_t)s;
                    o[0] = P.leaf_begin[s];
                    o[1] = P.leaf_begin[s + 1];
                    o[2] = P.leaf_level[s];
                    o[3] = __float_as_uint(P.leaf_h[s]);
                }
                break;
            case GDN_DUMP_LEAF_RHO_MED: if (s < nl) ((double*)dst)[s] = P.leaf_rho_med[s]; break;
            case GDN_DUMP_LEAF_NCAND: if (s < nl) ((uint32_t*)dst)[s] = P.leaf_ncand[s]; break;
            default: break;
        }
    }
}

__global__ void dump_scalars_kernel(Plan P, int what, void* dst) {
    if (what == GDN_DUMP_STATUS) {
        *(uint32_t*)dst = P.ctr->status;
    } else {
        int64_t* o = (int64_t*)dst;
        o[0] = P.ctr->n_leaves;
        o[1] = P.ctr->n_p1;
        o[2] = (int64_t)P.ctr->pairs;
        o[3] = P.ctr->n_kept;
    }
}

// Bytes the dump of `what` needs for a frame of n points (leaf dumps are sized
// for the largest possible leaf count, n).
size_t dump_bytes(uint32_t n, int k, int what) {
    switch (what) {
        case GDN_DUMP_STATUS: return 4;
        case GDN_DUMP_COUNTS: return 32;
        case GDN_DUMP_KEYS: return 8ull * n;
        case GDN_DUMP_ORDER: case GDN_DUMP_LEAF_OF: case GDN_DUMP_OCC: case GDN_DUMP_R2K:
        case GDN_DUMP_LEAF_NCAND: return 4ull * n;
        case GDN_DUMP_P1: case GDN_DUMP_P2: return n;
        case GDN_DUMP_NBR_IDX: case GDN_DUMP_NBR_D2: return 4ull * n * k;
        case GDN_DUMP_RHO: case GDN_DUMP_SCORE64: case GDN_DUMP_LEAF_RHO_MED: return 8ull * n;
        case GDN_DUMP_LEAF_TABLE: return 16ull * n;
        default: return 0;
    }
}

int launch_dump(const Plan& P, int what, void* dst, size_t dst_bytes, hipStream_t st) {
    const size_t need = dump_bytes(P.n, P.k, what);
    if (need == 0 || dst_bytes < need) return 1;
    if (what == GDN_DUMP_STATUS || what == GDN_DUMP_COUNTS) {
        hipLaunchKernelGGL(dump_scalars_kernel, dim3(1), dim3(1), 0, st, P, what, dst);
        return 0;
    }
    unsigned blocks = (P.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(dump_kernel, dim3(blocks), dim3(256), 0, st, P, what, dst);
    return 0;
}

}  // namespace gdn
