// Wave-level (64-lane) helpers for gfx950: lane ^ M exchanges without LDS,
// bitonic sorts and merges of one 64-bit key per lane, min / max reductions
// and a radix select of up to 256 keys.
#pragma once

#include "common.hpp"

namespace gdn {

// Value of lane ^ M without an LDS access: DPP quad permutes (1, 2) and row
// rotation (8), ds_swizzle in bitmask mode (4, 16: the exchange runs in the
// LDS unit's crossbar, which takes it off the VALU; with DPP, xor 4 needs two
// row rotations and a select), and the gfx950 permlane swap (32).
// Quad permutes and row rotations read a valid lane for every lane, so the
// DPP move needs no old value (one instruction, no zero to materialise).
// Every lane of the wave must be active (the sorts and reductions below are
// called by whole waves).
template <int M>
__device__ __forceinline__ uint32_t xor_lane(uint32_t x, uint32_t lane) {
    if constexpr (M == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
    } else if constexpr (M == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
    } else if constexpr (M == 4) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x101F);  // bitmask mode: xor 4
    } else if constexpr (M == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, true);  // row_ror:8
    } else if constexpr (M == 16) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x401F);  // bitmask mode: xor 16
    } else {
        static_assert(M == 32, "xor distance");
        const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        return (lane & 32u) ? (uint32_t)r[0] : (uint32_t)r[1];
    }
}

// Compare-exchange with lane ^ M: this lane keeps the smaller key iff
// keep_min.
template <int M>
__device__ __forceinline__ unsigned long long cx(unsigned long long v, uint32_t lane, bool keep_min) {
    const uint32_t lo = xor_lane<M>((uint32_t)v, lane);
    const uint32_t hi = xor_lane<M>((uint32_t)(v >> 32), lane);
    const unsigned long long o = ((unsigned long long)hi << 32) | lo;
    return ((o < v) == keep_min) ? o : v;
}

// One exchange step of the descending sort: blocks of SIZE lanes alternate
// direction so that each stage leaves bitonic blocks of twice the size.
template <int SIZE, int M>
__device__ __forceinline__ unsigned long long sort_step(unsigned long long v, uint32_t lane) {
    return cx<M>(v, lane, ((lane & (uint32_t)M) == 0u) == ((lane & (uint32_t)SIZE) != 0u));
}

// Bitonic sort of one key per lane, descending over lanes 0..63.
__device__ __forceinline__ unsigned long long sort64_desc(unsigned long long v, uint32_t lane) {
    v = sort_step<2, 1>(v, lane);
    v = sort_step<4, 2>(v, lane);
    v = sort_step<4, 1>(v, lane);
    v = sort_step<8, 4>(v, lane);
    v = sort_step<8, 2>(v, lane);
    v = sort_step<8, 1>(v, lane);
    v = sort_step<16, 8>(v, lane);
    v = sort_step<16, 4>(v, lane);
    v = sort_step<16, 2>(v, lane);
    v = sort_step<16, 1>(v, lane);
    v = sort_step<32, 16>(v, lane);
    v = sort_step<32, 8>(v, lane);
    v = sort_step<32, 4>(v, lane);
    v = sort_step<32, 2>(v, lane);
    v = sort_step<32, 1>(v, lane);
    v = sort_step<64, 32>(v, lane);
    v = sort_step<64, 16>(v, lane);
    v = sort_step<64, 8>(v, lane);
    v = sort_step<64, 4>(v, lane);
    v = sort_step<64, 2>(v, lane);
    v = sort_step<64, 1>(v, lane);
    return v;
}

// Bitonic sort of each 32-lane half (one key per lane), both halves
// descending: the stages of sort64_desc up to blocks of 16, then a final
// merge whose direction depends only on the exchange bit.
__device__ __forceinline__ unsigned long long sort32x2_desc(unsigned long long v, uint32_t lane) {
    v = sort_step<2, 1>(v, lane);
    v = sort_step<4, 2>(v, lane);
    v = sort_step<4, 1>(v, lane);
    v = sort_step<8, 4>(v, lane);
    v = sort_step<8, 2>(v, lane);
    v = sort_step<8, 1>(v, lane);
    v = sort_step<16, 8>(v, lane);
    v = sort_step<16, 4>(v, lane);
    v = sort_step<16, 2>(v, lane);
    v = sort_step<16, 1>(v, lane);
    v = sort_step<64, 16>(v, lane);
    v = sort_step<64, 8>(v, lane);
    v = sort_step<64, 4>(v, lane);
    v = sort_step<64, 2>(v, lane);
    v = sort_step<64, 1>(v, lane);
    return v;
}

template <int M>
__device__ __forceinline__ float xor_f32(float x, uint32_t lane) {
    return __uint_as_float(xor_lane<M>(__float_as_uint(x), lane));
}

// Wave-wide min / max, result in every lane (fminf/fmaxf skip NaN).
__device__ __forceinline__ float wave_min(float v, uint32_t lane) {
    v = fminf(v, xor_f32<1>(v, lane));
    v = fminf(v, xor_f32<2>(v, lane));
    v = fminf(v, xor_f32<4>(v, lane));
    v = fminf(v, xor_f32<8>(v, lane));
    v = fminf(v, xor_f32<16>(v, lane));
    return fminf(v, xor_f32<32>(v, lane));
}

__device__ __forceinline__ float wave_max(float v, uint32_t lane) {
    v = fmaxf(v, xor_f32<1>(v, lane));
    v = fmaxf(v, xor_f32<2>(v, lane));
    v = fmaxf(v, xor_f32<4>(v, lane));
    v = fmaxf(v, xor_f32<8>(v, lane));
    v = fmaxf(v, xor_f32<16>(v, lane));
    return fmaxf(v, xor_f32<32>(v, lane));
}

// Sort a bitonic sequence (one key per lane) ascending.
__device__ __forceinline__ unsigned long long merge64_asc(unsigned long long v, uint32_t lane) {
    v = cx<32>(v, lane, (lane & 32u) == 0u);
    v = cx<16>(v, lane, (lane & 16u) == 0u);
    v = cx<8>(v, lane, (lane & 8u) == 0u);
    v = cx<4>(v, lane, (lane & 4u) == 0u);
    v = cx<2>(v, lane, (lane & 2u) == 0u);
    v = cx<1>(v, lane, (lane & 1u) == 0u);
    return v;
}

// Sort a bitonic sequence in each 32-lane half ascending.
__device__ __forceinline__ unsigned long long merge32x2_asc(unsigned long long v, uint32_t lane) {
    v = cx<16>(v, lane, (lane & 16u) == 0u);
    v = cx<8>(v, lane, (lane & 8u) == 0u);
    v = cx<4>(v, lane, (lane & 4u) == 0u);
    v = cx<2>(v, lane, (lane & 2u) == 0u);
    v = cx<1>(v, lane, (lane & 1u) == 0u);
    return v;
}

// Orders this wave's LDS writes before its later LDS reads (no block barrier).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Value of ascending rank r (r < n) among the n <= 256 keys v[j] of elements
// j * 64 + lane < n (the rest are ignored). Radix select: the bits common to
// all keys are fixed first (a wave AND / OR), then MSD digits of up to 8 bits
// are counted in `hist` (this wave's 256 LDS words) from the highest
// differing bit down; once the chosen bin holds one key, that key is the
// answer. Whole wave, uniform arguments.
__device__ __forceinline__ unsigned long long wave_select(const unsigned long long (&v)[4], uint32_t n, uint32_t r,
                                                          uint32_t lane, uint32_t* hist) {
    unsigned long long a = ~0ull, o = 0ull;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if ((uint32_t)j * 64u + lane < n) {
            a &= v[j];
            o |= v[j];
        }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a &= (unsigned long long)__shfl_xor((long long)a, off, 64);
        o |= (unsigned long long)__shfl_xor((long long)o, off, 64);
    }
    if (a == o) return a;
    int top = 63 - __builtin_clzll(a ^ o);
    unsigned long long mask = top >= 63 ? 0ull : (~0ull << (top + 1));
    unsigned long long prefix = a & mask;
    while (true) {
        const int lo = top >= 7 ? top - 7 : 0;
        const uint32_t dm = (2u << (top - lo)) - 1u;
#pragma unroll
        for (int q = 0; q < 4; ++q) hist[(uint32_t)q * 64u + lane] = 0u;
        wave_lds_fence();
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if ((uint32_t)j * 64u + lane < n && (v[j] & mask) == prefix)
                atomicAdd(&hist[(uint32_t)(v[j] >> lo) & dm], 1u);
        wave_lds_fence();
        const uint32_t h0 = hist[4u * lane], h1 = hist[4u * lane + 1u], h2 = hist[4u * lane + 2u],
                       h3 = hist[4u * lane + 3u];
        const uint32_t s = h0 + h1 + h2 + h3;
        const uint32_t inc = wave_incl_scan(s);
        const uint32_t ex = inc - s;
        uint32_t acc = ex, b = 4u * lane, cnt = h0;
        if (r >= acc + h0) {
            acc += h0;
            ++b;
            cnt = h1;
            if (r >= acc + h1) {
                acc += h1;
                ++b;
                cnt = h2;
                if (r >= acc + h2) {
                    acc += h2;
                    ++b;
                    cnt = h3;
                }
            }
        }
        const int L = __ffsll((long long)__builtin_amdgcn_ballot_w64(ex <= r && r < inc)) - 1;
        b = (uint32_t)__builtin_amdgcn_readlane((int)b, L);
        acc = (uint32_t)__builtin_amdgcn_readlane((int)acc, L);
        cnt = (uint32_t)__builtin_amdgcn_readlane((int)cnt, L);
        wave_lds_fence();  // every lane has read hist before the next pass clears it
        r -= acc;
        prefix |= (unsigned long long)b << lo;
        mask |= (unsigned long long)dm << lo;
        if (lo == 0) return prefix;
        if (cnt == 1u) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const unsigned long long m =
                    __builtin_amdgcn_ballot_w64((uint32_t)j * 64u + lane < n && (v[j] & mask) == prefix);
                if (m) {
                    const int l = __ffsll((long long)m) - 1;
                    const uint32_t x = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v[j], l);
                    const uint32_t y = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v[j] >> 32), l);
                    return ((unsigned long long)y << 32) | x;
                }
            }
        }
        top = lo - 1;
    }
}

}  // namespace gdn
