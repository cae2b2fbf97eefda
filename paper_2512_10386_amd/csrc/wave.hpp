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

// Bitonic networks over the 64 lanes, one key per lane (32- or 64-bit).
//
// Every exchange keeps the smaller key in the lane whose M bit is clear, so
// the lane pattern it needs depends on M alone: six masks for all networks
// (left to the compiler, a pattern per (block size, M) pair fills the scalar
// registers and spills them). The direction of a block of the sort phase
// that merges blocks of 2^p lanes is folded into the keys instead: during
// that phase the lanes whose bit p is set, which sort descending, hold the
// complements of their keys (one XOR per phase).
template <int M>
__device__ __forceinline__ uint32_t xor_lane_key(uint32_t v, uint32_t lane) {
    return xor_lane<M>(v, lane);
}
template <int M>
__device__ __forceinline__ unsigned long long xor_lane_key(unsigned long long v, uint32_t lane) {
    const uint32_t lo = xor_lane<M>((uint32_t)v, lane);
    const uint32_t hi = xor_lane<M>((uint32_t)(v >> 32), lane);
    return ((unsigned long long)hi << 32) | lo;
}

// Compare-exchange with lane ^ M: the lane with the M bit clear keeps the
// smaller key.
template <int M, class K>
__device__ __forceinline__ K cx(K v, uint32_t lane) {
    const K o = xor_lane_key<M>(v, lane);
    return ((o < v) == ((lane & (uint32_t)M) == 0u)) ? o : v;
}

// All-ones where bit b of x is set.
template <class K>
__device__ __forceinline__ K bit_mask(uint32_t x, int b) {
    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)x, b, 1);
    if constexpr (sizeof(K) == 8) return ((unsigned long long)m << 32) | m;
    else return m;
}

// The steps of one merge phase: exchanges at lane distance 2^(P-1) .. 1.
template <int P, class K>
__device__ __forceinline__ K merge_steps(K w, uint32_t lane) {
    if constexpr (P >= 6) w = cx<32>(w, lane);
    if constexpr (P >= 5) w = cx<16>(w, lane);
    if constexpr (P >= 4) w = cx<8>(w, lane);
    if constexpr (P >= 3) w = cx<4>(w, lane);
    if constexpr (P >= 2) w = cx<2>(w, lane);
    return cx<1>(w, lane);
}

// Sort each block of 2^P lanes (P = 6: the wave), ascending or descending.
template <int P, bool ASC, class K>
__device__ __forceinline__ K bitonic_sort(K v, uint32_t lane) {
    // bit b of g: lane bits b and b + 1 differ (a phase boundary flips the
    // lanes whose direction changes)
    const uint32_t g = lane ^ (lane >> 1);
    K w = v ^ bit_mask<K>(lane, 1);
    w = merge_steps<1>(w, lane);
    if constexpr (P > 2) { w ^= bit_mask<K>(g, 1); w = merge_steps<2>(w, lane); }
    if constexpr (P > 3) { w ^= bit_mask<K>(g, 2); w = merge_steps<3>(w, lane); }
    if constexpr (P > 4) { w ^= bit_mask<K>(g, 3); w = merge_steps<4>(w, lane); }
    if constexpr (P > 5) { w ^= bit_mask<K>(g, 4); w = merge_steps<5>(w, lane); }
    // the last phase: every lane in the final direction
    w ^= bit_mask<K>(lane, P - 1);
    if constexpr (!ASC) w = ~w;
    w = merge_steps<P>(w, lane);
    return ASC ? w : ~w;
}

// Bitonic sort of one 64-bit key per lane, descending over lanes 0..63.
__device__ __forceinline__ unsigned long long sort64_desc(unsigned long long v, uint32_t lane) {
    return bitonic_sort<6, false>(v, lane);
}

// Each 32-lane half sorted descending.
__device__ __forceinline__ unsigned long long sort32x2_desc(unsigned long long v, uint32_t lane) {
    return bitonic_sort<5, false>(v, lane);
}

// The same sort with each exchange's direction taken from a lane pattern
// per (block size, M) pair: no XOR per phase, but 21 patterns held in scalar
// registers. Measured faster in the density select kernel; the kNN and
// top-lambda kernels use sort64_desc.
template <int SIZE, int M>
__device__ __forceinline__ unsigned long long cx_dir(unsigned long long v, uint32_t lane) {
    const unsigned long long o = xor_lane_key<M>(v, lane);
    const bool keep_min = ((lane & (uint32_t)M) == 0u) == ((lane & (uint32_t)SIZE) != 0u);
    return ((o < v) == keep_min) ? o : v;
}

__device__ __forceinline__ unsigned long long sort64_desc_dir(unsigned long long v, uint32_t lane) {
    v = cx_dir<2, 1>(v, lane);
    v = cx_dir<4, 2>(v, lane);
    v = cx_dir<4, 1>(v, lane);
    v = cx_dir<8, 4>(v, lane);
    v = cx_dir<8, 2>(v, lane);
    v = cx_dir<8, 1>(v, lane);
    v = cx_dir<16, 8>(v, lane);
    v = cx_dir<16, 4>(v, lane);
    v = cx_dir<16, 2>(v, lane);
    v = cx_dir<16, 1>(v, lane);
    v = cx_dir<32, 16>(v, lane);
    v = cx_dir<32, 8>(v, lane);
    v = cx_dir<32, 4>(v, lane);
    v = cx_dir<32, 2>(v, lane);
    v = cx_dir<32, 1>(v, lane);
    v = cx_dir<64, 32>(v, lane);
    v = cx_dir<64, 16>(v, lane);
    v = cx_dir<64, 8>(v, lane);
    v = cx_dir<64, 4>(v, lane);
    v = cx_dir<64, 2>(v, lane);
    v = cx_dir<64, 1>(v, lane);
    return v;
}

// 32-bit keys, ascending or descending over lanes 0..63.
template <bool ASC>
__device__ __forceinline__ uint32_t sort64_u32(uint32_t v, uint32_t lane) {
    return bitonic_sort<6, ASC>(v, lane);
}

// Sort a bitonic sequence (one key per lane) ascending.
__device__ __forceinline__ unsigned long long merge64_asc(unsigned long long v, uint32_t lane) {
    return merge_steps<6>(v, lane);
}

// Sort a bitonic sequence in each 32-lane half ascending.
__device__ __forceinline__ unsigned long long merge32x2_asc(unsigned long long v, uint32_t lane) {
    return merge_steps<5>(v, lane);
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
