// Single-pass exclusive scan with decoupled look-back.
//
// Workgroup b takes tiles b, b + G, b + 2G, ... (G workgroups). Each XCD
// starts its workgroups in index order, so a tile only waits on tiles of
// workgroups that have started and that wait only on lower tiles in turn;
// each wait is additionally bounded by SPIN_LIMIT (on expiry the device
// status word records DEV_WAIT_LIMIT and the scan carries on), so no launch
// can hang. (Tiles from an atomic counter cost a round trip before a tile's
// reads.) The status words must be zero before the launch.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace gdn {

// get(i)          -> value of element i (uint32, sum must stay < 2^30)
// emit(i, ex, v)  -> called once per element with its exclusive prefix
// fin(total)      -> called once with the grand total
// A tile's elements are read and emitted striped (element base + i*SCAN_BLOCK
// + thread: coalesced, and the get() calls of a thread are independent) and
// scanned blocked (ITEMS consecutive elements per thread), with an LDS
// transpose in between (padded one word per 32 against bank conflicts).
__device__ __forceinline__ uint32_t scan_lds_at(uint32_t e) { return e + (e >> 5); }

// True for a getter whose get() also stores outputs: its elements are read
// one by one (its stores keep its loads in order, so reading them all first
// gains nothing and costs registers).
template <class Get>
struct ScanGetWrites {
    static constexpr bool value = false;
};

// An emitter may split off its reads: with a member type Pre, pre(i) reads
// what emitting element i needs and operator()(i, ex, v, pre) writes, so
// the scan makes all of a thread's reads before any of its writes (which
// would otherwise keep the next element's reads waiting).
template <class Emit, class = void>
struct ScanEmitPre {
    static constexpr bool value = false;
};
template <class Emit>
struct ScanEmitPre<Emit, std::void_t<typename Emit::Pre>> {
    static constexpr bool value = true;
};

template <int ITEMS, class Get, class Emit, class Fin>
__global__ __launch_bounds__(SCAN_BLOCK) void scan_kernel(Get get, Emit emit, Fin fin,
                                                          const uint32_t* n_dev, uint32_t n_host,
                                                          uint32_t* status, uint32_t* dev_status) {
    __shared__ uint32_t s_excl;
    __shared__ uint32_t s_scan[SCAN_BLOCK / 64 + 1];
    constexpr uint32_t TILE = SCAN_BLOCK * ITEMS;
    __shared__ uint32_t s_val[TILE + TILE / 32];
    __shared__ uint32_t s_pre[TILE + TILE / 32];
    const uint32_t n = n_dev ? *n_dev : n_host;
    const uint32_t ntiles = (n + TILE - 1) / TILE;
    // The values are read into registers first and stored to LDS after, and
    // every read is made (past the end, of the last element, then dropped), so
    // a thread's reads, and the loads inside each get(), are in flight
    // together.
    constexpr bool writes = ScanGetWrites<Get>::value;
    auto read_tile = [&](uint32_t tbase, uint32_t* r) {
        if constexpr (writes) {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t idx = tbase + (uint32_t)i * SCAN_BLOCK + threadIdx.x;
                r[i] = idx < n ? get(idx) : 0u;
            }
            return;
        }
        if (n == 0u) {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) r[i] = 0u;
            return;
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t idx = tbase + (uint32_t)i * SCAN_BLOCK + threadIdx.x;
            const uint32_t v = get(idx < n ? idx : n - 1u);
            r[i] = idx < n ? v : 0u;
        }
    };
    uint32_t gv[ITEMS];
    for (uint32_t tile = blockIdx.x;; tile += gridDim.x) {
    if (tile >= ntiles) {
        if (n == 0 && tile == 0 && threadIdx.x == 0) fin(0u);
        return;
    }
    const uint32_t tbase = tile * TILE;
    read_tile(tbase, gv);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) s_val[scan_lds_at((uint32_t)i * SCAN_BLOCK + threadIdx.x)] = gv[i];
    __syncthreads();
    uint32_t v[ITEMS];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        v[i] = s_val[scan_lds_at(threadIdx.x * ITEMS + i)];
        sum += v[i];
    }
    uint32_t agg;
    const uint32_t ex = block_excl_scan(sum, s_scan, &agg);
    if (threadIdx.x < 64) {
        // first wave: look back over up to 64 predecessors per round trip
        // (lane l reads tile j - l); add the ready aggregates nearest first
        // up to and including an inclusive prefix, stop at one not ready
        const uint32_t lane = threadIdx.x;
        uint32_t* st = status + tile;
        if (tile == 0) {
            if (lane == 0) {
                st_relaxed_agent(st, LB_FLAG_PRE | agg);
                s_excl = 0;
            }
        } else {
            if (lane == 0) st_relaxed_agent(st, LB_FLAG_AGG | agg);
            uint32_t excl = 0, spins = 0;
            int j = (int)tile - 1;
            while (j >= 0) {
                const int jj = j - (int)lane;
                const uint32_t w = jj >= 0 ? ld_relaxed_agent(status + jj) : 0u;
                const unsigned long long nready = __builtin_amdgcn_ballot_w64(jj >= 0 && (w & ~LB_VALUE) == 0u);
                const unsigned long long pre = __builtin_amdgcn_ballot_w64(jj >= 0 && (w & LB_FLAG_PRE) != 0u);
                const unsigned long long stop = nready | pre;
                const uint32_t s = stop ? (uint32_t)__ffsll((long long)stop) - 1u : 64u;
                const bool done = s < 64u && ((pre >> s) & 1ull);
                const uint32_t take = (jj >= 0 && (lane < s || (done && lane == s))) ? (w & LB_VALUE) : 0u;
                excl += wave_sum(take);
                if (done) break;
                const uint32_t used = min(s, (uint32_t)(j + 1));
                j -= (int)used;
                if (used == 0u) {
                    if (++spins > SPIN_LIMIT) {
                        if (lane == 0) atomicOr(dev_status, DEV_WAIT_LIMIT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            if (lane == 0) {
                st_relaxed_agent(st, LB_FLAG_PRE | ((excl + agg) & LB_VALUE));
                s_excl = excl;
            }
        }
    }
    __syncthreads();
    uint32_t run = s_excl + ex;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        s_pre[scan_lds_at(threadIdx.x * ITEMS + i)] = run;
        run += v[i];
    }
    __syncthreads();
    if constexpr (ScanEmitPre<Emit>::value) {
        // (an element past n reads element n - 1 and is dropped)
        typename Emit::Pre pre[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t idx = tbase + (uint32_t)i * SCAN_BLOCK + threadIdx.x;
            pre[i] = emit.pre(idx < n ? idx : n - 1u);
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t e = (uint32_t)i * SCAN_BLOCK + threadIdx.x;
            const uint32_t idx = tbase + e;
            if (idx < n) emit(idx, s_pre[scan_lds_at(e)], s_val[scan_lds_at(e)], pre[i]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t e = (uint32_t)i * SCAN_BLOCK + threadIdx.x;
            const uint32_t idx = tbase + e;
            if (idx < n) emit(idx, s_pre[scan_lds_at(e)], s_val[scan_lds_at(e)]);
        }
    }
    if (tile == ntiles - 1 && threadIdx.x == 0) fin(s_excl + agg);
    __syncthreads();  // s_excl and the LDS tile are reused by the next tile
    }
}

// Items per thread for a scan over at most n_max elements: small scans use
// small tiles (more of them in flight), large ones full 16-item tiles. The
// status words must hold scan_tiles_for(n_max) entries.
inline uint32_t scan_items_for(uint32_t n_max) { return n_max <= SCAN_SMALL_N ? 4u : (uint32_t)SCAN_ITEMS; }
inline uint32_t scan_tiles_for(uint32_t n_max) {
    const uint32_t tile = SCAN_BLOCK * scan_items_for(n_max);
    const uint32_t t = (n_max + tile - 1) / tile;
    return t ? t : 1u;
}

// max_blocks > 0 caps the grid (workgroups then take several tiles): for
// scans whose device count is usually far below the host bound n_max.
template <class Get, class Emit, class Fin>
inline void launch_scan(Get get, Emit emit, Fin fin, const uint32_t* n_dev, uint32_t n_max,
                        uint32_t* status, uint32_t* dev_status, hipStream_t st,
                        uint32_t max_blocks = 0) {
    uint32_t tiles = scan_tiles_for(n_max);
    if (max_blocks > 0 && tiles > max_blocks) tiles = max_blocks;
    if (scan_items_for(n_max) == 4u)
        scan_kernel<4, Get, Emit, Fin><<<dim3(tiles), dim3(SCAN_BLOCK), 0, st>>>(get, emit, fin, n_dev, n_max,
                                                                                 status, dev_status);
    else
        scan_kernel<SCAN_ITEMS, Get, Emit, Fin><<<dim3(tiles), dim3(SCAN_BLOCK), 0, st>>>(
            get, emit, fin, n_dev, n_max, status, dev_status);
}

}  // namespace gdn
