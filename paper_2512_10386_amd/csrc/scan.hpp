// Single-pass exclusive scan with decoupled look-back.
//
// Every workgroup takes the next tile id from an atomic counter, so a tile
// only ever waits on tiles that were handed out earlier and are already
// resident; each wait is additionally bounded by SPIN_LIMIT (on expiry the
// device status word records DEV_WAIT_LIMIT and the scan carries on), so no
// launch can hang. The status words must be zero before the launch.
#pragma once

#include "common.hpp"

namespace gdn {

// get(i)          -> value of element i (uint32, sum must stay < 2^30)
// emit(i, ex, v)  -> called once per element with its exclusive prefix
// fin(total)      -> called once with the grand total
template <class Get, class Emit, class Fin>
__global__ __launch_bounds__(SCAN_BLOCK) void scan_kernel(Get get, Emit emit, Fin fin,
                                                          const uint32_t* n_dev, uint32_t n_host,
                                                          uint32_t* status, uint32_t* tile_ctr,
                                                          uint32_t* dev_status) {
    __shared__ uint32_t s_tile, s_excl;
    __shared__ uint32_t s_scan[SCAN_BLOCK / 64 + 1];
    const uint32_t n = n_dev ? *n_dev : n_host;
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tile >= ntiles) {
        if (n == 0 && tile == 0 && threadIdx.x == 0) fin(0u);
        return;
    }
    const uint32_t base = tile * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        uint32_t idx = base + i;
        v[i] = idx < n ? get(idx) : 0u;
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
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        uint32_t idx = base + i;
        if (idx < n) {
            emit(idx, run, v[i]);
            run += v[i];
        }
    }
    if (tile == ntiles - 1 && threadIdx.x == 0) fin(s_excl + agg);
}

template <class Get, class Emit, class Fin>
inline void launch_scan(Get get, Emit emit, Fin fin, const uint32_t* n_dev, uint32_t n_max,
                        uint32_t* status, uint32_t* tile_ctr, uint32_t* dev_status, hipStream_t st) {
    uint32_t tiles = (n_max + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles == 0) tiles = 1;
    scan_kernel<Get, Emit, Fin><<<dim3(tiles), dim3(SCAN_BLOCK), 0, st>>>(get, emit, fin, n_dev, n_max, status,
                                                                          tile_ctr, dev_status);
}

}  // namespace gdn
