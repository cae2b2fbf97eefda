// Shared device helpers and the workspace plan of the gfx950 denoiser.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gdn {

constexpr int MORTON_BITS = 21;
constexpr uint32_t QMAX = (1u << MORTON_BITS) - 1u;

// Tile sizes.
constexpr int SORT_BLOCK = 256;               // radix-sort workgroup
constexpr uint32_t SORT_BIG_N = 1u << 20;     // above: 16 keys per thread, else 4
constexpr int SORT_PASSES = 8;                // 8-bit digits over the 63-bit key
constexpr int SORT_FRAME_PASSES_MAX = 2;      // 8-bit digits of the frame id (batches)
constexpr int SORT_PASSES_MAX = SORT_PASSES + SORT_FRAME_PASSES_MAX;
constexpr uint32_t SORT_FOFF_LDS = 2048;      // frame offsets staged in LDS by frame passes (nf < this)
// Short sort: the radix passes cover only digits 4..7 (key bits 32..62),
// which hold every level-10 cell prefix (bits 33..62); the points end in
// (frame, bits 32..62, original index) order. A level-10 cell that holds
// more than leaf_cap points (and lies above the depth limit) splits further:
// such "deep" cells are found after the sort and each is sorted on its whole
// key by one workgroup, so the octree sees full key order wherever it goes
// below level 10.
constexpr int SORT_SHORT_LEVEL = 10;
constexpr int SORT_SHORT_FIRST = 4;
static_assert(3 * (MORTON_BITS - SORT_SHORT_LEVEL) >= 8 * SORT_SHORT_FIRST, "short sort must hold the cell prefix");
static_assert(SORT_SHORT_FIRST % 2 == 0, "skipped passes keep the ping-pong parity");
constexpr uint32_t MAX_FRAMES = 4096;         // frames per batched call (frame table staged in LDS)
constexpr int SCAN_BLOCK = 512;                // look-back scan workgroup (fewer tiles to look back over than 256)
constexpr int SCAN_ITEMS = 16;
constexpr uint32_t SCAN_SMALL_N = 1u << 20;   // scans up to this size: 4 items per thread
constexpr int SCAN_SLOTS = 6;                 // scans per call: leaves, P1, keep, 3 kNN plan scans
constexpr int PLAN_LEVELS = 8;                // candidate chunk lengths chunk0 << 0..7 (parallel plan)
constexpr int KNN_TQ = 16;                    // queries per kNN work item (one wave), at most
constexpr int KNN_TQ_SMALL = 8;               // ... for inputs of up to 2^20 points (shorter items, shorter tail)
constexpr uint32_t KNN_TQ_SMALL_MAX_N = 1u << 20;
constexpr int KNN_CC0 = 32768;                // default initial candidate chunk
constexpr int KNN_NCH_MAX = 32;               // max candidate chunks per leaf
constexpr int KNN_GRP = 64;                   // P1 positions per culling group of the kNN (one per lane)
constexpr uint32_t KNN_STREAMS = 8;           // kNN work-queue streams (cursors)
constexpr int HALO = 27;
constexpr int VOX_BLOCK = 256;
constexpr int VOX_LDS_SLOTS = 4096;           // LDS hash slots (leaves <= 2048 pts)
constexpr int SEL_BLOCK = 256;

// Status word packing for decoupled look-back: 2 flag bits + 30 value bits.
constexpr uint32_t LB_FLAG_AGG = 1u << 30;
constexpr uint32_t LB_FLAG_PRE = 2u << 30;
constexpr uint32_t LB_VALUE = (1u << 30) - 1u;
constexpr uint32_t SPIN_LIMIT = 1u << 22;

constexpr uint32_t DEV_NONFINITE = 1u;
constexpr uint32_t DEV_WAIT_LIMIT = 2u;
constexpr uint32_t DEV_BAD_FRAMES = 4u;

// Per-frame bounding-box accumulators (inside the zeroed block).
struct FrameStat {
    uint32_t bbox_max[3];   // ordered-uint max of x, y, z
    uint32_t bbox_nmin[3];  // ordered-uint max of ~x (i.e. the min)
    uint32_t nonfinite;
    uint32_t pad;
};

// Scalars the kernels share through device memory (inside the zeroed block).
struct Counters {
    uint32_t status;
    uint32_t n_leaves;
    uint32_t n_p1;
    uint32_t n_items;
    uint32_t n_kept;
    unsigned long long pairs;
    uint32_t n_chunked_items; // kNN items of chunked leaves (they come first)
    uint32_t plan_cc;         // chosen kNN chunk length (parallel plan)
    uint32_t pad[2];
    unsigned long long plan_acc[PLAN_LEVELS][3];  // per candidate chunk length: lists, items, chunked items
    unsigned long long plan_pairs;
    // kNN work queue: item i belongs to stream i % KNN_STREAMS; one cursor
    // per stream, each on its own 128-byte line
    uint32_t knn_q[KNN_STREAMS][32];
};

// Frame constants derived on the device from the bounding box.
struct FrameConst {
    float lo[3];
    int32_t dmax;
    double S;
    double scale;
};

// Bounding box of the P1 points at positions [KNN_GRP g, KNN_GRP (g + 1)).
struct GroupBox {
    float4 lo, hi;  // w unused
};

// One kNN work item: queries [q0, q1) of leaf `leaf` against candidate chunk
// `chunk`; `grp` indexes the arrival counter shared by the chunks of a tile.
struct KnnItem {
    uint32_t leaf, q0, q1, chunk, grp, pad;
};

// Method parameters as the kernels use them.
struct Params {
    int32_t k;
    int32_t leaf_cap;
    double min_leaf_side;
    double beta;
    int32_t min_vox_count;
    double rho_percentile;
    double alpha;
    double sigma;
    double eps;
    double keep_ratio;
    int32_t knn_chunk;        // initial kNN candidate chunk length (performance only)
    double gamma;             // kernel exponent: (d^2 + eps)^(-gamma/2); 2 = Eq. 20
    double log_thr;           // NaN: top-lambda; else keep P2 points with ln F >= log_thr
    int32_t stages;           // enabled modules: 1 voxel filter, 2 density filter, 4 score
};

// Parameters of the score fit (loss and gradient of a relaxed ln F threshold).
struct FitArgs {
    double alpha, sigma, gamma, tau, T, eps;
};

// Pointers into the caller's workspace for a batch of nf frames, n points in
// all (a plain call is the batch of one frame). Frames are contiguous runs of
// the input; after the sort (frame id most significant) frame f occupies the
// same positions [foff[f], foff[f+1]) in sorted order.
struct Plan {
    uint32_t n;
    int k;
    uint32_t nf;
    uint32_t sort_passes;     // SORT_PASSES + frame-id passes
    size_t bytes;
    // zero-initialised block
    char* zero_begin;
    size_t zero_bytes;
    Counters* ctr;
    FrameStat* fstat;         // [nf]
    uint32_t* sort_hist;      // [SORT_PASSES_MAX][256]
    uint32_t* sort_status;    // [SORT_PASSES_MAX][sort_tiles][256]
    uint32_t* scan_status;    // [SCAN_SLOTS][scan_tiles]
    uint32_t sort_tiles, scan_tiles;
    uint32_t sort_items;      // keys per thread of the radix passes (4 or 16)
    uint32_t tq;              // queries per kNN work item (KNN_TQ_SMALL or KNN_TQ)
    uint8_t* deepf;           // [n] 1 at sorted positions inside deep level-10 cells; between the two
                              // deep-cell kernels, 2 marks the start of a cell to re-sort (zeroed block)
    // frames
    uint32_t* foff;           // [nf+1] frame offsets (checked copy of the caller's)
    uint32_t* fid;            // [n] frame of each point (original order; nf > 1 only)
    uint32_t* bbox_part;      // [ceil(n / 1024)][8] per-chunk box (chunks inside one frame)
    FrameConst* fc;           // [nf]
    uint32_t* keep_ex;        // [n+1] exclusive count of kept points (original order; nf > 1)
    // sort (sorted order = s)
    uint64_t* keys_a;         // sorted keys end here
    uint64_t* keys_b;
    uint32_t* idx_a;          // sorted original indices end here
    uint32_t* idx_b;
    uint64_t* keys_src;       // where the keys are written before the sort (a or b by pass parity)
    uint32_t* idx_src;
    float4* pos4;             // [n] sorted x, y, z, original index bits
    uint32_t* leaf_of;        // [n] sorted
    uint32_t* occ;            // [n] sorted
    uint8_t* p1;              // [n] sorted
    uint8_t* bflag;           // [n] sorted: a leaf starts here
    uint32_t* p1pos;          // [n+1] exclusive scan of p1
    // leaves (at most n)
    uint32_t* leaf_begin;     // [n+1]
    uint32_t* leaf_level;     // [n]
    uint64_t* leaf_prefix;    // [n]
    float* leaf_h;            // [n]
    uint32_t* leaf_nr;        // [n] number of candidate ranges
    uint2* leaf_ranges;       // [n][HALO] compacted candidate ranges
    uint2* leaf_own;          // [n] the candidate range holding the leaf's own P1 points
    uint32_t* leaf_ncand;     // [n]
    uint32_t* leaf_nch;       // [n] candidate chunks
    uint32_t* leaf_cc;        // [n] chunk length
    uint32_t* leaf_plist;     // [n] first partial list of the leaf
    uint32_t* leaf_item;      // [n] queue index of the leaf's first kNN item
    double* leaf_rho_med;     // [n]
    float* leaf_r2cut;        // [n]
    uint32_t* leaf_m;         // [n]
    uint64_t* vox_keys;       // [2n] global hash fallback
    uint32_t* vox_cnt;        // [2n]
    // compacted P1 (query/candidate index q)
    float4* cand4;            // [n]
    uint32_t* cand_leaf;      // [n]
    uint32_t* nbr;            // [n][k] P1 positions of the neighbours (sorted by d2, then original index)
    uint32_t* inv_p1;         // [n] by original index: the P1 position of a P1 point
    float* nbr_d2;            // [n][k]
    float* r2k;               // [n] (written by the density kernel from krec)
    uint4* krec;              // [n] k-th neighbour's P1 position (none: 0xFFFFFFFF), fp32 bits of the (k-1)-th and k-th d2
    uint2* outrec;            // [n] by original index: fp32 score bits, stage (large inputs' outputs)
    float* tau_c;             // [n] per-query upper bound of r^2_K (-1: none)
    GroupBox* gbox;           // [ceil(n / KNN_GRP)] boxes of aligned groups of the P1 order
    double* rho_c;            // [n]
    double* r64_c;            // [n]
    double2* afac_c;          // [n] (rho_i / (rho_med^2 + eps))^(alpha/2), 1 / (2 (sigma r_K,i)^2)
    uint8_t* p2;              // [n]
    uint8_t* stage_c;         // [n] 1 density-removed, 2 score-removed, 3 kept
    double* score_c;          // [n]
    double* gpow_p;           // [n] P1 order: rho^(alpha/2)
    // kNN work
    KnnItem* items;           // [items_max]
    uint32_t items_max;
    uint64_t* plist;          // [plist_max][k] partial top-k keys
    uint32_t plist_max;
};

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint32_t f32_ordered(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float f32_from_ordered(uint32_t o) {
    uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
    return __uint_as_float(u);
}

// Look-back status words carry their whole payload (flag + count), so relaxed
// device-scope atomics suffice: no other data is published through them.
constexpr int LB_WINDOW = 4;                  // predecessors fetched per look-back round trip

__device__ __forceinline__ uint32_t ld_relaxed_agent(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed_agent(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-level inclusive scan (wave64).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block exclusive scan of one value per thread (blockDim multiple of 64, <= 1024).
// `smem` needs blockDim/64 + 1 words. Returns the exclusive prefix; *total gets
// the block sum. Contains __syncthreads.
// Workgroups are dealt to the chip's eight XCDs in turn (workgroup b runs on
// XCD b % 8). xcd_part gives the workgroups of one XCD one contiguous eighth
// of [0, n) to stride through: a kernel over sorted positions that gathers
// from, or scatters to, input order then touches only the lines of its own
// part's few frames, which stay in its XCD's L2 instead of being fetched by
// all eight. The grid must hold a whole number of workgroups per XCD
// (xcd_grid).
constexpr unsigned N_XCD = 8;
struct XcdPart {
    uint32_t first, end, step;
};
__device__ __forceinline__ XcdPart xcd_part(uint32_t n) {
    const uint32_t per = (n + N_XCD - 1u) / N_XCD;
    const uint32_t lo = min(n, (blockIdx.x % N_XCD) * per);
    return XcdPart{lo + (blockIdx.x / N_XCD) * blockDim.x + threadIdx.x, min(n, lo + per),
                   (gridDim.x / N_XCD) * blockDim.x};
}
inline unsigned xcd_grid(unsigned blocks) { return (blocks + N_XCD - 1u) / N_XCD * N_XCD; }

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* smem, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) smem[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < nw; ++w) { uint32_t t = smem[w]; smem[w] = run; run += t; }
        smem[nw] = run;
    }
    __syncthreads();
    uint32_t ex = smem[wave] + inc - v;
    *total = smem[nw];
    __syncthreads();
    return ex;
}

// 3D bit interleave (x in the lowest bit), magic-number spreading.
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x1F00000000FFFFull;
    x = (x | (x << 16)) & 0x1F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}
__device__ __forceinline__ uint32_t compact3(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10C30C30C30C30C3ull;
    x = (x ^ (x >> 4)) & 0x100F00F00F00F00Full;
    x = (x ^ (x >> 8)) & 0x1F0000FF0000FFull;
    x = (x ^ (x >> 16)) & 0x1F00000000FFFFull;
    x = (x ^ (x >> 32)) & 0x1FFFFFull;
    return (uint32_t)x;
}
__device__ __forceinline__ uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// Frame holding position j of a batch: frames are contiguous runs both of
// the input and of the sorted order (the frame id is the most significant
// sort digit), so the frame is the last f with foff[f] <= j (empty frames
// share their end with the next start). foff is tiny and stays in cache.
__device__ __forceinline__ uint32_t frame_of(const uint32_t* foff, uint32_t nf, uint32_t j) {
    uint32_t lo = 0, hi = nf;
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (foff[mid] <= j) lo = mid;
        else hi = mid;
    }
    return lo;
}

}  // namespace gdn
