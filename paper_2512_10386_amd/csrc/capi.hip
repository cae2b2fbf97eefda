// C ABI of the denoiser (include/gdn.h): parameter checks, workspace layout,
// the launch sequence of a frame or a batch of frames, graph capture of that
// sequence and the leaf-capacity / chunk-length autotuner.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gdn.h"
#include "kernels.hpp"
#include "scan.hpp"

// Events of one timed call: start, kNN start, kNN end, end.
constexpr int TIMING_RING = 256;
struct CallEvents {
    hipEvent_t ev[4];
};

struct gdn_ctx {
    int device = 0;
    int num_cus = 256;
    void* scratch = nullptr;  // this device's copy of the no-allocation scratch array
    std::string err;
    gdn::Plan last{};
    gdn::Params last_prm{};
    bool has_last = false;
    bool timing = false;
    std::vector<CallEvents> ring;
    int64_t timed_calls = 0;
};

namespace gdn {
size_t dump_bytes(uint32_t n, int k, int what);
int context_device(const gdn_ctx* ctx) { return ctx ? ctx->device : 0; }
}

// Scratch memory of gdn_denoise_noalloc: the workspace of one frame, in a
// fixed array that every GPU the library runs on holds (its own copy, at its
// own address) until the process ends. Host code never names the array
// itself in a kernel argument or copy: it uses the address
// hipGetSymbolAddress returns for the current device, kept per device.
static __device__ __align__(256) unsigned char scratch[GDN_NOALLOC_MAX_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on `device` (which must be current),
// looked up once per device.
hipError_t scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

constexpr int64_t MAX_POINTS = (1ll << 30) - 1;
static_assert(GDN_MAX_FRAMES == gdn::MAX_FRAMES, "frame limit of the ABI and the kernels");

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Carve the workspace into the batch's arrays (a plain call is one frame).
// With base == nullptr only the size is computed.
gdn::Plan make_plan(uint32_t n, uint32_t nf, int k, char* base) {
    using namespace gdn;
    Plan P{};
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? (void*)(base + off) : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    const size_t N = n;
    P.n = n;
    P.k = k;
    P.nf = nf;
    P.sort_passes = SORT_PASSES + (nf > 256u ? 2u : (nf > 1u ? 1u : 0u));
    P.sort_items = n > SORT_BIG_N ? 16u : 4u;
    P.tq = n > KNN_TQ_SMALL_MAX_N ? (uint32_t)KNN_TQ : (uint32_t)KNN_TQ_SMALL;
    const size_t sort_tile = (size_t)SORT_BLOCK * P.sort_items;
    P.sort_tiles = (uint32_t)((N + sort_tile - 1) / sort_tile);
    if (P.sort_tiles == 0) P.sort_tiles = 1;
    P.scan_tiles = scan_tiles_for(n);
    // capacities stay below 2^30 (the look-back scans carry 30-bit sums)
    P.items_max = (uint32_t)std::min<uint64_t>(2ull * n + 64u, (1ull << 30) - 64u);
    P.plist_max = (uint32_t)std::min<uint64_t>(3ull * n + 64u, (1ull << 30) - 64u);

    const size_t z0 = off;
    P.ctr = (Counters*)take(sizeof(Counters));  // first: status_word() reads the workspace start
    P.fstat = (FrameStat*)take(sizeof(FrameStat) * (size_t)nf);
    P.sort_hist = (uint32_t*)take(sizeof(uint32_t) * SORT_PASSES_MAX * 256);
    P.sort_status = (uint32_t*)take(sizeof(uint32_t) * (size_t)P.sort_passes * P.sort_tiles * 256);
    P.scan_status = (uint32_t*)take(sizeof(uint32_t) * SCAN_SLOTS * (size_t)P.scan_tiles);
    P.deepf = (uint8_t*)take(N);
    P.zero_begin = base ? base + z0 : nullptr;
    P.zero_bytes = off - z0;

    P.foff = (uint32_t*)take(4 * ((size_t)nf + 1));
    P.fc = (FrameConst*)take(sizeof(FrameConst) * (size_t)nf);
    P.bbox_part = (uint32_t*)take(32 * ((N + 1023) / 1024 + 1));
    if (nf > 1) {
        P.fid = (uint32_t*)take(4 * N);
        P.keep_ex = (uint32_t*)take(4 * (N + 1));
    }
    P.keys_a = (uint64_t*)take(8 * N);
    P.keys_b = (uint64_t*)take(8 * N);
    P.idx_a = (uint32_t*)take(4 * N);
    P.idx_b = (uint32_t*)take(4 * N);
    const bool odd = (P.sort_passes & 1u) != 0u;
    P.keys_src = odd ? P.keys_b : P.keys_a;
    P.idx_src = odd ? P.idx_b : P.idx_a;
    P.pos4 = (float4*)take(16 * N);
    P.leaf_of = (uint32_t*)take(4 * N);
    P.occ = (uint32_t*)take(4 * N);
    P.p1 = (uint8_t*)take(N);
    P.bflag = (uint8_t*)take(N);
    P.p1pos = (uint32_t*)take(4 * (N + 1));
    P.leaf_begin = (uint32_t*)take(4 * (N + 1));
    P.leaf_level = (uint32_t*)take(4 * N);
    P.leaf_prefix = (uint64_t*)take(8 * N);
    P.leaf_h = (float*)take(4 * N);
    P.leaf_nr = (uint32_t*)take(4 * N);
    P.leaf_ranges = (uint2*)take(sizeof(uint2) * HALO * N);
    P.leaf_own = (uint2*)take(sizeof(uint2) * N);
    P.leaf_ncand = (uint32_t*)take(4 * N);
    P.leaf_nch = (uint32_t*)take(4 * N);
    P.leaf_cc = (uint32_t*)take(4 * N);
    P.leaf_plist = (uint32_t*)take(4 * N);
    P.leaf_item = (uint32_t*)take(4 * N);
    P.leaf_rho_med = (double*)take(8 * N);
    P.leaf_r2cut = (float*)take(4 * N);
    P.leaf_m = (uint32_t*)take(4 * N);
    P.vox_keys = (uint64_t*)take(16 * N);
    P.vox_cnt = (uint32_t*)take(8 * N);
    P.cand4 = (float4*)take(16 * N);
    P.cand_leaf = (uint32_t*)take(4 * N);
    P.nbr = (uint32_t*)take(4 * N * k);
    P.inv_p1 = (uint32_t*)take(4 * N);
    P.nbr_d2 = (float*)take(4 * N * k);
    P.r2k = (float*)take(4 * N);
    P.krec = (uint4*)take(16 * N);
    P.outrec = (uint2*)take(8 * N);
    P.tau_c = (float*)take(4 * N);
    P.gbox = (GroupBox*)take(sizeof(GroupBox) * ((N + KNN_GRP - 1) / KNN_GRP));
    P.rho_c = (double*)take(8 * N);
    P.r64_c = (double*)take(8 * N);
    P.afac_c = (double2*)take(16 * N);
    P.p2 = (uint8_t*)take(N);
    P.stage_c = (uint8_t*)take(N);
    P.score_c = (double*)take(8 * N);
    P.gpow_p = (double*)take(sizeof(double) * N);
    P.items = (KnnItem*)take(sizeof(KnnItem) * (size_t)P.items_max);
    P.plist = (uint64_t*)take(8 * (size_t)P.plist_max * k);
    P.bytes = off;
    return P;
}

bool params_ok(const gdn_params* p, std::string* why) {
    auto bad = [&](const char* m) { *why = m; return false; };
    if (!p) return bad("params is NULL");
    if (p->k < 1 || p->k > 64) return bad("k must be in [1, 64]");
    if (p->leaf_cap < 1) return bad("leaf_cap must be >= 1");
    if (std::isnan(p->min_leaf_side)) return bad("min_leaf_side is NaN");
    if (!(p->beta > 0.0) || !std::isfinite(p->beta)) return bad("beta must be finite and > 0");
    if (p->min_vox_count < 1) return bad("min_vox_count must be >= 1");
    if (!(p->rho_percentile >= 0.0 && p->rho_percentile <= 100.0)) return bad("rho_percentile must be in [0, 100]");
    if (!(p->alpha >= 0.0) || !std::isfinite(p->alpha)) return bad("alpha must be finite and >= 0");
    if (!(p->sigma > 0.0) || !std::isfinite(p->sigma)) return bad("sigma must be finite and > 0");
    if (!(p->eps >= 0.0) || !std::isfinite(p->eps)) return bad("eps must be finite and >= 0");
    if (!(p->keep_ratio > 0.0 && p->keep_ratio <= 1.0)) return bad("keep_ratio must be in (0, 1]");
    if (p->knn_chunk < 0 || p->knn_chunk > (1 << 28)) return bad("knn_chunk must be in [0, 2^28]");
    if (!(p->gamma >= 0.0) || !std::isfinite(p->gamma)) return bad("gamma must be finite and >= 0");
    if (std::isinf(p->log_threshold)) return bad("log_threshold must be finite or NaN");
    if (p->stages < 0 || p->stages > GDN_STAGES_ALL) return bad("stages must be a subset of GDN_STAGES_ALL");
    return true;
}

gdn::Params to_params(const gdn_params* p) {
    gdn::Params q;
    q.k = p->k;
    q.leaf_cap = p->leaf_cap;
    q.min_leaf_side = p->min_leaf_side;
    q.beta = p->beta;
    q.min_vox_count = p->min_vox_count;
    q.rho_percentile = p->rho_percentile;
    q.alpha = p->alpha;
    q.sigma = p->sigma;
    q.eps = p->eps;
    q.keep_ratio = p->keep_ratio;
    q.knn_chunk = p->knn_chunk;
    q.gamma = p->gamma;
    q.log_thr = p->log_threshold;
    q.stages = p->stages;
    // A1 off: every voxel holds at least its own point, so n_v = 1 passes all.
    if (!(p->stages & GDN_STAGE_VOXEL)) q.min_vox_count = 1;
    // A2 off: with q = 0 the percentile rank is 1, the cut is the largest r^2,
    // and every point with k neighbours passes.
    if (!(p->stages & GDN_STAGE_DENSITY)) q.rho_percentile = 0.0;
    return q;
}

gdn_status fail(gdn_ctx* c, gdn_status s, const std::string& m) {
    if (c) c->err = m;
    return s;
}

// Make ctx->device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) changed = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" {

gdn_status gdn_default_params(gdn_params* out) {
    if (!out) return GDN_EINVAL;
    out->k = 12;
    out->leaf_cap = 512;
    out->min_leaf_side = 0.0;
    out->beta = 1.0;
    out->min_vox_count = 4;
    out->rho_percentile = 0.2;
    out->alpha = 1.0;
    out->sigma = 1.0;
    out->eps = 1e-12;
    out->keep_ratio = 0.98;
    out->knn_chunk = 0;
    out->gamma = 2.0;
    out->log_threshold = std::nan("");
    out->stages = GDN_STAGES_ALL;
    return GDN_OK;
}

gdn_status gdn_create(gdn_ctx** out, int device) {
    if (!out) return GDN_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return GDN_EINVAL;
    gdn_ctx* c = new (std::nothrow) gdn_ctx();
    if (!c) return GDN_EINTERNAL;
    c->device = device;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->num_cus = cus;
    {
        DeviceGuard guard(device);
        if (scratch_address(device, &c->scratch) != hipSuccess) {
            delete c;
            return GDN_EHIP;
        }
    }
    *out = c;
    return GDN_OK;
}

static void free_events(gdn_ctx* c) {
    for (auto& ce : c->ring)
        for (auto& e : ce.ev)
            if (e) (void)hipEventDestroy(e);
    c->ring.clear();
}

void gdn_destroy(gdn_ctx* ctx) {
    if (!ctx) return;
    DeviceGuard guard(ctx->device);
    free_events(ctx);
    delete ctx;
}

gdn_status gdn_set_timing(gdn_ctx* ctx, int enable) {
    if (!ctx) return GDN_EINVAL;
    DeviceGuard guard(ctx->device);
    if (!enable) {
        free_events(ctx);
        ctx->timing = false;
        return GDN_OK;
    }
    if (ctx->ring.empty()) {
        ctx->ring.resize(TIMING_RING);
        for (auto& ce : ctx->ring)
            for (auto& e : ce.ev)
                if (hipEventCreate(&e) != hipSuccess) {
                    free_events(ctx);
                    return fail(ctx, GDN_EHIP, "hipEventCreate failed");
                }
    }
    ctx->timing = true;
    ctx->timed_calls = 0;
    return GDN_OK;
}

gdn_status gdn_timing(gdn_ctx* ctx, int64_t back, float* total_ms, float* knn_ms) {
    if (!ctx || !total_ms || !knn_ms) return GDN_EINVAL;
    if (!ctx->timing) return fail(ctx, GDN_EINVAL, "timing is not enabled");
    if (back < 0 || back >= ctx->timed_calls || back >= TIMING_RING)
        return fail(ctx, GDN_EINVAL, "no such timed call");
    DeviceGuard guard(ctx->device);
    const CallEvents& ce = ctx->ring[(size_t)((ctx->timed_calls - 1 - back) % TIMING_RING)];
    if (hipEventSynchronize(ce.ev[3]) != hipSuccess) return fail(ctx, GDN_EHIP, "hipEventSynchronize failed");
    if (hipEventElapsedTime(total_ms, ce.ev[0], ce.ev[3]) != hipSuccess ||
        hipEventElapsedTime(knn_ms, ce.ev[1], ce.ev[2]) != hipSuccess)
        return fail(ctx, GDN_EHIP, "hipEventElapsedTime failed");
    return GDN_OK;
}

static gdn_status size_checks(gdn_ctx* ctx, const gdn_params* p, int64_t n, int64_t nf) {
    std::string why;
    if (!params_ok(p, &why)) return fail(ctx, GDN_EINVAL, why);
    if (n < 0) return fail(ctx, GDN_EINVAL, "n < 0");
    if (n > MAX_POINTS) return fail(ctx, GDN_ECAPACITY, "n exceeds 2^30-1 points");
    if (nf < 1) return fail(ctx, GDN_EINVAL, "a batch needs at least one frame");
    if (nf > (int64_t)gdn::MAX_FRAMES) return fail(ctx, GDN_ECAPACITY, "more than 4096 frames in one batch");
    return GDN_OK;
}

gdn_status gdn_workspace_size(gdn_ctx* ctx, const gdn_params* p, int64_t n, size_t* bytes) {
    return gdn_workspace_size_batch(ctx, p, n, 1, bytes);
}

gdn_status gdn_workspace_size_batch(gdn_ctx* ctx, const gdn_params* p, int64_t n, int64_t nf, size_t* bytes) {
    if (!bytes) return fail(ctx, GDN_EINVAL, "bytes is NULL");
    const gdn_status e = size_checks(ctx, p, n, nf);
    if (e != GDN_OK) return e;
    *bytes = n == 0 ? 0 : make_plan((uint32_t)n, (uint32_t)nf, p->k, nullptr).bytes;
    return GDN_OK;
}

// Enqueue the whole pipeline. frame_off == nullptr: one frame of n points.
static gdn_status run(gdn_ctx* ctx, const gdn_params* p, const float* xyz, int64_t n, const int64_t* frame_off,
                      int64_t nf, void* workspace, size_t workspace_bytes, uint8_t* keep, float* score,
                      uint8_t* stage, uint32_t* kept_idx, int64_t* n_kept, hipStream_t st, bool record) {
    gdn_status es = size_checks(ctx, p, n, nf);
    if (es != GDN_OK) return es;
    if (!n_kept) return fail(ctx, GDN_EINVAL, "n_kept is NULL");
    if (frame_off == nullptr && nf != 1) return fail(ctx, GDN_EINVAL, "frame_off is NULL");
    ctx->has_last = false;
    if (n == 0) {
        gdn::launch_write_zero_count(n_kept, (uint32_t)nf, st);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(ctx, GDN_EHIP, hipGetErrorString(e));
        ctx->err.clear();
        return GDN_OK;
    }
    if (!xyz || !keep || !score || !kept_idx) return fail(ctx, GDN_EINVAL, "NULL array argument");
    if (!workspace) return fail(ctx, GDN_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace & 255u) != 0) return fail(ctx, GDN_EINVAL, "workspace must be 256-byte aligned");
    const gdn::Plan P = make_plan((uint32_t)n, (uint32_t)nf, p->k, (char*)workspace);
    if (workspace_bytes < P.bytes) return fail(ctx, GDN_ENOMEM, "workspace too small");
    const gdn::Params prm = to_params(p);
    CallEvents* ce = nullptr;
    if (record && ctx->timing) {
        ce = &ctx->ring[(size_t)(ctx->timed_calls % TIMING_RING)];
        ++ctx->timed_calls;
        (void)hipEventRecord(ce->ev[0], st);
    }

    // a plain single-frame call clears the zeroed block inside the box kernel
    const bool clear_in_bbox = !frame_off && gdn::bbox_one_frame(P);
    if (!clear_in_bbox) gdn::launch_zero(P, st);
    if (frame_off) gdn::launch_frames(P, frame_off, st);
    gdn::launch_bbox(P, xyz, st, clear_in_bbox);
    gdn::launch_morton(P, prm, xyz, st);
    gdn::launch_sort(P, prm, st);
    gdn::launch_leaves(P, prm, xyz, st);
    gdn::launch_voxel(P, prm, st);
    gdn::launch_p1_compact(P, st);
    gdn::launch_halo(P, prm, st);
    gdn::launch_knn_plan(P, prm, st);
    gdn::launch_knn_bound(P, prm.k, ctx->num_cus, st);
    if (ce) (void)hipEventRecord(ce->ev[1], st);
    gdn::launch_knn(P, prm.k, ctx->num_cus, st);
    if (ce) (void)hipEventRecord(ce->ev[2], st);
    gdn::launch_knn_merge(P, prm.k, ctx->num_cus, st);
    gdn::launch_leaf_select(P, prm, xyz, st);
    bool written = false;  // outputs already written by the top-lambda pass
    if (prm.stages & GDN_STAGE_SCORE) {
        gdn::launch_score(P, prm, st);
        written = gdn::launch_topl(P, prm, keep, score, stage, st);
    } else {
        gdn::launch_keep_p2(P, st);
    }
    gdn::launch_outputs(P, keep, score, stage, kept_idx, n_kept, st, written);
    if (ce) (void)hipEventRecord(ce->ev[3], st);

    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, GDN_EHIP, hipGetErrorString(e));
    ctx->last = P;
    ctx->last_prm = prm;
    ctx->has_last = true;
    ctx->err.clear();
    return GDN_OK;
}

gdn_status gdn_denoise(gdn_ctx* ctx, const gdn_params* p, const float* xyz, int64_t n, void* workspace,
                       size_t workspace_bytes, uint8_t* keep, float* score, uint8_t* stage, uint32_t* kept_idx,
                       int64_t* n_kept, void* stream) {
    if (!ctx) return GDN_EINVAL;
    DeviceGuard guard(ctx->device);
    return run(ctx, p, xyz, n, nullptr, 1, workspace, workspace_bytes, keep, score, stage, kept_idx, n_kept,
               (hipStream_t)stream, true);
}

gdn_status gdn_denoise_noalloc(gdn_ctx* ctx, const gdn_params* p, const float* xyz, int64_t n, uint8_t* keep,
                               float* score, uint8_t* stage, uint32_t* kept_idx, int64_t* n_kept, void* stream) {
    if (!ctx) return GDN_EINVAL;
    size_t need = 0;
    const gdn_status e = gdn_workspace_size(ctx, p, n, &need);
    if (e != GDN_OK) return e;
    if (need > (size_t)GDN_NOALLOC_MAX_BYTES)
        return fail(ctx, GDN_ECAPACITY,
                    "frame needs " + std::to_string(need) + " bytes of scratch; gdn_denoise_noalloc holds " +
                        std::to_string((size_t)GDN_NOALLOC_MAX_BYTES) + " (use gdn_denoise with a workspace)");
    if (!ctx->scratch) return fail(ctx, GDN_EHIP, "no scratch address for this device");
    DeviceGuard guard(ctx->device);
    return run(ctx, p, xyz, n, nullptr, 1, ctx->scratch, (size_t)GDN_NOALLOC_MAX_BYTES, keep, score, stage,
               kept_idx, n_kept, (hipStream_t)stream, true);
}

gdn_status gdn_denoise_batch(gdn_ctx* ctx, const gdn_params* p, const float* xyz, int64_t n,
                             const int64_t* frame_off, int64_t nf, void* workspace, size_t workspace_bytes,
                             uint8_t* keep, float* score, uint8_t* stage, uint32_t* kept_idx, int64_t* n_kept,
                             void* stream) {
    if (!ctx) return GDN_EINVAL;
    if (!frame_off) return fail(ctx, GDN_EINVAL, "frame_off is NULL");
    DeviceGuard guard(ctx->device);
    return run(ctx, p, xyz, n, frame_off, nf, workspace, workspace_bytes, keep, score, stage, kept_idx, n_kept,
               (hipStream_t)stream, true);
}

// ---------------------------------------------------------------- graphs

struct gdn_graph {
    gdn_ctx* ctx = nullptr;
    hipGraphExec_t exec = nullptr;
    gdn::Plan plan{};
    gdn::Params prm{};
};

gdn_status gdn_graph_create(gdn_ctx* ctx, const gdn_params* p, const float* xyz, int64_t n,
                            const int64_t* frame_off, int64_t nf, void* workspace, size_t workspace_bytes,
                            uint8_t* keep, float* score, uint8_t* stage, uint32_t* kept_idx, int64_t* n_kept,
                            gdn_graph** out) {
    if (!ctx) return GDN_EINVAL;
    if (!out) return fail(ctx, GDN_EINVAL, "out is NULL");
    *out = nullptr;
    if (!frame_off) return fail(ctx, GDN_EINVAL, "frame_off is NULL");
    DeviceGuard guard(ctx->device);
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        return fail(ctx, GDN_EHIP, "hipStreamCreateWithFlags failed");
    gdn_status st = GDN_OK;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = fail(ctx, GDN_EHIP, "hipStreamBeginCapture failed");
    } else {
        st = run(ctx, p, xyz, n, frame_off, nf, workspace, workspace_bytes, keep, score, stage, kept_idx, n_kept,
                 cs, false);
        const hipError_t ec = hipStreamEndCapture(cs, &g);
        if (st == GDN_OK && ec != hipSuccess) st = fail(ctx, GDN_EHIP, "hipStreamEndCapture failed");
        if (st == GDN_OK && hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) != hipSuccess)
            st = fail(ctx, GDN_EHIP, "hipGraphInstantiate failed");
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (st != GDN_OK) {
        if (exec) (void)hipGraphExecDestroy(exec);
        ctx->has_last = false;
        return st;
    }
    gdn_graph* G = new (std::nothrow) gdn_graph();
    if (!G) {
        (void)hipGraphExecDestroy(exec);
        return fail(ctx, GDN_EINTERNAL, "out of host memory");
    }
    G->ctx = ctx;
    G->exec = exec;
    G->plan = ctx->last;
    G->prm = ctx->last_prm;
    ctx->has_last = false;  // nothing has run yet
    *out = G;
    return GDN_OK;
}

gdn_status gdn_graph_launch(gdn_graph* g, void* stream) {
    if (!g || !g->exec) return GDN_EINVAL;
    DeviceGuard guard(g->ctx->device);
    if (hipGraphLaunch(g->exec, (hipStream_t)stream) != hipSuccess)
        return fail(g->ctx, GDN_EHIP, "hipGraphLaunch failed");
    g->ctx->last = g->plan;
    g->ctx->last_prm = g->prm;
    g->ctx->has_last = true;
    return GDN_OK;
}

void gdn_graph_destroy(gdn_graph* g) {
    if (!g) return;
    DeviceGuard guard(g->ctx->device);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    delete g;
}

// ---------------------------------------------------------------- autotuner

gdn_status gdn_autotune(gdn_ctx* ctx, gdn_params* p, const int32_t* caps, int ncaps, const int32_t* chunks,
                        int nchunks, int reps, const float* xyz, int64_t n, const int64_t* frame_off, int64_t nf,
                        void* workspace, size_t workspace_bytes, uint8_t* keep, float* score, uint8_t* stage,
                        uint32_t* kept_idx, int64_t* n_kept, float* ms_out, void* stream) {
    if (!ctx) return GDN_EINVAL;
    if (!p || !caps || ncaps < 1 || reps < 1) return fail(ctx, GDN_EINVAL, "bad autotune arguments");
    if (!frame_off) return fail(ctx, GDN_EINVAL, "frame_off is NULL");
    const int32_t zero_chunk = 0;
    if (!chunks || nchunks < 1) {
        chunks = &zero_chunk;
        nchunks = 1;
    }
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(ctx, GDN_EHIP, "hipEventCreate failed");
    }
    gdn_params best = *p;
    float best_ms = INFINITY;
    gdn_status status = GDN_OK;
    std::vector<float> t((size_t)reps);
    for (int a = 0; a < ncaps && status == GDN_OK; ++a) {
        for (int b = 0; b < nchunks && status == GDN_OK; ++b) {
            gdn_params q = *p;
            q.leaf_cap = caps[a];
            q.knn_chunk = chunks[b];
            status = run(ctx, &q, xyz, n, frame_off, nf, workspace, workspace_bytes, keep, score, stage, kept_idx,
                         n_kept, st, false);  // warm-up
            for (int r = 0; r < reps && status == GDN_OK; ++r) {
                (void)hipEventRecord(e0, st);
                status = run(ctx, &q, xyz, n, frame_off, nf, workspace, workspace_bytes, keep, score, stage,
                             kept_idx, n_kept, st, false);
                (void)hipEventRecord(e1, st);
                if (status != GDN_OK) break;
                if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t[(size_t)r], e0, e1) != hipSuccess)
                    status = fail(ctx, GDN_EHIP, "event timing failed");
            }
            if (status != GDN_OK) break;
            std::vector<float> srt = t;
            std::sort(srt.begin(), srt.end());
            const float med = srt[srt.size() / 2];
            if (ms_out) ms_out[a * nchunks + b] = med;
            if (med < best_ms) {
                best_ms = med;
                best = q;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != GDN_OK) return status;
    *p = best;
    ctx->has_last = false;  // the workspace holds the last candidate's frame, not the chosen one
    return GDN_OK;
}

gdn_status gdn_debug_dump(gdn_ctx* ctx, int what, void* dst, size_t dst_bytes, void* stream) {
    if (!ctx) return GDN_EINVAL;
    if (!ctx->has_last) return fail(ctx, GDN_EINVAL, "no frame has been denoised on this context");
    if (!dst) return fail(ctx, GDN_EINVAL, "dst is NULL");
    DeviceGuard guard(ctx->device);
    if (gdn::launch_dump(ctx->last, what, dst, dst_bytes, (hipStream_t)stream) != 0)
        return fail(ctx, GDN_EINVAL, "unknown dump item or dst too small");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, GDN_EHIP, hipGetErrorString(e));
    return GDN_OK;
}

gdn_status gdn_fit_workspace_size(gdn_ctx* ctx, int64_t n, size_t* bytes) {
    if (!bytes) return fail(ctx, GDN_EINVAL, "bytes is NULL");
    if (n < 0) return fail(ctx, GDN_EINVAL, "n < 0");
    if (n > MAX_POINTS) return fail(ctx, GDN_ECAPACITY, "n exceeds 2^30-1 points");
    *bytes = gdn::fit_workspace_bytes((uint32_t)n);
    return GDN_OK;
}

gdn_status gdn_fit_loss_grad(gdn_ctx* ctx, const gdn_fit_params* fp, const float* xyz, const uint8_t* label,
                             int64_t n, void* workspace, size_t workspace_bytes, double* out, void* stream) {
    if (!ctx) return GDN_EINVAL;
    if (!fp || !xyz || !label || !workspace || !out) return fail(ctx, GDN_EINVAL, "NULL argument");
    if (!(fp->alpha >= 0.0) || !std::isfinite(fp->alpha)) return fail(ctx, GDN_EINVAL, "alpha must be finite and >= 0");
    if (!(fp->sigma > 0.0) || !std::isfinite(fp->sigma)) return fail(ctx, GDN_EINVAL, "sigma must be finite and > 0");
    if (!(fp->gamma >= 0.0) || !std::isfinite(fp->gamma)) return fail(ctx, GDN_EINVAL, "gamma must be finite and >= 0");
    if (!std::isfinite(fp->tau)) return fail(ctx, GDN_EINVAL, "tau must be finite");
    if (!(fp->temperature > 0.0) || !std::isfinite(fp->temperature))
        return fail(ctx, GDN_EINVAL, "temperature must be finite and > 0");
    if (!ctx->has_last) return fail(ctx, GDN_EINVAL, "no frame has been denoised on this context");
    if (n != (int64_t)ctx->last.n) return fail(ctx, GDN_EINVAL, "n differs from the last denoised frame or batch");
    if (((uintptr_t)workspace & 255u) != 0) return fail(ctx, GDN_EINVAL, "workspace must be 256-byte aligned");
    if (workspace_bytes < gdn::fit_workspace_bytes((uint32_t)n)) return fail(ctx, GDN_ENOMEM, "workspace too small");
    DeviceGuard guard(ctx->device);
    const gdn::FitArgs a{fp->alpha, fp->sigma, fp->gamma, fp->tau, fp->temperature, ctx->last_prm.eps};
    gdn::launch_fit(ctx->last, xyz, label, a, workspace, out, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, GDN_EHIP, hipGetErrorString(e));
    ctx->err.clear();
    return GDN_OK;
}

static gdn_status cloud_size(gdn_ctx* ctx, int64_t n, const char* what) {
    if (n < 1) return fail(ctx, GDN_EINVAL, std::string(what) + " is empty");
    if (n > MAX_POINTS) return fail(ctx, GDN_ECAPACITY, std::string(what) + " exceeds 2^30-1 points");
    return GDN_OK;
}

gdn_status gdn_nearest_workspace_size(gdn_ctx* ctx, int64_t na, size_t* bytes) {
    if (!bytes) return fail(ctx, GDN_EINVAL, "bytes is NULL");
    const gdn_status e = cloud_size(ctx, na, "the query cloud");
    if (e != GDN_OK) return e;
    *bytes = gdn::nearest_workspace_bytes((uint32_t)na);
    return GDN_OK;
}

gdn_status gdn_nearest(gdn_ctx* ctx, const float* a, int64_t na, const float* b, int64_t nb, void* workspace,
                       size_t workspace_bytes, uint32_t* idx, float* d2, void* stream) {
    if (!ctx) return GDN_EINVAL;
    gdn_status e = cloud_size(ctx, na, "the query cloud");
    if (e == GDN_OK) e = cloud_size(ctx, nb, "the reference cloud");
    if (e != GDN_OK) return e;
    if (!a || !b || !workspace || !idx || !d2) return fail(ctx, GDN_EINVAL, "NULL argument");
    if (((uintptr_t)workspace & 255u) != 0) return fail(ctx, GDN_EINVAL, "workspace must be 256-byte aligned");
    if (workspace_bytes < gdn::nearest_workspace_bytes((uint32_t)na))
        return fail(ctx, GDN_ENOMEM, "workspace too small");
    DeviceGuard guard(ctx->device);
    gdn::launch_nearest(a, (uint32_t)na, b, (uint32_t)nb, workspace, idx, d2, (hipStream_t)stream);
    hipError_t he = hipGetLastError();
    if (he != hipSuccess) return fail(ctx, GDN_EHIP, hipGetErrorString(he));
    ctx->err.clear();
    return GDN_OK;
}

gdn_status gdn_eval_workspace_size(gdn_ctx* ctx, int64_t nc, int64_t nd, size_t* bytes) {
    if (!bytes) return fail(ctx, GDN_EINVAL, "bytes is NULL");
    gdn_status e = cloud_size(ctx, nc, "the clean cloud");
    if (e == GDN_OK) e = cloud_size(ctx, nd, "the denoised cloud");
    if (e != GDN_OK) return e;
    *bytes = gdn::eval_workspace_bytes((uint32_t)nc, (uint32_t)nd);
    return GDN_OK;
}

gdn_status gdn_eval_metrics(gdn_ctx* ctx, const float* clean, int64_t nc, const float* den, int64_t nd,
                            void* workspace, size_t workspace_bytes, double* out, void* stream) {
    if (!ctx) return GDN_EINVAL;
    gdn_status e = cloud_size(ctx, nc, "the clean cloud");
    if (e == GDN_OK) e = cloud_size(ctx, nd, "the denoised cloud");
    if (e != GDN_OK) return e;
    if (!clean || !den || !workspace || !out) return fail(ctx, GDN_EINVAL, "NULL argument");
    if (((uintptr_t)workspace & 255u) != 0) return fail(ctx, GDN_EINVAL, "workspace must be 256-byte aligned");
    if (workspace_bytes < gdn::eval_workspace_bytes((uint32_t)nc, (uint32_t)nd))
        return fail(ctx, GDN_ENOMEM, "workspace too small");
    DeviceGuard guard(ctx->device);
    gdn::launch_eval(clean, (uint32_t)nc, den, (uint32_t)nd, workspace, out, (hipStream_t)stream);
    hipError_t he = hipGetLastError();
    if (he != hipSuccess) return fail(ctx, GDN_EHIP, hipGetErrorString(he));
    ctx->err.clear();
    return GDN_OK;
}

const char* gdn_status_string(gdn_status s) {
    switch (s) {
        case GDN_OK: return "ok";
        case GDN_EINVAL: return "invalid argument";
        case GDN_ENOMEM: return "workspace too small";
        case GDN_ECAPACITY: return "input too large";
        case GDN_EHIP: return "HIP runtime error";
        case GDN_EINTERNAL: return "internal error";
    }
    return "unknown status";
}

const char* gdn_last_error(gdn_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

#ifndef GDN_SOURCE_HASH
#define GDN_SOURCE_HASH "unknown"
#endif
const char* gdn_source_hash(void) { return GDN_SOURCE_HASH; }

}  // extern "C"
