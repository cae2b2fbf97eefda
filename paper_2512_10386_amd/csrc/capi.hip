// C ABI of the denoiser (include/gdn.h): parameter checks, workspace layout
// and the launch sequence of one frame.
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "gdn.h"
#include "kernels.hpp"

// Events of one timed call: start, kNN start, kNN end, end.
constexpr int TIMING_RING = 256;
struct CallEvents {
    hipEvent_t ev[4];
};

struct gdn_ctx {
    int device = 0;
    int num_cus = 256;
    std::string err;
    gdn::Plan last{};
    bool has_last = false;
    bool timing = false;
    std::vector<CallEvents> ring;
    int64_t timed_calls = 0;
};

namespace gdn {
size_t dump_bytes(uint32_t n, int k, int what);
}

namespace {

constexpr int64_t MAX_POINTS = (1ll << 30) - 1;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Carve the workspace into the frame's arrays. With base == nullptr only the
// size is computed.
gdn::Plan make_plan(uint32_t n, int k, char* base) {
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
    P.sort_tiles = (uint32_t)((N + SORT_TILE - 1) / SORT_TILE);
    if (P.sort_tiles == 0) P.sort_tiles = 1;
    P.scan_tiles = (uint32_t)((N + SCAN_TILE - 1) / SCAN_TILE);
    if (P.scan_tiles == 0) P.scan_tiles = 1;
    P.items_max = 2u * n + 64u;
    P.plist_max = 3u * n + 64u;

    const size_t z0 = off;
    P.ctr = (Counters*)take(sizeof(Counters));
    P.sort_hist = (uint32_t*)take(sizeof(uint32_t) * SORT_PASSES * 256);
    P.sort_status = (uint32_t*)take(sizeof(uint32_t) * (size_t)SORT_PASSES * P.sort_tiles * 256);
    P.scan_status = (uint32_t*)take(sizeof(uint32_t) * 4 * (size_t)P.scan_tiles);
    P.zero_begin = base ? base + z0 : nullptr;
    P.zero_bytes = off - z0;

    P.fc = (FrameConst*)take(sizeof(FrameConst));
    P.keys_a = (uint64_t*)take(8 * N);
    P.keys_b = (uint64_t*)take(8 * N);
    P.idx_a = (uint32_t*)take(4 * N);
    P.idx_b = (uint32_t*)take(4 * N);
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
    P.nbr_d2 = (float*)take(4 * N * k);
    P.r2k = (float*)take(4 * N);
    P.tau_c = (float*)take(4 * N);
    P.rho_c = (double*)take(8 * N);
    P.r64_c = (double*)take(8 * N);
    P.afac_c = (double*)take(8 * N);
    P.p2 = (uint8_t*)take(N);
    P.stage_c = (uint8_t*)take(N);
    P.score_c = (double*)take(8 * N);
    P.gpow_o = (double*)take(8 * N);
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

gdn_status gdn_workspace_size(gdn_ctx* ctx, const gdn_params* p, int64_t n, size_t* bytes) {
    std::string why;
    if (!bytes) return fail(ctx, GDN_EINVAL, "bytes is NULL");
    if (!params_ok(p, &why)) return fail(ctx, GDN_EINVAL, why);
    if (n < 0) return fail(ctx, GDN_EINVAL, "n < 0");
    if (n > MAX_POINTS) return fail(ctx, GDN_ECAPACITY, "n exceeds 2^30-1 points");
    *bytes = n == 0 ? 0 : make_plan((uint32_t)n, p->k, nullptr).bytes;
    return GDN_OK;
}

gdn_status gdn_denoise(gdn_ctx* ctx, const gdn_params* p, const float* xyz, int64_t n, void* workspace,
                       size_t workspace_bytes, uint8_t* keep, float* score, uint8_t* stage, uint32_t* kept_idx,
                       int64_t* n_kept, void* stream) {
    if (!ctx) return GDN_EINVAL;
    std::string why;
    if (!params_ok(p, &why)) return fail(ctx, GDN_EINVAL, why);
    if (n < 0) return fail(ctx, GDN_EINVAL, "n < 0");
    if (n > MAX_POINTS) return fail(ctx, GDN_ECAPACITY, "n exceeds 2^30-1 points");
    if (!n_kept) return fail(ctx, GDN_EINVAL, "n_kept is NULL");
    hipStream_t st = (hipStream_t)stream;
    DeviceGuard guard(ctx->device);
    ctx->has_last = false;
    if (n == 0) {
        gdn::launch_write_zero_count(n_kept, st);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(ctx, GDN_EHIP, hipGetErrorString(e));
        ctx->err.clear();
        return GDN_OK;
    }
    if (!xyz || !keep || !score || !kept_idx) return fail(ctx, GDN_EINVAL, "NULL array argument");
    if (!workspace) return fail(ctx, GDN_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace & 255u) != 0) return fail(ctx, GDN_EINVAL, "workspace must be 256-byte aligned");
    const gdn::Plan P = make_plan((uint32_t)n, p->k, (char*)workspace);
    if (workspace_bytes < P.bytes) return fail(ctx, GDN_ENOMEM, "workspace too small");
    const gdn::Params prm = to_params(p);
    CallEvents* ce = nullptr;
    if (ctx->timing) {
        ce = &ctx->ring[(size_t)(ctx->timed_calls % TIMING_RING)];
        ++ctx->timed_calls;
        (void)hipEventRecord(ce->ev[0], st);
    }

    gdn::launch_zero(P, st);
    gdn::launch_bbox(P, xyz, st);
    gdn::launch_morton(P, prm, xyz, st);
    gdn::launch_sort(P, st);
    gdn::launch_permute(P, xyz, st);
    gdn::launch_leaves(P, prm, st);
    gdn::launch_voxel(P, prm, st);
    gdn::launch_p1_compact(P, st);
    gdn::launch_halo(P, st);
    gdn::launch_knn_plan(P, st);
    gdn::launch_knn_bound(P, prm.k, ctx->num_cus, st);
    if (ce) (void)hipEventRecord(ce->ev[1], st);
    gdn::launch_knn(P, prm.k, ctx->num_cus, st);
    if (ce) (void)hipEventRecord(ce->ev[2], st);
    gdn::launch_knn_merge(P, prm.k, ctx->num_cus, st);
    gdn::launch_density(P, prm, xyz, st);
    gdn::launch_leaf_select(P, prm, st);
    gdn::launch_score(P, prm, xyz, st);
    gdn::launch_topl(P, prm, st);
    gdn::launch_outputs(P, keep, score, stage, kept_idx, n_kept, st);
    if (ce) (void)hipEventRecord(ce->ev[3], st);

    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, GDN_EHIP, hipGetErrorString(e));
    ctx->last = P;
    ctx->has_last = true;
    ctx->err.clear();
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

}  // extern "C"
