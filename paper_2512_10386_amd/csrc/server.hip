// Continuous-batching request server (include/gdn.h, gdn_server_*): streamed
// frames are admitted into slots as slots free up, each slot running one
// batch of frames through the batched pipeline on its own stream, so the
// batches of different slots overlap on the device. The HBM budget given at
// creation fixes the number of slots; every slot owns its input buffer,
// workspace (its frames' octrees stay resident there until the slot is
// reused) and outputs. Requests are gathered into a slot's input and their
// results scattered back to the caller's buffers by two small kernels.
#include <algorithm>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "gdn.h"
#include "kernels.hpp"

namespace {

// One request of a batch, as the gather/scatter kernels see it.
struct ReqDesc {
    const float* xyz;
    uint8_t* keep;
    float* score;
    uint8_t* stage;
    uint32_t* kept_idx;
    int64_t* n_kept;
    int64_t off;  // first point in the slot's batch
    int64_t n;
};

__device__ __forceinline__ uint32_t req_of(const ReqDesc* d, uint32_t nr, int64_t p) {
    uint32_t lo = 0, hi = nr;  // last request with off <= p
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (d[mid].off <= p) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void gather_kernel(const ReqDesc* __restrict__ d, uint32_t nr, int64_t total,
                                                     float* __restrict__ xyz, int64_t* __restrict__ foff) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nt = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = tid; p < total; p += nt) {
        const ReqDesc& r = d[req_of(d, nr, p)];
        const int64_t i = p - r.off;
        xyz[3 * p] = r.xyz[3 * i];
        xyz[3 * p + 1] = r.xyz[3 * i + 1];
        xyz[3 * p + 2] = r.xyz[3 * i + 2];
    }
    for (int64_t f = tid; f <= (int64_t)nr; f += nt) foff[f] = f < (int64_t)nr ? d[f].off : total;
}

__global__ __launch_bounds__(256) void scatter_kernel(const ReqDesc* __restrict__ d, uint32_t nr, int64_t total,
                                                      const uint8_t* keep, const float* score, const uint8_t* stage,
                                                      const uint32_t* kept_idx, const int64_t* n_kept) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nt = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = tid; p < total; p += nt) {
        const uint32_t f = req_of(d, nr, p);
        const ReqDesc& r = d[f];
        const int64_t i = p - r.off;
        r.keep[i] = keep[p];
        r.score[i] = score[p];
        if (r.stage) r.stage[i] = stage[p];
        if (i < n_kept[f]) r.kept_idx[i] = kept_idx[p];
    }
    for (int64_t f = tid; f < (int64_t)nr; f += nt) *d[f].n_kept = n_kept[f];
}

struct Req {
    int64_t ticket;
    ReqDesc desc;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    float* xyz = nullptr;
    int64_t* foff = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    uint8_t* keep = nullptr;
    float* score = nullptr;
    uint8_t* stage = nullptr;
    uint32_t* kept_idx = nullptr;
    int64_t* n_kept = nullptr;
    ReqDesc* desc_dev = nullptr;
    ReqDesc* desc_host = nullptr;  // pinned
    uint32_t* status_host = nullptr;  // pinned: the batch's device status word
    std::vector<int64_t> tickets;
    bool busy = false;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct gdn_server {
    gdn_ctx* ctx = nullptr;
    gdn_params params{};
    int64_t cap_points = 0;
    int cap_frames = 0;
    std::vector<Slot> slots;
    std::deque<Req> waiting;
    std::vector<int64_t> done;  // finished tickets not yet reported
    std::vector<uint32_t> done_status;  // their batches' device status words
    int64_t next_ticket = 0;
    std::string err;
};

namespace {

gdn_status srv_fail(gdn_server* s, gdn_status st, const char* m) {
    if (s) s->err = m;
    return st;
}

void free_slot(Slot& sl) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.xyz) (void)hipFree(sl.xyz);  // one allocation holds all device arrays
    if (sl.desc_host) (void)hipHostFree(sl.desc_host);
    if (sl.status_host) (void)hipHostFree(sl.status_host);
    sl = Slot{};
}

// Start a batch in a free slot from the head of the queue.
gdn_status launch_slot(gdn_server* S, Slot& sl) {
    uint32_t nr = 0;
    int64_t total = 0;
    sl.tickets.clear();
    while (!S->waiting.empty() && (int)nr < S->cap_frames && total + S->waiting.front().desc.n <= S->cap_points) {
        Req r = S->waiting.front();
        S->waiting.pop_front();
        r.desc.off = total;
        sl.desc_host[nr++] = r.desc;
        sl.tickets.push_back(r.ticket);
        total += r.desc.n;
    }
    if (nr == 0) return GDN_OK;
    if (hipMemcpyAsync(sl.desc_dev, sl.desc_host, sizeof(ReqDesc) * nr, hipMemcpyHostToDevice, sl.stream) !=
        hipSuccess)
        return srv_fail(S, GDN_EHIP, "hipMemcpyAsync of the request table failed");
    unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256 + 1, 4096);
    hipLaunchKernelGGL(gather_kernel, dim3(blocks), dim3(256), 0, sl.stream, sl.desc_dev, nr, total, sl.xyz,
                       sl.foff);
    const gdn_status st = gdn_denoise_batch(S->ctx, &S->params, sl.xyz, total, sl.foff, nr, sl.ws, sl.ws_bytes,
                                            sl.keep, sl.score, sl.stage, sl.kept_idx, sl.n_kept, sl.stream);
    if (st != GDN_OK) return srv_fail(S, st, gdn_last_error(S->ctx));
    hipLaunchKernelGGL(scatter_kernel, dim3(blocks), dim3(256), 0, sl.stream, sl.desc_dev, nr, total, sl.keep,
                       sl.score, sl.stage, sl.kept_idx, sl.n_kept);
    if (hipMemcpyAsync(sl.status_host, gdn::status_word(sl.ws), sizeof(uint32_t), hipMemcpyDeviceToHost,
                       sl.stream) != hipSuccess)
        return srv_fail(S, GDN_EHIP, "hipMemcpyAsync of the status word failed");
    if (hipEventRecord(sl.done, sl.stream) != hipSuccess) return srv_fail(S, GDN_EHIP, "hipEventRecord failed");
    if (hipGetLastError() != hipSuccess) return srv_fail(S, GDN_EHIP, "kernel launch failed");
    sl.busy = true;
    return GDN_OK;
}

}  // namespace

extern "C" {

gdn_status gdn_server_create(gdn_ctx* ctx, const gdn_params* p, size_t hbm_budget, int max_slots,
                             int64_t slot_points, int slot_frames, gdn_server** out) {
    if (!ctx || !p || !out) return GDN_EINVAL;
    *out = nullptr;
    if (max_slots < 1 || slot_points < 1 || slot_frames < 1 || slot_frames > GDN_MAX_FRAMES) return GDN_EINVAL;
    size_t ws = 0;
    gdn_status st = gdn_workspace_size_batch(ctx, p, slot_points, slot_frames, &ws);
    if (st != GDN_OK) return st;
    const size_t P = (size_t)slot_points, F = (size_t)slot_frames;
    const size_t bytes = align256(12 * P) + align256(8 * (F + 1)) + align256(ws) + align256(P) + align256(4 * P) +
                         align256(P) + align256(4 * P) + align256(8 * F) + align256(sizeof(ReqDesc) * F);
    const size_t nslots = std::min<size_t>((size_t)max_slots, hbm_budget / bytes);
    if (nslots == 0) return GDN_ENOMEM;
    gdn_server* S = new (std::nothrow) gdn_server();
    if (!S) return GDN_EINTERNAL;
    S->ctx = ctx;
    S->params = *p;
    S->cap_points = slot_points;
    S->cap_frames = slot_frames;
    S->slots.resize(nslots);
    gdn::CurrentDevice guard(gdn::context_device(ctx));
    for (Slot& sl : S->slots) {
        char* b = nullptr;
        bool ok = hipMalloc((void**)&b, bytes) == hipSuccess;
        ok = ok && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
        ok = ok && hipHostMalloc((void**)&sl.desc_host, sizeof(ReqDesc) * F) == hipSuccess;
        ok = ok && hipHostMalloc((void**)&sl.status_host, sizeof(uint32_t)) == hipSuccess;
        if (!ok) {
            if (b) (void)hipFree(b);
            for (Slot& x : S->slots) free_slot(x);
            delete S;
            return GDN_ENOMEM;
        }
        size_t o = 0;
        auto take = [&](size_t n) {
            char* q = b + o;
            o += align256(n);
            return q;
        };
        sl.xyz = (float*)take(12 * P);
        sl.foff = (int64_t*)take(8 * (F + 1));
        sl.ws = take(ws);
        sl.ws_bytes = ws;
        sl.keep = (uint8_t*)take(P);
        sl.score = (float*)take(4 * P);
        sl.stage = (uint8_t*)take(P);
        sl.kept_idx = (uint32_t*)take(4 * P);
        sl.n_kept = (int64_t*)take(8 * F);
        sl.desc_dev = (ReqDesc*)take(sizeof(ReqDesc) * F);
    }
    *out = S;
    return GDN_OK;
}

gdn_status gdn_server_info(gdn_server* s, int* n_slots, size_t* bytes_per_slot) {
    if (!s) return GDN_EINVAL;
    if (n_slots) *n_slots = (int)s->slots.size();
    if (bytes_per_slot) {
        size_t ws = 0;
        (void)gdn_workspace_size_batch(s->ctx, &s->params, s->cap_points, s->cap_frames, &ws);
        const size_t P = (size_t)s->cap_points, F = (size_t)s->cap_frames;
        *bytes_per_slot = align256(12 * P) + align256(8 * (F + 1)) + align256(ws) + align256(P) + align256(4 * P) +
                          align256(P) + align256(4 * P) + align256(8 * F) + align256(sizeof(ReqDesc) * F);
    }
    return GDN_OK;
}

gdn_status gdn_server_submit(gdn_server* s, const float* xyz, int64_t n, uint8_t* keep, float* score,
                             uint8_t* stage, uint32_t* kept_idx, int64_t* n_kept, int64_t* ticket) {
    if (!s) return GDN_EINVAL;
    if (n < 1) return srv_fail(s, GDN_EINVAL, "a request needs at least one point");
    if (n > s->cap_points) return srv_fail(s, GDN_ECAPACITY, "request larger than a slot");
    if (!xyz || !keep || !score || !kept_idx || !n_kept || !ticket)
        return srv_fail(s, GDN_EINVAL, "NULL argument");
    Req r;
    r.ticket = s->next_ticket++;
    r.desc = ReqDesc{xyz, keep, score, stage, kept_idx, n_kept, 0, n};
    s->waiting.push_back(r);
    *ticket = r.ticket;
    return GDN_OK;
}

gdn_status gdn_server_poll(gdn_server* s, int64_t* done_tickets, uint32_t* done_status, int max_done, int* n_done,
                           int* n_waiting, int* n_busy) {
    if (!s || !n_done) return GDN_EINVAL;
    gdn::CurrentDevice guard(gdn::context_device(s->ctx));
    for (Slot& sl : s->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipSuccess) {
            sl.busy = false;
            s->done.insert(s->done.end(), sl.tickets.begin(), sl.tickets.end());
            s->done_status.insert(s->done_status.end(), sl.tickets.size(), *sl.status_host);
            sl.tickets.clear();
        } else if (q != hipErrorNotReady) {
            return srv_fail(s, GDN_EHIP, "hipEventQuery failed");
        }
    }
    for (Slot& sl : s->slots) {
        if (s->waiting.empty()) break;
        if (sl.busy) continue;
        const gdn_status st = launch_slot(s, sl);
        if (st != GDN_OK) return st;
    }
    const int k = std::min<int>((int)s->done.size(), std::max(max_done, 0));
    for (int i = 0; i < k; ++i) {
        done_tickets[i] = s->done[(size_t)i];
        if (done_status) done_status[i] = s->done_status[(size_t)i];
    }
    s->done.erase(s->done.begin(), s->done.begin() + k);
    s->done_status.erase(s->done_status.begin(), s->done_status.begin() + k);
    *n_done = k;
    if (n_waiting) *n_waiting = (int)s->waiting.size();
    if (n_busy) {
        int b = 0;
        for (const Slot& sl : s->slots) b += sl.busy ? 1 : 0;
        *n_busy = b;
    }
    return GDN_OK;
}

void gdn_server_destroy(gdn_server* s) {
    if (!s) return;
    gdn::CurrentDevice guard(gdn::context_device(s->ctx));
    for (Slot& sl : s->slots) free_slot(sl);
    delete s;
}

const char* gdn_server_last_error(gdn_server* s) { return s ? s->err.c_str() : ""; }

}  // extern "C"
