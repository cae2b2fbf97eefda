/*
 * gdn.h - C ABI of the MI355X (gfx950) library for the adaptive dual-weight
 * gravitational point-cloud denoiser (arxiv 2512.10386, Section 3).
 *
 * Problem statement (Sec. 3): a frame P = {p_1..p_N} of xyz points goes in;
 * out come the denoised subset P_denoise (Eq. 22) as a keep-mask and a list of
 * kept indices, and the per-point weighted gravitational score F_i (Eq. 21).
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers on the context's GPU, allocated and
 *     owned by the caller. The library allocates no device memory on the
 *     denoise path: all scratch lives in the caller's workspace.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *     No call synchronises the host except gdn_create/gdn_destroy, the
 *     profiling/tuning calls gdn_timing and gdn_autotune, and graph creation
 *     and destruction.
 *   - Parameter and size errors are reported synchronously by the return
 *     value, with nothing enqueued. Conditions only the GPU can see
 *     (non-finite coordinates, an exhausted internal wait) are recorded in a
 *     device status word readable with gdn_debug_dump(GDN_DUMP_STATUS).
 *   - A context is not thread-safe; use one context per host thread/stream.
 *   - No C++ exception crosses this interface.
 */
#ifndef GDN_H
#define GDN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GDN_OK = 0,
    GDN_EINVAL = 1,      /* bad parameter, size or pointer */
    GDN_ENOMEM = 2,      /* workspace too small */
    GDN_ECAPACITY = 3,   /* input larger than the library supports */
    GDN_EHIP = 4,        /* a HIP runtime call failed */
    GDN_EINTERNAL = 5
} gdn_status;

/* Device status word bits (GDN_DUMP_STATUS). */
#define GDN_DEV_NONFINITE   1u  /* some coordinate was NaN/inf: outputs unspecified */
#define GDN_DEV_WAIT_LIMIT  2u  /* an inter-workgroup wait hit its spin limit */
#define GDN_DEV_BAD_FRAMES  4u  /* a batch's frame table was not 0 = off[0] <= ... <= off[nf] = n;
                                   it was clamped/repaired: outputs unspecified */

#define GDN_MAX_FRAMES 4096     /* frames per gdn_denoise_batch call */

typedef struct {
    int32_t k;              /* K of Eq. 13 and Eq. 15: neighbours per point, 1..64 */
    int32_t leaf_cap;       /* octree: max points per leaf (Sec. 3), >= 1 */
    double  min_leaf_side;  /* octree: min leaf side in input units; <= 0: depth 21 */
    double  beta;           /* voxel enlargement coefficient of Eq. 11, > 0 */
    int32_t min_vox_count;  /* n_v of Eq. 12, >= 1 */
    double  rho_percentile; /* q of Eq. 14 in PERCENT (MATLAB prctile), 0..100 */
    double  alpha;          /* density-weight exponent of Eq. 17, >= 0 */
    double  sigma;          /* bandwidth scale of Eq. 18, > 0 */
    double  eps;            /* epsilon of Eq. 17 and Eq. 20, >= 0 */
    double  keep_ratio;     /* lambda: top fraction of P2 kept per leaf, (0, 1] */
    int32_t knn_chunk;      /* initial candidate chunk length of the kNN work split;
                               changes speed only, never results; 0 = default (32768) */
    double  gamma;          /* exponent of the gravitational kernel, (d^2 + eps)^(-gamma/2):
                               2 is Eq. 20 (computed as 1/(d^2+eps)); finite, >= 0 */
    double  log_threshold;  /* NaN: the per-leaf top-lambda rule (Sec. 3); a finite value
                               keeps instead every P2 point with ln F_i >= log_threshold */
    int32_t stages;         /* enabled modules, GDN_STAGE_* bits (the switches of Table 9);
                               GDN_STAGES_ALL = the method. A1 off: P1 = every point.
                               A2 off: P2 = the P1 points with k neighbours. A3 off: no
                               score (-1) and every P2 point is kept. */
} gdn_params;

#define GDN_STAGE_VOXEL   1  /* A1: voxel occupancy filter, Eq. 12 */
#define GDN_STAGE_DENSITY 2  /* A2: kNN density percentile filter, Eq. 14 */
#define GDN_STAGE_SCORE   4  /* A3: weighted gravitational score and top-lambda, Eq. 15-21 */
#define GDN_STAGES_ALL    7

typedef struct gdn_ctx gdn_ctx;

/* Defaults: k=12, rho_percentile=0.2, min_vox_count=4 (the paper's defaults,
 * Sec. 4.3.1); beta=1, alpha=1, sigma=1, eps=1e-12, keep_ratio=0.98,
 * leaf_cap=512, min_leaf_side=0 (not valued in the paper); knn_chunk=0;
 * gamma=2 (Eq. 20); log_threshold=NaN (top-lambda); stages=GDN_STAGES_ALL. */
gdn_status gdn_default_params(gdn_params *out);

/* Create a context bound to HIP device `device`. */
gdn_status gdn_create(gdn_ctx **out, int device);
void gdn_destroy(gdn_ctx *ctx);

/* Workspace bytes gdn_denoise needs for a frame of n points (n <= 2^30-1). */
gdn_status gdn_workspace_size(gdn_ctx *ctx, const gdn_params *p, int64_t n, size_t *bytes);

/*
 * Denoise one frame.
 *   xyz       [n][3] float32, row-major, input points (read only)
 *   workspace >= gdn_workspace_size bytes, 256-byte aligned; contents on entry
 *             are ignored; it holds this frame's intermediates until reused
 *   keep      [n] uint8: 1 if the point is in P_denoise (Eq. 22)
 *   score     [n] float32: F_i of Eq. 21 for points scored (the set P2 of
 *             Eq. 14); -1 for points removed before scoring
 *   stage     [n] uint8 or NULL: 0 removed by the voxel filter (Eq. 12),
 *             1 removed by the density filter (Eq. 14), 2 removed by the
 *             per-leaf top-lambda rule, 3 kept
 *   kept_idx  [n] uint32: the first *n_kept entries are the kept point
 *             indices in ascending order
 *   n_kept    device int64 scalar
 * Returns GDN_EINVAL for bad parameters/null pointers, GDN_ENOMEM if
 * workspace_bytes is too small, GDN_ECAPACITY if n > 2^30-1.
 */
gdn_status gdn_denoise(gdn_ctx *ctx, const gdn_params *p, const float *xyz, int64_t n,
                       void *workspace, size_t workspace_bytes,
                       uint8_t *keep, float *score, uint8_t *stage,
                       uint32_t *kept_idx, int64_t *n_kept, void *stream);

/*
 * Denoise one frame without allocating anything, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation. Same arguments, results and errors as
 * gdn_denoise, without the workspace: the frame's intermediates live in a
 * fixed scratch array of GDN_NOALLOC_MAX_BYTES inside the library, one per
 * GPU, held from the library's first use on that GPU until the process ends.
 * A frame whose gdn_workspace_size exceeds it is refused with GDN_ECAPACITY
 * (a 120k-point frame at k = 32 needs about 179 MiB). Every call on one GPU
 * shares that GPU's array and it keeps the last call's contents
 * (gdn_debug_dump reads them): calls that overlap on one GPU, on any streams
 * or contexts, race and give unspecified results. The call never allocates
 * or frees device memory and never synchronises the host.
 */
#define GDN_NOALLOC_MAX_BYTES (192u << 20)
gdn_status gdn_denoise_noalloc(gdn_ctx *ctx, const gdn_params *p, const float *xyz, int64_t n,
                               uint8_t *keep, float *score, uint8_t *stage,
                               uint32_t *kept_idx, int64_t *n_kept, void *stream);

/* Workspace bytes gdn_denoise_batch needs for nf frames of n points in all
 * (1 <= nf <= GDN_MAX_FRAMES). */
gdn_status gdn_workspace_size_batch(gdn_ctx *ctx, const gdn_params *p, int64_t n, int64_t nf, size_t *bytes);

/*
 * Denoise a batch of nf independent frames in one pass of the pipeline: the
 * method of Sec. 3 runs on every frame on its own (own bounding box and
 * octree, own percentiles), with results equal to nf gdn_denoise calls.
 *   xyz       [n][3] float32: the frames' points back to back
 *   frame_off DEVICE int64[nf+1]: frame f is points [frame_off[f],
 *             frame_off[f+1]); frame_off[0] = 0, non-decreasing,
 *             frame_off[nf] = n (empty frames allowed). A table breaking this
 *             is repaired on the device and GDN_DEV_BAD_FRAMES is set.
 *   keep, score, stage  [n], as gdn_denoise, at the points' batch positions
 *   kept_idx  [n] uint32: frame f's kept points, as FRAME-LOCAL indices in
 *             ascending order, start at kept_idx[frame_off[f]]
 *   n_kept    DEVICE int64[nf]: kept points per frame
 * Errors as gdn_denoise; GDN_ECAPACITY also for nf > GDN_MAX_FRAMES.
 */
gdn_status gdn_denoise_batch(gdn_ctx *ctx, const gdn_params *p, const float *xyz, int64_t n,
                             const int64_t *frame_off, int64_t nf,
                             void *workspace, size_t workspace_bytes,
                             uint8_t *keep, float *score, uint8_t *stage,
                             uint32_t *kept_idx, int64_t *n_kept, void *stream);

/*
 * A gdn_denoise_batch call recorded once as a HIP graph and replayed with
 * one launch. Every pointer and the sizes n, nf are fixed at creation; the
 * CONTENTS of xyz and frame_off may change between launches (same n and nf).
 * Creation captures on a private stream and runs nothing; each launch
 * enqueues the whole pipeline on `stream`. Launches of one graph must not
 * overlap (they share the workspace). gdn_debug_dump reads the workspace of
 * the latest launch. Destroy before the context.
 */
typedef struct gdn_graph gdn_graph;
gdn_status gdn_graph_create(gdn_ctx *ctx, const gdn_params *p, const float *xyz, int64_t n,
                            const int64_t *frame_off, int64_t nf,
                            void *workspace, size_t workspace_bytes,
                            uint8_t *keep, float *score, uint8_t *stage,
                            uint32_t *kept_idx, int64_t *n_kept, gdn_graph **out);
gdn_status gdn_graph_launch(gdn_graph *g, void *stream);
void gdn_graph_destroy(gdn_graph *g);

/*
 * Autotuner: runs the batch with every (leaf_cap, knn_chunk) pair from
 * caps[ncaps] x chunks[nchunks] (chunks may be NULL: default only), one
 * warm-up and `reps` timed runs each (HIP events on `stream`; this call waits
 * for them), and writes the fastest pair into *p. The leaf capacity changes
 * the octree and therefore the results (Sec. 3); knn_chunk does not. The
 * outputs and workspace hold the last run's results afterwards, not the
 * chosen pair's; gdn_debug_dump is unavailable until the next denoise.
 *   ms_out  float[ncaps * nchunks] or NULL: median ms per pair (row = cap)
 */
gdn_status gdn_autotune(gdn_ctx *ctx, gdn_params *p, const int32_t *caps, int ncaps,
                        const int32_t *chunks, int nchunks, int reps,
                        const float *xyz, int64_t n, const int64_t *frame_off, int64_t nf,
                        void *workspace, size_t workspace_bytes,
                        uint8_t *keep, float *score, uint8_t *stage,
                        uint32_t *kept_idx, int64_t *n_kept, float *ms_out, void *stream);

/*
 * Continuous-batching request server for streamed frames (serving form of the
 * batched path). gdn_server_create splits an HBM budget into slots (at most
 * max_slots), each able to run one batch of up to slot_frames frames and
 * slot_points points: its input buffer, workspace and outputs are allocated
 * here (hipMalloc; the only calls that allocate device memory). Each slot has
 * its own stream, so batches of different slots overlap on the device.
 *   gdn_server_submit queues one frame (host side only; nothing runs).
 *     xyz [n][3] and the outputs keep/score/stage(NULL ok)/kept_idx [n] and
 *     n_kept (int64 scalar) are the caller's device buffers, laid out as for
 *     gdn_denoise; they must stay valid until the ticket is reported done,
 *     and xyz must be completely written before submit (the slots' streams
 *     do not wait for the caller's). A frame larger than slot_points is
 *     refused with GDN_ECAPACITY, an empty one with GDN_EINVAL.
 *   gdn_server_poll retires finished batches, then packs waiting frames (in
 *     arrival order) into every free slot and launches them; it never waits
 *     for the GPU. It reports up to max_done finished tickets, and optionally
 *     (done_status, NULL ok) for each the device status word (GDN_DEV_*) of
 *     the batch it ran in: non-zero means that batch's outputs are
 *     unspecified; and optionally the queue length and the number of busy
 *     slots.
 * Results of a frame equal those of gdn_denoise on it alone. Not thread-safe;
 * poll from one thread. After a GDN_EHIP from poll the server is unusable.
 * Destroy waits for running slots, drops frames still queued and frees the
 * slots; destroy the server before its context. GDN_ENOMEM from create if
 * the budget holds no slot (gdn_server_info gives the bytes per slot).
 */
typedef struct gdn_server gdn_server;
gdn_status gdn_server_create(gdn_ctx *ctx, const gdn_params *p, size_t hbm_budget, int max_slots,
                             int64_t slot_points, int slot_frames, gdn_server **out);
gdn_status gdn_server_info(gdn_server *s, int *n_slots, size_t *bytes_per_slot);
gdn_status gdn_server_submit(gdn_server *s, const float *xyz, int64_t n, uint8_t *keep, float *score,
                             uint8_t *stage, uint32_t *kept_idx, int64_t *n_kept, int64_t *ticket);
gdn_status gdn_server_poll(gdn_server *s, int64_t *done_tickets, uint32_t *done_status, int max_done,
                           int *n_done, int *n_waiting, int *n_busy);
void gdn_server_destroy(gdn_server *s);
const char *gdn_server_last_error(gdn_server *s);

/*
 * Score fit: loss and gradient of a relaxed threshold on the score, for
 * fitting the weight parameters to labelled frames. It reads the neighbour
 * sets, densities, medians and P2 of the last gdn_denoise / gdn_denoise_batch
 * / graph launch on this context (workspace untouched since; those stay
 * fixed) and recomputes F_i of Eq. 21 at the given alpha (Eq. 17), sigma
 * (Eq. 18, 19) and kernel exponent gamma ((d^2+eps)^(-gamma/2); Eq. 20 is
 * gamma = 2), with eps of the last call. With y_i = 1 for a clean point
 * (label 0) and 0 for noise (label 1), z_i = (ln F_i - tau) / temperature:
 *   L = mean over the P2 points with 0 < F_i < inf of
 *       BCE(sigmoid(z_i), y_i) = ln(1 + e^z_i) - y_i z_i.
 *   xyz       [n][3] float32: the points of that last call
 *   label     [n] uint8 device: 1 = noise, 0 = clean (batch positions)
 *   workspace >= gdn_fit_workspace_size(n) bytes, 256-byte aligned
 *   out       DEVICE double[6]: L, dL/dalpha, dL/dsigma, dL/dgamma,
 *             dL/dtau, number of terms (FP64; L and gradients 0 if none)
 * The sums are taken in a fixed order: equal inputs give equal bits.
 * GDN_EINVAL if nothing was denoised, n differs from the last call, or a
 * parameter is out of range (alpha, gamma >= 0, sigma, temperature > 0,
 * all finite); GDN_ENOMEM if the workspace is too small.
 */
typedef struct {
    double alpha;        /* density-weight exponent of Eq. 17 */
    double sigma;        /* bandwidth scale of Eq. 18 */
    double gamma;        /* kernel exponent, 2 = Eq. 20 */
    double tau;          /* threshold on ln F */
    double temperature;  /* sigmoid temperature T */
} gdn_fit_params;
gdn_status gdn_fit_workspace_size(gdn_ctx *ctx, int64_t n, size_t *bytes);
gdn_status gdn_fit_loss_grad(gdn_ctx *ctx, const gdn_fit_params *fp, const float *xyz, const uint8_t *label,
                             int64_t n, void *workspace, size_t workspace_bytes, double *out, void *stream);

/*
 * Evaluation (Sec. 4.1): exact nearest neighbours and the quality metrics of
 * a denoised cloud.
 * gdn_nearest: for every point of a [na][3] its nearest point of b [nb][3],
 *   brute force, fp32 squared distance (dx*dx + dy*dy) + dz*dz, ties to the
 *   smaller index: idx [na] uint32, d2 [na] float (device arrays). A query
 *   with a NaN coordinate gets idx 0, d2 +inf.
 * gdn_eval_metrics: clean [nc][3] against denoised [nd][3]; each point is
 *   matched to its nearest point of the other cloud, squared distances of
 *   the matched pairs in FP64; out DEVICE double[4]:
 *     MSE = mean over clean of the squared distance to the denoised cloud,
 *     the mean over denoised of the squared distance to the clean cloud,
 *     CD = the sum of the two (Eq. 30),
 *     PSNR = 10 log10(M^2 / MSE) dB with M the diagonal of the clean cloud's
 *     bounding box (Eq. 29); +inf when MSE = 0.
 * Both need 1 <= na, nb, nc, nd <= 2^30-1 (GDN_EINVAL / GDN_ECAPACITY) and a
 * 256-byte aligned workspace of the reported size (GDN_ENOMEM).
 */
gdn_status gdn_nearest_workspace_size(gdn_ctx *ctx, int64_t na, size_t *bytes);
gdn_status gdn_nearest(gdn_ctx *ctx, const float *a, int64_t na, const float *b, int64_t nb,
                       void *workspace, size_t workspace_bytes, uint32_t *idx, float *d2, void *stream);
gdn_status gdn_eval_workspace_size(gdn_ctx *ctx, int64_t nc, int64_t nd, size_t *bytes);
gdn_status gdn_eval_metrics(gdn_ctx *ctx, const float *clean, int64_t nc, const float *den, int64_t nd,
                            void *workspace, size_t workspace_bytes, double *out, void *stream);

/* Intermediates of the last gdn_denoise / gdn_denoise_batch / graph launch
 * on this context (its workspace must be untouched since). Per-point arrays
 * are in ORIGINAL (batch) point order; leaf arrays cover the whole batch. */
enum {
    GDN_DUMP_STATUS = 0,     /* uint32 device status word (GDN_DEV_*) */
    GDN_DUMP_COUNTS = 1,     /* int64[4]: n_leaves, |P1|, kNN pair count W, n_kept */
    GDN_DUMP_KEYS = 2,       /* uint64[n] Morton keys */
    GDN_DUMP_ORDER = 3,      /* uint32[n] original index at each sorted position: leaves in
                                Morton order, each over its [begin, end); inside a leaf the
                                order is unspecified (keys are sorted only as deep as the
                                octree reaches) */
    GDN_DUMP_LEAF_OF = 4,    /* uint32[n] leaf id of each point */
    GDN_DUMP_LEAF_TABLE = 5, /* uint32[n_leaves][4]: begin, end, level, fp32 bits of h */
    GDN_DUMP_OCC = 6,        /* uint32[n] voxel occupancy n(voxel(p)) of Eq. 12 */
    GDN_DUMP_P1 = 7,         /* uint8[n] */
    GDN_DUMP_NBR_IDX = 8,    /* uint32[n][k] neighbours (original idx) of P1 points,
                                (d2, idx) ascending, 0xFFFFFFFF padding */
    GDN_DUMP_NBR_D2 = 9,     /* float[n][k] fp32 squared distances, +inf padding */
    GDN_DUMP_R2K = 10,       /* float[n] squared k-th distance (+inf: fewer than k) */
    GDN_DUMP_RHO = 11,       /* double[n] density of Eq. 13 */
    GDN_DUMP_P2 = 12,        /* uint8[n] */
    GDN_DUMP_LEAF_RHO_MED = 13, /* double[n_leaves] median density of Eq. 16 */
    GDN_DUMP_SCORE64 = 14,   /* double[n] score of Eq. 21 (-1 if not scored) */
    GDN_DUMP_LEAF_NCAND = 15 /* uint32[n_leaves] candidate count |C_t| */
};
/* Copy one intermediate into device buffer dst (dst_bytes must hold it;
 * rows not defined for a point are filled with the padding values). */
gdn_status gdn_debug_dump(gdn_ctx *ctx, int what, void *dst, size_t dst_bytes, void *stream);

/* Profiling aid. With timing enabled, each gdn_denoise records HIP events on
 * its stream (call start, kNN kernel start, kNN kernel end, call end) into a
 * ring of the last 256 calls. gdn_timing reads call `back` (0 = the latest),
 * waiting for its events; it returns the whole call's and the brute-force kNN
 * kernel's elapsed milliseconds. Enabling creates the events (no device
 * memory); disabling destroys them. */
gdn_status gdn_set_timing(gdn_ctx *ctx, int enable);
gdn_status gdn_timing(gdn_ctx *ctx, int64_t back, float *total_ms, float *knn_ms);

const char *gdn_status_string(gdn_status s);
/* Message of the last failed call on ctx ("" if none). */
const char *gdn_last_error(gdn_ctx *ctx);

/* Hex SHA-256 of the sources and flags this library was built from (a static
 * string; "unknown" if the build did not set it). Loaders compare it with the
 * sources beside the library to refuse a stale build. */
const char *gdn_source_hash(void);

#ifdef __cplusplus
}
#endif
#endif
