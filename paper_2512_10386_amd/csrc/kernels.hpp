// Host-side launchers of the denoiser's kernels (one group per source file).
#pragma once

#include "common.hpp"

struct gdn_ctx;

namespace gdn {

// frame.hip: zero-fill, frame table, frame bboxes, Morton keys, radix sort (and
// the re-sort of deep level-10 cells)
void launch_zero(const Plan& P, hipStream_t st);
void launch_frames(const Plan& P, const int64_t* frame_off, hipStream_t st);
// A single frame of up to 2^20 points: one box kernel that can also clear
// the zeroed block (clear: the fill launch is skipped).
bool bbox_one_frame(const Plan& P);
void launch_bbox(const Plan& P, const float* xyz, hipStream_t st, bool clear = false);
void launch_morton(const Plan& P, const Params& prm, const float* xyz, hipStream_t st);
void launch_sort(const Plan& P, const Params& prm, hipStream_t st);

// octree.hip: sorted coordinates and leaves, voxel filter, P1 compaction, halo
// ranges, kNN plan
void launch_leaves(const Plan& P, const Params& prm, const float* xyz, hipStream_t st);
void launch_voxel(const Plan& P, const Params& prm, hipStream_t st);
void launch_p1_compact(const Plan& P, hipStream_t st);
void launch_halo(const Plan& P, const Params& prm, hipStream_t st);
void launch_knn_plan(const Plan& P, const Params& prm, hipStream_t st);

// knn.hip: brute-force kNN over leaf + halo candidates (chunk merge included)
void launch_knn_bound(const Plan& P, int k, int num_cus, hipStream_t st);
void launch_knn(const Plan& P, int k, int num_cus, hipStream_t st);
void launch_knn_merge(const Plan& P, int k, int num_cus, hipStream_t st);

// score.hip: density with percentile/median, score, top-lambda, outputs
void launch_leaf_select(const Plan& P, const Params& prm, const float* xyz, hipStream_t st);
void launch_score(const Plan& P, const Params& prm, hipStream_t st);
// Returns true when top-lambda also wrote keep, score and stage (single
// frames); launch_outputs then only builds the kept list.
bool launch_topl(const Plan& P, const Params& prm, uint8_t* keep, float* score, uint8_t* stage, hipStream_t st);
void launch_keep_p2(const Plan& P, hipStream_t st);
void launch_outputs(const Plan& P, uint8_t* keep, float* score, uint8_t* stage,
                    uint32_t* kept_idx, int64_t* n_kept, hipStream_t st, bool written = false);
void launch_write_zero_count(int64_t* n_kept, uint32_t nf, hipStream_t st);

// fit.hip: score-fit loss and gradient over the last pass's intermediates
size_t fit_workspace_bytes(uint32_t n);
void launch_fit(const Plan& P, const float* xyz, const uint8_t* label, const FitArgs& a, void* workspace,
                double* out, hipStream_t st);

// eval.hip: exact nearest neighbours between clouds, PSNR / Chamfer metrics
size_t nearest_workspace_bytes(uint32_t na);
void launch_nearest(const float* a, uint32_t na, const float* b, uint32_t nb, void* ws, uint32_t* idx, float* d2,
                    hipStream_t st);
size_t eval_workspace_bytes(uint32_t nc, uint32_t nd);
void launch_eval(const float* clean, uint32_t nc, const float* den, uint32_t nd, void* ws, double* out,
                 hipStream_t st);

// The device status word of a pass: the Counters block opens the workspace.
inline const uint32_t* status_word(const void* workspace) {
    return &static_cast<const Counters*>(workspace)->status;
}

// dump.hip: intermediates back in original point order
int launch_dump(const Plan& P, int what, void* dst, size_t dst_bytes, hipStream_t st);

// capi.hip: the device a context is bound to, and a scope that makes a
// device current (restoring the previous one)
int context_device(const ::gdn_ctx* ctx);
struct CurrentDevice {
    int prev = -1;
    bool changed = false;
    explicit CurrentDevice(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) changed = hipSetDevice(dev) == hipSuccess;
    }
    ~CurrentDevice() {
        if (changed) (void)hipSetDevice(prev);
    }
};

}  // namespace gdn
