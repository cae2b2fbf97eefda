/*
 * CPU oracle for the adaptive dual-weight gravitational denoiser
 * (arxiv 2512.10386, Section 3, Eq. 10-22).
 *
 * TEST INFRASTRUCTURE ONLY. This library is the plain, slow reference that the
 * HIP path is checked against. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never calls
 * it and shares no code with it.
 *
 * Numeric policy: every discrete decision (Morton keys, octree leaves, voxel
 * indices, kNN sets, ranks) is taken in the precision the method fixes for it
 * (fp32 squared distances summed as (dx*dx+dy*dy)+dz*dz, FP64 quantisation);
 * continuous outputs (density, median, score) are FP64. Built with
 * -ffp-contract=off and no fast-math.
 */
#ifndef GDN_ORACLE_H
#define GDN_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t k;              /* K of Eq. 13 / 15 */
    int32_t leaf_cap;       /* max points per octree leaf (Sec. 3, octree) */
    double  min_leaf_side;  /* min leaf side; <= 0 means depth limit 21 */
    double  beta;           /* voxel enlargement coefficient, Eq. 11 */
    int32_t min_vox_count;  /* n_v, Eq. 12 */
    double  rho_percentile; /* q of Eq. 14, in percent (prctile semantics) */
    double  alpha;          /* density-weight exponent, Eq. 17 */
    double  sigma;          /* bandwidth scale, Eq. 18 */
    double  eps;            /* epsilon of Eq. 17 and Eq. 20 */
    double  keep_ratio;     /* lambda of the per-leaf top-lambda rule */
    double  gamma;          /* exponent of the gravitational kernel (d^2+eps)^(-gamma/2);
                               2 gives Eq. 20 exactly (computed as 1/(d^2+eps)) */
    double  log_threshold;  /* NaN: per-leaf top-lambda rule; otherwise keep the
                               P2 points with ln F_i >= log_threshold instead */
    int32_t stages;         /* enabled modules (Table 9): bit 0 A1 voxel filter (Eq. 12),
                               bit 1 A2 density filter (Eq. 14), bit 2 A3 score and
                               top-lambda (Eq. 15-21); 7 = the full method.
                               A1 off: P1 = all points. A2 off: P2 = the P1 points with
                               k neighbours. A3 off: no score (-1), P2 is kept. */
} orc_params;

/* Every array is caller-allocated. Per-point arrays are indexed by ORIGINAL
 * point index and hold n entries (nbr_* hold n*k). Leaf arrays hold up to n
 * entries (a frame of n points has at most n leaves). Any pointer may be NULL
 * except the ones the caller wants filled. */
typedef struct {
    /* per point */
    uint64_t *key;        /* Morton key */
    uint32_t *order;      /* order[s] = original index at sorted position s */
    uint32_t *leaf_of;    /* leaf id of each point */
    uint32_t *occ;        /* occupancy of the point's voxel, Eq. 12 */
    uint8_t  *p1;         /* 1 if the point is in P1 */
    uint32_t *nbr_idx;    /* [n][k] neighbour original indices, (d2, idx) ascending;
                             0xFFFFFFFF padding; rows of non-P1 points untouched */
    float    *nbr_d2;     /* [n][k] fp32 squared distances (+inf padding) */
    float    *r2k;        /* fp32 squared k-th distance, +inf if insufficient */
    double   *rho;        /* Eq. 13 density (0 if insufficient) */
    uint8_t  *p2;         /* 1 if the point is in P2 (Eq. 14) */
    double   *score;      /* Eq. 21 score, -1 for points not scored */
    uint8_t  *stage;      /* 0 voxel-removed, 1 density-removed, 2 score-removed, 3 kept */
    uint8_t  *keep;       /* 1 if in the output set (Eq. 22) */
    uint32_t *kept_idx;   /* ascending original indices of kept points */
    /* per leaf */
    uint32_t *leaf_begin; /* sorted-position range [begin, end) */
    uint32_t *leaf_end;
    uint32_t *leaf_level;
    uint64_t *leaf_prefix;
    float    *leaf_h;     /* fp32 voxel size h (0 = single voxel) */
    uint32_t *leaf_n1;    /* |P1 in leaf| */
    uint32_t *leaf_n2;    /* |P2 in leaf| */
    uint32_t *leaf_m;     /* points kept by top-lambda */
    double   *leaf_rho_med;
    uint32_t *leaf_ncand; /* |C_t|: P1 points in the leaf's 27-cell block */
    /* scalars out */
    int64_t  n_kept;
    int64_t  n_leaves;
    uint64_t pairs;       /* sum over leaves of |Q_t| * (|C_t| - 1) */
    int32_t  threads;     /* OpenMP threads used */
} orc_out;

void orc_default_params(orc_params *p);

/* Whole pipeline. Returns 0 on success, -1 on invalid parameters. */
int orc_denoise(const float *xyz, int64_t n, const orc_params *p, orc_out *o);

/*
 * Score-fit loss and its gradient (FP64), over the intermediates of a prior
 * orc_denoise on the same points (o must hold nbr_idx, rho, p2, leaf_of and
 * leaf_rho_med; the neighbour sets, densities, medians and P2 stay fixed).
 * With F_i the score of Eq. 21 (kernel exponent gamma) at the given alpha,
 * sigma, gamma, and y_i = 1 for a clean point (label 0), 0 for noise:
 *   z_i = (ln F_i - tau) / T,  L = mean over i in P2 with 0 < F_i < inf of
 *   BCE(sigmoid(z_i), y_i).
 * out[6] = {L, dL/dalpha, dL/dsigma, dL/dgamma, dL/dtau, number of terms}.
 * Returns -1 for T <= 0 or sigma <= 0.
 */
int orc_fit_loss_grad(const float *xyz, int64_t n, int k, double eps, const orc_out *o,
                      const uint8_t *label, double alpha, double sigma, double gamma,
                      double tau, double T, double *out);

/*
 * Nearest neighbour of every point of a in b (brute force): fp32 squared
 * distance ((dx*dx + dy*dy) + dz*dz), ties to the smaller index of b.
 * idx[na], d2[na]. Returns -1 if nb == 0.
 */
int orc_nearest(const float *a, int64_t na, const float *b, int64_t nb, uint32_t *idx, float *d2);

/*
 * Quality of a denoised cloud against the clean one (Eq. 29, 30), with each
 * clean point matched to its nearest denoised point and vice versa
 * (orc_nearest), squared distances of the matched pairs in FP64:
 *   out[0] = MSE = mean over clean of the squared distance to the denoised set
 *   out[1] = mean over denoised of the squared distance to the clean set
 *   out[2] = CD = out[0] + out[1]                                   (Eq. 30)
 *   out[3] = PSNR = 10 log10(M^2 / MSE), M = diagonal of the clean
 *            cloud's bounding box (from its fp32 min/max)           (Eq. 29)
 * Returns -1 if either cloud is empty.
 */
int orc_eval_metrics(const float *clean, int64_t nc, const float *den, int64_t nd, double *out);

/* Individual steps exposed for pinning. */
uint64_t orc_morton_interleave(uint32_t qx, uint32_t qy, uint32_t qz);
/* MATLAB-prctile keep count: 1-based rank c of the cut (Eq. 14). */
int64_t orc_percentile_rank(int64_t n, double q_percent);

#ifdef __cplusplus
}
#endif
#endif
