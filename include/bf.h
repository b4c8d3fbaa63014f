/*
 * bf.h - C ABI of the MI355X (gfx950) BayesFusion-SDF narrow-band solver.
 *
 * The library computes, on one GPU, the probabilistic signed-distance fusion of
 * the paper "BayesFusion-SDF: Probabilistic Signed Distance Fusion with View
 * Planning on CPU" (arXiv 2602.19697): coarse TSDF and narrow band (Sec. 3.3,
 * eq. 1), observation assembly under a heteroscedastic noise model (Sec. 3.5,
 * eqs. 3-5), the GMRF posterior precision Q = Lambda_obs + lambda L + eps I and
 * its mean (Sec. 3.6, eqs. 7-11), the Hutchinson estimate of diag(Q^-1)
 * (Sec. 3.7, eq. 12) and next-best-view scoring (Sec. 3.8, eq. 13).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Units are metres.  A pose is the row-major 3x4 camera-to-world matrix
 *    [R | t] (T_{w<-c} of Sec. 3.1); cameras follow the pinhole model with x
 *    right, y down, z forward and integer pixel centres.  Depth is camera-z
 *    depth (eq. 2), float32, with 0 meaning "no return".
 *  - Pointers named *_dev are device pointers on the context's device; the
 *    caller owns them.  Pointers named *_host are host memory.  Struct
 *    arguments are read during the call only.
 *  - Every call is ordered on the context's HIP stream.  Calls that write a
 *    host out-parameter (a count, a report, an argmax) synchronise that stream
 *    before returning; all others are asynchronous.
 *  - Every call returns a bf_status.  On failure the context's message
 *    (bf_last_error) says what went wrong; outputs are then unspecified unless
 *    the call's comment says otherwise.  No C++ exception crosses the ABI.
 *  - Band and system objects are opaque, own their device arrays and are
 *    released with bf_band_free / bf_system_free on the context that made them.
 *    Arrays exposed by the *_view calls stay valid until that free.
 *  - A band of zero voxels is valid: later calls launch nothing and succeed.
 */
#ifndef BF_H
#define BF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bf_status {
  BF_OK = 0,
  BF_ERR_INVALID_ARG = 1,    /* bad size, NULL pointer, NaN/negative depth, ... */
  BF_ERR_OOM = 2,            /* device allocation failed */
  BF_ERR_CAPACITY = 3,       /* band too large for 32-bit band indices */
  BF_ERR_BREAKDOWN = 4,      /* CG met p.Qp <= 0 or a non-finite scalar */
  BF_ERR_NOT_CONVERGED = 5,  /* max_iter reached; result and report are written */
  BF_ERR_HIP = 6             /* a HIP runtime call failed */
} bf_status;

typedef struct bf_ctx bf_ctx;
typedef struct bf_band bf_band;
typedef struct bf_system bf_system;

/* Regular grid of G^3 voxels of edge h whose low corner is `origin`; voxel
 * (i,j,k) has centre origin + (index + 1/2) h.  tau is the TSDF truncation
 * distance and `band` the half-width of the narrow band (eq. 1 with
 * alpha*tau = band), both in metres.  G <= 2048. */
typedef struct bf_grid {
  int32_t G;
  double h;
  double origin[3];
  double tau;
  double band;
} bf_grid;

typedef struct bf_camera {
  int32_t width, height;
  double fx, fy, cx, cy;
} bf_camera;

/* Observation variance of eq. (5): sigma^2 = sigma_depth(D)^2 + sigma2_pose[t]
 * + sigma2_model with sigma_depth(D) = a + c (D - z0)^2 of the measured depth.
 * sigma2_pose_dev is a device array [T] or NULL (all zero). */
typedef struct bf_noise {
  double a, c, z0;
  const double* sigma2_pose_dev;
  double sigma2_model;
} bf_noise;

/* GMRF prior of eqs. (6)-(7): lambda weights the 6-neighbour Laplacian of the
 * band (unit edge weights), eps >= 0 adds eps*I, and lambda_b >= 0 anchors the
 * band boundary (voxels with fewer than 6 band neighbours) to the TSDF. */
typedef struct bf_prior {
  double lambda, eps, lambda_b;
} bf_prior;

enum { BF_PREC_FP64 = 0, BF_PREC_MIXED = 1 };
enum { BF_BAND_KEEP_DENSE = 1 };
enum { BF_UTILITY_SUM_VAR = 0, BF_UTILITY_VAR_REDUCTION = 1 };
enum { BF_SYSTEM_VOXEL = 0, BF_SYSTEM_TRILINEAR = 1 };

/* CG stopping rule: ||rhs - Q x|| <= tol ||rhs|| with the residual recomputed
 * in FP64 before stopping.  precision: BF_PREC_FP64 runs every vector
 * operation in double; BF_PREC_MIXED runs the matrix-vector products and
 * vector updates in float with double dot products, alpha/beta and an FP64
 * residual-correction loop.  use_x0 != 0 starts from the values in x_dev.
 * check_every: host convergence polls, 0 = automatic. */
typedef struct bf_solve_opts {
  double tol;
  int32_t max_iter;
  int32_t precision;
  int32_t use_x0;
  int32_t check_every;
} bf_solve_opts;

typedef struct bf_solve_report {
  int32_t iters;            /* CG iterations (the largest over probe columns) */
  int32_t status;           /* bf_status of the solve */
  int32_t refinements;      /* FP64 residual corrections taken (mixed precision) */
  int32_t used_warm_start;  /* 1 if a start was supplied and kept.  A supplied start whose FP64
                               residual ||rhs - Q x0|| is not below ||rhs|| (no better than
                               zero) is dropped and that solve (or probe column) runs from
                               x = 0; this is 0 if any column's start was dropped. */
  double rel_res;           /* final FP64 ||rhs - Q x|| / ||rhs|| (max over columns) */
  double seconds;           /* device time of the solve */
  int64_t col_iters;        /* iterations summed over right-hand sides (probe columns) */
} bf_solve_report;

/* Hutchinson probes of eq. (12): K Rademacher vectors z_k with z_k[i] = -1 when
 * the top bit of output i of SplitMix64 started at u_k is set (else +1), u_k
 * being output k of SplitMix64 started at `seed`.  K in {1..64}. */
typedef struct bf_probe_opts {
  int32_t K;
  int32_t precision;
  uint64_t seed;
  double tol;
  int32_t max_iter;
} bf_probe_opts;

typedef struct bf_band_arrays {
  int64_t n;               /* band voxel count N */
  int32_t dense_side;      /* P = smallest power of two >= G */
  const uint64_t* keys;    /* [N] Morton keys, strictly ascending: bit 3b = bit b of i,
                              bit 3b+1 = bit b of j, bit 3b+2 = bit b of k */
  const double* tsdf;      /* [N] coarse TSDF */
  const int32_t* w;        /* [N] number of views fused */
  const int32_t* nbr;      /* [N][6] band index of the -x,+x,-y,+y,-z,+z neighbour or -1 */
  const int32_t* deg;      /* [N] number of band neighbours */
  const double* dense_tsdf;   /* [P^3] Morton-ordered dense TSDF, or NULL */
  const int32_t* dense_w;     /* [P^3] Morton-ordered dense weights, or NULL */
  int64_t tsdf_voxel_views;   /* voxel x view projections the coarse TSDF evaluated; 4^3 cells that
                                 provably hold no band voxel are skipped (not with BF_BAND_KEEP_DENSE) */
  int64_t tsdf_box_tests;     /* (box, view) screening tests made for that skipping; a box is a
                                 32x16x16 super tile, a 16x8x8 block tile or a 4^3 cell */
  int64_t tsdf_tile_tests;    /* ... of them, those of super tiles and block tiles */
} bf_band_arrays;

typedef struct bf_system_arrays {
  int64_t n;
  const double* Lambda;    /* [N] diagonal of A^T W A (eq. 10) */
  const double* b;         /* [N] A^T W y (eq. 11) */
  const double* rhs;       /* [N] h = A^T W y + b0 (anchor term included) */
  const double* diag;      /* [N] diagonal of Q */
  const float* diag32;     /* [N] diag rounded to float */
  const double* acc;       /* [N][5] n_obs, sum y, sum y^2, sum sigma, min sigma (voxel rows only) */
  int32_t kind;            /* BF_SYSTEM_VOXEL or BF_SYSTEM_TRILINEAR */
  const double* off;       /* [26][N] trilinear couplings Q_vu, slot-major (see bf_assemble_trilinear), or NULL */
  const int32_t* nb26;     /* [26][N] band index of each coupling's voxel or -1, slot-major, or NULL */
  int64_t n_samples;       /* trilinear samples kept */
  int64_t n_cells;         /* 2x2x2 cells holding at least one kept sample */
} bf_system_arrays;

/* ---------------------------------------------------------------- context */

/* Device memory for the arrays that bands, systems and meshes own (the
 * objects the caller keeps and frees).  alloc returns a device pointer of at
 * least `bytes` bytes on the context's device, usable in the order of work on
 * `hip_stream` (the context's stream), or NULL on failure (the call then
 * fails with BF_ERR_OOM); release hands a pointer back once the work queued on
 * `hip_stream` before the call no longer needs it.  Both are called on the
 * thread that makes the library call, with `user` passed through; a caller can
 * route them to its framework's caching allocator (torch's, for instance). */
typedef struct bf_allocator {
  void* user;
  void* (*alloc)(void* user, size_t bytes, void* hip_stream);
  void (*release)(void* user, void* ptr, void* hip_stream);
} bf_allocator;

/* Create a context on HIP device `device` that orders its work on
 * `hip_stream` (a hipStream_t, NULL = the null stream).  alloc (copied; NULL =
 * the library's own stream-ordered pool, which keeps freed memory for reuse)
 * provides the memory of bands, systems and meshes.  The context owns
 * reusable device workspaces (from its pool) and a pinned host staging
 * buffer. */
bf_status bf_create(bf_ctx** out, int32_t device, void* hip_stream, const bf_allocator* alloc);
bf_status bf_destroy(bf_ctx* ctx);
/* Change the stream later calls are ordered on. */
bf_status bf_set_stream(bf_ctx* ctx, void* hip_stream);
/* Message of the last failure on this context ("" if none); owned by ctx. */
const char* bf_last_error(const bf_ctx* ctx);
/* Library version string, static storage. */
const char* bf_version(void);

/* ---------------------------------------------------------------- band */

/* Sec. 3.3-3.4, eq. (1), Algorithm 1 steps 1-2.  Fuses the T depth maps
 * depth_dev [T][H][W] with poses c2w_dev [T][3][4] into a coarse TSDF over the
 * whole grid (unit weight per view; a view counts when the projective distance
 * D - Z of the nearest pixel is >= -tau, and contributes min(D - Z, tau)),
 * then activates B = { v : W(v) > 0 and |TSDF(v)| <= band } in ascending
 * Morton order, builds the key -> index map (direct 4^3-block records) and the
 * 6-neighbour table.
 * flags: BF_BAND_KEEP_DENSE keeps the dense grid in the band object.
 * Writes *out (new band) and *n_out (host; synchronises).  Errors:
 * INVALID_ARG for bad sizes (G outside [1, 2048], T outside [0, 65535]) or
 * depth that is NaN, infinite or negative;
 * CAPACITY if the band exceeds 2^31 - 1 voxels; OOM; HIP. */
bf_status bf_build_band(bf_ctx* ctx, const bf_grid* grid, const bf_camera* cam, int32_t T,
                        const float* depth_dev, const double* c2w_dev, uint32_t flags,
                        bf_band** out, int64_t* n_out);
bf_status bf_band_view(const bf_band* band, bf_band_arrays* out);
bf_status bf_band_free(bf_ctx* ctx, bf_band* band);

/* ---------------------------------------------------------------- system */

/* Sec. 3.5-3.6, eqs. (3)-(5), (8)-(11), Algorithm 1 steps 3-4.  Voxel-centric
 * observation rows: each band voxel gets one observation per accepted view
 * (same acceptance as the TSDF), y = min(D - Z, tau) with weight 1/sigma^2.
 * Builds Lambda, b, the anchored right-hand side and diag(Q) =
 * Lambda + lambda deg + eps (+ lambda_b on the boundary); the off-diagonal
 * entries -lambda on band edges are implicit.  Writes *out.
 * Given the depth maps and poses the band was built from (the same device
 * arrays, T and camera, unchanged since), a screened band's per-cell view
 * masks let each voxel skip the views proved to observe no voxel of its 4^3
 * cell; the sums, taken in view order, are the same bits either way. */
bf_status bf_assemble(bf_ctx* ctx, const bf_band* band, const bf_camera* cam, int32_t T,
                      const float* depth_dev, const double* c2w_dev, const bf_noise* noise,
                      const bf_prior* prior, bf_system** out);

/* Sec. 3.5-3.6, eqs. (3)-(5), (10)-(11): the voxel-centric system sys with T
 * more views appended (depth_dev [T][H][W], c2w_dev [T][3][4], noise's pose
 * variances [T] for the new views).  Each band voxel continues its running
 * sums (Lambda, b and the feature statistics) over the new views in order, so
 * *out is, bit for bit, the system bf_assemble builds from all the views at
 * once (camera and prior as sys; the band must still be alive).  *out is a new
 * system (free with bf_system_free); sys is unchanged.  Errors: INVALID_ARG
 * for a trilinear system, T < 0, bad camera or NULL arrays; OOM; HIP. */
bf_status bf_assemble_more(bf_ctx* ctx, const bf_system* sys, const bf_camera* cam, int32_t T,
                           const float* depth_dev, const double* c2w_dev, const bf_noise* noise,
                           bf_system** out);

/* Sec. 3.2, eqs. (2)-(5), (7), (10)-(11): trilinear pixel-centric observation
 * rows (eq. 4, up to 8 non-zeros).  Every valid pixel (row, col) of view t
 * gives 2S+1 samples (S = samples_per_side, 0..15) along its camera ray at
 * camera depths z = D + s h, s = -S..S (eq. 2); y = clamp(D - z, -tau, tau)
 * (eq. 3, normal = viewing axis); the row holds the trilinear weights of the
 * sample point on the 8 surrounding voxel centres, and the sample is kept only
 * when all 8 are band voxels; weight 1/sigma^2 as in bf_assemble (eq. 5).
 * Q = A^T W A + lambda L + eps I (+ lambda_b on the boundary) is stored as
 * diag(Q) and 26 couplings per row, stored slot-major ([26][N], so the
 * rows of a wave read them coalesced): slot order of the offsets d in
 * {-1,0,1}^3 \ {0} by (dx+1) + 3(dy+1) + 9(dz+1) ascending, centre removed;
 * face slots include -lambda; absent voxels have nb26 = -1 and coupling 0.
 * FP64 results are reproducible bit for bit: samples are summed per 2x2x2
 * cell (the cube whose lowest voxel is the sample's floor corner) in
 * ascending sample id ((t H + row) W + col)(2S+1) + (s + S), and each voxel
 * sums its 8 cells in the order of its corner index q = dx + 2dy + 4dz inside
 * the cell.  The system works with bf_apply_Q, bf_pcg_solve and
 * bf_diag_estimate (without a log-variance start); bf_features, the warm
 * start and the batched solves reject it.  n_samples_out (host, may be NULL)
 * receives the kept sample count.  Synchronises.  Errors: INVALID_ARG (bad
 * sizes, S outside [0, 15], more samples than a 64-bit sort key holds), OOM,
 * HIP. */
bf_status bf_assemble_trilinear(bf_ctx* ctx, const bf_band* band, const bf_camera* cam, int32_t T,
                                const float* depth_dev, const double* c2w_dev, const bf_noise* noise,
                                const bf_prior* prior, int32_t samples_per_side, bf_system** out,
                                int64_t* n_samples_out);
bf_status bf_system_view(const bf_system* sys, bf_system_arrays* out);
bf_status bf_system_free(bf_ctx* ctx, bf_system* sys);

/* The (band voxel, view) pairs bf_assemble went through for sys (eqs. 3-5):
 * N T without the band's view masks, fewer with them (views the screen
 * proved to observe nothing of a voxel's cell are skipped), counted from the
 * band's masks, so the band must still exist.  For rates, not results.  *out
 * is a host int64.  Synchronises with the context's stream.  Errors:
 * INVALID_ARG (NULL argument, or a system not made by bf_assemble), HIP. */
bf_status bf_system_assembly_views(bf_ctx* ctx, const bf_system* sys, int64_t* out);

/* q_dev = Q p_dev for device vectors of N doubles (eq. 10). */
bf_status bf_apply_Q(bf_ctx* ctx, const bf_system* sys, const double* p_dev, double* q_dev);

/* ---------------------------------------------------------------- surface */

typedef struct bf_mesh bf_mesh;

typedef struct bf_mesh_arrays {
  int64_t n_vert, n_tri;
  const double* verts;     /* [n_vert][3] world positions (m) */
  const int32_t* tris;     /* [n_tri][3] vertex indices, normal (b-a)x(c-a) towards mu > iso */
} bf_mesh_arrays;

/* Algorithm 1 step 7: the iso-surface mu = iso of a field over the band
 * (mu_dev [N], e.g. the posterior mean) by marching tetrahedra, the
 * tetrahedral form of marching cubes.  A voxel is inside when mu < iso.  Each
 * cube of 8 band voxel centres is split into the 6 tetrahedra of the
 * Freudenthal split along its main diagonal (the split matches across cubes,
 * so the mesh is watertight inside the band).  Vertices lie on grid edges
 * from a band voxel v along one of the 7 directions {0,1}^3 \ 0 (x, y, z, xy,
 * xz, yz, xyz) to a band voxel with the other inside state, at
 * x_v + t (x_u - x_v), t = (mu_v - iso) / (mu_v - mu_u); they are numbered by
 * band index, then direction; triangles by cube (band index of its lowest
 * voxel), tetrahedron (axis orders 012, 021, 102, 120, 201, 210), position.
 * Writes *out (a new mesh; free with bf_mesh_free on this context) and the
 * host counts (may be NULL).  Synchronises.  Errors: INVALID_ARG, CAPACITY
 * (2^31 vertices or more), OOM, HIP. */
bf_status bf_extract_surface(bf_ctx* ctx, const bf_band* band, const double* mu_dev, double iso,
                             bf_mesh** out, int64_t* n_vert, int64_t* n_tri);
bf_status bf_mesh_view(const bf_mesh* mesh, bf_mesh_arrays* out);
bf_status bf_mesh_free(bf_ctx* ctx, bf_mesh* mesh);

/* Geometry metrics of Sec. 4.2 between predicted points P and ground-truth
 * points G (both [n][3] device arrays, m): with d(x, S) the distance to the
 * nearest point of S (exact, by brute force over all pairs),
 * chamfer = mean_P d(p,G)^2 + mean_G d(g,P)^2 (eq. 14), accuracy =
 * mean_P d(p,G), completeness = mean_G d(g,P), and per threshold thr[t]
 * (n_thr <= 8): precision = fraction of P with d < thr, recall = fraction of
 * G with d < thr, F = 2 P R / (P + R).  d_pred_dev [n_pred] and d_gt_dev
 * [n_gt] (may be NULL) receive the squared distances.  Synchronises. */
typedef struct bf_metrics {
  int64_t n_pred, n_gt;
  double chamfer, accuracy, completeness;
  int32_t n_thr;
  double thr[8], precision[8], recall[8], fscore[8];
} bf_metrics;
bf_status bf_surface_metrics(bf_ctx* ctx, const double* pred_dev, int64_t n_pred, const double* gt_dev,
                             int64_t n_gt, int32_t n_thr, const double* thr_host, bf_metrics* out,
                             double* d_pred_dev, double* d_gt_dev);

/* ---------------------------------------------------------------- solves */

/* Sec. 3.6, eq. (11), Algorithm 1 step 5: Jacobi-preconditioned CG for
 * Q x = rhs with rhs_dev [N] (NULL = the system's right-hand side h).  x_dev
 * [N] receives the posterior mean (and holds the start if opts->use_x0).
 * rep (host, may be NULL) is filled; synchronises.  Returns NOT_CONVERGED
 * (with x and report written) when max_iter is reached, BREAKDOWN when
 * p.Qp <= 0 or non-finite. */
bf_status bf_pcg_solve(bf_ctx* ctx, const bf_system* sys, const bf_solve_opts* opts,
                       const double* rhs_dev, double* x_dev, bf_solve_report* rep);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * solve as bf_pcg_solve, same kernels and results, with every temporary (the
 * CG vectors r, z, p, q, the float correction, block partials and the solver
 * state) in one static device array of BF_PCG_NOALLOC_BYTES per GPU.  That
 * array is loaded with the library's code object and held until the process
 * ends; its address is looked up once per device by bf_create.  The caller
 * still passes rhs and x.  The call allocates nothing (no device, pinned or
 * pooled memory, no events): the solver state is read back into host stack
 * memory, per-kernel timing records are not taken and rep->seconds is host
 * time.  Every call on one GPU shares that GPU's array, so calls that overlap
 * on one GPU (from several contexts, streams or threads) race; the array keeps
 * the last call's contents and each call initialises what it reads.
 * Errors: as bf_pcg_solve, plus CAPACITY when the system needs more scratch
 * than the array holds (bf_pcg_noalloc_max_n gives the largest N per
 * precision: about 1.67M voxels in FP64, 2.79M mixed). */
#define BF_PCG_NOALLOC_BYTES (64u << 20)
bf_status bf_pcg_solve_noalloc(bf_ctx* ctx, const bf_system* sys, const bf_solve_opts* opts,
                               const double* rhs_dev, double* x_dev, bf_solve_report* rep);
/* Largest band size bf_pcg_solve_noalloc accepts in the given precision. */
int64_t bf_pcg_noalloc_max_n(int32_t precision);

/* Sec. 3.7, eq. (12), Algorithm 1 step 6: s_dev [N] = (1/K) sum_k z_k * u_k
 * with Q u_k = z_k, all K probe solves run together as one block CG whose
 * columns keep their own alpha/beta and stop independently.  logvar_dev
 * [N] (NULL = none) is a predicted log of diag(Q^-1) * diag(Q); when given,
 * each probe solve starts from u = exp(logvar) z / diag.  Synchronises. */
bf_status bf_diag_estimate(bf_ctx* ctx, const bf_system* sys, const bf_probe_opts* opts,
                           const float* logvar_dev, double* s_dev, bf_solve_report* rep);

/* ---------------------------------------------------------------- NBV */

/* Sec. 3.8, eq. (13), Algorithm 1 step 8.  Scores n_cand candidate poses
 * cand_c2w_dev [n][3][4] by casting one ray per pixel of ray_cam through the
 * grid (voxel walk, lowest axis first on ties) and summing, over the band
 * voxels crossed up to and including the first with mu <= 0, the quantised
 * variance q_v = rint(s_v / max(s) * 2^32) (BF_UTILITY_SUM_VAR) or the
 * quantised expected reduction s_v^2 / (s_v + sigma(Z)^2) scaled the same way
 * (BF_UTILITY_VAR_REDUCTION, Z = the voxel's depth in the candidate view).
 * scores_dev [n] int64 receives the exact integer utilities; *best_host the
 * lowest index attaining the maximum (synchronises).  noise is used by the
 * variance-reduction utility only (may be NULL otherwise). */
bf_status bf_nbv_score(bf_ctx* ctx, const bf_band* band, const double* mu_dev,
                       const double* s_dev, int32_t n_cand, const double* cand_c2w_dev,
                       const bf_camera* ray_cam, int32_t utility, const bf_noise* noise,
                       int64_t* scores_dev, int32_t* best_host);

/* Sec. 3.8: the depth map [H][W] (float, device) that a sensor with camera
 * cam would return from pose c2w_dev [3][4], predicted from the mean mu_dev
 * [N]: pixel (row, col) walks the ray of bf_nbv_score's rays (direction
 * R ((col - cx)/fx, (row - cy)/fy, 1), voxel by voxel, lowest axis first on
 * ties) to the first band voxel with mu <= 0, and gets the camera-z depth of
 * that voxel's centre, (R e_z) . (x - t), rounded to float; 0 (no return)
 * when the ray leaves the grid first.  Stream-ordered.  Errors: INVALID_ARG
 * for NULL arrays or a bad camera; HIP. */
bf_status bf_predict_depth(bf_ctx* ctx, const bf_band* band, const double* mu_dev,
                           const double* c2w_dev, const bf_camera* cam, float* depth_dev);

/* Sec. 3.8, eq. (13) with the post-view variance:
 *   U(v) = sum over the band voxels with |mu| <= eps_band of (s_i - s'_i),
 * where s' = diag(Q'^-1) and Q' is the precision once the view from candidate
 * v has been fused.  For each of the n_sel candidates cand_idx_host[i] (into
 * cand_c2w_dev [n_cand][3][4]) the view of sensor camera `cam` is predicted
 * (bf_predict_depth), appended to sys as one more view (bf_assemble_more with
 * noise's a, c, z0 and sigma2_model; the planned pose is taken as exact, no
 * pose variance), and s' is estimated by bf_diag_estimate with opts.  Pass
 * the seed s was estimated with, so s and s' share the probes and the
 * difference does not carry their independent noise.  warm != 0 starts the
 * probe solves from u0 = z clamp(s diag', 1e-3, 1e3) / diag' (a start no
 * better than zero is dropped per column, as in bf_diag_estimate).
 * util_host [n_sel] receives U; *best_host the candidate index (from
 * cand_idx_host) with the largest U, the first on ties.  Optional: s_post_dev
 * [n_sel][N] receives each s', reps_host [n_sel] each solve's report.
 * Synchronises.  Errors: INVALID_ARG (trilinear system, eps_band < 0, an
 * index outside [0, n_cand), NULL arrays), the errors of bf_diag_estimate. */
bf_status bf_nbv_postview(bf_ctx* ctx, const bf_system* sys, const double* mu_dev, const double* s_dev,
                          int32_t n_cand, const double* cand_c2w_dev, int32_t n_sel,
                          const int32_t* cand_idx_host, const bf_camera* cam, const bf_noise* noise,
                          const bf_probe_opts* opts, double eps_band, int32_t warm, double* util_host,
                          int32_t* best_host, double* s_post_dev, bf_solve_report* reps_host);

/* Voxel visits of the plain Amanatides-Woo walk summed over every ray of the
 * last bf_nbv_score call on ctx (voxels visited, plus voxels skipped by the
 * exact empty-space jumps, which the plain walk would have visited): the
 * "DDA steps" of that call.  Host only; valid after bf_nbv_score returned. */
bf_status bf_nbv_walk_steps(bf_ctx* ctx, int64_t* steps);

/* ---------------------------------------------------------------- batched solves */
/* Many systems (scenes of uneven band size) solved together: the work list is
 * every system's row tiles in the schedule's order.  Persistent: one
 * cooperative launch whose co-resident workgroups walk the list phase by
 * phase and meet at grid barriers between CG phases.  Phased: one launch per
 * CG phase over the whole list.  Every system and probe column keeps its own
 * scalars and stopping test, and converged systems leave the work list.
 * Results equal the single-system calls up to the order of the dot-product
 * reductions. */
enum { BF_ORDER_SCENE_MAJOR = 0, BF_ORDER_INTERLEAVED = 1, BF_ORDER_LARGEST_FIRST = 2 };
typedef struct bf_schedule {
  int32_t rows_per_tile;  /* band rows per work item, 16..4096 */
  int32_t blocks_per_cu;  /* workgroups per CU, 0..16 (persistent: 0 = as many as fit;
                             phased: 0 = 4) */
  int32_t order;          /* BF_ORDER_* tile order across systems */
  int32_t xcd_aware;      /* 1: contiguous runs of tiles stay on one XCD's workgroups */
  int32_t persistent;     /* 1: one cooperative launch with grid barriers (probe solves
                             only); 0: one launch per CG phase, host polls convergence */
} bf_schedule;

/* Hutchinson probes (as bf_diag_estimate, no warm start) for n_sys systems;
 * s_dev[i] receives system i's estimate, reps[i] (host, may be NULL) its
 * report.  sched NULL = a default schedule.  Synchronises. */
bf_status bf_diag_estimate_batched(bf_ctx* ctx, const bf_system* const* systems, int32_t n_sys,
                                   const bf_probe_opts* opts, const bf_schedule* sched,
                                   double* const* s_dev, bf_solve_report* reps);
/* Posterior means (as bf_pcg_solve from x = 0 with each system's rhs).  Runs
 * phased only: a schedule with persistent = 1 is rejected (BF_ERR_INVALID_ARG). */
bf_status bf_pcg_solve_batched(bf_ctx* ctx, const bf_system* const* systems, int32_t n_sys,
                               const bf_solve_opts* opts, const bf_schedule* sched,
                               double* const* x_dev, bf_solve_report* reps);
/* Times every candidate schedule (launch kind x rows per tile x blocks per CU
 * x order x XCD mapping) on the batched probe solve and returns the fastest in *best;
 * json (host, may be NULL) receives every candidate's time as a JSON array. */
bf_status bf_autotune_batch(bf_ctx* ctx, const bf_system* const* systems, int32_t n_sys,
                            const bf_probe_opts* opts, double* const* s_dev, bf_schedule* best,
                            char* json, size_t json_len);

/* ---------------------------------------------------------------- learned warm start */
/* The paper names learned priors as future work (Sec. 6-7).  This extension
 * proposes starting points only; every solve still runs CG to its tolerance.
 * Network: 12 features -> 64 -> 64 -> 64 -> 2 with SiLU, BF16 weights on the
 * matrix cores with FP32 accumulation.  params_dev is a float32 device vector
 * of BF_MLP_PARAMS values: W1[64][12] b1[64] W2[64][64] b2[64] W3[64][64]
 * b3[64] W4[2][64] b4[2] (BF_MLP_TRAIN trainable values), then the fixed
 * input standardisation in_mean[12] in_std[12] and output scaling
 * out_mean[2] out_std[2].  Outputs: o0 = (mu - rhs/diag) / h (the mean's
 * correction to the Jacobi estimate, in voxels) and o1 = log(s * diag) (the
 * variance relative to 1/diag). */
enum { BF_MLP_TRAIN = 9282, BF_MLP_PARAMS = 9310 };

/* feat_dev [N][12] float: TSDF/h, log(1+W), deg/6, n_obs/T, mean y/h,
 * var y/h^2, mean sigma/h, min sigma/h, log(1 + Lambda h^2), and the TSDF
 * central differences along x, y, z over 2h (own value where a band
 * neighbour is absent). */
bf_status bf_features(bf_ctx* ctx, const bf_system* sys, float* feat_dev);
/* out_dev [n][2] = network outputs (physical units) for feat_dev [n][12]. */
bf_status bf_mlp_forward(bf_ctx* ctx, const float* params_dev, const float* feat_dev, int64_t n,
                         float* out_dev);
/* Features -> network -> x0_dev [N] = rhs/diag + h*o0 (mean start) and
 * logvar_dev [N] = o1 (probe start for bf_diag_estimate); either may be NULL.
 * feat_dev [N][12] as bf_features writes it, or NULL: the features are then
 * computed in the same pass (the same values), without the [N][12] array. */
bf_status bf_warm_start(bf_ctx* ctx, const bf_system* sys, const float* params_dev,
                        const float* feat_dev, double* x0_dev, float* logvar_dev);
/* Training targets of the network from the method's own solves of sys:
 * target_dev [N][2] float = ((mu - rhs/diag) / h, log(clamp(s * diag,
 * clamp_lo, clamp_hi))), with mu_dev [N] a converged mean (eq. 11) and s_dev
 * [N] a Hutchinson estimate of diag(Q^-1) (eq. 12); the clamp keeps the log
 * finite where a few-probe estimate is not positive.  Voxel-centric systems;
 * 0 < clamp_lo <= clamp_hi.  Asynchronous. */
bf_status bf_warm_start_targets(bf_ctx* ctx, const bf_system* sys, const double* mu_dev, const double* s_dev,
                                double clamp_lo, double clamp_hi, float* target_dev);
/* Gradient of L = 1/(2M) sum_m |o_m - t_m|^2 (outputs and targets in the
 * standardised units (t - out_mean) / out_std) over the batch rows idx_dev[M]
 * of feat_dev [nrows][12] / target_dev [nrows][2]; rows outside [0, nrows)
 * are skipped.  grad_dev [BF_MLP_TRAIN]; loss_dev (device float, may be NULL). */
bf_status bf_mlp_grad(bf_ctx* ctx, const float* params_dev, const float* feat_dev,
                      const float* target_dev, int64_t nrows, const int32_t* idx_dev, int64_t M,
                      float* grad_dev, float* loss_dev);
/* One Adam step (Kingma & Ba 2015, bias-corrected, step >= 1) on the
 * trainable part of params_dev with moment vectors m_dev, v_dev. */
bf_status bf_adam_step(bf_ctx* ctx, float* params_dev, float* m_dev, float* v_dev,
                       const float* grad_dev, int32_t step, float lr, float beta1, float beta2,
                       float eps);

/* ---------------------------------------------------------------- instrumentation */

/* Per-kernel device time, accumulated while timing is on: the library
 * brackets each hot kernel launch with HIP events on the context stream. */
typedef struct bf_kernel_time {
  char name[48];
  int64_t launches;
  double total_ms;
} bf_kernel_time;

bf_status bf_set_timing(bf_ctx* ctx, int32_t enable);
/* Synchronises, aggregates the recorded launches by kernel name into out
 * [cap] (host), writes the number of names to *n_out and clears the record. */
bf_status bf_get_timings(bf_ctx* ctx, bf_kernel_time* out, int32_t cap, int32_t* n_out);

#ifdef __cplusplus
}
#endif
#endif /* BF_H */
