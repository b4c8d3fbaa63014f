/*
 * Plain FP64 CPU oracle for the BayesFusion-SDF narrow-band solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header or constant table with
 * the GPU library.
 *
 * Every routine is a slow, scalar, obviously-correct statement of one step of
 * the method (Sec. 3 of the paper); each function below cites the passage it
 * follows.  Layouts:
 *   depth  float  [T][H][W], camera-z depth in metres, 0 = no return
 *   c2w    double [T][3][4], row-major camera-to-world [R | t]
 *   dense grid arrays: linear index (k*G + j)*G + i
 *   band arrays: in ascending Morton-key order
 *   nbr    int32  [N][6] neighbour band index in the order -x,+x,-y,+y,-z,+z, -1 if absent
 */
#ifndef BF_ORACLE_H
#define BF_ORACLE_H
#include <stdint.h>

typedef struct {
  int32_t G;          /* voxels per axis */
  double h;           /* voxel edge (m) */
  double origin[3];   /* world position of the grid's low corner */
  double tau;         /* truncation distance (m) */
  double band;        /* band half-width (m): |TSDF| <= band */
} orc_grid;

typedef struct {
  int32_t width, height;
  double fx, fy, cx, cy;
} orc_cam;

typedef struct {
  double a, c, z0;            /* sigma_depth(D) = a + c (D - z0)^2 */
  const double* sigma2_pose;  /* [T] or NULL (= 0) */
  double sigma2_model;
} orc_noise;

typedef struct {
  int32_t iters;
  int32_t status;      /* 0 ok, 4 breakdown, 5 not converged */
  double rel_res;      /* ||b - Q x|| / ||b|| recomputed at exit */
} orc_report;

void orc_set_threads(int32_t n);
int32_t orc_max_threads(void);
uint64_t orc_morton_encode(int32_t i, int32_t j, int32_t k);
void orc_morton_decode(uint64_t key, int32_t* i, int32_t* j, int32_t* k);

int orc_observe(const orc_grid* g, const orc_cam* cam, const float* depth_t, const double* c2w_t,
                int32_t i, int32_t j, int32_t k, double* D_out, double* Z_out);
void orc_tsdf_voxel(const orc_grid* g, const orc_cam* cam, int32_t T, const float* depth,
                    const double* c2w, int32_t i, int32_t j, int32_t k, double* tsdf, int32_t* w);
void orc_tsdf_dense(const orc_grid* g, const orc_cam* cam, int32_t T, const float* depth,
                    const double* c2w, double* tsdf, int32_t* w);
void orc_tsdf_points(const orc_grid* g, const orc_cam* cam, int32_t T, const float* depth,
                     const double* c2w, int64_t n, const int32_t* ijk, double* tsdf, int32_t* w);
int64_t orc_band(const orc_grid* g, const double* tsdf_dense, const int32_t* w_dense, int64_t cap,
                 uint64_t* keys, double* tsdf, int32_t* w);
void orc_neighbours(int32_t G, const uint64_t* keys, int64_t N, int32_t* nbr, int32_t* deg);

void orc_assemble(const orc_grid* g, const orc_cam* cam, int32_t T, const float* depth,
                  const double* c2w, const orc_noise* nz, const uint64_t* keys, int64_t N,
                  double* Lambda, double* b, double* acc /* [N][5] or NULL */);
void orc_precision_diag(int64_t N, const double* Lambda, const int32_t* deg, double lam,
                        double eps, double lam_b, double* diag);
void orc_anchor_rhs(int64_t N, const double* b, const int32_t* deg, const double* tsdf,
                    double lam_b, double* h_out);

void orc_apply_Q(int64_t N, const int32_t* nbr, const double* diag, double lam, const double* p,
                 double* q);
void orc_pcg(int64_t N, const int32_t* nbr, const double* diag, double lam, const double* rhs,
             const double* x0, double tol, int32_t max_iter, double* x, orc_report* rep);

uint64_t orc_splitmix_output(uint64_t start, uint64_t n);
int32_t orc_probe_sign(uint64_t seed, int32_t k, int64_t i);
void orc_hutchinson(int64_t N, const int32_t* nbr, const double* diag, double lam, int32_t K,
                    uint64_t seed, double tol, int32_t max_iter, double* s_out,
                    int32_t* iters_out /* [K] or NULL */);

typedef struct {
  int32_t utility;    /* 0: sum of quantised variance, 1: expected variance reduction */
  double a, c, z0;    /* sensor model sigma(Z) = a + c (Z - z0)^2 (utility 1) */
  const double* s;    /* [N] variance (utility 1) */
  double smax;        /* max(0, max s) (utility 1) */
} orc_utility;

void orc_quantize_variance(int64_t N, const double* s, int64_t* q);
void orc_pred_depth(const orc_grid* g, const orc_cam* cam, const uint64_t* keys, int64_t N,
                    const double* mu, const double* P, float* depth);
int64_t orc_nbv_ray_u(const orc_grid* g, const uint64_t* keys, int64_t N, const double* mu,
                      const int64_t* q, const orc_utility* u, const double* P, const double* o,
                      const double* d, int64_t* steps_out);
int64_t orc_nbv_candidate_u(const orc_grid* g, const orc_cam* cam, const uint64_t* keys,
                            int64_t N, const double* mu, const int64_t* q, const orc_utility* u,
                            const double* P);
int64_t orc_nbv_ray(const orc_grid* g, const uint64_t* keys, int64_t N, const double* mu,
                    const int64_t* q, const double* o, const double* d, int64_t* steps_out);
int64_t orc_nbv_candidate(const orc_grid* g, const orc_cam* ray_cam, const uint64_t* keys,
                          int64_t N, const double* mu, const int64_t* q, const double* c2w);
/* Voxels visited by the walks of every ray of one candidate. */
int64_t orc_nbv_candidate_steps(const orc_grid* g, const orc_cam* ray_cam, const uint64_t* keys, int64_t N,
                                const double* mu, const int64_t* q, const double* P);
void orc_nbv_scores(const orc_grid* g, const orc_cam* cam, const uint64_t* keys, int64_t N,
                    const double* mu, const int64_t* q, const orc_utility* u, int32_t n,
                    const double* c2w, int64_t* scores, int64_t* steps /* [n] or NULL */);
int32_t orc_nbv_argmax(int32_t n, const int64_t* scores);
void orc_features(int64_t N, int32_t T, double h, const double* tsdf, const int32_t* w,
                  const int32_t* nbr, const int32_t* deg, const double* Lambda, const double* acc,
                  double* feat);


/* Trilinear observation rows (trilinear.c; Sec. 3.2, eqs. 2-5, 7, 10-12). */
int32_t orc_tri_slot(int32_t dx, int32_t dy, int32_t dz);
int orc_tri_sample(const orc_grid* g, const orc_cam* cam, const float* depth_t, const double* P,
                   const orc_noise* nz, double sigma2_pose_t, int32_t row, int32_t col, int32_t s,
                   int32_t* base, double* a, double* y, double* wv);
int64_t orc_tri_sample_list(const orc_grid* g, const orc_cam* cam, int32_t T, const float* depth,
                            const double* c2w, const orc_noise* nz, int32_t S, const uint64_t* keys, int64_t N,
                            int64_t cap, int32_t* base, double* a, double* y, double* wv, int32_t* tcrs);
int64_t orc_tri_assemble(const orc_grid* g, const orc_cam* cam, int32_t T, const float* depth,
                         const double* c2w, const orc_noise* nz, int32_t S, const uint64_t* keys, int64_t N,
                         const int32_t* deg, const double* tsdf, double lam, double eps, double lam_b,
                         double* Lambda, double* b, double* rhs, double* diag, double* off, int32_t* nb26,
                         int64_t* ncells_out);
void orc_apply_Q27(int64_t N, const double* diag, const double* off, const int32_t* nb26, const double* p,
                   double* q);
void orc_pcg27(int64_t N, const double* diag, const double* off, const int32_t* nb26, const double* rhs,
               const double* x0, double tol, int32_t max_iter, double* x, orc_report* rep);
void orc_hutchinson27(int64_t N, const double* diag, const double* off, const int32_t* nb26, int32_t K,
                      uint64_t seed, double tol, int32_t max_iter, double* s_out, int32_t* iters_out);

/* Surface extraction and geometry-metric distances (surface.c; Alg. 1 step 7, eq. 14). */
int32_t orc_surf_dir(int32_t dx, int32_t dy, int32_t dz);
void orc_extract_surface(const orc_grid* g, const uint64_t* keys, int64_t N, const double* mu, double iso,
                         int64_t cap_v, int64_t cap_t, double* verts, int32_t* tris, int64_t* nv, int64_t* nt);
void orc_nn_dist2(const double* a, int64_t na, const double* b, int64_t nb, double* d_out);

#endif
