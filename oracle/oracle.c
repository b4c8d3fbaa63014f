/*
 * Plain FP64 CPU oracle for the BayesFusion-SDF narrow-band solve.
 * TEST INFRASTRUCTURE ONLY: see oracle.h.  Built by gcc with
 * -O2 -fno-fast-math -ffp-contract=off so every + - * / is a separately
 * rounded IEEE double operation in the order written.
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Threads of the oracle's parallel loops (results do not depend on it). */
void orc_set_threads(int32_t n) { omp_set_num_threads(n > 0 ? n : 1); }
int32_t orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* Morton keys.  The paper stores the band in a sparse voxel structure  */
/* (Sec. 3.4, "hashed blocks"); the band is ordered by the 64-bit key   */
/* whose bit 3b is bit b of i, bit 3b+1 bit b of j, bit 3b+2 bit b of k.*/
/* ------------------------------------------------------------------ */
uint64_t orc_morton_encode(int32_t i, int32_t j, int32_t k) {
  uint64_t key = 0;
  for (int b = 0; b < 21; ++b) {
    key |= (uint64_t)((i >> b) & 1) << (3 * b);
    key |= (uint64_t)((j >> b) & 1) << (3 * b + 1);
    key |= (uint64_t)((k >> b) & 1) << (3 * b + 2);
  }
  return key;
}

void orc_morton_decode(uint64_t key, int32_t* i, int32_t* j, int32_t* k) {
  int32_t a = 0, bb = 0, c = 0;
  for (int b = 0; b < 21; ++b) {
    a |= (int32_t)((key >> (3 * b)) & 1) << b;
    bb |= (int32_t)((key >> (3 * b + 1)) & 1) << b;
    c |= (int32_t)((key >> (3 * b + 2)) & 1) << b;
  }
  *i = a;
  *j = bb;
  *k = c;
}

/* ------------------------------------------------------------------ */
/* Projective observation of one voxel centre in one view (eqs. 2-3).   */
/* The voxel centre x = origin + (i + 1/2) h is moved into the camera   */
/* frame with the inverse pose, x_c = R^T (x - t), and projected with   */
/* the pinhole K to the nearest pixel.  Returns 1 and the measured depth*/
/* D and the voxel's camera depth Z when the pixel is inside the image  */
/* and holds a return; the projective signed distance along the viewing */
/* axis is then D - Z.                                                  */
/* ------------------------------------------------------------------ */
int orc_observe(const orc_grid* g, const orc_cam* cam, const float* depth_t, const double* P,
                int32_t i, int32_t j, int32_t k, double* D_out, double* Z_out) {
  double x = g->origin[0] + ((double)i + 0.5) * g->h;
  double y = g->origin[1] + ((double)j + 0.5) * g->h;
  double z = g->origin[2] + ((double)k + 0.5) * g->h;
  double dx = x - P[3];
  double dy = y - P[7];
  double dz = z - P[11];
  /* column a of R is (P[a], P[4+a], P[8+a]); x_c[a] = column_a . (x - t) */
  double X = (P[0] * dx + P[4] * dy) + P[8] * dz;
  double Y = (P[1] * dx + P[5] * dy) + P[9] * dz;
  double Z = (P[2] * dx + P[6] * dy) + P[10] * dz;
  if (!(Z > 0.0)) return 0;
  double u = (cam->fx * X) / Z + cam->cx;
  double v = (cam->fy * Y) / Z + cam->cy;
  double cu = u + 0.5;   /* nearest pixel: floor(u + 1/2) */
  double cv = v + 0.5;
  if (!(cu >= 0.0 && cu < (double)cam->width)) return 0;
  if (!(cv >= 0.0 && cv < (double)cam->height)) return 0;
  int32_t col = (int32_t)floor(cu);
  int32_t row = (int32_t)floor(cv);
  double D = (double)depth_t[(int64_t)row * cam->width + col];
  if (!(D > 0.0) || !isfinite(D)) return 0;
  *D_out = D;
  *Z_out = Z;
  return 1;
}

/* ------------------------------------------------------------------ */
/* Coarse TSDF bootstrap (Sec. 3.3): weighted-average fusion with unit  */
/* weight per accepted view, views in ascending order.  A view is       */
/* accepted when the projective distance d = D - Z is >= -tau (voxels   */
/* further behind the surface are occluded); d is truncated to tau.     */
/* TSDF = (sum of truncated d) / W.                                     */
/* ------------------------------------------------------------------ */
void orc_tsdf_voxel(const orc_grid* g, const orc_cam* cam, int32_t T, const float* depth,
                    const double* c2w, int32_t i, int32_t j, int32_t k, double* tsdf,
                    int32_t* w) {
  double S = 0.0;
  int32_t W = 0;
  int64_t plane = (int64_t)cam->width * cam->height;
  for (int32_t t = 0; t < T; ++t) {
    double D, Z;
    if (!orc_observe(g, cam, depth + t * plane, c2w + 12 * t, i, j, k, &D, &Z)) continue;
    double d = D - Z;
    if (d < -g->tau) continue;
    double yv = d < g->tau ? d : g->tau;
    S = S + yv;
    W = W + 1;
  }
  *w = W;
  *tsdf = W > 0 ? S / (double)W : 0.0;
}

void orc_tsdf_dense(const orc_grid* g, const orc_cam* cam, int32_t T, const float* depth,
                    const double* c2w, double* tsdf, int32_t* w) {
  int32_t G = g->G;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t k = 0; k < G; ++k)
    for (int32_t j = 0; j < G; ++j)
      for (int32_t i = 0; i < G; ++i) {
        int64_t lin = ((int64_t)k * G + j) * G + i;
        orc_tsdf_voxel(g, cam, T, depth, c2w, i, j, k, &tsdf[lin], &w[lin]);
      }
}

/* Coarse TSDF of a list of voxels ijk [n][3] (voxels in parallel). */
void orc_tsdf_points(const orc_grid* g, const orc_cam* cam, int32_t T, const float* depth,
                     const double* c2w, int64_t n, const int32_t* ijk, double* tsdf, int32_t* w) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t p = 0; p < n; ++p)
    orc_tsdf_voxel(g, cam, T, depth, c2w, ijk[3 * p], ijk[3 * p + 1], ijk[3 * p + 2], &tsdf[p], &w[p]);
}

/* ------------------------------------------------------------------ */
/* Narrow-band activation, eq. (1): B = { v : W(v) > 0, |TSDF(v)| <= band }.*/
/* The band is listed in ascending Morton key (sorted with qsort).      */
/* ------------------------------------------------------------------ */
typedef struct {
  uint64_t key;
  double tsdf;
  int32_t w;
} orc_entry;

static int cmp_entry(const void* a, const void* b) {
  uint64_t ka = ((const orc_entry*)a)->key, kb = ((const orc_entry*)b)->key;
  return ka < kb ? -1 : (ka > kb ? 1 : 0);
}

int64_t orc_band(const orc_grid* g, const double* tsdf_dense, const int32_t* w_dense, int64_t cap,
                 uint64_t* keys, double* tsdf, int32_t* w) {
  int32_t G = g->G;
  int64_t total = (int64_t)G * G * G;
  int64_t n = 0;
  for (int64_t lin = 0; lin < total; ++lin)
    if (w_dense[lin] > 0 && fabs(tsdf_dense[lin]) <= g->band) ++n;
  if (keys == NULL || n > cap) return n;
  orc_entry* e = (orc_entry*)malloc(sizeof(orc_entry) * (size_t)(n > 0 ? n : 1));
  int64_t m = 0;
  for (int32_t k = 0; k < G; ++k)
    for (int32_t j = 0; j < G; ++j)
      for (int32_t i = 0; i < G; ++i) {
        int64_t lin = ((int64_t)k * G + j) * G + i;
        if (w_dense[lin] > 0 && fabs(tsdf_dense[lin]) <= g->band) {
          e[m].key = orc_morton_encode(i, j, k);
          e[m].tsdf = tsdf_dense[lin];
          e[m].w = w_dense[lin];
          ++m;
        }
      }
  qsort(e, (size_t)n, sizeof(orc_entry), cmp_entry);
  for (int64_t q = 0; q < n; ++q) {
    keys[q] = e[q].key;
    tsdf[q] = e[q].tsdf;
    w[q] = e[q].w;
  }
  free(e);
  return n;
}

/* ------------------------------------------------------------------ */
/* 6-neighbour connectivity of the band (Sec. 3.4): binary search of the */
/* sorted keys.  Edges only join band voxels (induced subgraph).        */
/* ------------------------------------------------------------------ */
static int64_t find_key(const uint64_t* keys, int64_t N, uint64_t key) {
  int64_t lo = 0, hi = N - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (keys[mid] == key) return mid;
    if (keys[mid] < key) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

void orc_neighbours(int32_t G, const uint64_t* keys, int64_t N, int32_t* nbr, int32_t* deg) {
  static const int off[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < N; ++v) {
    int32_t i, j, k;
    orc_morton_decode(keys[v], &i, &j, &k);
    int32_t dcount = 0;
    for (int s = 0; s < 6; ++s) {
      int32_t a = i + off[s][0], b = j + off[s][1], c = k + off[s][2];
      int64_t idx = -1;
      if (a >= 0 && a < G && b >= 0 && b < G && c >= 0 && c < G)
        idx = find_key(keys, N, orc_morton_encode(a, b, c));
      nbr[v * 6 + s] = (int32_t)idx;
      if (idx >= 0) ++dcount;
    }
    deg[v] = dcount;
  }
}

/* ------------------------------------------------------------------ */
/* Observation assembly (eqs. 3-5, 8-11) with voxel-centric rows a_i =  */
/* e_v: one observation per (band voxel, accepted view), with           */
/* y = min(D - Z, tau) and variance sigma^2 = sigma_depth(D)^2 +        */
/* sigma_pose(t)^2 + sigma_model^2.  Then A^T W A = diag(Lambda) and    */
/* A^T W y = b with Lambda_v = sum w, b_v = sum w y, w = 1/sigma^2.     */
/* acc (optional) collects per-voxel statistics [n, sum y, sum y^2,     */
/* sum sigma, min sigma] for the learned warm start's features.         */
/* ------------------------------------------------------------------ */
void orc_assemble(const orc_grid* g, const orc_cam* cam, int32_t T, const float* depth,
                  const double* c2w, const orc_noise* nz, const uint64_t* keys, int64_t N,
                  double* Lambda, double* b, double* acc) {
  int64_t plane = (int64_t)cam->width * cam->height;
  /* voxels are independent; each one's sums run over t in ascending order */
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < N; ++v) {
    int32_t i, j, k;
    orc_morton_decode(keys[v], &i, &j, &k);
    double L = 0.0, B = 0.0, n = 0.0, sy = 0.0, syy = 0.0, ss = 0.0, smin = INFINITY;
    for (int32_t t = 0; t < T; ++t) {
      double D, Z;
      if (!orc_observe(g, cam, depth + t * plane, c2w + 12 * t, i, j, k, &D, &Z)) continue;
      double d = D - Z;
      if (d < -g->tau) continue;
      double yv = d < g->tau ? d : g->tau;
      double e = D - nz->z0;
      double sd = nz->a + nz->c * (e * e);
      double var = sd * sd + (nz->sigma2_pose ? nz->sigma2_pose[t] : 0.0);
      var = var + nz->sigma2_model;
      double wv = 1.0 / var;
      L = L + wv;
      B = B + wv * yv;
      n = n + 1.0;
      sy = sy + yv;
      syy = syy + yv * yv;
      ss = ss + sd;
      if (sd < smin) smin = sd;
    }
    Lambda[v] = L;
    b[v] = B;
    if (acc) {
      acc[v * 5 + 0] = n;
      acc[v * 5 + 1] = sy;
      acc[v * 5 + 2] = syy;
      acc[v * 5 + 3] = ss;
      acc[v * 5 + 4] = n > 0.0 ? smin : 0.0;
    }
  }
}

/* ------------------------------------------------------------------ */
/* Posterior precision diagonal, eqs. (7) and (10):                     */
/* Q = diag(Lambda) + lam L + eps I (+ lam_b on the band boundary, the  */
/* voxels with fewer than 6 band neighbours).  L = deg - adjacency, so  */
/* Q_vv = Lambda_v + lam deg_v + eps and Q_uv = -lam on each band edge. */
/* ------------------------------------------------------------------ */
void orc_precision_diag(int64_t N, const double* Lambda, const int32_t* deg, double lam,
                        double eps, double lam_b, double* diag) {
  for (int64_t v = 0; v < N; ++v) {
    double d = Lambda[v] + lam * (double)deg[v];
    d = d + eps;
    if (lam_b != 0.0 && deg[v] < 6) d = d + lam_b;
    diag[v] = d;
  }
}

/* Right-hand side h = A^T W y + b0 of eq. (11); b0 = lam_b * TSDF on the boundary. */
void orc_anchor_rhs(int64_t N, const double* b, const int32_t* deg, const double* tsdf,
                    double lam_b, double* h_out) {
  for (int64_t v = 0; v < N; ++v) {
    double h = b[v];
    if (lam_b != 0.0 && deg[v] < 6) h = h + lam_b * tsdf[v];
    h_out[v] = h;
  }
}

/* q = Q p with Q_vv = diag_v and Q_uv = -lam on band edges. */
void orc_apply_Q(int64_t N, const int32_t* nbr, const double* diag, double lam, const double* p,
                 double* q) {
  for (int64_t v = 0; v < N; ++v) {
    double s = 0.0;
    for (int t = 0; t < 6; ++t) {
      int32_t u = nbr[v * 6 + t];
      if (u >= 0) s = s + p[u];
    }
    q[v] = diag[v] * p[v] - lam * s;
  }
}

static double dot(int64_t N, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t v = 0; v < N; ++v) s = s + a[v] * b[v];
  return s;
}

/* ------------------------------------------------------------------ */
/* MAP mean (eq. 11, Sec. 3.6): Jacobi-preconditioned conjugate         */
/* gradients on Q mu = rhs.  Stops when ||r|| <= tol ||rhs||, confirmed */
/* with a recomputed residual rhs - Q x (a stale recursive residual is  */
/* replaced and the iteration continues).                               */
/* ------------------------------------------------------------------ */
void orc_pcg(int64_t N, const int32_t* nbr, const double* diag, double lam, const double* rhs,
             const double* x0, double tol, int32_t max_iter, double* x, orc_report* rep) {
  double* r = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  double* z = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  double* p = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  double* q = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  rep->iters = 0;
  rep->status = 0;
  rep->rel_res = 0.0;
  double bnorm = sqrt(dot(N, rhs, rhs));
  if (bnorm == 0.0) {
    for (int64_t v = 0; v < N; ++v) x[v] = 0.0;
    goto done;
  }
  for (int64_t v = 0; v < N; ++v) x[v] = x0 ? x0[v] : 0.0;
  orc_apply_Q(N, nbr, diag, lam, x, q);
  for (int64_t v = 0; v < N; ++v) r[v] = rhs[v] - q[v];
  if (sqrt(dot(N, r, r)) <= tol * bnorm) goto done;
  for (int64_t v = 0; v < N; ++v) {
    z[v] = r[v] / diag[v];
    p[v] = z[v];
  }
  double rho = dot(N, r, z);
  rep->status = 5;
  for (int32_t it = 1; it <= max_iter; ++it) {
    orc_apply_Q(N, nbr, diag, lam, p, q);
    double pq = dot(N, p, q);
    if (!(pq > 0.0) || !isfinite(pq)) {
      rep->status = 4;
      rep->iters = it;
      break;
    }
    double alpha = rho / pq;
    for (int64_t v = 0; v < N; ++v) {
      x[v] = x[v] + alpha * p[v];
      r[v] = r[v] - alpha * q[v];
    }
    rep->iters = it;
    if (sqrt(dot(N, r, r)) <= tol * bnorm) {
      orc_apply_Q(N, nbr, diag, lam, x, q);
      for (int64_t v = 0; v < N; ++v) r[v] = rhs[v] - q[v];
      if (sqrt(dot(N, r, r)) <= tol * bnorm) {
        rep->status = 0;
        break;
      }
    }
    for (int64_t v = 0; v < N; ++v) z[v] = r[v] / diag[v];
    double rho_new = dot(N, r, z);
    double beta = rho_new / rho;
    rho = rho_new;
    for (int64_t v = 0; v < N; ++v) p[v] = z[v] + beta * p[v];
  }
done:
  if (bnorm > 0.0) {
    orc_apply_Q(N, nbr, diag, lam, x, q);
    for (int64_t v = 0; v < N; ++v) r[v] = rhs[v] - q[v];
    rep->rel_res = sqrt(dot(N, r, r)) / bnorm;
  }
  free(r);
  free(z);
  free(p);
  free(q);
}

/* ------------------------------------------------------------------ */
/* Rademacher probes for eq. (12).  The paper does not fix a generator; */
/* z_k[i] is taken from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014):  */
/* with next(s): s += 0x9E3779B97F4A7C15, return mix(s), the probe seed */
/* u_k is output k (0-based) of the generator started at `seed`, and    */
/* z_k[i] = -1 if the top bit of output i of the generator started at   */
/* u_k is set, else +1.                                                 */
/* ------------------------------------------------------------------ */
static uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t orc_splitmix_output(uint64_t start, uint64_t n) {
  uint64_t s = start;
  /* stepping n+1 times from `start`, written as a multiply */
  s = s + (n + 1) * 0x9E3779B97F4A7C15ULL;
  return splitmix_mix(s);
}

int32_t orc_probe_sign(uint64_t seed, int32_t k, int64_t i) {
  uint64_t u = orc_splitmix_output(seed, (uint64_t)k);
  uint64_t v = orc_splitmix_output(u, (uint64_t)i);
  return (v >> 63) ? -1 : 1;
}

/* ------------------------------------------------------------------ */
/* Hutchinson / Bekas diagonal estimator, eq. (12): solve Q u_k = z_k   */
/* for each probe with the same PCG and average z_k * u_k.              */
/* ------------------------------------------------------------------ */
/* The K probe solves are independent and run in parallel (each one is the  */
/* serial PCG above); their products z_k * u_k are then summed per voxel in */
/* ascending k, so the result does not depend on the thread count.          */
void orc_hutchinson(int64_t N, const int32_t* nbr, const double* diag, double lam, int32_t K,
                    uint64_t seed, double tol, int32_t max_iter, double* s_out,
                    int32_t* iters_out) {
  size_t n1 = (size_t)(N > 0 ? N : 1);
  double* zu = (double*)malloc(sizeof(double) * n1 * (size_t)(K > 0 ? K : 1));
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t k = 0; k < K; ++k) {
    double* z = (double*)malloc(sizeof(double) * n1);
    double* u = (double*)malloc(sizeof(double) * n1);
    for (int64_t v = 0; v < N; ++v) z[v] = (double)orc_probe_sign(seed, k, v);
    orc_report rep;
    orc_pcg(N, nbr, diag, lam, z, NULL, tol, max_iter, u, &rep);
    if (iters_out) iters_out[k] = rep.iters;
    for (int64_t v = 0; v < N; ++v) zu[(size_t)k * n1 + (size_t)v] = z[v] * u[v];
    free(z);
    free(u);
  }
  for (int64_t v = 0; v < N; ++v) s_out[v] = 0.0;
  for (int32_t k = 0; k < K; ++k)
    for (int64_t v = 0; v < N; ++v) s_out[v] = s_out[v] + zu[(size_t)k * n1 + (size_t)v];
  for (int64_t v = 0; v < N; ++v) s_out[v] = s_out[v] / (double)K;
  free(zu);
}

/* ------------------------------------------------------------------ */
/* Next-best-view scoring (eq. 13, Sec. 3.8).  The default utility sums */
/* posterior variance over the band voxels each candidate ray crosses,  */
/* up to and including the first voxel whose mean is <= 0 (the surface  */
/* is reached).  Variances are quantised to integers first so the sum  */
/* is exact: q_v = rint(s_v / max(s) * 2^32).                           */
/* ------------------------------------------------------------------ */
void orc_quantize_variance(int64_t N, const double* s, int64_t* q) {
  double smax = 0.0;
  for (int64_t v = 0; v < N; ++v)
    if (s[v] > smax) smax = s[v];
  for (int64_t v = 0; v < N; ++v) q[v] = smax > 0.0 ? (int64_t)rint((s[v] / smax) * 4294967296.0) : 0;
}

/* Amanatides-Woo voxel walk of the ray o + t d (t >= 0) through the grid.  */
/* The next boundary on axis a is computed directly from the voxel index:   */
/* t_a = (origin_a + (i_a + [d_a > 0]) h - o_a) / d_a (as a product with    */
/* 1/d_a); the smallest t_a is stepped, the lowest axis first on ties.      */
/* Utility 0 sums q_v.  Utility 1 sums, per crossed band voxel, the         */
/* quantised expected variance reduction of one new observation taken at    */
/* the voxel's depth Z in the candidate view: s^2 / (s + sigma(Z)^2) for    */
/* s > 0, scaled by 2^32 / max(s) and rounded to an integer.                */
/* walk_ray is that walk; *stop_out (may be NULL) receives the band index of */
/* the voxel where it stopped (the first band voxel with mu <= 0), or -1.    */
static int64_t walk_ray(const orc_grid* g, const uint64_t* keys, int64_t N, const double* mu,
                        const int64_t* q, const orc_utility* u, const double* P, const double* o,
                        const double* d, int64_t* steps_out, int64_t* stop_out) {
  int32_t G = g->G;
  if (stop_out) *stop_out = -1;
  double inv[3];
  double tnear = 0.0, tfar = INFINITY;
  for (int a = 0; a < 3; ++a) {
    double lo = g->origin[a];
    double hi = g->origin[a] + (double)G * g->h;
    if (d[a] == 0.0) {
      inv[a] = 0.0;
      if (o[a] < lo || o[a] > hi) return 0;
      continue;
    }
    inv[a] = 1.0 / d[a];
    double t0 = (lo - o[a]) * inv[a];
    double t1 = (hi - o[a]) * inv[a];
    double tmin = t0 < t1 ? t0 : t1;
    double tmax = t0 < t1 ? t1 : t0;
    if (tmin > tnear) tnear = tmin;
    if (tmax < tfar) tfar = tmax;
  }
  if (!(tnear < tfar)) return 0;
  int32_t idx[3];
  double tn[3];
  int32_t step[3];
  for (int a = 0; a < 3; ++a) {
    double pa = o[a] + tnear * d[a];
    double f = floor((pa - g->origin[a]) / g->h);
    int32_t ia = f < 0.0 ? 0 : (f > (double)(G - 1) ? G - 1 : (int32_t)f);
    idx[a] = ia;
    step[a] = d[a] > 0.0 ? 1 : (d[a] < 0.0 ? -1 : 0);
  }
  for (int a = 0; a < 3; ++a) {
    if (step[a] == 0) tn[a] = INFINITY;
    else tn[a] = ((g->origin[a] + (double)(idx[a] + (step[a] > 0 ? 1 : 0)) * g->h) - o[a]) * inv[a];
  }
  int64_t score = 0, steps = 0;
  for (int64_t it = 0; it < 3 * (int64_t)G + 3; ++it) {
    ++steps;
    int64_t v = find_key(keys, N, orc_morton_encode(idx[0], idx[1], idx[2]));
    if (v >= 0) {
      if (u == NULL || u->utility == 0) {
        if (q) score += q[v];
      } else {
        double x = g->origin[0] + ((double)idx[0] + 0.5) * g->h;
        double y = g->origin[1] + ((double)idx[1] + 0.5) * g->h;
        double z = g->origin[2] + ((double)idx[2] + 0.5) * g->h;
        double dx = x - P[3], dy = y - P[7], dz = z - P[11];
        double Z = (P[2] * dx + P[6] * dy) + P[10] * dz;
        double e = Z - u->z0;
        double sd = u->a + u->c * (e * e);
        double sv = u->s[v];
        double term = sv > 0.0 ? (sv * sv) / (sv + sd * sd) : 0.0;
        score += u->smax > 0.0 ? (int64_t)rint((term / u->smax) * 4294967296.0) : 0;
      }
      if (mu[v] <= 0.0) {
        if (stop_out) *stop_out = v;
        break;
      }
    }
    int a = 0;
    if (tn[1] < tn[a]) a = 1;
    if (tn[2] < tn[a]) a = 2;
    idx[a] += step[a];
    if (idx[a] < 0 || idx[a] >= G) break;
    tn[a] = ((g->origin[a] + (double)(idx[a] + (step[a] > 0 ? 1 : 0)) * g->h) - o[a]) * inv[a];
  }
  if (steps_out) *steps_out += steps;
  return score;
}

int64_t orc_nbv_ray_u(const orc_grid* g, const uint64_t* keys, int64_t N, const double* mu,
                      const int64_t* q, const orc_utility* u, const double* P, const double* o,
                      const double* d, int64_t* steps_out) {
  return walk_ray(g, keys, N, mu, q, u, P, o, d, steps_out, NULL);
}

int64_t orc_nbv_ray(const orc_grid* g, const uint64_t* keys, int64_t N, const double* mu,
                    const int64_t* q, const double* o, const double* d, int64_t* steps_out) {
  return orc_nbv_ray_u(g, keys, N, mu, q, NULL, NULL, o, d, steps_out);
}

/* One candidate pose: rays through every pixel centre of ray_cam, with the */
/* unnormalised direction R ((col - cx)/fx, (row - cy)/fy, 1).              */
int64_t orc_nbv_candidate_u(const orc_grid* g, const orc_cam* cam, const uint64_t* keys,
                            int64_t N, const double* mu, const int64_t* q, const orc_utility* u,
                            const double* P) {
  int64_t total = 0;
  double o[3] = {P[3], P[7], P[11]};
  for (int32_t row = 0; row < cam->height; ++row)
    for (int32_t col = 0; col < cam->width; ++col) {
      double a = ((double)col - cam->cx) / cam->fx;
      double b = ((double)row - cam->cy) / cam->fy;
      double d[3];
      d[0] = (P[0] * a + P[1] * b) + P[2];
      d[1] = (P[4] * a + P[5] * b) + P[6];
      d[2] = (P[8] * a + P[9] * b) + P[10];
      total += orc_nbv_ray_u(g, keys, N, mu, q, u, P, o, d, NULL);
    }
  return total;
}

int64_t orc_nbv_candidate(const orc_grid* g, const orc_cam* cam, const uint64_t* keys, int64_t N,
                          const double* mu, const int64_t* q, const double* P) {
  return orc_nbv_candidate_u(g, cam, keys, N, mu, q, NULL, P);
}

/* Voxels visited by the walks of every ray of one candidate (the same rays */
/* and walk as orc_nbv_candidate; only the visit count is returned).         */
int64_t orc_nbv_candidate_steps(const orc_grid* g, const orc_cam* cam, const uint64_t* keys, int64_t N,
                                const double* mu, const int64_t* q, const double* P) {
  int64_t steps = 0;
  double o[3] = {P[3], P[7], P[11]};
  for (int32_t row = 0; row < cam->height; ++row)
    for (int32_t col = 0; col < cam->width; ++col) {
      double a = ((double)col - cam->cx) / cam->fx;
      double b = ((double)row - cam->cy) / cam->fy;
      double d[3];
      d[0] = (P[0] * a + P[1] * b) + P[2];
      d[1] = (P[4] * a + P[5] * b) + P[6];
      d[2] = (P[8] * a + P[9] * b) + P[10];
      orc_nbv_ray_u(g, keys, N, mu, q, NULL, NULL, o, d, &steps);
    }
  return steps;
}

/* Utilities (or plain-walk visit counts, when steps is not NULL) of n       */
/* candidates c2w [n][3][4], candidates in parallel.  Each is an exact       */
/* integer sum, so the thread count cannot change a result.                  */
void orc_nbv_scores(const orc_grid* g, const orc_cam* cam, const uint64_t* keys, int64_t N,
                    const double* mu, const int64_t* q, const orc_utility* u, int32_t n,
                    const double* c2w, int64_t* scores, int64_t* steps) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t c = 0; c < n; ++c) {
    scores[c] = orc_nbv_candidate_u(g, cam, keys, N, mu, q, u, c2w + 12 * c);
    if (steps) steps[c] = orc_nbv_candidate_steps(g, cam, keys, N, mu, q, c2w + 12 * c);
  }
}

/* The view a sensor with camera cam would take from pose P, predicted from  */
/* the current mean (Sec. 3.8: the post-view variance of eq. 13 needs the    */
/* observations the candidate would add).  Pixel (row, col) looks along the  */
/* ray of orc_nbv_candidate_u; its depth is the camera-z depth, as in eq. 2, */
/* of the centre of the first band voxel with mu <= 0 that the walk meets,   */
/* rounded to float like a depth map, and 0 (no return) when it meets none.  */
void orc_pred_depth(const orc_grid* g, const orc_cam* cam, const uint64_t* keys, int64_t N,
                    const double* mu, const double* P, float* depth) {
  double o[3] = {P[3], P[7], P[11]};
#pragma omp parallel for schedule(dynamic, 4)
  for (int32_t row = 0; row < cam->height; ++row)
    for (int32_t col = 0; col < cam->width; ++col) {
      double a = ((double)col - cam->cx) / cam->fx;
      double b = ((double)row - cam->cy) / cam->fy;
      double d[3];
      d[0] = (P[0] * a + P[1] * b) + P[2];
      d[1] = (P[4] * a + P[5] * b) + P[6];
      d[2] = (P[8] * a + P[9] * b) + P[10];
      int64_t v;
      walk_ray(g, keys, N, mu, NULL, NULL, P, o, d, NULL, &v);
      float z = 0.0f;
      if (v >= 0) {
        int32_t i, j, k;
        orc_morton_decode(keys[v], &i, &j, &k);
        double x = g->origin[0] + ((double)i + 0.5) * g->h;
        double y = g->origin[1] + ((double)j + 0.5) * g->h;
        double zz = g->origin[2] + ((double)k + 0.5) * g->h;
        double dx = x - P[3], dy = y - P[7], dz = zz - P[11];
        z = (float)((P[2] * dx + P[6] * dy) + P[10] * dz);
      }
      depth[(int64_t)row * cam->width + col] = z;
    }
}

int32_t orc_nbv_argmax(int32_t n, const int64_t* scores) {
  int32_t best = 0;
  for (int32_t c = 1; c < n; ++c)
    if (scores[c] > scores[best]) best = c;
  return best;
}

/* ------------------------------------------------------------------ */
/* Per-voxel input features of the learned warm start (not in the paper;*/
/* the paper names learned priors as future work in Sec. 6-7).  Lengths */
/* are in units of the voxel edge h:                                    */
/*  0 TSDF/h   1 log(1+W)   2 deg/6   3 n_obs/T   4 mean y/h            */
/*  5 var y/h^2   6 mean sigma/h   7 min sigma/h   8 log(1+Lambda h^2)  */
/*  9-11 central difference of the TSDF along x, y, z over 2h, using    */
/*       the voxel's own value where a band neighbour is absent.        */
/* ------------------------------------------------------------------ */
void orc_features(int64_t N, int32_t T, double h, const double* tsdf, const int32_t* w,
                  const int32_t* nbr, const int32_t* deg, const double* Lambda, const double* acc,
                  double* feat) {
  for (int64_t v = 0; v < N; ++v) {
    double* f = feat + v * 12;
    double n = acc[v * 5 + 0];
    double my = n > 0.0 ? acc[v * 5 + 1] / n : 0.0;
    double vy = n > 0.0 ? acc[v * 5 + 2] / n - my * my : 0.0;
    double ms = n > 0.0 ? acc[v * 5 + 3] / n : 0.0;
    f[0] = tsdf[v] / h;
    f[1] = log(1.0 + (double)w[v]);
    f[2] = (double)deg[v] / 6.0;
    f[3] = n / (double)T;
    f[4] = my / h;
    f[5] = vy / (h * h);
    f[6] = ms / h;
    f[7] = acc[v * 5 + 4] / h;
    f[8] = log(Lambda[v] * (h * h) + 1.0);
    for (int a = 0; a < 3; ++a) {
      int32_t m = nbr[v * 6 + 2 * a], p = nbr[v * 6 + 2 * a + 1];
      double tm = m >= 0 ? tsdf[m] : tsdf[v];
      double tp = p >= 0 ? tsdf[p] : tsdf[v];
      f[9 + a] = (tp - tm) / (2.0 * h);
    }
  }
}
