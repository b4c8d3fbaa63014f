/*
 * Trilinear observation rows (Sec. 3.2, eqs. 2-5) for the FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: nothing in the product library
 * links, loads or calls this code.
 *
 * Observation model (the readings are the oracle's, stated once here):
 *  - every valid depth pixel u of view t gives 2S+1 samples along its camera
 *    ray (eq. 2), at camera depths z_s = D + s h, s = -S..S;
 *  - the sample's signed distance is y = clamp(D - z_s, -tau, tau) (eq. 3 with
 *    the normal read as the viewing axis, as in the voxel-centric rows);
 *  - its row a_i holds the trilinear weights of the sample point on the 8
 *    voxel centres around it (eq. 4, "up to 8 non-zeros"); a sample is kept
 *    only when those 8 voxels are all band voxels;
 *  - its variance is sigma_depth(D)^2 + sigma2_pose[t] + sigma2_model (eq. 5).
 * Then Q = A^T W A + lam L + eps I (+ lam_b on the band boundary), eqs. (7),
 * (10), and h = A^T W y (+ lam_b TSDF on the boundary), eq. (11).
 *
 * Summation order (the definition of the FP64 result): samples are grouped
 * by their cell (the 2x2x2 voxel cube whose lowest voxel is the sample's
 * floor corner) and, inside a cell, taken in ascending sample id
 * ((t H + row) W + col) (2S+1) + (s + S).  Per cell c,
 *   M_c[j][k] = sum_i (w_i a_ij) a_ik   for corners j <= k (also used for k, j)
 *   g_c[j]    = sum_i (w_i y_i) a_ij.
 * A voxel v is corner q of the cell v - off(q); over q = 0..7 ascending,
 *   Lambda_v += M_c[q][q], b_v += g_c[q], and coupling(v, u) += M_c[q][k]
 * for every other corner k (u = c + off(k)).  Corner q has offset
 * off(q) = (q & 1, (q >> 1) & 1, q >> 2).
 * Off-diagonal slots: the 26 offsets d in {-1,0,1}^3 \ {0} ordered by
 * (dx+1) + 3 (dy+1) + 9 (dz+1) ascending with the centre removed; the six
 * face slots also carry -lam when the neighbour is in the band.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int32_t corner_off(int32_t q, int32_t axis) { return (q >> axis) & 1; }

int32_t orc_tri_slot(int32_t dx, int32_t dy, int32_t dz) {
  int32_t idx = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
  if (idx == 13) return -1;
  return idx < 13 ? idx : idx - 1;
}

/* Band index of voxel (i, j, k) by binary search over the sorted keys, or -1. */
static int64_t band_find(int32_t G, const uint64_t* keys, int64_t N, int32_t i, int32_t j, int32_t k) {
  if (i < 0 || j < 0 || k < 0 || i >= G || j >= G || k >= G) return -1;
  uint64_t key = orc_morton_encode(i, j, k);
  int64_t lo = 0, hi = N;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (keys[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return (lo < N && keys[lo] == key) ? lo : -1;
}

/* One sample (eqs. 2-5).  Returns 1 and fills the cell's lowest voxel, the 8
 * corner weights, y and the weight 1/sigma^2 when the sample point has all 8
 * surrounding voxel centres inside the grid; 0 otherwise. */
int orc_tri_sample(const orc_grid* g, const orc_cam* cam, const float* depth_t, const double* P,
                   const orc_noise* nz, double sigma2_pose_t, int32_t row, int32_t col, int32_t s,
                   int32_t* base, double* a, double* y, double* wv) {
  double D = (double)depth_t[(int64_t)row * cam->width + col];
  if (!(D > 0.0) || !isfinite(D)) return 0;
  double z = D + (double)s * g->h;
  if (!(z > 0.0)) return 0;
  double yv = D - z;
  if (yv < -g->tau) yv = -g->tau;
  if (yv > g->tau) yv = g->tau;
  /* camera ray through the pixel centre, K^-1 (col, row, 1) */
  double ra = ((double)col - cam->cx) / cam->fx;
  double rb = ((double)row - cam->cy) / cam->fy;
  double wgt[3][2];
  for (int r = 0; r < 3; ++r) {
    double dw = (P[4 * r] * ra + P[4 * r + 1] * rb) + P[4 * r + 2];
    double x = P[4 * r + 3] + z * dw;
    double gc = (x - g->origin[r]) / g->h - 0.5;
    double fl = floor(gc);
    if (!(fl >= 0.0) || !(fl + 1.0 <= (double)(g->G - 1))) return 0;
    double f = gc - fl;
    base[r] = (int32_t)fl;
    wgt[r][0] = 1.0 - f;
    wgt[r][1] = f;
  }
  for (int32_t q = 0; q < 8; ++q)
    a[q] = (wgt[0][corner_off(q, 0)] * wgt[1][corner_off(q, 1)]) * wgt[2][corner_off(q, 2)];
  double e = D - nz->z0;
  double sd = nz->a + nz->c * (e * e);
  double var = sd * sd + sigma2_pose_t;
  var = var + nz->sigma2_model;
  *y = yv;
  *wv = 1.0 / var;
  return 1;
}

typedef struct {
  uint64_t cell;  /* Morton key of the cell's lowest voxel */
  uint64_t id;    /* sample id */
} tri_item;

static int cmp_item(const void* pa, const void* pb) {
  const tri_item* x = (const tri_item*)pa;
  const tri_item* y = (const tri_item*)pb;
  if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
  if (x->id != y->id) return x->id < y->id ? -1 : 1;
  return 0;
}

static void id_decode(uint64_t id, int32_t S, int32_t W, int32_t H, int32_t* t, int32_t* row, int32_t* col,
                      int32_t* s) {
  uint64_t ns = (uint64_t)(2 * S + 1);
  *s = (int32_t)(id % ns) - S;
  id /= ns;
  *col = (int32_t)(id % (uint64_t)W);
  id /= (uint64_t)W;
  *row = (int32_t)(id % (uint64_t)H);
  *t = (int32_t)(id / (uint64_t)H);
}

/* Kept samples in (cell, id) order: writes up to cap items into cells/ids and
 * returns the total count (call with cap = 0 to size). */
static int64_t collect(const orc_grid* g, const orc_cam* cam, int32_t T, const float* depth, const double* c2w,
                       const orc_noise* nz, int32_t S, const uint64_t* keys, int64_t N, tri_item** out) {
  int64_t plane = (int64_t)cam->width * cam->height;
  int64_t cap = 1024, n = 0;
  tri_item* items = (tri_item*)malloc(sizeof(tri_item) * (size_t)cap);
  for (int32_t t = 0; t < T; ++t)
    for (int32_t row = 0; row < cam->height; ++row)
      for (int32_t col = 0; col < cam->width; ++col)
        for (int32_t s = -S; s <= S; ++s) {
          int32_t base[3];
          double a[8], y, wv;
          if (!orc_tri_sample(g, cam, depth + t * plane, c2w + 12 * t, nz,
                              nz->sigma2_pose ? nz->sigma2_pose[t] : 0.0, row, col, s, base, a, &y, &wv))
            continue;
          int inside = 1;
          for (int32_t q = 0; q < 8 && inside; ++q)
            inside = band_find(g->G, keys, N, base[0] + corner_off(q, 0), base[1] + corner_off(q, 1),
                               base[2] + corner_off(q, 2)) >= 0;
          if (!inside) continue;
          if (n == cap) {
            cap *= 2;
            items = (tri_item*)realloc(items, sizeof(tri_item) * (size_t)cap);
          }
          items[n].cell = orc_morton_encode(base[0], base[1], base[2]);
          items[n].id = (((uint64_t)t * (uint64_t)cam->height + (uint64_t)row) * (uint64_t)cam->width +
                         (uint64_t)col) * (uint64_t)(2 * S + 1) + (uint64_t)(s + S);
          ++n;
        }
  qsort(items, (size_t)n, sizeof(tri_item), cmp_item);
  *out = items;
  return n;
}

/* The kept samples as explicit rows (for checks against a dense A^T W A):
 * base[n][3], a[n][8], y[n], wv[n] and the sample's (t, row, col, s) in
 * tcrs[n][4], in (cell, id) order.  Returns n; with cap < n nothing is
 * written. */
int64_t orc_tri_sample_list(const orc_grid* g, const orc_cam* cam, int32_t T, const float* depth,
                            const double* c2w, const orc_noise* nz, int32_t S, const uint64_t* keys, int64_t N,
                            int64_t cap, int32_t* base, double* a, double* y, double* wv, int32_t* tcrs) {
  tri_item* items = NULL;
  int64_t n = collect(g, cam, T, depth, c2w, nz, S, keys, N, &items);
  if (n <= cap) {
    int64_t plane = (int64_t)cam->width * cam->height;
    for (int64_t i = 0; i < n; ++i) {
      int32_t t, row, col, s;
      id_decode(items[i].id, S, cam->width, cam->height, &t, &row, &col, &s);
      orc_tri_sample(g, cam, depth + t * plane, c2w + 12 * t, nz, nz->sigma2_pose ? nz->sigma2_pose[t] : 0.0,
                     row, col, s, base + 3 * i, a + 8 * i, y + i, wv + i);
      tcrs[4 * i] = t;
      tcrs[4 * i + 1] = row;
      tcrs[4 * i + 2] = col;
      tcrs[4 * i + 3] = s;
    }
  }
  free(items);
  return n;
}

/* Assembly of the trilinear system; see the file comment for the order.
 * Outputs [N]: Lambda, b, rhs, diag; [N][26]: off (couplings incl. -lam on
 * band faces), nb26 (band index of each offset's voxel or -1).  Returns the
 * number of kept samples; *ncells_out = cells holding at least one. */
int64_t orc_tri_assemble(const orc_grid* g, const orc_cam* cam, int32_t T, const float* depth,
                         const double* c2w, const orc_noise* nz, int32_t S, const uint64_t* keys, int64_t N,
                         const int32_t* deg, const double* tsdf, double lam, double eps, double lam_b,
                         double* Lambda, double* b, double* rhs, double* diag, double* off, int32_t* nb26,
                         int64_t* ncells_out) {
  tri_item* items = NULL;
  int64_t n = collect(g, cam, T, depth, c2w, nz, S, keys, N, &items);
  int64_t plane = (int64_t)cam->width * cam->height;
  /* per-cell sums M (36 upper-triangle entries, row-major over j <= k) and g */
  int64_t ncell = 0;
  for (int64_t i = 0; i < n; ++i)
    if (i == 0 || items[i].cell != items[i - 1].cell) ++ncell;
  uint64_t* ckey = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(ncell > 0 ? ncell : 1));
  double* M = (double*)calloc((size_t)(ncell > 0 ? ncell : 1) * 36, sizeof(double));
  double* gv = (double*)calloc((size_t)(ncell > 0 ? ncell : 1) * 8, sizeof(double));
  int64_t c = -1;
  for (int64_t i = 0; i < n; ++i) {
    if (i == 0 || items[i].cell != items[i - 1].cell) ckey[++c] = items[i].cell;
    int32_t t, row, col, s, base[3];
    double a[8], y, wv;
    id_decode(items[i].id, S, cam->width, cam->height, &t, &row, &col, &s);
    orc_tri_sample(g, cam, depth + t * plane, c2w + 12 * t, nz, nz->sigma2_pose ? nz->sigma2_pose[t] : 0.0, row,
                   col, s, base, a, &y, &wv);
    int e = 0;
    for (int j = 0; j < 8; ++j) {
      double wa = wv * a[j];
      for (int k = j; k < 8; ++k, ++e) M[c * 36 + e] = M[c * 36 + e] + wa * a[k];
      gv[c * 8 + j] = gv[c * 8 + j] + (wv * y) * a[j];
    }
  }
  /* gather per band voxel */
  for (int64_t v = 0; v < N; ++v) {
    int32_t vi, vj, vk;
    orc_morton_decode(keys[v], &vi, &vj, &vk);
    double L = 0.0, B = 0.0;
    double cpl[26];
    for (int t = 0; t < 26; ++t) cpl[t] = 0.0;
    for (int32_t q = 0; q < 8; ++q) {
      int32_t ci = vi - corner_off(q, 0), cj = vj - corner_off(q, 1), ck = vk - corner_off(q, 2);
      if (ci < 0 || cj < 0 || ck < 0) continue;
      uint64_t key = orc_morton_encode(ci, cj, ck);
      int64_t lo = 0, hi = ncell;
      while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (ckey[mid] < key) lo = mid + 1;
        else hi = mid;
      }
      if (!(lo < ncell && ckey[lo] == key)) continue;
      const double* Mc = M + lo * 36;
      for (int32_t k = 0; k < 8; ++k) {
        int32_t jj = q < k ? q : k, kk = q < k ? k : q;
        int32_t e = jj * 8 - (jj * (jj - 1)) / 2 + (kk - jj);  /* row-major upper triangle index */
        if (k == q) {
          L = L + Mc[e];
        } else {
          int32_t slot = orc_tri_slot(corner_off(k, 0) - corner_off(q, 0), corner_off(k, 1) - corner_off(q, 1),
                                      corner_off(k, 2) - corner_off(q, 2));
          cpl[slot] = cpl[slot] + Mc[e];
        }
      }
      B = B + gv[lo * 8 + q];
    }
    Lambda[v] = L;
    b[v] = B;
    for (int32_t dz = -1; dz <= 1; ++dz)
      for (int32_t dy = -1; dy <= 1; ++dy)
        for (int32_t dx = -1; dx <= 1; ++dx) {
          int32_t slot = orc_tri_slot(dx, dy, dz);
          if (slot < 0) continue;
          int64_t u = band_find(g->G, keys, N, vi + dx, vj + dy, vk + dz);
          nb26[v * 26 + slot] = (int32_t)u;
          double o = cpl[slot];
          int face = (dx != 0) + (dy != 0) + (dz != 0) == 1;
          if (face && u >= 0) o = o - lam;
          off[v * 26 + slot] = u >= 0 ? o : 0.0;
        }
  }
  orc_precision_diag(N, Lambda, deg, lam, eps, lam_b, diag);
  orc_anchor_rhs(N, b, deg, tsdf, lam_b, rhs);
  free(items);
  free(ckey);
  free(M);
  free(gv);
  if (ncells_out) *ncells_out = ncell;
  return n;
}

/* q = Q p for the trilinear system: q_v = diag_v p_v + sum over the 26 slots
 * (ascending) of off[v][slot] p[nb26[v][slot]]. */
void orc_apply_Q27(int64_t N, const double* diag, const double* off, const int32_t* nb26, const double* p,
                   double* q) {
  for (int64_t v = 0; v < N; ++v) {
    double s = 0.0;
    for (int t = 0; t < 26; ++t) {
      int32_t u = nb26[v * 26 + t];
      if (u >= 0) s = s + off[v * 26 + t] * p[u];
    }
    q[v] = diag[v] * p[v] + s;
  }
}

static double dot27(int64_t N, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t v = 0; v < N; ++v) s = s + a[v] * b[v];
  return s;
}

/* Jacobi PCG on the trilinear system; the same iteration and stopping rule
 * as orc_pcg (eq. 11), with the 27-point product. */
void orc_pcg27(int64_t N, const double* diag, const double* off, const int32_t* nb26, const double* rhs,
               const double* x0, double tol, int32_t max_iter, double* x, orc_report* rep) {
  size_t sz = sizeof(double) * (size_t)(N > 0 ? N : 1);
  double *r = (double*)malloc(sz), *z = (double*)malloc(sz), *p = (double*)malloc(sz), *q = (double*)malloc(sz);
  rep->iters = 0;
  rep->status = 0;
  rep->rel_res = 0.0;
  double bnorm = sqrt(dot27(N, rhs, rhs));
  if (bnorm == 0.0) {
    for (int64_t v = 0; v < N; ++v) x[v] = 0.0;
  } else {
    for (int64_t v = 0; v < N; ++v) x[v] = x0 ? x0[v] : 0.0;
    orc_apply_Q27(N, diag, off, nb26, x, q);
    for (int64_t v = 0; v < N; ++v) r[v] = rhs[v] - q[v];
    if (!(sqrt(dot27(N, r, r)) <= tol * bnorm)) {
      for (int64_t v = 0; v < N; ++v) {
        z[v] = r[v] / diag[v];
        p[v] = z[v];
      }
      double rho = dot27(N, r, z);
      rep->status = 5;
      for (int32_t it = 1; it <= max_iter; ++it) {
        orc_apply_Q27(N, diag, off, nb26, p, q);
        double pq = dot27(N, p, q);
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
        if (sqrt(dot27(N, r, r)) <= tol * bnorm) {
          orc_apply_Q27(N, diag, off, nb26, x, q);
          for (int64_t v = 0; v < N; ++v) r[v] = rhs[v] - q[v];
          if (sqrt(dot27(N, r, r)) <= tol * bnorm) {
            rep->status = 0;
            break;
          }
        }
        for (int64_t v = 0; v < N; ++v) z[v] = r[v] / diag[v];
        double rho_new = dot27(N, r, z);
        double beta = rho_new / rho;
        rho = rho_new;
        for (int64_t v = 0; v < N; ++v) p[v] = z[v] + beta * p[v];
      }
    }
    orc_apply_Q27(N, diag, off, nb26, x, q);
    for (int64_t v = 0; v < N; ++v) r[v] = rhs[v] - q[v];
    rep->rel_res = sqrt(dot27(N, r, r)) / bnorm;
  }
  free(r);
  free(z);
  free(p);
  free(q);
}

/* Hutchinson estimate of diag(Q^-1) on the trilinear system (eq. 12), with
 * the probes of orc_hutchinson. */
void orc_hutchinson27(int64_t N, const double* diag, const double* off, const int32_t* nb26, int32_t K,
                      uint64_t seed, double tol, int32_t max_iter, double* s_out, int32_t* iters_out) {
  size_t sz = sizeof(double) * (size_t)(N > 0 ? N : 1);
  double *z = (double*)malloc(sz), *u = (double*)malloc(sz);
  for (int64_t v = 0; v < N; ++v) s_out[v] = 0.0;
  for (int32_t k = 0; k < K; ++k) {
    for (int64_t v = 0; v < N; ++v) z[v] = (double)orc_probe_sign(seed, k, v);
    orc_report rep;
    orc_pcg27(N, diag, off, nb26, z, NULL, tol, max_iter, u, &rep);
    if (iters_out) iters_out[k] = rep.iters;
    for (int64_t v = 0; v < N; ++v) s_out[v] = s_out[v] + z[v] * u[v];
  }
  for (int64_t v = 0; v < N; ++v) s_out[v] = s_out[v] / (double)K;
  free(z);
  free(u);
}
