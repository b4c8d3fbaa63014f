/*
 * Surface extraction (Algorithm 1 step 7) and the nearest-point distances of
 * the geometry metrics (Sec. 4.2, eq. 14) for the FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: nothing in the product library
 * links, loads or calls this code.
 *
 * Readings (the oracle's, stated once here):
 *  - the iso-surface mu = iso is extracted with marching tetrahedra, the
 *    tetrahedral form of marching cubes: each 2x2x2 cube of band voxel centres
 *    (all 8 corners in the band) is split into the 6 tetrahedra of the
 *    Freudenthal split along its main diagonal, one per axis order (a, b, c):
 *    corners 0, e_a, e_a + e_b, (1,1,1).  The split matches across
 *    neighbouring cubes, so the mesh is watertight;
 *  - a voxel is inside when mu < iso;
 *  - mesh vertices sit on grid edges: from a band voxel v along one of the 7
 *    directions d in {0,1}^3 \ 0 (order: x, y, z, xy, xz, yz, xyz) to the band
 *    voxel v + d, when exactly one end is inside; the vertex is
 *    x_v + t (x_{v+d} - x_v) per coordinate with t = (mu_v - iso) /
 *    (mu_v - mu_{v+d}), computed from the lower end v.  Vertices are numbered
 *    by band index of v, then by d;
 *  - a tetrahedron with one (or three) inside corners gives one triangle on
 *    the three edges of the lone corner, with two a quad split into the
 *    triangles (e0, e1, e2), (e0, e2, e3) in the order listed in tri_tet();
 *    each triangle is turned so that (b - a) x (c - a) has a non-negative
 *    product with n_in * (sum of outside corners) - n_out * (sum of inside
 *    corners), i.e. points from the inside corners towards the outside ones;
 *  - triangles are listed by cube (band index of its lowest voxel), then by
 *    tetrahedron (axis orders (0,1,2), (0,2,1), (1,0,2), (1,2,0), (2,0,1),
 *    (2,1,0)), then in the order above.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "oracle.h"

static const int32_t kDir[7][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}};
static const int32_t kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

static int64_t find(int32_t G, const uint64_t* keys, int64_t N, int32_t i, int32_t j, int32_t k) {
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

int32_t orc_surf_dir(int32_t dx, int32_t dy, int32_t dz) {
  for (int32_t d = 0; d < 7; ++d)
    if (kDir[d][0] == dx && kDir[d][1] == dy && kDir[d][2] == dz) return d;
  return -1;
}

/* Crossing mask of band voxel v: bit d set when v + dir_d is a band voxel
 * and exactly one of the two is inside. */
static uint32_t crossing_mask(const orc_grid* g, const uint64_t* keys, int64_t N, const double* mu, double iso,
                              int64_t v) {
  int32_t i, j, k;
  orc_morton_decode(keys[v], &i, &j, &k);
  uint32_t m = 0;
  for (int32_t d = 0; d < 7; ++d) {
    int64_t u = find(g->G, keys, N, i + kDir[d][0], j + kDir[d][1], k + kDir[d][2]);
    if (u < 0) continue;
    int in_v = mu[v] < iso, in_u = mu[u] < iso;
    if (in_v != in_u) m |= 1u << d;
  }
  return m;
}

static int popc(uint32_t x) {
  int c = 0;
  while (x) {
    c += (int)(x & 1u);
    x >>= 1;
  }
  return c;
}

/* Vertex id of the crossing on the edge from voxel (i,j,k) along d. */
static int64_t vertex_id(const orc_grid* g, const uint64_t* keys, int64_t N, const int64_t* vstart,
                         const uint32_t* vmask, int32_t i, int32_t j, int32_t k, int32_t d) {
  int64_t v = find(g->G, keys, N, i, j, k);
  return vstart[v] + popc(vmask[v] & ((1u << d) - 1u));
}

/* The marching-tetrahedra triangles of one tetrahedron with corner offsets
 * c[4][3] (from the cube's lowest voxel) and values f[4]: writes up to 2
 * triangles as pairs of corner indices per vertex, tri[t][vert][2]; returns
 * the count. */
static int tri_tet(const double* f, double iso, int32_t tri[2][3][2]) {
  int in[4], n_in = 0;
  for (int q = 0; q < 4; ++q) {
    in[q] = f[q] < iso;
    n_in += in[q];
  }
  if (n_in == 0 || n_in == 4) return 0;
  if (n_in == 1 || n_in == 3) {
    int lone = -1;
    for (int q = 0; q < 4; ++q)
      if (in[q] == (n_in == 1)) lone = q;
    int e = 0;
    for (int q = 0; q < 4; ++q) {
      if (q == lone) continue;
      tri[0][e][0] = lone;
      tri[0][e][1] = q;
      ++e;
    }
    return 1;
  }
  /* two inside (a, b), two outside (c, d): quad a-c, a-d, b-d, b-c */
  int ins[2], outs[2], ni = 0, no = 0;
  for (int q = 0; q < 4; ++q) {
    if (in[q]) ins[ni++] = q;
    else outs[no++] = q;
  }
  int32_t quad[4][2] = {{ins[0], outs[0]}, {ins[0], outs[1]}, {ins[1], outs[1]}, {ins[1], outs[0]}};
  const int order[2][3] = {{0, 1, 2}, {0, 2, 3}};
  for (int t = 0; t < 2; ++t)
    for (int e = 0; e < 3; ++e) {
      tri[t][e][0] = quad[order[t][e]][0];
      tri[t][e][1] = quad[order[t][e]][1];
    }
  return 2;
}

/* Extraction.  Pass 1 (cap = 0): returns vertex and triangle counts through
 * *nv, *nt.  With room (cap_v >= nv, cap_t >= nt) also writes verts[nv][3]
 * and tris[nt][3]. */
void orc_extract_surface(const orc_grid* g, const uint64_t* keys, int64_t N, const double* mu, double iso,
                         int64_t cap_v, int64_t cap_t, double* verts, int32_t* tris, int64_t* nv, int64_t* nt) {
  uint32_t* vmask = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(N > 0 ? N : 1));
  int64_t* vstart = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
  int64_t V = 0;
  for (int64_t v = 0; v < N; ++v) {
    vmask[v] = crossing_mask(g, keys, N, mu, iso, v);
    vstart[v] = V;
    V += popc(vmask[v]);
  }
  *nv = V;
  int write = cap_v >= V;
  if (write) {
    for (int64_t v = 0; v < N; ++v) {
      int32_t i, j, k;
      orc_morton_decode(keys[v], &i, &j, &k);
      int64_t id = vstart[v];
      for (int32_t d = 0; d < 7; ++d) {
        if (!((vmask[v] >> d) & 1u)) continue;
        int64_t u = find(g->G, keys, N, i + kDir[d][0], j + kDir[d][1], k + kDir[d][2]);
        double t = (mu[v] - iso) / (mu[v] - mu[u]);
        int32_t a[3] = {i, j, k};
        for (int r = 0; r < 3; ++r) {
          double xa = g->origin[r] + ((double)a[r] + 0.5) * g->h;
          double xb = g->origin[r] + ((double)(a[r] + kDir[d][r]) + 0.5) * g->h;
          verts[3 * id + r] = xa + t * (xb - xa);
        }
        ++id;
      }
    }
  }
  int64_t T = 0;
  for (int64_t v = 0; v < N; ++v) {
    int32_t i, j, k;
    orc_morton_decode(keys[v], &i, &j, &k);
    double fc[8];
    int full = 1;
    for (int32_t q = 0; q < 8 && full; ++q) {
      int64_t u = find(g->G, keys, N, i + (q & 1), j + ((q >> 1) & 1), k + ((q >> 2) & 1));
      if (u < 0) full = 0;
      else fc[q] = mu[u];
    }
    if (!full) continue;
    for (int p = 0; p < 6; ++p) {
      int32_t c[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 1}};
      c[1][kPerm[p][0]] = 1;
      c[2][kPerm[p][0]] = 1;
      c[2][kPerm[p][1]] = 1;
      double f[4];
      for (int q = 0; q < 4; ++q) f[q] = fc[c[q][0] | (c[q][1] << 1) | (c[q][2] << 2)];
      int32_t tr[2][3][2];
      int ntr = tri_tet(f, iso, tr);
      for (int t = 0; t < ntr; ++t) {
        if (write && cap_t > T) {
          int64_t id[3];
          double P[3][3];
          for (int e = 0; e < 3; ++e) {
            const int32_t* ca = c[tr[t][e][0]];
            const int32_t* cb = c[tr[t][e][1]];
            /* the edge's lower end and direction (cb - ca or ca - cb is in {0,1}^3) */
            int lower_is_a = (cb[0] - ca[0]) >= 0 && (cb[1] - ca[1]) >= 0 && (cb[2] - ca[2]) >= 0;
            const int32_t* lo = lower_is_a ? ca : cb;
            const int32_t* hi = lower_is_a ? cb : ca;
            int32_t d = orc_surf_dir(hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]);
            id[e] = vertex_id(g, keys, N, vstart, vmask, i + lo[0], j + lo[1], k + lo[2], d);
            for (int r = 0; r < 3; ++r) P[e][r] = verts[3 * id[e] + r];
          }
          /* turn so that the normal points from inside to outside corners */
          double ab[3], ac[3], nrm[3], gdir[3] = {0.0, 0.0, 0.0};
          for (int r = 0; r < 3; ++r) {
            ab[r] = P[1][r] - P[0][r];
            ac[r] = P[2][r] - P[0][r];
          }
          nrm[0] = ab[1] * ac[2] - ab[2] * ac[1];
          nrm[1] = ab[2] * ac[0] - ab[0] * ac[2];
          nrm[2] = ab[0] * ac[1] - ab[1] * ac[0];
          /* mean of the outside corners minus mean of the inside ones, times
             n_in n_out (exact integers): it has a positive product with the
             gradient of the tetrahedron's linear interpolant */
          int n_in = 0;
          for (int q = 0; q < 4; ++q) n_in += f[q] < iso;
          for (int q = 0; q < 4; ++q)
            for (int r = 0; r < 3; ++r) gdir[r] += (double)((f[q] < iso ? -(4 - n_in) : n_in) * c[q][r]);
          double s = (nrm[0] * gdir[0] + nrm[1] * gdir[1]) + nrm[2] * gdir[2];
          tris[3 * T] = (int32_t)id[0];
          tris[3 * T + 1] = (int32_t)(s < 0.0 ? id[2] : id[1]);
          tris[3 * T + 2] = (int32_t)(s < 0.0 ? id[1] : id[2]);
        }
        ++T;
      }
    }
  }
  *nt = T;
  free(vmask);
  free(vstart);
}

/* Geometry metrics (eq. 14): d_out[i] = min over j of |a_i - b_j|^2 with
 * |x|^2 = (x0 x0 + x1 x1) + x2 x2, by brute force over all pairs. */
void orc_nn_dist2(const double* a, int64_t na, const double* b, int64_t nb, double* d_out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < na; ++i) {
    double best = INFINITY;
    for (int64_t j = 0; j < nb; ++j) {
      double dx = a[3 * i] - b[3 * j];
      double dy = a[3 * i + 1] - b[3 * j + 1];
      double dz = a[3 * i + 2] - b[3 * j + 2];
      double d = (dx * dx + dy * dy) + dz * dz;
      if (d < best) best = d;
    }
    d_out[i] = best;
  }
}
