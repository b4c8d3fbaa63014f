// Surface extraction (Algorithm 1 step 7) by marching tetrahedra over the
// band, and the nearest-point distances and geometry metrics of Sec. 4.2
// (eq. 14: Chamfer; mean accuracy and completeness; F-scores).
//
// Extraction: a voxel is inside when mu < iso.  A mesh vertex lies on the
// grid edge from band voxel v along one of the 7 directions d in {0,1}^3 \ 0
// (x, y, z, xy, xz, yz, xyz) to band voxel v + d when exactly one end is
// inside, at x_v + t (x_{v+d} - x_v), t = (mu_v - iso) / (mu_v - mu_{v+d}),
// numbered by band index of v, then d (a 7-bit crossing mask and a scan).
// Each cube of 8 band voxels is split into the 6 Freudenthal tetrahedra (axis
// orders 012, 021, 102, 120, 201, 210: corners 0, e_a, e_a + e_b, 111), which
// match across neighbouring cubes, so the mesh is watertight; a tetrahedron
// gives one triangle (one or three corners inside) or two (a quad), turned
// so that its normal points from the inside corners to the outside ones.
// Triangles are numbered by cube, tetrahedron, then position (a scan).
//
// Metrics: the nearest point of a set is found by brute force over all
// pairs, FP64, the other set staged through LDS in tiles; minima are exact,
// so the distances are reproducible bit for bit.
#include <hipcub/hipcub.hpp>

#include "bf_internal.h"

struct bf_mesh {
  int64_t nv = 0, nt = 0;
  double* verts = nullptr;  // [nv][3]
  int32_t* tris = nullptr;  // [nt][3]
};

namespace {

constexpr int kThreads = 256;

__constant__ int8_t kDir[7][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}};
__constant__ int8_t kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

struct surf_k {
  int32_t G, ncell;
  double h, org[3], iso;
  const bf_cell* cells;
  const uint64_t* keys;
  const double* mu;
  int64_t n;
};

__device__ __forceinline__ void decode(uint64_t key, int32_t& i, int32_t& j, int32_t& k) {
  i = (int32_t)bf_compact3(key);
  j = (int32_t)bf_compact3(key >> 1);
  k = (int32_t)bf_compact3(key >> 2);
}

// Pass 1: crossing mask and vertex count of each band voxel.
__global__ __launch_bounds__(256) void k_surf_mask(surf_k S, uint8_t* __restrict__ mask, uint32_t* __restrict__ cnt) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= S.n) return;
  int32_t i, j, k;
  decode(S.keys[v], i, j, k);
  const bool in_v = S.mu[v] < S.iso;
  uint32_t m = 0;
#pragma unroll
  for (int d = 0; d < 7; ++d) {
    const int32_t u = bf_band_index(S.cells, S.ncell, S.G, i + kDir[d][0], j + kDir[d][1], k + kDir[d][2]);
    if (u >= 0 && (S.mu[u] < S.iso) != in_v) m |= 1u << d;
  }
  mask[v] = (uint8_t)m;
  cnt[v] = (uint32_t)__popc(m);
}

// Pass 2: vertex positions.
__global__ __launch_bounds__(256) void k_surf_verts(surf_k S, const uint8_t* __restrict__ mask,
                                                    const uint64_t* __restrict__ vstart, double* __restrict__ verts) {
#pragma clang fp contract(off)
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= S.n) return;
  const uint32_t m = mask[v];
  if (!m) return;
  int32_t a[3];
  decode(S.keys[v], a[0], a[1], a[2]);
  uint64_t id = vstart[v];
  for (int d = 0; d < 7; ++d) {
    if (!((m >> d) & 1u)) continue;
    const int32_t u = bf_band_index(S.cells, S.ncell, S.G, a[0] + kDir[d][0], a[1] + kDir[d][1], a[2] + kDir[d][2]);
    const double t = (S.mu[v] - S.iso) / (S.mu[v] - S.mu[u]);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double xa = S.org[r] + ((double)a[r] + 0.5) * S.h;
      const double xb = S.org[r] + ((double)(a[r] + kDir[d][r]) + 0.5) * S.h;
      verts[3 * id + r] = xa + t * (xb - xa);
    }
    ++id;
  }
}

// Corner values of the cube whose lowest voxel is (i, j, k); false unless
// all 8 are band voxels.
__device__ __forceinline__ bool cube_values(const surf_k& S, int32_t i, int32_t j, int32_t k, double (&fc)[8]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int32_t u = bf_band_index(S.cells, S.ncell, S.G, i + (q & 1), j + ((q >> 1) & 1), k + ((q >> 2) & 1));
    if (u < 0) return false;
    fc[q] = S.mu[u];
  }
  return true;
}

// Corner offsets of tetrahedron p (bits x | y << 1 | z << 2 per corner).
__device__ __forceinline__ void tet_corners(int p, int (&c)[4]) {
  c[0] = 0;
  c[1] = 1 << kPerm[p][0];
  c[2] = c[1] | (1 << kPerm[p][1]);
  c[3] = 7;
}

__device__ __forceinline__ int tet_count(const double (&f)[4], double iso) {
  int n_in = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) n_in += f[q] < iso;
  return (n_in == 0 || n_in == 4) ? 0 : (n_in == 2 ? 2 : 1);
}

// Pass 3: triangles per cube.
__global__ __launch_bounds__(256) void k_surf_tcount(surf_k S, uint32_t* __restrict__ cnt) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= S.n) return;
  int32_t i, j, k;
  decode(S.keys[v], i, j, k);
  double fc[8];
  uint32_t total = 0;
  if (cube_values(S, i, j, k, fc)) {
    for (int p = 0; p < 6; ++p) {
      int c[4];
      tet_corners(p, c);
      const double f[4] = {fc[c[0]], fc[c[1]], fc[c[2]], fc[c[3]]};
      total += (uint32_t)tet_count(f, S.iso);
    }
  }
  cnt[v] = total;
}

// Vertex id of the crossing on the edge between cube corners ca and cb (one
// is componentwise below the other).
__device__ __forceinline__ int64_t edge_vertex(const surf_k& S, const uint8_t* __restrict__ mask,
                                               const uint64_t* __restrict__ vstart, int32_t i, int32_t j, int32_t k,
                                               int ca, int cb) {
  const bool a_low = (ca & cb) == ca;  // ca's set bits are a subset of cb's
  const int lo = a_low ? ca : cb, hi = a_low ? cb : ca;
  const int dm = hi & ~lo;  // direction bits
  const int d = dm == 1 ? 0 : dm == 2 ? 1 : dm == 4 ? 2 : dm == 3 ? 3 : dm == 5 ? 4 : dm == 6 ? 5 : 6;
  const int32_t u = bf_band_index(S.cells, S.ncell, S.G, i + (lo & 1), j + ((lo >> 1) & 1), k + ((lo >> 2) & 1));
  return (int64_t)vstart[u] + __popc(mask[u] & ((1u << d) - 1u));
}

// Pass 4: triangles (vertex ids), oriented from inside to outside.
__global__ __launch_bounds__(256) void k_surf_tris(surf_k S, const uint8_t* __restrict__ mask,
                                                   const uint64_t* __restrict__ vstart,
                                                   const double* __restrict__ verts,
                                                   const uint64_t* __restrict__ tstart, int32_t* __restrict__ tris) {
#pragma clang fp contract(off)
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= S.n) return;
  int32_t i, j, k;
  decode(S.keys[v], i, j, k);
  double fc[8];
  if (!cube_values(S, i, j, k, fc)) return;
  uint64_t out = tstart[v];
  for (int p = 0; p < 6; ++p) {
    int c[4];
    tet_corners(p, c);
    const double f[4] = {fc[c[0]], fc[c[1]], fc[c[2]], fc[c[3]]};
    int in[4], n_in = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      in[q] = f[q] < S.iso;
      n_in += in[q];
    }
    if (n_in == 0 || n_in == 4) continue;
    int tri[2][3][2], ntr;
    if (n_in == 1 || n_in == 3) {
      int lone = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (in[q] == (n_in == 1)) lone = q;
      int e = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q == lone) continue;
        tri[0][e][0] = lone;
        tri[0][e][1] = q;
        ++e;
      }
      ntr = 1;
    } else {
      int ins[2], outs[2], ni = 0, no = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (in[q]) ins[ni++] = q;
        else outs[no++] = q;
      }
      const int quad[4][2] = {{ins[0], outs[0]}, {ins[0], outs[1]}, {ins[1], outs[1]}, {ins[1], outs[0]}};
      const int order[2][3] = {{0, 1, 2}, {0, 2, 3}};
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          tri[t][e][0] = quad[order[t][e]][0];
          tri[t][e][1] = quad[order[t][e]][1];
        }
      ntr = 2;
    }
    // n_in * (sum of outside corners) - n_out * (sum of inside corners)
    double gdir[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 3; ++r) gdir[r] += (double)((in[q] ? -(4 - n_in) : n_in) * ((c[q] >> r) & 1));
    for (int t = 0; t < ntr; ++t) {
      int64_t id[3];
      double P[3][3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        id[e] = edge_vertex(S, mask, vstart, i, j, k, c[tri[t][e][0]], c[tri[t][e][1]]);
#pragma unroll
        for (int r = 0; r < 3; ++r) P[e][r] = verts[3 * id[e] + r];
      }
      double ab[3], ac[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        ab[r] = P[1][r] - P[0][r];
        ac[r] = P[2][r] - P[0][r];
      }
      const double n0 = ab[1] * ac[2] - ab[2] * ac[1];
      const double n1 = ab[2] * ac[0] - ab[0] * ac[2];
      const double n2 = ab[0] * ac[1] - ab[1] * ac[0];
      const double sgn = (n0 * gdir[0] + n1 * gdir[1]) + n2 * gdir[2];
      tris[3 * out] = (int32_t)id[0];
      tris[3 * out + 1] = (int32_t)(sgn < 0.0 ? id[2] : id[1]);
      tris[3 * out + 2] = (int32_t)(sgn < 0.0 ? id[1] : id[2]);
      ++out;
    }
  }
}

// d_out[i] = min_j |a_i - b_j|^2, |x|^2 = (x0 x0 + x1 x1) + x2 x2.  Each thread
// keeps two points of a; b goes through LDS in tiles of kThreads points.
constexpr int kNNPerThread = 2;
__global__ __launch_bounds__(256) void k_nn_dist2(const double* __restrict__ a, int64_t na,
                                                  const double* __restrict__ b, int64_t nb,
                                                  double* __restrict__ d_out) {
#pragma clang fp contract(off)
  __shared__ double sx[kThreads], sy[kThreads], sz[kThreads];
  const int64_t i0 = (int64_t)blockIdx.x * kThreads * kNNPerThread + threadIdx.x;
  double ax[kNNPerThread], ay[kNNPerThread], az[kNNPerThread], best[kNNPerThread];
#pragma unroll
  for (int p = 0; p < kNNPerThread; ++p) {
    const int64_t i = i0 + (int64_t)p * kThreads;
    const bool ok = i < na;
    ax[p] = ok ? a[3 * i] : 0.0;
    ay[p] = ok ? a[3 * i + 1] : 0.0;
    az[p] = ok ? a[3 * i + 2] : 0.0;
    best[p] = INFINITY;
  }
  for (int64_t j0 = 0; j0 < nb; j0 += kThreads) {
    const int64_t jt = j0 + threadIdx.x;
    __syncthreads();
    sx[threadIdx.x] = jt < nb ? b[3 * jt] : INFINITY;
    sy[threadIdx.x] = jt < nb ? b[3 * jt + 1] : INFINITY;
    sz[threadIdx.x] = jt < nb ? b[3 * jt + 2] : INFINITY;
    __syncthreads();
    const int m = (int)(nb - j0 < kThreads ? nb - j0 : kThreads);
    for (int jj = 0; jj < m; ++jj) {
      const double bx = sx[jj], by = sy[jj], bz = sz[jj];
#pragma unroll
      for (int p = 0; p < kNNPerThread; ++p) {
        const double dx = ax[p] - bx, dy = ay[p] - by, dz = az[p] - bz;
        const double d = (dx * dx + dy * dy) + dz * dz;
        best[p] = d < best[p] ? d : best[p];
      }
    }
  }
#pragma unroll
  for (int p = 0; p < kNNPerThread; ++p) {
    const int64_t i = i0 + (int64_t)p * kThreads;
    if (i < na) d_out[i] = best[p];
  }
}

// Block partials of sum d, sum sqrt(d) and, per threshold, the count of
// sqrt(d) < thr (as doubles, exact below 2^53).
constexpr int kMaxThr = 8;
__global__ __launch_bounds__(256) void k_metric_partials(const double* __restrict__ d, int64_t n, int nthr,
                                                         const double* __restrict__ thr,
                                                         double* __restrict__ part) {
  __shared__ double lds[16];
  double s2 = 0.0, s1 = 0.0, c[kMaxThr];
#pragma unroll
  for (int t = 0; t < kMaxThr; ++t) c[t] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const double di = d[i], r = sqrt(di);
    s2 += di;
    s1 += r;
#pragma unroll
    for (int t = 0; t < kMaxThr; ++t)
      if (t < nthr && r < thr[t]) c[t] += 1.0;
  }
  const int W = 2 + kMaxThr;
  double* out = part + (int64_t)blockIdx.x * W;
  s2 = bf_block_sum(s2, lds);
  s1 = bf_block_sum(s1, lds);
  if (threadIdx.x == 0) {
    out[0] = s2;
    out[1] = s1;
  }
#pragma unroll
  for (int t = 0; t < kMaxThr; ++t) {
    const double ct = bf_block_sum(c[t], lds);
    if (threadIdx.x == 0) out[2 + t] = ct;
  }
}

// Sum of the block partials in ascending block order (one thread).
__global__ void k_metric_total(const double* __restrict__ part, int nb, double* __restrict__ tot) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int W = 2 + kMaxThr;
  double acc[2 + kMaxThr];
  for (int w = 0; w < W; ++w) acc[w] = 0.0;
  for (int b = 0; b < nb; ++b)
    for (int w = 0; w < W; ++w) acc[w] += part[(int64_t)b * W + w];
  for (int w = 0; w < W; ++w) tot[w] = acc[w];
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" bf_status bf_extract_surface(bf_ctx* ctx, const bf_band* band, const double* mu_dev, double iso,
                                        bf_mesh** out, int64_t* n_vert, int64_t* n_tri) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, band && out, "bf_extract_surface: NULL argument");
  BF_CHECK(ctx, isfinite(iso), "bf_extract_surface: iso must be finite");
  *out = nullptr;
  if (n_vert) *n_vert = 0;
  if (n_tri) *n_tri = 0;
  BF_HIP(ctx, hipSetDevice(ctx->device));
  bf_mesh* mesh = new (std::nothrow) bf_mesh();
  if (!mesh) return bf_fail(ctx, BF_ERR_OOM, "bf_extract_surface: host allocation");
  auto fail = [&](bf_status st) {
    bf_mesh_free(ctx, mesh);
    return st;
  };
  const int64_t N = band->n;
  if (N == 0) {
    *out = mesh;
    return BF_OK;
  }
  if (!mu_dev) return fail(bf_fail(ctx, BF_ERR_INVALID_ARG, "bf_extract_surface: NULL mu"));
  surf_k S{band->G, band->ncell, band->h, {band->origin[0], band->origin[1], band->origin[2]}, iso,
           band->cells, band->keys, mu_dev, N};
  // workspace: mask [N] | vcount [N] | vstart [N] | tcount [N] | tstart [N] | scan temp
  size_t scan_tmp = 0;
  if (hipcub::DeviceScan::ExclusiveSum(nullptr, scan_tmp, (const uint32_t*)nullptr, (uint64_t*)nullptr, (int)N,
                                       ctx->stream) != hipSuccess)
    return fail(bf_fail(ctx, BF_ERR_HIP, "bf_extract_surface: scan sizing failed"));
  const size_t s8 = al256(N), s4 = al256(N * 4), s64 = al256(N * 8);
  char* ws = nullptr;
  if (bf_status s = bf_ws(ctx, bf_ctx::WS_SURF, s8 + 2 * s4 + 2 * s64 + al256(scan_tmp), (void**)&ws)) return fail(s);
  uint8_t* mask = (uint8_t*)ws;
  uint32_t* vcnt = (uint32_t*)(ws + s8);
  uint32_t* tcnt = (uint32_t*)(ws + s8 + s4);
  uint64_t* vstart = (uint64_t*)(ws + s8 + 2 * s4);
  uint64_t* tstart = (uint64_t*)(ws + s8 + 2 * s4 + s64);
  void* tmp = ws + s8 + 2 * s4 + 2 * s64;
  const unsigned g = (unsigned)bf_cdiv(N, kThreads);
  BF_LAUNCH(ctx, "surf_mask", k_surf_mask, dim3(g), dim3(kThreads), 0, S, mask, vcnt);
  BF_LAUNCH(ctx, "surf_tcount", k_surf_tcount, dim3(g), dim3(kThreads), 0, S, tcnt);
  if (hipcub::DeviceScan::ExclusiveSum(tmp, scan_tmp, vcnt, vstart, (int)N, ctx->stream) != hipSuccess ||
      hipcub::DeviceScan::ExclusiveSum(tmp, scan_tmp, tcnt, tstart, (int)N, ctx->stream) != hipSuccess)
    return fail(bf_fail(ctx, BF_ERR_HIP, "bf_extract_surface: scan failed"));
  uint64_t* pin = nullptr;
  if (bf_status s = bf_pinned(ctx, 32, (void**)&pin)) return fail(s);
  if (hipMemcpyAsync(pin, vstart + N - 1, 8, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipMemcpyAsync(pin + 1, tstart + N - 1, 8, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipMemcpyAsync((char*)(pin + 2), vcnt + N - 1, 4, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipMemcpyAsync((char*)(pin + 2) + 4, tcnt + N - 1, 4, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess)
    return fail(bf_fail(ctx, BF_ERR_HIP, "bf_extract_surface: count read-back failed"));
  const uint32_t* lastc = (const uint32_t*)(pin + 2);
  mesh->nv = (int64_t)pin[0] + lastc[0];
  mesh->nt = (int64_t)pin[1] + lastc[1];
  if (mesh->nv >= (1ll << 31)) return fail(bf_fail(ctx, BF_ERR_CAPACITY, "bf_extract_surface: too many vertices"));
  if (bf_status s = bf_obj_alloc(ctx, (void**)&mesh->verts, mesh->nv * 3 * sizeof(double))) return fail(s);
  if (bf_status s = bf_obj_alloc(ctx, (void**)&mesh->tris, mesh->nt * 3 * sizeof(int32_t))) return fail(s);
  BF_LAUNCH(ctx, "surf_verts", k_surf_verts, dim3(g), dim3(kThreads), 0, S, mask, vstart, mesh->verts);
  BF_LAUNCH(ctx, "surf_tris", k_surf_tris, dim3(g), dim3(kThreads), 0, S, mask, vstart, mesh->verts, tstart,
            mesh->tris);
  if (bf_status s = bf_launch_check(ctx, "surface extraction")) return fail(s);
  if (n_vert) *n_vert = mesh->nv;
  if (n_tri) *n_tri = mesh->nt;
  *out = mesh;
  return BF_OK;
}

extern "C" bf_status bf_mesh_view(const bf_mesh* mesh, bf_mesh_arrays* out) {
  if (!mesh || !out) return BF_ERR_INVALID_ARG;
  out->n_vert = mesh->nv;
  out->n_tri = mesh->nt;
  out->verts = mesh->verts;
  out->tris = mesh->tris;
  return BF_OK;
}

extern "C" bf_status bf_mesh_free(bf_ctx* ctx, bf_mesh* mesh) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  if (!mesh) return BF_OK;
  bf_obj_free(ctx, mesh->verts);
  bf_obj_free(ctx, mesh->tris);
  delete mesh;
  return BF_OK;
}

extern "C" bf_status bf_surface_metrics(bf_ctx* ctx, const double* pred_dev, int64_t n_pred, const double* gt_dev,
                                        int64_t n_gt, int32_t n_thr, const double* thr_host, bf_metrics* out,
                                        double* d_pred_dev, double* d_gt_dev) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, out, "bf_surface_metrics: NULL output");
  BF_CHECK(ctx, n_pred > 0 && n_gt > 0 && pred_dev && gt_dev, "bf_surface_metrics: empty or NULL point set");
  BF_CHECK(ctx, n_thr >= 0 && n_thr <= kMaxThr && (n_thr == 0 || thr_host),
           "bf_surface_metrics: n_thr=%d outside [0, %d]", n_thr, kMaxThr);
  BF_HIP(ctx, hipSetDevice(ctx->device));
  const int nbp = (int)std::min<int64_t>(bf_cdiv(std::max(n_pred, n_gt), kThreads), 1024);
  const int W = 2 + kMaxThr;
  // workspace: thresholds | partials | totals (2 x W) | distances (if not given)
  const size_t sthr = 256, spart = al256((size_t)nbp * W * 8), stot = al256(2 * W * 8);
  const size_t sdp = d_pred_dev ? 0 : al256(n_pred * 8), sdg = d_gt_dev ? 0 : al256(n_gt * 8);
  char* ws = nullptr;
  BF_TRY(bf_ws(ctx, bf_ctx::WS_SURF, sthr + spart + stot + sdp + sdg, (void**)&ws));
  double* dthr = (double*)ws;
  double* part = (double*)(ws + sthr);
  double* tot = (double*)(ws + sthr + spart);
  double* dp = d_pred_dev ? d_pred_dev : (double*)(ws + sthr + spart + stot);
  double* dg = d_gt_dev ? d_gt_dev : (double*)(ws + sthr + spart + stot + sdp);
  double hthr[kMaxThr] = {0.0};
  for (int t = 0; t < n_thr; ++t) hthr[t] = thr_host[t];
  BF_HIP(ctx, hipMemcpyAsync(dthr, hthr, sizeof(hthr), hipMemcpyHostToDevice, ctx->stream));
  BF_LAUNCH(ctx, "nn_dist2", k_nn_dist2, dim3((unsigned)bf_cdiv(n_pred, kThreads * kNNPerThread)), dim3(kThreads), 0,
            pred_dev, n_pred, gt_dev, n_gt, dp);
  BF_LAUNCH(ctx, "nn_dist2", k_nn_dist2, dim3((unsigned)bf_cdiv(n_gt, kThreads * kNNPerThread)), dim3(kThreads), 0,
            gt_dev, n_gt, pred_dev, n_pred, dg);
  const int nb1 = (int)std::min<int64_t>(bf_cdiv(n_pred, kThreads), nbp);
  const int nb2 = (int)std::min<int64_t>(bf_cdiv(n_gt, kThreads), nbp);
  hipLaunchKernelGGL(k_metric_partials, dim3(nb1), dim3(kThreads), 0, ctx->stream, dp, n_pred, n_thr, dthr, part);
  hipLaunchKernelGGL(k_metric_total, dim3(1), dim3(64), 0, ctx->stream, part, nb1, tot);
  hipLaunchKernelGGL(k_metric_partials, dim3(nb2), dim3(kThreads), 0, ctx->stream, dg, n_gt, n_thr, dthr, part);
  hipLaunchKernelGGL(k_metric_total, dim3(1), dim3(64), 0, ctx->stream, part, nb2, tot + W);
  BF_TRY(bf_launch_check(ctx, "surface metrics"));
  double* pin = nullptr;
  BF_TRY(bf_pinned(ctx, 2 * W * 8, (void**)&pin));
  BF_HIP(ctx, hipMemcpyAsync(pin, tot, 2 * W * 8, hipMemcpyDeviceToHost, ctx->stream));
  BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *out = bf_metrics{};
  out->n_pred = n_pred;
  out->n_gt = n_gt;
  out->chamfer = pin[0] / (double)n_pred + pin[W] / (double)n_gt;
  out->accuracy = pin[1] / (double)n_pred;
  out->completeness = pin[W + 1] / (double)n_gt;
  out->n_thr = n_thr;
  for (int t = 0; t < n_thr; ++t) {
    const double pr = pin[2 + t] / (double)n_pred, rc = pin[W + 2 + t] / (double)n_gt;
    out->thr[t] = thr_host[t];
    out->precision[t] = pr;
    out->recall[t] = rc;
    out->fscore[t] = pr + rc > 0.0 ? 2.0 * pr * rc / (pr + rc) : 0.0;
  }
  return BF_OK;
}
