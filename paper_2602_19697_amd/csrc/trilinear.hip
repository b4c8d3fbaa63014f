// Trilinear pixel-centric observation rows (Sec. 3.2, eqs. 2-5) and the
// 27-point posterior precision they give (eqs. 7, 10-11).
//
// Samples: every valid pixel (row, col) of view t gives samples at camera
// depths z = D + s h (s = -S..S) along its ray; y = clamp(D - z, -tau, tau);
// the row a_i holds the trilinear weights of the sample point on the 8 voxel
// centres around it, and the sample is kept when all 8 are band voxels.
//
// Deterministic FP64 assembly in four passes:
//   1. count the kept samples of each (view, pixel); exclusive scan;
//   2. emit one 64-bit key per kept sample: the Morton key of its cell (the
//      2x2x2 cube whose lowest voxel is the sample's floor corner) above its
//      sample id ((t H + row) W + col)(2S+1) + (s + S);
//   3. radix-sort the keys (unique, so the order is unique): every cell's
//      samples are then one run in ascending id;
//   4. one thread per cell sums M_c[j][k] = sum (w a_j) a_k (j <= k) and
//      g_c[j] = sum (w y) a_j in that order; one thread per band voxel adds
//      its 8 cells, in the order of its corner index q inside the cell, into
//      Lambda, b and the 26 couplings.
// The sample arithmetic is recomputed from the id in pass 4 with the same
// operation order as in pass 1, so each sum sees the same bits.
#include <hipcub/hipcub.hpp>

#include <cstring>

#include "bf_internal.h"

namespace {

constexpr int kThreads = 256;

struct tri_k {
  bf_grid_k g;
  bf_cam_k c;
  int32_t T, S;
  double na, nc, nz0, nmodel;
  const double* npose;  // [T] or null
  const bf_cell* cells;
  int32_t ncell;
};

// Slot of offset (dx, dy, dz) among the 26 couplings (compile-time when the
// offsets are).
__host__ __device__ constexpr int tri_slot(int dx, int dy, int dz) {
  return ((dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)) < 13 ? ((dx + 1) + 3 * (dy + 1) + 9 * (dz + 1))
                                                       : ((dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)) - 1;
}

// Index of entry (j, k), j <= k, in the row-major upper triangle of an 8x8.
__host__ __device__ constexpr int tri_upper(int j, int k) { return j * 8 - (j * (j - 1)) / 2 + (k - j); }

// One sample in the operation order of the definition; false when the sample
// point does not have all 8 surrounding voxel centres inside the grid.
__device__ __forceinline__ bool tri_sample(const tri_k& K, const float* __restrict__ depth,
                                           const double* __restrict__ poses, int32_t t, int32_t row, int32_t col,
                                           int32_t s, int32_t (&base)[3], double (&a)[8], double& y, double& wv) {
#pragma clang fp contract(off)
  const double D = (double)depth[((int64_t)t * K.c.H + row) * K.c.W + col];
  if (!(D > 0.0) || !isfinite(D)) return false;
  const double z = D + (double)s * K.g.h;
  if (!(z > 0.0)) return false;
  double yv = D - z;
  yv = yv < -K.g.tau ? -K.g.tau : yv;
  yv = yv > K.g.tau ? K.g.tau : yv;
  const double ra = ((double)col - K.c.cx) / K.c.fx;
  const double rb = ((double)row - K.c.cy) / K.c.fy;
  const double* P = poses + 12 * t;
  const double org[3] = {K.g.ox, K.g.oy, K.g.oz};
  double w0[3], w1[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double dw = (P[4 * r] * ra + P[4 * r + 1] * rb) + P[4 * r + 2];
    const double x = P[4 * r + 3] + z * dw;
    const double gc = (x - org[r]) / K.g.h - 0.5;
    const double fl = floor(gc);
    if (!(fl >= 0.0) || !(fl + 1.0 <= (double)(K.g.G - 1))) return false;
    const double f = gc - fl;
    base[r] = (int32_t)fl;
    w0[r] = 1.0 - f;
    w1[r] = f;
  }
#pragma unroll
  for (int q = 0; q < 8; ++q)
    a[q] = (((q & 1) ? w1[0] : w0[0]) * (((q >> 1) & 1) ? w1[1] : w0[1])) * (((q >> 2) & 1) ? w1[2] : w0[2]);
  const double e = D - K.nz0;
  const double sd = K.na + K.nc * (e * e);
  double var = sd * sd + (K.npose ? K.npose[t] : 0.0);
  var = var + K.nmodel;
  y = yv;
  wv = 1.0 / var;
  return true;
}

__device__ __forceinline__ bool tri_corners_in_band(const tri_k& K, const int32_t (&base)[3]) {
  bool in = true;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    in = in && bf_band_index(K.cells, K.ncell, K.g.G, base[0] + (q & 1), base[1] + ((q >> 1) & 1),
                             base[2] + ((q >> 2) & 1)) >= 0;
  return in;
}

// Pass 1: kept samples per (view, pixel).
__global__ __launch_bounds__(256) void k_tri_count(tri_k K, const float* __restrict__ depth,
                                                   const double* __restrict__ poses, int64_t npix_all,
                                                   uint32_t* __restrict__ counts) {
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (tid >= npix_all) return;
  const int64_t plane = (int64_t)K.c.W * K.c.H;
  const int32_t t = (int32_t)(tid / plane);
  const int32_t pix = (int32_t)(tid % plane), row = pix / K.c.W, col = pix % K.c.W;
  uint32_t n = 0;
  for (int32_t s = -K.S; s <= K.S; ++s) {
    int32_t base[3];
    double a[8], y, wv;
    if (tri_sample(K, depth, poses, t, row, col, s, base, a, y, wv) && tri_corners_in_band(K, base)) ++n;
  }
  counts[tid] = n;
}

// Pass 2: one key per kept sample at the (view, pixel)'s scanned offset.
__global__ __launch_bounds__(256) void k_tri_emit(tri_k K, const float* __restrict__ depth,
                                                  const double* __restrict__ poses, int64_t npix_all,
                                                  const uint64_t* __restrict__ offs, int idbits,
                                                  uint64_t* __restrict__ keys) {
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (tid >= npix_all) return;
  const int64_t plane = (int64_t)K.c.W * K.c.H;
  const int32_t t = (int32_t)(tid / plane);
  const int32_t pix = (int32_t)(tid % plane), row = pix / K.c.W, col = pix % K.c.W;
  uint64_t o = offs[tid];
  for (int32_t s = -K.S; s <= K.S; ++s) {
    int32_t base[3];
    double a[8], y, wv;
    if (!tri_sample(K, depth, poses, t, row, col, s, base, a, y, wv) || !tri_corners_in_band(K, base)) continue;
    const uint64_t id = (uint64_t)tid * (uint64_t)(2 * K.S + 1) + (uint64_t)(s + K.S);
    keys[o++] = (bf_morton((uint32_t)base[0], (uint32_t)base[1], (uint32_t)base[2]) << idbits) | id;
  }
}

// Pass 3b: run heads of the sorted keys (a new cell starts).
__global__ __launch_bounds__(256) void k_tri_heads(const uint64_t* __restrict__ keys, int64_t n, int idbits,
                                                   int32_t* __restrict__ head) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  head[i] = (i == 0 || (keys[i] >> idbits) != (keys[i - 1] >> idbits)) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_tri_starts(const uint64_t* __restrict__ keys, int64_t n, int idbits,
                                                    const int32_t* __restrict__ head,
                                                    const int32_t* __restrict__ cidx, int64_t* __restrict__ cstart,
                                                    uint64_t* __restrict__ ckey) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n || !head[i]) return;
  cstart[cidx[i]] = i;
  ckey[cidx[i]] = keys[i] >> idbits;
}

// Pass 4a: per-cell sums in ascending sample id.
__global__ __launch_bounds__(256) void k_tri_cellsum(tri_k K, const float* __restrict__ depth,
                                                     const double* __restrict__ poses,
                                                     const uint64_t* __restrict__ keys, int idbits,
                                                     const int64_t* __restrict__ cstart, int64_t ncells,
                                                     double* __restrict__ cellM, double* __restrict__ cellG) {
#pragma clang fp contract(off)
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  double M[36], Gv[8];
#pragma unroll
  for (int e = 0; e < 36; ++e) M[e] = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) Gv[j] = 0.0;
  const uint64_t idmask = (1ull << idbits) - 1ull, ns = (uint64_t)(2 * K.S + 1);
  for (int64_t i = cstart[c]; i < cstart[c + 1]; ++i) {
    uint64_t id = keys[i] & idmask;
    const int32_t s = (int32_t)(id % ns) - K.S;
    id /= ns;
    const int32_t col = (int32_t)(id % (uint64_t)K.c.W);
    id /= (uint64_t)K.c.W;
    const int32_t row = (int32_t)(id % (uint64_t)K.c.H);
    const int32_t t = (int32_t)(id / (uint64_t)K.c.H);
    int32_t base[3];
    double a[8], y, wv;
    tri_sample(K, depth, poses, t, row, col, s, base, a, y, wv);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double wa = wv * a[j];
#pragma unroll
      for (int k = j; k < 8; ++k) M[tri_upper(j, k)] = M[tri_upper(j, k)] + wa * a[k];
      Gv[j] = Gv[j] + (wv * y) * a[j];
    }
  }
#pragma unroll
  for (int e = 0; e < 36; ++e) cellM[c * 36 + e] = M[e];
#pragma unroll
  for (int j = 0; j < 8; ++j) cellG[c * 8 + j] = Gv[j];
}

__device__ __forceinline__ int64_t tri_find_cell(const uint64_t* __restrict__ ckey, int64_t ncells, uint64_t key) {
  int64_t lo = 0, hi = ncells;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (ckey[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return (lo < ncells && ckey[lo] == key) ? lo : -1;
}

// Pass 4b: per band voxel, its 8 cells in corner order -> Lambda, b, the 26
// couplings and their neighbour indices, diag(Q), rhs.
__global__ __launch_bounds__(256) void k_tri_gather(tri_k K, const uint64_t* __restrict__ keys,
                                                    const double* __restrict__ tsdf, const int32_t* __restrict__ deg,
                                                    int64_t n, const uint64_t* __restrict__ ckey, int64_t ncells,
                                                    const double* __restrict__ cellM,
                                                    const double* __restrict__ cellG, double lam, double eps,
                                                    double lam_b, double* __restrict__ Lambda,
                                                    double* __restrict__ b, double* __restrict__ rhs,
                                                    double* __restrict__ diag, double* __restrict__ dinv,
                                                    float* __restrict__ diag32, float* __restrict__ dinv32,
                                                    double* __restrict__ off, float* __restrict__ off32,
                                                    int32_t* __restrict__ nb26) {
#pragma clang fp contract(off)
  const int64_t v = bf_xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  if (v >= n) return;
  const uint64_t key = keys[v];
  const int32_t i = (int32_t)bf_compact3(key), j = (int32_t)bf_compact3(key >> 1), k = (int32_t)bf_compact3(key >> 2);
  double L = 0.0, B = 0.0, cpl[26];
#pragma unroll
  for (int t = 0; t < 26; ++t) cpl[t] = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int32_t ci = i - (q & 1), cj = j - ((q >> 1) & 1), ck = k - ((q >> 2) & 1);
    if (ci < 0 || cj < 0 || ck < 0) continue;
    const int64_t c = tri_find_cell(ckey, ncells, bf_morton((uint32_t)ci, (uint32_t)cj, (uint32_t)ck));
    if (c < 0) continue;
    const double* Mc = cellM + c * 36;
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const double m = Mc[tri_upper(q < kk ? q : kk, q < kk ? kk : q)];
      if (kk == q) {
        L = L + m;
      } else {
        const int slot = tri_slot((kk & 1) - (q & 1), ((kk >> 1) & 1) - ((q >> 1) & 1),
                                  ((kk >> 2) & 1) - ((q >> 2) & 1));
        cpl[slot] = cpl[slot] + m;
      }
    }
    B = B + cellG[c * 8 + q];
  }
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx == 0 && dy == 0 && dz == 0) continue;
        const int slot = tri_slot(dx, dy, dz);
        const int32_t u = bf_band_index(K.cells, K.ncell, K.g.G, i + dx, j + dy, k + dz);
        double o = cpl[slot];
        if ((dx != 0) + (dy != 0) + (dz != 0) == 1 && u >= 0) o = o - lam;
        o = u >= 0 ? o : 0.0;
        nb26[slot * n + v] = u;  // slot-major [26][N]: coalesced across the rows of a wave
        off[slot * n + v] = o;
        off32[slot * n + v] = (float)o;
      }
  const int32_t dg = deg[v];
  double dq = L + lam * (double)dg;
  dq = dq + eps;
  double h = B;
  if (lam_b != 0.0 && dg < 6) {
    dq = dq + lam_b;
    h = h + lam_b * tsdf[v];
  }
  Lambda[v] = L;
  b[v] = B;
  rhs[v] = h;
  diag[v] = dq;
  const double inv = 1.0 / dq;
  dinv[v] = inv;
  diag32[v] = (float)dq;
  dinv32[v] = (float)inv;
}

__global__ __launch_bounds__(256) void k_tri_set_i64(int64_t* p, int64_t v) { *p = v; }

int bits_for(uint64_t n) {  // bits needed to hold the values 0..n-1
  int b = 0;
  while (b < 64 && (n - 1) >> b) ++b;
  return b;
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" bf_status bf_assemble_trilinear(bf_ctx* ctx, const bf_band* band, const bf_camera* cam, int32_t T,
                                           const float* depth_dev, const double* c2w_dev, const bf_noise* noise,
                                           const bf_prior* prior, int32_t samples_per_side, bf_system** out,
                                           int64_t* n_samples_out) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, band && cam && noise && prior && out, "bf_assemble_trilinear: NULL argument");
  *out = nullptr;
  if (n_samples_out) *n_samples_out = 0;
  BF_CHECK(ctx, T >= 0, "bf_assemble_trilinear: T < 0");
  BF_CHECK(ctx, samples_per_side >= 0 && samples_per_side <= 15,
           "bf_assemble_trilinear: samples_per_side=%d outside [0, 15]", samples_per_side);
  BF_CHECK(ctx, T == 0 || band->n == 0 || (depth_dev && c2w_dev && cam->width > 0 && cam->height > 0),
           "bf_assemble_trilinear: bad camera or NULL depth/poses");
  BF_CHECK(ctx, prior->lambda >= 0.0 && prior->eps >= 0.0 && prior->lambda_b >= 0.0,
           "bf_assemble_trilinear: lambda, eps and lambda_b must be >= 0");
  BF_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t N = band->n;
  const int S = samples_per_side;
  const int64_t npix_all = N > 0 ? (int64_t)T * cam->width * cam->height : 0;
  const int idbits = bits_for((uint64_t)std::max<int64_t>(npix_all, 1) * (uint64_t)(2 * S + 1));
  const int cellbits = 3 * band->log2P;
  BF_CHECK(ctx, idbits + cellbits <= 64, "bf_assemble_trilinear: %d-bit sample ids and %d-bit cells exceed 64 bits",
           idbits, cellbits);
  // candidate samples below 2^31: the 32-bit per-pixel counts, their scan and
  // the cell scan cannot overflow
  BF_CHECK(ctx, npix_all * (int64_t)(2 * S + 1) < (1ll << 31),
           "bf_assemble_trilinear: %lld candidate samples exceed 2^31", (long long)(npix_all * (2 * S + 1)));
  int64_t* pin = nullptr;
  BF_TRY(bf_pinned(ctx, 16, (void**)&pin));
  bf_system* sys = new (std::nothrow) bf_system();
  if (!sys) return bf_fail(ctx, BF_ERR_OOM, "bf_assemble_trilinear: host allocation");
  sys->n = N;
  sys->band = band;
  sys->lambda = prior->lambda;
  sys->eps = prior->eps;
  sys->lambda_b = prior->lambda_b;
  sys->T = T;
  sys->kind = BF_SYSTEM_TRILINEAR;
  auto fail = [&](bf_status st) {
    bf_system_free(ctx, sys);
    return st;
  };
  if (N == 0) {
    *out = sys;
    return BF_OK;
  }
  if (bf_status s = bf_obj_alloc_parts(ctx, &sys->block,
                                       {{(void**)&sys->Lambda, (size_t)N * 8}, {(void**)&sys->b, (size_t)N * 8},
                                        {(void**)&sys->rhs, (size_t)N * 8}, {(void**)&sys->diag, (size_t)N * 8},
                                        {(void**)&sys->dinv, (size_t)N * 8}, {(void**)&sys->diag32, (size_t)N * 4},
                                        {(void**)&sys->dinv32, (size_t)N * 4}, {(void**)&sys->off, (size_t)N * 26 * 8},
                                        {(void**)&sys->off32, (size_t)N * 26 * 4},
                                        {(void**)&sys->nb26, (size_t)N * 26 * 4}}))
    return fail(s);

  tri_k K{};
  K.g = bf_grid_k{band->G, band->h, band->origin[0], band->origin[1], band->origin[2], band->tau, band->band};
  K.c = bf_cam_k{cam->width, cam->height, cam->fx, cam->fy, cam->cx, cam->cy};
  K.T = T;
  K.S = S;
  K.na = noise->a;
  K.nc = noise->c;
  K.nz0 = noise->z0;
  K.nmodel = noise->sigma2_model;
  K.npose = noise->sigma2_pose_dev;
  K.cells = band->cells;
  K.ncell = band->ncell;

  // passes 1-2 workspace: counts | offsets | scan temp
  int64_t total = 0;
  size_t scan_tmp = 0;
  if (npix_all > 0 && hipcub::DeviceScan::ExclusiveSum(nullptr, scan_tmp, (const uint32_t*)nullptr,
                                                       (uint64_t*)nullptr, (int)npix_all, ctx->stream) != hipSuccess)
    return fail(bf_fail(ctx, BF_ERR_HIP, "bf_assemble_trilinear: scan sizing failed"));
  char* ws = nullptr;
  const size_t w1 = al256(npix_all * 4), w2 = al256(npix_all * 8);
  if (bf_status s = bf_ws(ctx, bf_ctx::WS_TRI, w1 + w2 + al256(scan_tmp) + 256, (void**)&ws)) return fail(s);
  uint32_t* counts = (uint32_t*)ws;
  uint64_t* offs = (uint64_t*)(ws + w1);
  void* tmp = ws + w1 + w2;
  if (npix_all > 0) {
    const unsigned g1 = (unsigned)bf_cdiv(npix_all, kThreads);
    BF_LAUNCH(ctx, "tri_count", k_tri_count, dim3(g1), dim3(kThreads), 0, K, depth_dev, c2w_dev, npix_all, counts);
    if (hipcub::DeviceScan::ExclusiveSum(tmp, scan_tmp, counts, offs, (int)npix_all, ctx->stream) != hipSuccess)
      return fail(bf_fail(ctx, BF_ERR_HIP, "bf_assemble_trilinear: scan failed"));
    uint32_t last = 0;
    if (hipMemcpyAsync(pin, offs + npix_all - 1, 8, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(pin + 1, counts + npix_all - 1, 4, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      return fail(bf_fail(ctx, BF_ERR_HIP, "bf_assemble_trilinear: count read-back failed"));
    memcpy(&last, pin + 1, 4);
    total = pin[0] + (int64_t)last;
  }
  sys->n_samples = total;

  // passes 2-4 workspace (after the counts are consumed): keys x2 | head | cidx | cstart | ckey | M | G | temp
  const int64_t tn = std::max<int64_t>(total, 1);
  size_t sort_tmp = 0, scan2_tmp = 0;
  if (total > 0) {
    if (hipcub::DeviceRadixSort::SortKeys(nullptr, sort_tmp, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                          (int)total, 0, idbits + cellbits, ctx->stream) != hipSuccess ||
        hipcub::DeviceScan::ExclusiveSum(nullptr, scan2_tmp, (const int32_t*)nullptr, (int32_t*)nullptr, (int)total,
                                         ctx->stream) != hipSuccess)
      return fail(bf_fail(ctx, BF_ERR_HIP, "bf_assemble_trilinear: sort sizing failed"));
  }
  // cells <= samples; M and G sized by samples until the cell count is known
  const size_t sz_keys = al256(tn * 8), sz_i32 = al256(tn * 4), sz_cs = al256((tn + 1) * 8), sz_ck = al256(tn * 8);
  const size_t sz_M = al256(tn * 36 * 8), sz_G = al256(tn * 8 * 8);
  const size_t sz_tmp = al256(std::max(sort_tmp, scan2_tmp));
  const size_t need = w1 + w2 + 2 * sz_keys + 2 * sz_i32 + sz_cs + sz_ck + sz_M + sz_G + sz_tmp;
  // grow the workspace keeping the offsets (they are still needed by pass 2)
  char* ws2 = nullptr;
  if (bf_status s = bf_dev_alloc(ctx, (void**)&ws2, need - w1 - w2)) return fail(s);
  uint64_t* keys_a = (uint64_t*)ws2;
  uint64_t* keys_b = (uint64_t*)(ws2 + sz_keys);
  int32_t* head = (int32_t*)(ws2 + 2 * sz_keys);
  int32_t* cidx = (int32_t*)(ws2 + 2 * sz_keys + sz_i32);
  int64_t* cstart = (int64_t*)(ws2 + 2 * sz_keys + 2 * sz_i32);
  uint64_t* ckey = (uint64_t*)(ws2 + 2 * sz_keys + 2 * sz_i32 + sz_cs);
  double* cellM = (double*)(ws2 + 2 * sz_keys + 2 * sz_i32 + sz_cs + sz_ck);
  double* cellG = (double*)(ws2 + 2 * sz_keys + 2 * sz_i32 + sz_cs + sz_ck + sz_M);
  void* tmp2 = ws2 + 2 * sz_keys + 2 * sz_i32 + sz_cs + sz_ck + sz_M + sz_G;
  auto fail2 = [&](bf_status st) {
    bf_dev_free(ctx, ws2);
    return fail(st);
  };
  int64_t ncells = 0;
  if (total > 0) {
    const unsigned g1 = (unsigned)bf_cdiv(npix_all, kThreads);
    BF_LAUNCH(ctx, "tri_emit", k_tri_emit, dim3(g1), dim3(kThreads), 0, K, depth_dev, c2w_dev, npix_all, offs, idbits,
              keys_a);
    if (hipcub::DeviceRadixSort::SortKeys(tmp2, sort_tmp, keys_a, keys_b, (int)total, 0, idbits + cellbits,
                                          ctx->stream) != hipSuccess)
      return fail2(bf_fail(ctx, BF_ERR_HIP, "bf_assemble_trilinear: sort failed"));
    const unsigned g2 = (unsigned)bf_cdiv(total, kThreads);
    BF_LAUNCH(ctx, "tri_heads", k_tri_heads, dim3(g2), dim3(kThreads), 0, keys_b, total, idbits, head);
    if (hipcub::DeviceScan::ExclusiveSum(tmp2, scan2_tmp, head, cidx, (int)total, ctx->stream) != hipSuccess)
      return fail2(bf_fail(ctx, BF_ERR_HIP, "bf_assemble_trilinear: cell scan failed"));
    int32_t* p32 = (int32_t*)pin;
    if (hipMemcpyAsync(p32, cidx + total - 1, 4, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(p32 + 1, head + total - 1, 4, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      return fail2(bf_fail(ctx, BF_ERR_HIP, "bf_assemble_trilinear: cell count read-back failed"));
    ncells = (int64_t)p32[0] + p32[1];
    BF_LAUNCH(ctx, "tri_starts", k_tri_starts, dim3(g2), dim3(kThreads), 0, keys_b, total, idbits, head, cidx, cstart,
              ckey);
    hipLaunchKernelGGL(k_tri_set_i64, dim3(1), dim3(1), 0, ctx->stream, cstart + ncells, total);
    BF_LAUNCH(ctx, "tri_cellsum", k_tri_cellsum, dim3((unsigned)bf_cdiv(ncells, kThreads)), dim3(kThreads), 0, K,
              depth_dev, c2w_dev, keys_b, idbits, cstart, ncells, cellM, cellG);
  }
  sys->n_cells = ncells;
  BF_LAUNCH(ctx, "tri_gather", k_tri_gather, dim3((unsigned)bf_round8(bf_cdiv(N, kThreads))), dim3(kThreads), 0, K,
            band->keys, band->tsdf, band->deg, N, ckey, ncells, cellM, cellG, prior->lambda, prior->eps,
            prior->lambda_b, sys->Lambda, sys->b, sys->rhs, sys->diag, sys->dinv, sys->diag32, sys->dinv32,
            sys->off, sys->off32, sys->nb26);
  if (bf_status s = bf_launch_check(ctx, "trilinear assembly")) return fail2(s);
  bf_dev_free(ctx, ws2);
  BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (n_samples_out) *n_samples_out = total;
  *out = sys;
  return BF_OK;
}
