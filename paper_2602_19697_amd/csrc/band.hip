// Coarse TSDF bootstrap, narrow-band activation in Morton order, key->index
// block records and 6-neighbour table (Sec. 3.3-3.4, eq. 1; Algorithm 1
// steps 1-2).
//
// Layout: the dense coarse TSDF lives on a P^3 cube (P = next power of two
// >= G) indexed by Morton code m, so walking m = 0..P^3-1 visits voxels in
// key order and a block-wise stream compaction emits the band already sorted.
// Morton-local voxels also project to nearby pixels, which keeps the depth
// gathers of a block inside a few cache lines.
//
// Screening: only voxels of the band need an exact TSDF.  Before fusing a
// block, every 4^3 cell of it is tested against every view with a min/max
// pyramid of the valid depths (block tiles first, then cells; see
// k_tsdf_count): if in each view every voxel of the cell either sees free
// space further than the band half-width in front of the surface (all its
// observations exceed the band, as the truncation does) or lies more than tau
// behind it (occluded: skipped), no voxel of the cell can be in the band, and
// the cell is not fused, nor are its dense values stored or read back by the
// scatter.  The band (keys, TSDF, weights) is the same bit for bit; screening
// is off when the dense grid is kept for inspection.
#include "bf_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 4;                    // voxels per thread per block tile
constexpr int kTile = kThreads * kItems;     // Morton codes per block

__global__ __launch_bounds__(256) void k_validate_depth(const float* __restrict__ depth, int64_t n,
                                                        int* __restrict__ flag) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float d = depth[i];
    if (!(d >= 0.0f) || d == INFINITY) bad = 1;
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// Min/max pyramid of the valid depths of every view: level l holds, per
// 2^l x 2^l pixel block, the smallest and largest depth D > 0 (+inf / -1 when
// the block has none).  Levels are packed per view at offsets off[l].  Level
// 0 is the depth map itself under that rule, so it is read from there and its
// slots stay unwritten.
constexpr int kMaxLevels = 16;
struct Pyr {
  int nl;
  int32_t w[kMaxLevels], h[kMaxLevels];
  int64_t off[kMaxLevels];
  int64_t per_view;
};

// Levels 0..kTileLevels of one 32x32 pixel tile of one view.  A level-l cell
// holds the extremes over its 2^l x 2^l base pixels inside the image, so the
// tile-local reduction equals the level-by-level one (min and max are exact in
// any order).  Thread t holds 4 adjacent pixels of row t / 8 (one 16-byte load
// when W is a multiple of 4), so a wave holds 8 full rows: levels 1-3 combine
// within the wave by lane exchanges (rows y ^ 1, y ^ 2, y ^ 4 are lanes ^ 8,
// ^ 16, ^ 32; quads x ^ 4 are lanes ^ 1), and only levels 4-5 go through LDS.
constexpr int kPyrTile = 32;
constexpr int kTileLevels = 5;  // 32 >> 5 = 1
__device__ __forceinline__ void pyr_pair(float& a, float& b, int lanemask) {
  a = fminf(a, __shfl_xor(a, lanemask, 64));
  b = fmaxf(b, __shfl_xor(b, lanemask, 64));
}
// The kernel reads every pixel once, so it also flags invalid depth (NaN,
// inf or negative) as k_validate_depth does.
__global__ __launch_bounds__(256) void k_pyr_tiles(const float* __restrict__ depth, int32_t W, int32_t H, Pyr P,
                                                   float* __restrict__ dmin, float* __restrict__ dmax,
                                                   int* __restrict__ flag) {
  __shared__ float l3lo[16], l3hi[16];
  const int t = blockIdx.z;
  const int32_t x0 = blockIdx.x * kPyrTile, y0 = blockIdx.y * kPyrTile;
  const float* D = depth + (int64_t)t * W * H;
  float* mn = dmin + (int64_t)t * P.per_view;
  float* mx = dmax + (int64_t)t * P.per_view;
  const int ly = threadIdx.x >> 3, lx = (threadIdx.x & 7) * 4;  // tile row, first column
  const int32_t gy = y0 + ly, gx = x0 + lx;
  float d[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  bool in[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) in[k] = gy < H && gx + k < W;
  if ((W & 3) == 0) {
    if (in[0]) {
      const float4 v = *reinterpret_cast<const float4*>(D + (int64_t)gy * W + gx);
      d[0] = v.x;
      d[1] = v.y;
      d[2] = v.z;
      d[3] = v.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (in[k]) d[k] = D[(int64_t)gy * W + gx + k];
  }
  int bad = 0;
  float a[4], b[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (in[k] && (!(d[k] >= 0.0f) || d[k] == INFINITY)) bad = 1;
    const bool ok = in[k] && d[k] > 0.0f;
    a[k] = ok ? d[k] : INFINITY;
    b[k] = ok ? d[k] : -1.0f;
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
  // level 1: pixel pairs of the thread, rows y and y ^ 1
  float a1[2], b1[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    a1[h] = fminf(a[2 * h], a[2 * h + 1]);
    b1[h] = fmaxf(b[2 * h], b[2 * h + 1]);
    pyr_pair(a1[h], b1[h], 8);
  }
  if (P.nl > 1 && (ly & 1) == 0) {
    const int32_t cy = gy >> 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int32_t cx = (gx >> 1) + h;
      if (cx < P.w[1] && cy < P.h[1]) {
        mn[P.off[1] + (int64_t)cy * P.w[1] + cx] = a1[h];
        mx[P.off[1] + (int64_t)cy * P.w[1] + cx] = b1[h];
      }
    }
  }
  // level 2: the thread's 4 columns, rows y .. y ^ 3
  float a2 = fminf(a1[0], a1[1]), b2 = fmaxf(b1[0], b1[1]);
  pyr_pair(a2, b2, 16);
  if (P.nl > 2 && (ly & 3) == 0) {
    const int32_t cx = gx >> 2, cy = gy >> 2;
    if (cx < P.w[2] && cy < P.h[2]) {
      mn[P.off[2] + (int64_t)cy * P.w[2] + cx] = a2;
      mx[P.off[2] + (int64_t)cy * P.w[2] + cx] = b2;
    }
  }
  // level 3: quads x, x ^ 4 (lanes ^ 1) and rows y .. y ^ 7 (lanes ^ 32)
  pyr_pair(a2, b2, 1);
  pyr_pair(a2, b2, 32);
  if ((threadIdx.x & 63) < 8 && (threadIdx.x & 1) == 0) {
    if (P.nl > 3) {
      const int32_t cx = gx >> 3, cy = gy >> 3;
      if (cx < P.w[3] && cy < P.h[3]) {
        mn[P.off[3] + (int64_t)cy * P.w[3] + cx] = a2;
        mx[P.off[3] + (int64_t)cy * P.w[3] + cx] = b2;
      }
    }
    // level-3 grid of the tile: 4 x 4, row = wave, column = quad / 2
    l3lo[(threadIdx.x >> 6) * 4 + ((threadIdx.x & 7) >> 1)] = a2;
    l3hi[(threadIdx.x >> 6) * 4 + ((threadIdx.x & 7) >> 1)] = b2;
  }
  __syncthreads();
  if (threadIdx.x < 4 && P.nl > 4) {
    // level 4: the 2 x 2 cells of 16 x 16 pixels, each over 2 x 2 level-3 cells
    const int i = threadIdx.x & 1, j = threadIdx.x >> 1;
    float a4 = INFINITY, b4 = -1.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = (2 * j + (q >> 1)) * 4 + 2 * i + (q & 1);
      a4 = fminf(a4, l3lo[e]);
      b4 = fmaxf(b4, l3hi[e]);
    }
    const int32_t cx = (x0 >> 4) + i, cy = (y0 >> 4) + j;
    if (cx < P.w[4] && cy < P.h[4]) {
      mn[P.off[4] + (int64_t)cy * P.w[4] + cx] = a4;
      mx[P.off[4] + (int64_t)cy * P.w[4] + cx] = b4;
    }
    if (threadIdx.x == 0 && P.nl > 5) {
      // level 5: the whole tile
      float a5 = INFINITY, b5 = -1.0f;
      for (int e = 0; e < 16; ++e) {
        a5 = fminf(a5, l3lo[e]);
        b5 = fmaxf(b5, l3hi[e]);
      }
      const int32_t cx5 = x0 >> 5, cy5 = y0 >> 5;
      if (cx5 < P.w[5] && cy5 < P.h[5]) {
        mn[P.off[5] + (int64_t)cy5 * P.w[5] + cx5] = a5;
        mx[P.off[5] + (int64_t)cy5 * P.w[5] + cx5] = b5;
      }
    }
  }
}

// The remaining levels of one view (one block per view), each from the one
// below it in global memory.
__global__ __launch_bounds__(1024) void k_pyr_top(Pyr P, float* __restrict__ dmin, float* __restrict__ dmax) {
  const int t = blockIdx.x;
  float* mn = dmin + (int64_t)t * P.per_view;
  float* mx = dmax + (int64_t)t * P.per_view;
  for (int l = kTileLevels + 1; l < P.nl; ++l) {
    __threadfence_block();
    __syncthreads();
    const int32_t pw = P.w[l - 1], ph = P.h[l - 1];
    const int64_t cells = (int64_t)P.w[l] * P.h[l];
    for (int64_t q = threadIdx.x; q < cells; q += blockDim.x) {
      const int32_t x = (int32_t)(q % P.w[l]), y = (int32_t)(q / P.w[l]);
      float a = INFINITY, b = -1.0f;
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int32_t cx = 2 * x + dx, cy = 2 * y + dy;
          if (cx < pw && cy < ph) {
            a = fminf(a, mn[P.off[l - 1] + (int64_t)cy * pw + cx]);
            b = fmaxf(b, mx[P.off[l - 1] + (int64_t)cy * pw + cx]);
          }
        }
      mn[P.off[l] + q] = a;
      mx[P.off[l] + q] = b;
    }
  }
}

// What can view t do to the voxels of the box of voxel centres from
// (i0, j0, k0) to (i0, j0, k0) + (ni, nj, nk) - 1 (a 4^3 cell or a block tile)?  kViewNone: provably nothing (behind the camera, outside the
// image, no valid depth under the cell, or occluded), so no voxel of the cell
// takes an observation from it; kViewFar: each voxel it observes sees free
// space further than the band in front of the surface, so it adds to the TSDF
// but cannot bring a voxel into the band; kViewMay: anything else (see the
// file comment).  The corner
// centres are the lowest one plus sums of the three rotated cell edges (FP64);
// the Z range over the cell follows from the edge signs, and the extremes of
// the projected u, v over the box are at its 8 corners.  The test is a filter,
// not part of the result, so the projection runs in FP32: its error is a few
// 1e-7 of |u| (the coordinates stay FP64), which the twentieth-of-a-pixel
// widening covers wherever an endpoint can fall near the image.
constexpr int kViewNone = 0, kViewFar = 1, kViewMay = 2;

__device__ int cell_view_class(const bf_grid_k& g, const bf_cam_k& c, const Pyr& P,
                                     const float* __restrict__ depth_t,
                                     const float* __restrict__ dmin, const float* __restrict__ dmax,
                                     const double* __restrict__ Pose, int t, int32_t i0, int32_t j0, int32_t k0,
                                     int32_t ni, int32_t nj, int32_t nk) {
  const double x = g.ox + ((double)i0 + 0.5) * g.h;
  const double y = g.oy + ((double)j0 + 0.5) * g.h;
  const double z = g.oz + ((double)k0 + 0.5) * g.h;
  const double dx = x - Pose[3], dy = y - Pose[7], dz = z - Pose[11];
  const double X0 = Pose[0] * dx + Pose[4] * dy + Pose[8] * dz;
  const double Y0 = Pose[1] * dx + Pose[5] * dy + Pose[9] * dz;
  const double Z0 = Pose[2] * dx + Pose[6] * dy + Pose[10] * dz;
  // lowest to highest voxel centre of the box along each axis
  const double ex = (ni - 1) * g.h, ey = (nj - 1) * g.h, ez = (nk - 1) * g.h;
  const double ax = ex * Pose[0], ay = ex * Pose[1], az = ex * Pose[2];  // per grid-x edge
  const double bx = ey * Pose[4], by = ey * Pose[5], bz = ey * Pose[6];  // per grid-y edge
  const double qx = ez * Pose[8], qy = ez * Pose[9], qz = ez * Pose[10];  // per grid-z edge
  const double zlo = Z0 + fmin(az, 0.0) + fmin(bz, 0.0) + fmin(qz, 0.0);
  const double zhi = Z0 + fmax(az, 0.0) + fmax(bz, 0.0) + fmax(qz, 0.0);
  const double zmargin = 1e-9 + 1e-12 * fabs(zhi);
  if (zhi < -zmargin) return kViewNone;  // the whole cell is behind the camera: never observed
  if (zlo <= 1e-6) return kViewMay;      // straddles the camera plane: no projection bound
  const float fx = (float)c.fx, fy = (float)c.fy;
  float ulo = INFINITY, uhi = -INFINITY, vlo = INFINITY, vhi = -INFINITY;
#pragma unroll
  for (int corner = 0; corner < 8; ++corner) {
    const double X = X0 + ((corner & 1) ? ax : 0.0) + ((corner & 2) ? bx : 0.0) + ((corner & 4) ? qx : 0.0);
    const double Y = Y0 + ((corner & 1) ? ay : 0.0) + ((corner & 2) ? by : 0.0) + ((corner & 4) ? qy : 0.0);
    const double Z = Z0 + ((corner & 1) ? az : 0.0) + ((corner & 2) ? bz : 0.0) + ((corner & 4) ? qz : 0.0);
    const float rz = __builtin_amdgcn_rcpf((float)Z);  // v_rcp_f32, within 1 ulp
    const float u = (fx * (float)X) * rz, v = (fy * (float)Y) * rz;
    ulo = fminf(ulo, u);
    uhi = fmaxf(uhi, u);
    vlo = fminf(vlo, v);
    vhi = fmaxf(vhi, v);
  }
  // pixel (floor(u + cx + 1/2)) range, widened by a twentieth of a pixel
  const float hcx = (float)c.cx + 0.5f, hcy = (float)c.cy + 0.5f;
  const float c0f = floorf(ulo + hcx - 0.05f), c1f = floorf(uhi + hcx + 0.05f);
  const float r0f = floorf(vlo + hcy - 0.05f), r1f = floorf(vhi + hcy + 0.05f);
  if (c1f < 0.0f || r1f < 0.0f || c0f >= (float)c.W || r0f >= (float)c.H) return kViewNone;  // outside the image
  const int32_t c0 = (int32_t)fmaxf(c0f, 0.0f), c1 = (int32_t)fminf(c1f, (float)(c.W - 1));
  const int32_t r0 = (int32_t)fmaxf(r0f, 0.0f), r1 = (int32_t)fminf(r1f, (float)(c.H - 1));
  int l = 0;
  while (l < P.nl - 1 && (((c1 >> l) - (c0 >> l)) > 1 || ((r1 >> l) - (r0 >> l)) > 1)) ++l;
  // level 0 is the depth map (invalid: +inf / -1); the sources are chosen per
  // lane so that every lane runs the same loads
  const bool l0 = l == 0;
  const int64_t base = (int64_t)t * P.per_view + P.off[l];
  const float* smin = l0 ? depth_t : dmin + base;
  const float* smax = l0 ? depth_t : dmax + base;
  const int64_t pitch = l0 ? c.W : P.w[l];
  float lo = INFINITY, hi = -1.0f;
  const int32_t xs[2] = {c0 >> l, c1 >> l}, ys[2] = {r0 >> l, r1 >> l};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t q = (int64_t)ys[a] * pitch + xs[b];
      const float vmin = smin[q], vmax = smax[q];
      lo = fminf(lo, (l0 && !(vmin > 0.0f)) ? INFINITY : vmin);
      hi = fmaxf(hi, (l0 && !(vmax > 0.0f)) ? -1.0f : vmax);
    }
  if (hi < 0.0f) return kViewNone;                               // no valid depth under the cell
  if ((double)hi - zlo < -g.tau - zmargin) return kViewNone;     // occluded: skipped by every voxel
  if ((double)lo - zhi > g.band + zmargin) return kViewFar;      // free space beyond the band
  return kViewMay;
}

// One block tile of Morton codes: fuse every view into the coarse TSDF of each
// voxel (unit weights, truncation, occlusion test), store the dense grid and
// count the band predicate |TSDF| <= band, W > 0.  With screening, a cell is
// fused only if some view may bring one of its voxels into the band, and then
// only over the views that can observe it at all: a view of class kViewNone
// adds nothing to any voxel of the cell, so leaving it out keeps every sum
// (taken in view order) bit for bit.  Per-view masks cover the first
// 32 * kMaskWords views; later views are always fused.
//
// The screen has three levels: k_super_screen tests each super tile (8 block
// tiles, a 32 x 16 x 16 voxel box) against each of the first kTileViews views,
// k_tile_screen each block tile (16 x 8 x 8) against the views its super tile
// left undecided, and k_cell_screen each cell against those its block tile
// left undecided, and against every view past kTileViews.  What holds for a
// box holds for every box inside it, so a kViewNone needs no test below and a
// kViewFar marks the view as contributing for every cell (a cell the view does
// not in fact observe gets no observation from it in the fused loop).
constexpr int kCells = kTile / 64;  // 4^3 cells per block tile; one wave fuses one cell
constexpr int kMaskWords = 8;
constexpr int kTileViews = 32 * kMaskWords;
constexpr int kViewBatch = 4;  // views whose depth loads the fused loop has in flight together
constexpr int kTileI = 16, kTileJ = 8, kTileK = 8;  // Morton tile of kTile codes (x takes the low bit)
static_assert(kTileI * kTileJ * kTileK == kTile, "block tile box");

// The screen's first level: one wave per (super tile, 64 views), a super tile
// being kSuper consecutive block tiles in Morton order (a 32 x 16 x 16 voxel
// box): its kViewFar and kViewMay view masks, smask[sup][0 | 1][word], from
// the ballots of the lanes' tests.
constexpr int kSuper = 8;
constexpr int kSupI = 2 * kTileI, kSupJ = 2 * kTileJ, kSupK = 2 * kTileK;
constexpr int kChunks = kTileViews / 64;  // 64-view chunks of the masks
__global__ __launch_bounds__(256) void k_super_screen(bf_grid_k g, bf_cam_k c, int32_t T, int64_t nsup,
                                                      const float* __restrict__ depth,
                                                      const double* __restrict__ poses, Pyr P,
                                                      const float* __restrict__ dmin,
                                                      const float* __restrict__ dmax, uint32_t* __restrict__ smask) {
#pragma clang fp contract(off)
  const int32_t tv = min(T, kTileViews);
  const int nchunk = (tv + 63) >> 6;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= nsup * nchunk) return;  // whole waves: nsup * nchunk waves exactly
  const int64_t sup = wave / nchunk;
  const int chunk = (int)(wave % nchunk);
  const uint64_t base = (uint64_t)sup * (kSuper * kTile);
  const int32_t si = (int32_t)bf_compact3(base), sj = (int32_t)bf_compact3(base >> 1),
                sk = (int32_t)bf_compact3(base >> 2);
  const int t = chunk * 64 + lane;
  int cls = kViewNone;
  // a super tile with no voxel in the grid needs no test; one reaching past
  // the grid is tested as the whole box (a larger box only widens the classes)
  const bool test = t < tv && si < g.G && sj < g.G && sk < g.G;
  if (test)
    cls = cell_view_class(g, c, P, depth + t * ((int64_t)c.W * c.H), dmin, dmax, poses + 12 * t, t, si, sj, sk,
                          kSupI, kSupJ, kSupK);
  const uint64_t far = __ballot(cls == kViewFar), may = __ballot(cls == kViewMay);
  uint32_t* sm = smask + sup * (2 * kMaskWords);
  if (lane < 2) {
    sm[2 * chunk + lane] = (uint32_t)(far >> (32 * lane));
    sm[kMaskWords + 2 * chunk + lane] = (uint32_t)(may >> (32 * lane));
  }
}

// The second level: one wave per (super tile, 64 views) writes the block
// tiles' masks tmask[tile][0 | 1][word].  Every voxel of a block tile is a
// voxel of its super tile, so a view that is kViewNone or kViewFar for the
// super tile is that for each of its block tiles; only the super tile's
// kViewMay views are tested tile by tile, the lanes taking the (tile, view)
// pairs in turn.  tests[tile][chunk]: the tile's tests in this chunk.
__global__ __launch_bounds__(256) void k_tile_screen(bf_grid_k g, bf_cam_k c, int32_t T, int64_t ntiles,
                                                     const float* __restrict__ depth,
                                                     const double* __restrict__ poses, Pyr P,
                                                     const float* __restrict__ dmin, const float* __restrict__ dmax,
                                                     const uint32_t* __restrict__ smask,
                                                     uint32_t* __restrict__ tmask, uint32_t* __restrict__ tests) {
#pragma clang fp contract(off)
  __shared__ int vlist[kThreads / 64][64];
  __shared__ uint32_t res[kThreads / 64][kSuper][2][2];  // [wave][tile][far | may][word]
  const int32_t tv = min(T, kTileViews);
  const int nchunk = (tv + 63) >> 6;
  const int64_t nsup = bf_cdiv(ntiles, kSuper);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63, wl = threadIdx.x >> 6;
  if (wave >= nsup * nchunk) return;  // whole waves; no workgroup barrier below
  const int64_t sup = wave / nchunk;
  const int chunk = (int)(wave % nchunk);
  const uint32_t* sm = smask + sup * (2 * kMaskWords);
  const uint64_t sfar = (uint64_t)sm[2 * chunk] | ((uint64_t)sm[2 * chunk + 1] << 32);
  const uint64_t smay = (uint64_t)sm[kMaskWords + 2 * chunk] | ((uint64_t)sm[kMaskWords + 2 * chunk + 1] << 32);
  const int m = __popcll(smay);
  // the super tile's kViewMay views of the chunk, in view order
  if ((smay >> lane) & 1ull) vlist[wl][__popcll(smay & ((1ull << lane) - 1ull))] = chunk * 64 + lane;
  if (lane < kSuper * 4) (&res[wl][0][0][0])[lane] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // the wave's LDS writes are done
  for (int q = lane; q < kSuper * m; q += 64) {
    const int kt = q / m, t = vlist[wl][q % m];
    const int64_t tile = sup * kSuper + kt;
    if (tile >= ntiles) continue;
    const uint64_t base = (uint64_t)tile * kTile;
    const int32_t ti = (int32_t)bf_compact3(base), tj = (int32_t)bf_compact3(base >> 1),
                  tk = (int32_t)bf_compact3(base >> 2);
    if (ti >= g.G || tj >= g.G || tk >= g.G) continue;  // no voxel of the tile exists
    const int cls = cell_view_class(g, c, P, depth + t * ((int64_t)c.W * c.H), dmin, dmax, poses + 12 * t, t, ti,
                                    tj, tk, kTileI, kTileJ, kTileK);
    const int bit = t - chunk * 64;
    if (cls == kViewFar) atomicOr(&res[wl][kt][0][bit >> 5], 1u << (bit & 31));
    if (cls == kViewMay) atomicOr(&res[wl][kt][1][bit >> 5], 1u << (bit & 31));
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  if (lane < kSuper * 2) {
    const int kt = lane >> 1, wd = lane & 1;
    const int64_t tile = sup * kSuper + kt;
    if (tile < ntiles) {
      const uint64_t base = (uint64_t)tile * kTile;
      const bool exists = (int32_t)bf_compact3(base) < g.G && (int32_t)bf_compact3(base >> 1) < g.G &&
                          (int32_t)bf_compact3(base >> 2) < g.G;
      uint32_t* tm = tmask + tile * (2 * kMaskWords);
      tm[2 * chunk + wd] = exists ? (uint32_t)(sfar >> (32 * wd)) | res[wl][kt][0][wd] : 0u;
      tm[kMaskWords + 2 * chunk + wd] = exists ? res[wl][kt][1][wd] : 0u;
      if (wd == 0) tests[tile * kChunks + chunk] = exists ? (uint32_t)m : 0u;
    }
  }
}

// Cell tests of one block tile per wave (most tiles leave few views
// undecided): each cell starts with the tile's kViewFar views marked, then is
// tested against the tile's kViewMay views (in view order) and every view past
// kTileViews, the lanes taking the (cell, view) pairs in turn.  Writes the
// tile's live-cell bits and, for its live cells only (the only ones read), the
// view masks cmask[tile][cell][word]; the test count goes to the high word of
// work[tile].  The waves of a workgroup share nothing.
__global__ __launch_bounds__(256) void k_cell_screen(bf_grid_k g, bf_cam_k c, int32_t T,
                                                     const float* __restrict__ depth,
                                                     const double* __restrict__ poses, uint64_t total,
                                                     int64_t ntiles, Pyr P, const float* __restrict__ dmin,
                                                     const float* __restrict__ dmax,
                                                     const uint32_t* __restrict__ tmask,
                                                     uint32_t* __restrict__ cmask, uint32_t* __restrict__ live_bits,
                                                     uint2* __restrict__ work) {
#pragma clang fp contract(off)
  constexpr int NW = kThreads / 64;
  __shared__ int live[NW][kCells];
  __shared__ uint32_t vmask[NW][kCells][kMaskWords];
  __shared__ int may_pre[NW][kMaskWords + 1];
  __shared__ int mlist[NW][kTileViews];  // the tile's kViewMay views in view order
  const int wl = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tile = (int64_t)blockIdx.x * NW + wl;
  if (tile >= ntiles) return;  // whole waves; no workgroup barrier below
  const uint64_t base = (uint64_t)tile * kTile;
  const int64_t plane = (int64_t)c.W * c.H;
  const int32_t tv = min(T, kTileViews);  // views the tile screen tested
  const int tvw = (tv + 31) >> 5;
  const uint32_t* tm = tmask + tile * (2 * kMaskWords);
  if (lane < kCells) live[wl][lane] = 0;
  for (int i = lane; i < kCells * kMaskWords; i += 64) {
    const int w = i % kMaskWords;
    vmask[wl][i / kMaskWords][w] = w < tvw ? tm[w] : 0u;
  }
  // kViewMay views per mask word, and their running count before each word
  const uint32_t mw = lane < tvw ? tm[kMaskWords + lane] : 0u;
  int pre = lane < kMaskWords ? __popc(mw) : 0;
  for (int off = 1; off < kMaskWords; off <<= 1) {
    const int v = __shfl_up(pre, off, 64);
    if (lane >= off) pre += v;
  }
  if (lane < kMaskWords) may_pre[wl][lane + 1] = pre;  // inclusive through word `lane`
  if (lane == 0) may_pre[wl][0] = 0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // the wave's LDS writes are done
  for (int w = 0; w < tvw; ++w) {
    const uint32_t word = (uint32_t)__shfl((int)mw, w, 64);
    const int t = 32 * w + (lane & 31);
    if (lane < 32 && ((word >> (t & 31)) & 1u))
      mlist[wl][may_pre[wl][w] + __popc(word & ((1u << (t & 31)) - 1u))] = t;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  uint32_t tests = 0;
  const int nm_tile = may_pre[wl][kMaskWords];
  const int nm = nm_tile + (T - tv);
  for (int e = lane; e < kCells * nm; e += 64) {
    const int cell = e % kCells, r = e / kCells;
    const int t = r < nm_tile ? mlist[wl][r] : tv + (r - nm_tile);
    const uint64_t m0 = base + (uint64_t)cell * 64;
    if (m0 >= total) continue;
    const int32_t i0 = (int32_t)bf_compact3(m0), j0 = (int32_t)bf_compact3(m0 >> 1),
                  k0 = (int32_t)bf_compact3(m0 >> 2);
    if (i0 >= g.G || j0 >= g.G || k0 >= g.G) continue;
    ++tests;
    const int cls = cell_view_class(g, c, P, depth + t * plane, dmin, dmax, poses + 12 * t, t, i0, j0, k0, 4, 4, 4);
    if (cls != kViewNone && t < kTileViews) atomicOr(&vmask[wl][cell][t >> 5], 1u << (t & 31));
    if (cls == kViewMay) atomicOr(&live[wl][cell], 1);
  }
  for (int off = 32; off > 0; off >>= 1) tests += __shfl_xor(tests, off, 64);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  for (int i = lane; i < kCells * kMaskWords; i += 64)
    if (live[wl][i / kMaskWords])
      cmask[tile * (kCells * kMaskWords) + i] = vmask[wl][i / kMaskWords][i % kMaskWords];
  if (lane == 0) {
    uint32_t lm = 0;
    for (int q = 0; q < kCells; ++q) lm |= live[wl][q] ? 1u << q : 0u;
    live_bits[tile] = lm;
    reinterpret_cast<uint32_t*>(work)[2 * tile + 1] = tests;
  }
}

// Fusion of one block tile over the views the cell masks keep (all views
// without screening); see the comment above kCells.
__global__ __launch_bounds__(256) void k_tsdf_count(bf_grid_k g, bf_cam_k c, int32_t T,
                                                    const float* __restrict__ depth,
                                                    const double* __restrict__ poses,
                                                    uint64_t total, double* __restrict__ dense_t,
                                                    int32_t* __restrict__ dense_w,
                                                    uint32_t* __restrict__ counts, int screen,
                                                    const uint32_t* __restrict__ cmask,
                                                    const uint32_t* __restrict__ live_bits,
                                                    uint2* __restrict__ work, uint32_t* __restrict__ cellmask) {
#pragma clang fp contract(off)
  __shared__ uint32_t wave_cnt[kThreads / 64], wave_fused[kThreads / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kTile;
  const int64_t plane = (int64_t)c.W * c.H;
  const uint32_t lm = screen ? live_bits[blockIdx.x] : (1u << kCells) - 1u;
  if (lm == 0) {  // no live cell: nothing fused, stored or counted
    if (threadIdx.x == 0) {
      counts[blockIdx.x] = 0;
      reinterpret_cast<uint32_t*>(work)[2 * blockIdx.x] = 0;
      cellmask[blockIdx.x] = 0;
    }
    return;
  }
  const uint32_t* cm = cmask + (int64_t)blockIdx.x * (kCells * kMaskWords);
  uint32_t cnt = 0, fused = 0;
  const int nwords = (T + 31) >> 5;
  for (int it = 0; it < kItems; ++it) {
    const uint64_t m = base + (uint64_t)it * kThreads + threadIdx.x;
    if (m >= total) break;
    const int32_t i = (int32_t)bf_compact3(m), j = (int32_t)bf_compact3(m >> 1),
                  k = (int32_t)bf_compact3(m >> 2);
    const int cell = (int)((m - base) >> 6);  // the same for every lane of the wave
    // a screened cell holds no band voxel: its dense values are never read
    // (the scatter skips it by cellmask), so they are not stored either
    if (!((lm >> cell) & 1u)) continue;
    double tsdf = 0.0;
    int32_t W = 0;
    if (i < g.G && j < g.G && k < g.G) {
      double S = 0.0;
      for (int w = 0; w < nwords; ++w) {
        uint32_t bits = (screen && w < kMaskWords) ? cm[cell * kMaskWords + w] : ~0u;
        bits = (uint32_t)__builtin_amdgcn_readfirstlane((int)bits);
        if (w == nwords - 1 && (T & 31)) bits &= (1u << (T & 31)) - 1u;
        fused += (uint32_t)__popc(bits);
        while (bits) {
          // up to kViewBatch views at a time: project, issue every depth
          // load, then add in view order (the sum's order is unchanged)
          int32_t tq[kViewBatch];
          int64_t px[kViewBatch];
          double Zq[kViewBatch];
          float Dq[kViewBatch];
#pragma unroll
          for (int q = 0; q < kViewBatch; ++q) {
            tq[q] = bits ? 32 * w + __builtin_ctz(bits) : -1;
            bits &= bits - 1u;  // 0 stays 0
          }
#pragma unroll
          for (int q = 0; q < kViewBatch; ++q) {
            Zq[q] = 0.0;
            px[q] = -1;
            if (tq[q] >= 0) {
              // the whole pose in one round of scalar loads (the projection
              // would otherwise load the rest only after its depth test)
              double P[12];
#pragma unroll
              for (int e = 0; e < 12; ++e) P[e] = poses[12 * tq[q] + e];
              asm volatile("" ::"s"(P[0]), "s"(P[1]), "s"(P[2]), "s"(P[3]), "s"(P[4]), "s"(P[5]), "s"(P[6]),
                           "s"(P[7]), "s"(P[8]), "s"(P[9]), "s"(P[10]), "s"(P[11]));
              px[q] = bf_project(g, c, P, i, j, k, Zq[q]);
            }
          }
#pragma unroll
          for (int q = 0; q < kViewBatch; ++q) Dq[q] = px[q] >= 0 ? depth[tq[q] * plane + px[q]] : 0.0f;
          // a view that adds nothing adds +0.0: S starts at +0.0 and a sum of
          // doubles never gives -0.0 from a +0.0 operand, so S is unchanged;
          // d is finite, so fmin(d, tau) is d < tau ? d : tau
#pragma unroll
          for (int q = 0; q < kViewBatch; ++q) {
            const double D = (double)Dq[q];
            const double d = D - Zq[q];
            const bool keep = px[q] >= 0 && D > 0.0 && !(d < -g.tau);
            S = S + (keep ? fmin(d, g.tau) : 0.0);
            W = W + (keep ? 1 : 0);
          }
        }
      }
      if (W > 0) tsdf = S / (double)W;
    }
    dense_t[m] = tsdf;
    dense_w[m] = W;
    cnt += (W > 0 && fabs(tsdf) <= g.band) ? 1u : 0u;
  }
  // block counts (integer: any order is exact); the work counts are summed
  // by the scan, as one atomic per wave on a single address serialises in L2
  for (int off = 32; off > 0; off >>= 1) {
    cnt += __shfl_xor(cnt, off, 64);
    fused += __shfl_xor(fused, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    wave_cnt[threadIdx.x >> 6] = cnt;
    wave_fused[threadIdx.x >> 6] = fused;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0, f = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
      s += wave_cnt[w];
      f += wave_fused[w];
    }
    counts[blockIdx.x] = s;
    reinterpret_cast<uint32_t*>(work)[2 * blockIdx.x] = f;
    if (!screen) reinterpret_cast<uint32_t*>(work)[2 * blockIdx.x + 1] = 0;  // no cell tests made
    cellmask[blockIdx.x] = lm;
  }
}

// Exclusive scan of the per-block counts in two passes over contiguous
// segments of them, one workgroup per segment (at most kScanBlocks): the
// first sums each segment's counts and work counts (fused voxel-views, cell
// tests, block tile tests of nchunk view chunks); the second starts each
// segment from the sum of the segments before it and scans the segment 256
// counts at a time, writing offsets[nb], the total to *n_total and the work
// totals to work_total[0..2].  Integer sums:
// any order is exact.
constexpr int kScanBlocks = 256;

// Sum over the workgroup of 256 threads; lds holds 4 values.
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* lds) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();  // lds is free
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  return lds[0] + lds[1] + lds[2] + lds[3];
}

__global__ __launch_bounds__(256) void k_scan_part(const uint32_t* __restrict__ counts,
                                                   const uint2* __restrict__ work,
                                                   const uint32_t* __restrict__ ttests, int nchunk, int64_t nb,
                                                   int64_t seg, uint64_t* __restrict__ part) {
  __shared__ uint64_t lds[4];
  const int64_t lo = (int64_t)blockIdx.x * seg, hi = lo + seg < nb ? lo + seg : nb;
  uint64_t s = 0, sf = 0, st = 0, sb = 0;
  for (int64_t b = lo + threadIdx.x; b < hi; b += 256) {
    s += counts[b];
    const uint2 wk = work[b];
    sf += wk.x;
    st += wk.y;
    for (int q = 0; q < nchunk; ++q) sb += ttests[b * kChunks + q];
  }
  s = block_sum_u64(s, lds);
  sf = block_sum_u64(sf, lds);
  st = block_sum_u64(st, lds);
  sb = block_sum_u64(sb, lds);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s;
    part[gridDim.x + blockIdx.x] = sf;
    part[2 * gridDim.x + blockIdx.x] = st;
    part[3 * gridDim.x + blockIdx.x] = sb;
  }
}

__global__ __launch_bounds__(256) void k_scan_final(const uint32_t* __restrict__ counts, int64_t nb, int64_t seg,
                                                    const uint64_t* __restrict__ part,
                                                    uint64_t* __restrict__ offsets, uint64_t* __restrict__ n_total,
                                                    unsigned long long* __restrict__ work_total) {
  __shared__ uint64_t lds[4], wtot[4];
  const int G = gridDim.x, g = blockIdx.x;
  uint64_t pre = 0;
  for (int i = threadIdx.x; i < g; i += 256) pre += part[i];
  pre = block_sum_u64(pre, lds);
  if (g == 0) {
    uint64_t sf = 0, st = 0, sb = 0;
    for (int i = threadIdx.x; i < G; i += 256) {
      sf += part[G + i];
      st += part[2 * G + i];
      sb += part[3 * G + i];
    }
    sf = block_sum_u64(sf, lds);
    st = block_sum_u64(st, lds);
    sb = block_sum_u64(sb, lds);
    if (threadIdx.x == 0) {
      work_total[0] = sf;
      work_total[1] = st;
      work_total[2] = sb;
    }
  }
  const int64_t lo = (int64_t)g * seg, hi = lo + seg < nb ? lo + seg : nb;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int64_t b0 = lo; b0 < hi; b0 += 256) {  // the same trip count for every thread
    const int64_t b = b0 + threadIdx.x;
    const uint64_t cnt = b < hi ? counts[b] : 0;
    uint64_t inc = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t v = __shfl_up(inc, off, 64);
      if (lane >= off) inc += v;
    }
    __syncthreads();  // the previous strip's wave totals are read
    if (lane == 63) wtot[wid] = inc;
    __syncthreads();
    uint64_t before = pre;
    for (int w = 0; w < wid; ++w) before += wtot[w];
    if (b < hi) offsets[b] = before + inc - cnt;
    pre += wtot[0] + wtot[1] + wtot[2] + wtot[3];
  }
  if (g == G - 1 && threadIdx.x == 0) *n_total = pre;
}

// Scatter of the band voxels of one block tile in Morton order.
__global__ __launch_bounds__(256) void k_band_scatter(uint64_t total, double band,
                                                      const double* __restrict__ dense_t,
                                                      const int32_t* __restrict__ dense_w,
                                                      const uint64_t* __restrict__ offsets,
                                                      const uint32_t* __restrict__ counts,
                                                      const uint32_t* __restrict__ cellmask,
                                                      uint64_t* __restrict__ keys,
                                                      double* __restrict__ tsdf,
                                                      int32_t* __restrict__ w,
                                                      const uint32_t* __restrict__ cmask, int vw,
                                                      uint32_t* __restrict__ vmask) {
  constexpr int NW = kThreads / 64;
  __shared__ uint32_t wave_cnt[kItems][NW];
  if (counts[blockIdx.x] == 0) return;  // the whole block: no band voxel in the tile
  const uint64_t base = (uint64_t)blockIdx.x * kTile;
  const uint32_t lm = cellmask[blockIdx.x];  // cells whose dense values were stored
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // every item's loads first, then one barrier for all the wave counts
  double t[kItems];
  int32_t W[kItems];
  bool sel[kItems];
  uint32_t rank[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const uint64_t m = base + (uint64_t)it * kThreads + threadIdx.x;
    t[it] = 0.0;
    W[it] = 0;
    if (m < total && ((lm >> (it * NW + wid)) & 1u)) {
      t[it] = dense_t[m];
      W[it] = dense_w[m];
    }
  }
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const uint64_t m = base + (uint64_t)it * kThreads + threadIdx.x;
    sel[it] = m < total && W[it] > 0 && fabs(t[it]) <= band;
    const uint64_t mask = __ballot(sel[it]);
    rank[it] = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wave_cnt[it][wid] = (uint32_t)__popcll(mask);
  }
  __syncthreads();
  uint64_t out = offsets[blockIdx.x];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    uint32_t before = 0, row = 0;
#pragma unroll
    for (int v = 0; v < NW; ++v) {
      if (v < wid) before += wave_cnt[it][v];
      row += wave_cnt[it][v];
    }
    if (sel[it]) {
      const uint64_t o = out + before + rank[it];
      keys[o] = base + (uint64_t)it * kThreads + threadIdx.x;
      tsdf[o] = t[it];
      w[o] = W[it];
      if (vmask) {  // the screen's view mask of the voxel's cell (one wave = one cell)
        const uint32_t* cm = cmask + (int64_t)blockIdx.x * (kCells * kMaskWords) + (it * NW + wid) * kMaskWords;
        if ((vw & 3) == 0)  // 16-byte pieces (both arrays 16-byte aligned, rows a multiple of 16 bytes)
          for (int q = 0; q < vw; q += 4)
            *reinterpret_cast<uint4*>(vmask + o * vw + q) = *reinterpret_cast<const uint4*>(cm + q);
        else
          for (int q = 0; q < vw; ++q) vmask[o * vw + q] = cm[q];
      }
    }
    out += row;
  }
}

__global__ __launch_bounds__(256) void k_fill_u64(uint64_t* __restrict__ p, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// 6-neighbour table: each neighbour's band index through the 4^3 cell records
// (the same key -> index map the ray walker uses).
__global__ __launch_bounds__(256) void k_neighbours(const uint64_t* __restrict__ keys, int64_t n, int32_t G,
                                                    const bf_cell* __restrict__ cells, int32_t ncell,
                                                    int32_t* __restrict__ nbr, int32_t* __restrict__ deg) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint64_t key = keys[v];
  const int32_t c[3] = {(int32_t)bf_compact3(key), (int32_t)bf_compact3(key >> 1),
                        (int32_t)bf_compact3(key >> 2)};
  int32_t d = 0, idx[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    int32_t q[3] = {c[0], c[1], c[2]};
    q[s >> 1] += (s & 1) ? 1 : -1;
    idx[s] = bf_band_index(cells, ncell, G, q[0], q[1], q[2]);
    d += idx[s] >= 0;
  }
  // the row's 24 bytes as three 8-byte stores (8-byte aligned: the band's
  // arrays start on 256-byte boundaries)
  int2* o = reinterpret_cast<int2*>(nbr + v * 6);
  o[0] = make_int2(idx[0], idx[1]);
  o[1] = make_int2(idx[2], idx[3]);
  o[2] = make_int2(idx[4], idx[5]);
  deg[v] = d;
}

__global__ __launch_bounds__(256) void k_brick_bits(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                    int nbrick, uint32_t* __restrict__ bits) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint64_t key = keys[v];
  // a brick is a Morton range of 2^(3 shift) keys and the band is sorted, so
  // only the first band voxel of each brick sets its bit
  if (v > 0 && (keys[v - 1] >> (3 * shift)) == (key >> (3 * shift))) return;
  const uint32_t bi = bf_compact3(key) >> shift, bj = bf_compact3(key >> 1) >> shift,
                 bk = bf_compact3(key >> 2) >> shift;
  const uint32_t bit = (bk * nbrick + bj) * nbrick + bi;
  atomicOr(&bits[bit >> 5], 1u << (bit & 31));
}

// Cell records (the key -> band index map of the neighbour table and the ray
// walker): occupancy mask and first band index of every 4^3 cell, addressed
// directly by the cell's coordinates, so a lookup never collides or probes.
// A cell is a range of 64 Morton codes and the band is sorted, so a cell's
// voxels are consecutive: each wave ORs its runs of one cell with a segmented
// shuffle scan, and the run's last lane writes the mask (an atomic OR where
// the run may continue in the neighbouring wave, a plain store otherwise).
__global__ __launch_bounds__(256) void k_cell_tables(const uint64_t* __restrict__ keys, int64_t n, int ncell,
                                                     bf_cell* __restrict__ cells) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = v < n;
  const uint64_t key = valid ? keys[v] : ~0ull;
  const uint64_t ck = key >> 6;  // cell of the key (lanes past n share an impossible one)
  uint64_t m = valid ? 1ull << (key & 63) : 0ull;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t om = __shfl_up(m, off, 64);
    const uint64_t oc = __shfl_up(ck, off, 64);
    if (lane >= off && oc == ck) m |= om;  // sorted keys: lanes in between are in the same cell
  }
  const uint64_t next_ck = __shfl_down(ck, 1, 64);
  const uint64_t first_ck = __shfl(ck, 0, 64);
  const bool last = lane == 63 || next_ck != ck;
  if (!valid) return;
  const uint32_t ci = bf_compact3(key) >> 2, cj = bf_compact3(key >> 1) >> 2, ck3 = bf_compact3(key >> 2) >> 2;
  const int64_t c = ((int64_t)ck3 * ncell + cj) * ncell + ci;
  if (last) {
    const bool edge = lane == 63 || first_ck == ck;  // the run may go on in the next or previous wave
    if (edge)
      atomicOr(&cells[c].mask, m);
    else
      cells[c].mask = m;
  }
  if (v == 0 || (keys[v - 1] >> 6) != ck) cells[c].start = (int32_t)v;
}

// Forward-octant Chebyshev distances over the brick grid (empty-space skipping
// for the ray walker).  Octant o has bit a set when the ray moves towards lower
// coordinates on axis a.  For brick b, dist_o(b) = min over occupied bricks b'
// ahead of b in that octant (b'_a - b_a of the octant's sign, or 0, on every
// axis) of max_a |b'_a - b_a|, capped at 255 (also: no such brick).  So the
// box from b to b + (dist - 1) bricks along the octant holds no occupied brick.
// The min of max separates into one pass per axis,
//   out(x) = min over t >= 0 of max(t, in(x + sign t)),
// each pass doubling the variants (bit a of a variant = sign on axis a): 2 after
// the x pass (which reads the bitmap, in = 0 on occupied bricks, else 255), 4
// after y, 8 after z.  Variant v's grid is at offset v nb^3.
__global__ __launch_bounds__(256) void k_brick_oct(const uint32_t* __restrict__ bits, const uint8_t* __restrict__ in,
                                                   uint8_t* __restrict__ out, int lnb, int axis) {
  // nb = 2^lnb <= 64 bricks per axis: every index fits 32 bits and splits by shifts
  const int nb = 1 << lnb;
  const int32_t id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (1 << (3 * lnb + axis + 1))) return;
  const int vout = id >> (3 * lnb);
  const int32_t e = id & ((1 << (3 * lnb)) - 1);
  const int vin = vout & ((1 << axis) - 1);
  const int dir = ((vout >> axis) & 1) ? -1 : 1;
  const int pos = (e >> (axis * lnb)) & (nb - 1);
  const int32_t stride = 1 << (axis * lnb);
  const int32_t base = e - pos * stride;
  if (axis == 0) {
    // in = 0 on occupied bricks, 255 elsewhere: the result is the distance to
    // the nearest occupied brick from pos on along the line (255: none), read
    // off the line's occupancy bits.  A line starts at a multiple of nb bits.
    uint64_t line;
    if (lnb == 6) line = (uint64_t)bits[base >> 5] | ((uint64_t)bits[(base >> 5) + 1] << 32);
    else line = (uint64_t)(bits[base >> 5] >> (base & 31)) & ((1ull << nb) - 1ull);  // nb <= 32: one word
    int best;
    if (dir > 0) {
      const uint64_t ahead = line >> pos;
      best = ahead ? __builtin_ctzll(ahead) : 255;
    } else {
      const uint64_t behind = pos == 63 ? line : line & ((2ull << pos) - 1ull);
      best = behind ? pos - (63 - __builtin_clzll(behind)) : 255;
    }
    out[id] = (uint8_t)best;
    return;
  }
  const uint8_t* src = in + (vin << (3 * lnb));
  // Candidates are taken 8 at a time so their loads are in flight together.
  // Taking more than needed changes nothing: max(t, .) >= t >= best once
  // t >= best, and positions outside the grid count as 255.
  const int tend = dir > 0 ? nb - pos : pos + 1;  // positions along the line from pos on
  int best = 255;
  for (int t0 = 0; t0 < best && t0 < tend; t0 += 8) {
    int dv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u;
      const int q = min(max(pos + dir * t, 0), nb - 1);  // in the grid even where unused
      const int32_t j = base + q * stride;
      dv[u] = t >= tend ? 255 : (int)src[j];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int m = dv[u] > t0 + u ? dv[u] : t0 + u;
      best = m < best ? m : best;
    }
  }
  out[id] = (uint8_t)best;
}

}  // namespace

extern "C" bf_status bf_build_band(bf_ctx* ctx, const bf_grid* grid, const bf_camera* cam, int32_t T,
                                   const float* depth_dev, const double* c2w_dev, uint32_t flags,
                                   bf_band** out, int64_t* n_out) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, grid && cam && out && n_out, "bf_build_band: NULL argument");
  *out = nullptr;
  *n_out = 0;
  BF_CHECK(ctx, grid->G >= 1 && grid->G <= 2048, "bf_build_band: G=%d outside [1, 2048]", grid->G);
  BF_CHECK(ctx, grid->h > 0.0 && grid->tau >= 0.0 && grid->band >= 0.0,
           "bf_build_band: h must be > 0, tau and band >= 0");
  BF_CHECK(ctx, T >= 0 && T <= 65535, "bf_build_band: T=%d outside [0, 65535]", T);
  BF_CHECK(ctx, T == 0 || (cam->width > 0 && cam->height > 0 && depth_dev && c2w_dev),
           "bf_build_band: bad camera size or NULL depth/poses");
  BF_HIP(ctx, hipSetDevice(ctx->device));

  bf_band* band = new (std::nothrow) bf_band();
  if (!band) return bf_fail(ctx, BF_ERR_OOM, "bf_build_band: host allocation");
  band->G = grid->G;
  band->h = grid->h;
  for (int a = 0; a < 3; ++a) band->origin[a] = grid->origin[a];
  band->tau = grid->tau;
  band->band = grid->band;
  int l2 = 0;
  while ((1 << l2) < grid->G) ++l2;
  band->P = 1 << l2;
  band->log2P = l2;
  const uint64_t total = (uint64_t)band->P * band->P * band->P;
  const int64_t nblocks = (int64_t)((total + kTile - 1) / kTile);

  auto fail = [&](bf_status st) {
    bf_band_free(ctx, band);
    return st;
  };

  // flags[0]: depth invalid; then the band count
  void* scan_ws = nullptr;
  // layout: flags and counters (64 B) | counts [nblocks] | offsets [nblocks + 1] | work counts
  // [nblocks] | tile view masks [nblocks][2][kMaskWords] | scattered-cell masks [nblocks] | live-cell
  // bits [nblocks] | cell view masks [nblocks][kCells][kMaskWords] | scan partials [4][kScanBlocks]
  // | super tile view masks [nsup][2][kMaskWords] | block tile test counts [nblocks][kChunks]
  const size_t off_counts = 64, off_offsets = off_counts + ((nblocks * sizeof(uint32_t) + 63) / 64) * 64;
  const size_t off_work = (off_offsets + (nblocks + 1) * sizeof(uint64_t) + 255) / 256 * 256;
  const size_t off_tmask = (off_work + nblocks * sizeof(uint2) + 255) / 256 * 256;
  const size_t off_cmask = off_tmask + nblocks * (2 * kMaskWords * sizeof(uint32_t));
  const size_t off_live = off_cmask + nblocks * sizeof(uint32_t);
  const size_t off_vmask = (off_live + nblocks * sizeof(uint32_t) + 255) / 256 * 256;
  const size_t off_part = (off_vmask + nblocks * (kCells * kMaskWords * sizeof(uint32_t)) + 255) / 256 * 256;
  const int64_t nsup = bf_cdiv(nblocks, kSuper);
  const size_t off_smask = off_part + 4 * kScanBlocks * sizeof(uint64_t);
  const size_t off_ttests = (off_smask + nsup * (2 * kMaskWords * sizeof(uint32_t)) + 255) / 256 * 256;
  const size_t scan_bytes = off_ttests + nblocks * (kChunks * sizeof(uint32_t));
  if (bf_status s = bf_ws(ctx, bf_ctx::WS_SCAN, scan_bytes, &scan_ws)) return fail(s);
  int* dflags = (int*)scan_ws;
  uint64_t* d_ntotal = (uint64_t*)((char*)scan_ws + 16);
  uint32_t* counts = (uint32_t*)((char*)scan_ws + off_counts);
  uint64_t* offsets = (uint64_t*)((char*)scan_ws + off_offsets);
  uint2* work = (uint2*)((char*)scan_ws + off_work);
  uint32_t* tmask = (uint32_t*)((char*)scan_ws + off_tmask);
  uint32_t* cellmask = (uint32_t*)((char*)scan_ws + off_cmask);
  uint32_t* live_bits = (uint32_t*)((char*)scan_ws + off_live);
  uint32_t* ttests = (uint32_t*)((char*)scan_ws + off_ttests);
  uint32_t* vmask = (uint32_t*)((char*)scan_ws + off_vmask);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, ctx->stream, (uint64_t*)scan_ws, (uint64_t)8, 0ull);

  double* dense_t = nullptr;
  int32_t* dense_w = nullptr;
  if (flags & BF_BAND_KEEP_DENSE) {
    if (bf_status s = bf_obj_alloc(ctx, (void**)&band->dense_tsdf, total * sizeof(double))) return fail(s);
    if (bf_status s = bf_obj_alloc(ctx, (void**)&band->dense_w, total * sizeof(int32_t))) return fail(s);
    dense_t = band->dense_tsdf;
    dense_w = band->dense_w;
  } else {
    if (bf_status s = bf_ws(ctx, bf_ctx::WS_DENSE_T, total * sizeof(double), (void**)&dense_t)) return fail(s);
    if (bf_status s = bf_ws(ctx, bf_ctx::WS_DENSE_W, total * sizeof(int32_t), (void**)&dense_w)) return fail(s);
  }

  const int64_t npix = (int64_t)T * cam->width * cam->height;
  bf_grid_k gk{grid->G, grid->h, grid->origin[0], grid->origin[1], grid->origin[2], grid->tau, grid->band};
  bf_cam_k ck{cam->width, cam->height, cam->fx, cam->fy, cam->cx, cam->cy};
  // screening pyramid (off when the dense grid is kept, or when truncation does not exceed the band)
  const int screen = (!(flags & BF_BAND_KEEP_DENSE) && grid->tau > grid->band && npix > 0) ? 1 : 0;
  // words of the per-voxel view masks kept for the assembly (views past kTileViews are never masked)
  const int vw = screen ? (std::min<int32_t>(T, kTileViews) + 31) / 32 : 0;
  if (npix > 0 && !screen) {  // with screening the pyramid kernel validates the depth
    const int vb = (int)std::min<int64_t>(bf_cdiv(npix, 256), 8192);
    BF_LAUNCH(ctx, "validate_depth", k_validate_depth, dim3(vb), dim3(256), 0, depth_dev, npix, dflags);
    if (bf_status s = bf_launch_check(ctx, "k_validate_depth")) return fail(s);
  }
  Pyr pyr{};
  float* dmin = nullptr;
  float* dmax = nullptr;
  if (screen) {
    int32_t w = cam->width, h = cam->height;
    int64_t off = 0;
    for (;;) {
      if (pyr.nl >= kMaxLevels) return fail(bf_fail(ctx, BF_ERR_INVALID_ARG, "bf_build_band: depth image too large"));
      pyr.w[pyr.nl] = w;
      pyr.h[pyr.nl] = h;
      pyr.off[pyr.nl] = off;
      off += (int64_t)w * h;
      ++pyr.nl;
      if (w == 1 && h == 1) break;
      w = (w + 1) / 2;
      h = (h + 1) / 2;
    }
    pyr.per_view = off;
    void* pw = nullptr;
    const size_t half = ((size_t)off * T * sizeof(float) + 255) / 256 * 256;
    if (bf_status s = bf_ws(ctx, bf_ctx::WS_PYR, 2 * half, &pw)) return fail(s);
    dmin = (float*)pw;
    dmax = (float*)((char*)pw + half);
    BF_LAUNCH(ctx, "depth_pyramid", k_pyr_tiles,
              dim3((unsigned)bf_cdiv(cam->width, kPyrTile), (unsigned)bf_cdiv(cam->height, kPyrTile), (unsigned)T),
              dim3(256), 0, depth_dev, cam->width, cam->height, pyr, dmin, dmax, dflags);
    if (pyr.nl > kTileLevels + 1)
      BF_LAUNCH(ctx, "depth_pyramid", k_pyr_top, dim3((unsigned)T), dim3(1024), 0, pyr, dmin, dmax);
    // one wave per (super tile, 64 of the first kTileViews views), in both levels
    const int64_t waves = nsup * ((std::min<int32_t>(T, kTileViews) + 63) / 64);
    uint32_t* smask = (uint32_t*)((char*)scan_ws + off_smask);
    BF_LAUNCH(ctx, "super_screen", k_super_screen, dim3((unsigned)bf_cdiv(waves, 4)), dim3(256), 0, gk, ck, T, nsup,
              depth_dev, c2w_dev, pyr, dmin, dmax, smask);
    BF_LAUNCH(ctx, "tile_screen", k_tile_screen, dim3((unsigned)bf_cdiv(waves, 4)), dim3(256), 0, gk, ck, T,
              (int64_t)nblocks, depth_dev, c2w_dev, pyr, dmin, dmax, smask, tmask, ttests);
    BF_LAUNCH(ctx, "cell_screen", k_cell_screen, dim3((unsigned)bf_cdiv(nblocks, kThreads / 64)), dim3(kThreads), 0,
              gk, ck, T, depth_dev, c2w_dev, total, (int64_t)nblocks, pyr, dmin, dmax, tmask, vmask, live_bits, work);
  }
  BF_LAUNCH(ctx, "tsdf_count", k_tsdf_count, dim3((unsigned)nblocks), dim3(kThreads), 0, gk, ck, T,
                     depth_dev, c2w_dev, total, dense_t, dense_w, counts, screen, vmask, live_bits, work,
                     cellmask);
  if (bf_status s = bf_launch_check(ctx, "k_tsdf_count")) return fail(s);
  {
    // segments of at least 1024 counts, at most kScanBlocks of them (one, holding nothing, for an empty grid)
    const int sg = (int)std::max<int64_t>(1, std::min<int64_t>(kScanBlocks, bf_cdiv(nblocks, 1024)));
    const int64_t seg = std::max<int64_t>(1, bf_cdiv(nblocks, sg));
    uint64_t* part = (uint64_t*)((char*)scan_ws + off_part);
    BF_LAUNCH(ctx, "scan_counts", k_scan_part, dim3(sg), dim3(256), 0, counts, work, ttests,
              screen ? (std::min<int32_t>(T, kTileViews) + 63) / 64 : 0, (int64_t)nblocks, seg, part);
    BF_LAUNCH(ctx, "scan_counts", k_scan_final, dim3(sg), dim3(256), 0, counts, (int64_t)nblocks, seg, part, offsets,
              d_ntotal, (unsigned long long*)((char*)scan_ws + 24));
  }
  if (bf_status s = bf_launch_check(ctx, "k_scan_counts")) return fail(s);

  void* pin = nullptr;
  if (bf_status s = bf_pinned(ctx, 64, &pin)) return fail(s);
  if (hipMemcpyAsync(pin, scan_ws, 48, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess)
    return fail(bf_fail(ctx, BF_ERR_HIP, "bf_build_band: count read-back failed"));
  if (((int*)pin)[0] & 1)
    return fail(bf_fail(ctx, BF_ERR_INVALID_ARG, "bf_build_band: depth holds NaN, inf or negative values"));
  const uint64_t N = *(uint64_t*)((char*)pin + 16);
  band->tsdf_voxel_views = *(const int64_t*)((char*)pin + 24);
  // cell tests, block tile tests, and one super tile test per (super tile
  // holding a grid voxel, screened view)
  band->tsdf_tile_tests = *(const int64_t*)((char*)pin + 40);
  if (screen)
    band->tsdf_tile_tests += bf_cdiv(grid->G, kSupI) * bf_cdiv(grid->G, kSupJ) * bf_cdiv(grid->G, kSupK) *
                             (int64_t)std::min<int32_t>(T, kTileViews);
  band->tsdf_box_tests = *(const int64_t*)((char*)pin + 32) + band->tsdf_tile_tests;
  if (N >= (1ull << 31) - 1)
    return fail(bf_fail(ctx, BF_ERR_CAPACITY, "bf_build_band: band of %llu voxels exceeds int32 indexing",
                        (unsigned long long)N));
  band->n = (int64_t)N;

  if (N > 0) {
    // 4^3 cell records (key -> band index) for the neighbour table and the
    // ray walker; brick occupancy bitmap for the ray walker (brick edge
    // 2^shift, at most 64 bricks per axis) and its forward-octant distances
    band->ncell = std::max(1, band->P >> 2);
    const int64_t nc3 = (int64_t)band->ncell * band->ncell * band->ncell;
    int shift = 2;
    while ((band->P >> shift) > 64) ++shift;
    band->brick_shift = shift;
    band->nbrick = std::max(1, band->P >> shift);
    const int64_t nbr3 = (int64_t)band->nbrick * band->nbrick * band->nbrick;
    const size_t words = ((size_t)nbr3 + 31) / 32;
    if (bf_status s = bf_obj_alloc_parts(
            ctx, &band->block,
            {{(void**)&band->keys, N * sizeof(uint64_t)}, {(void**)&band->tsdf, N * sizeof(double)},
             {(void**)&band->w, N * sizeof(int32_t)}, {(void**)&band->nbr, N * 6 * sizeof(int32_t)},
             {(void**)&band->deg, N * sizeof(int32_t)}, {(void**)&band->cells, (size_t)nc3 * sizeof(bf_cell)},
             {(void**)&band->bricks, words * 4}, {(void**)&band->brick_dist, (size_t)(8 * nbr3)},
             {(void**)&band->vmask, screen ? N * vw * sizeof(uint32_t) : 0}}))
      return fail(s);
    if (screen) {
      band->vmask_words = vw;
      band->view_depth = depth_dev;
      band->view_poses = c2w_dev;
      band->view_T = T;
      band->view_W = cam->width;
      band->view_H = cam->height;
      band->view_f[0] = cam->fx;
      band->view_f[1] = cam->fy;
      band->view_f[2] = cam->cx;
      band->view_f[3] = cam->cy;
    } else {
      band->vmask = nullptr;
    }
    BF_LAUNCH(ctx, "band_scatter", k_band_scatter, dim3((unsigned)nblocks), dim3(kThreads), 0, total,
                       grid->band, dense_t, dense_w, offsets, counts, cellmask, band->keys, band->tsdf, band->w, vmask,
                       vw, screen ? band->vmask : nullptr);
    if (bf_status s = bf_launch_check(ctx, "k_band_scatter")) return fail(s);

    const unsigned nb = (unsigned)bf_cdiv((int64_t)N, 256);
    // clear the cell records and the brick bitmap, which follows them in the block
    const uint64_t nclear = (uint64_t)(((char*)band->bricks + words * 4 - (char*)band->cells + 7) / 8);
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)std::min<uint64_t>(bf_cdiv((int64_t)nclear, 256), 16384)),
                       dim3(256), 0, ctx->stream, (uint64_t*)band->cells, nclear, 0ull);
    BF_LAUNCH(ctx, "cell_tables", k_cell_tables, dim3(nb), dim3(256), 0, band->keys, (int64_t)N, band->ncell,
              band->cells);
    BF_LAUNCH(ctx, "neighbours", k_neighbours, dim3(nb), dim3(256), 0, band->keys, (int64_t)N, grid->G, band->cells,
              band->ncell, band->nbr, band->deg);
    BF_LAUNCH(ctx, "brick_bits", k_brick_bits, dim3(nb), dim3(256), 0, band->keys, (int64_t)N, shift, band->nbrick,
              band->bricks);
    // forward-octant brick distances (empty-space skipping) for the ray walker
    uint8_t* dtmp = nullptr;  // 2 nbr3 after the x pass, then 4 nbr3 after y
    if (bf_status s = bf_ws(ctx, bf_ctx::WS_NBV_TMP, 6 * nbr3, (void**)&dtmp)) return fail(s);
    int lnb = 0;  // nbrick is a power of two, at most 64
    while ((1 << lnb) < band->nbrick) ++lnb;
    for (int axis = 0; axis < 3; ++axis) {
      const uint8_t* in = axis == 0 ? nullptr : (axis == 1 ? dtmp : dtmp + 2 * nbr3);
      uint8_t* o = axis == 0 ? dtmp : (axis == 1 ? dtmp + 2 * nbr3 : band->brick_dist);
      BF_LAUNCH(ctx, "brick_dist", k_brick_oct, dim3((unsigned)bf_cdiv(nbr3 << (axis + 1), 256)), dim3(256), 0,
                band->bricks, in, o, lnb, axis);
    }
    if (bf_status s = bf_launch_check(ctx, "neighbours/bricks/cells")) return fail(s);
  }
  *out = band;
  *n_out = band->n;
  return BF_OK;
}
