// Next-best-view scoring (Sec. 3.8, eq. 13; Algorithm 1 step 8).
//
// Each candidate pose casts one ray per pixel of the ray camera.  A thread
// walks its ray through the voxel grid (Amanatides-Woo, with the next
// boundary on each axis computed directly from the voxel index so the walk is
// reproducible) and sums the quantised variance of the band voxels it crosses
// up to and including the first voxel whose posterior mean is <= 0.  Band
// membership is tested only in occupied bricks (a bitmap in LDS), through the
// 4^3 cell masks; across empty bricks the walk jumps (see walk()).  Variances are quantised to int64
// (q = rint(s / max s * 2^32)) before summation, so the per-candidate
// utility is an exact integer independent of summation order: block sums
// are combined with 64-bit integer atomics.
#include "bf_internal.h"

#include <climits>

namespace {

constexpr int kThreads = 256;
constexpr double kScale = 4294967296.0;  // 2^32

// max(0, max_v s_v): non-negative doubles order like their bit patterns, so an
// integer atomic max on the bits is exact and order independent.
__global__ __launch_bounds__(256) void k_max(const double* __restrict__ s, int64_t n,
                                             unsigned long long* __restrict__ out_bits) {
  __shared__ double lds[kThreads / 64];
  double m = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    m = fmax(m, s[i]);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) b = fmax(b, lds[w]);
    atomicMax(out_bits, (unsigned long long)__double_as_longlong(b));
  }
}

__global__ __launch_bounds__(256) void k_quantize(const double* __restrict__ s, int64_t n,
                                                  const double* __restrict__ smax, int64_t* __restrict__ q) {
#pragma clang fp contract(off)
  const int64_t v = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (v >= n) return;
  const double m = *smax;
  q[v] = m > 0.0 ? (int64_t)rint((s[v] / m) * kScale) : 0;
}

struct ray_k {
  bf_grid_k g;
  bf_cam_k cam;
  int utility;
  double na, nc, nz0;  // sensor model for the variance-reduction utility
  int brick_shift, nbrick, ncell;
  int64_t tiles_per_cand, ntiles;
};

constexpr int kMaxBrickWords = 64 * 64 * 64 / 32;
// Empty-space jumps start at bricks whose nearest occupied brick is at least
// this many bricks away (Chebyshev); closer to the band the walk steps voxel by voxel.
constexpr int kJumpMinDist = 2;

// Time at which the ray crosses plane p of one axis (the plane between voxels
// p - 1 and p).  Every step and every jump evaluates plane times with this one
// expression, so a jump lands on exactly the state the voxel steps reach.
__device__ __forceinline__ double plane_t(double org, double h, double o, double inv, int32_t p) {
#pragma clang fp contract(off)
  return ((org + (double)p * h) - o) * inv;
}

// Walk of one ray; returns the ray's integer utility.
//
// The voxel sequence is the Amanatides-Woo walk: each step crosses the
// nearest next plane (lowest axis on ties), with plane times from plane_t.
// Since every plane time depends only on the plane index, the walk is the
// merge, ordered by (time, axis), of the three axes' plane sequences, and
// "every crossing earlier than time c" is a prefix of it.  Inside a cube of
// bricks known to hold no band voxel the walk jumps: c = the earliest time at
// which a plane bounding the cube is crossed, and each axis advances by the
// number of its planes with time < c (estimated from the continuous ray, then
// corrected with plane_t).  The voxels skipped hold no band voxel, so the
// visited band voxels, the utility and the stopping voxel are those of the
// plain walk.
__device__ int64_t walk(const ray_k& R, const double* __restrict__ P, int32_t row, int32_t col,
                        const unsigned long long* __restrict__ cmask, const int32_t* __restrict__ cstart,
                        const uint8_t* __restrict__ bdist, const double* __restrict__ mu,
                        const double* __restrict__ s, const int64_t* __restrict__ q, double smax,
                        const uint32_t* __restrict__ bricks) {
#pragma clang fp contract(off)
  const bf_grid_k& g = R.g;
  const double o[3] = {P[3], P[7], P[11]};
  const double a = ((double)col - R.cam.cx) / R.cam.fx;
  const double b = ((double)row - R.cam.cy) / R.cam.fy;
  double d[3];
  d[0] = (P[0] * a + P[1] * b) + P[2];
  d[1] = (P[4] * a + P[5] * b) + P[6];
  d[2] = (P[8] * a + P[9] * b) + P[10];
  const double org[3] = {g.ox, g.oy, g.oz};
  double inv[3];
  double tnear = 0.0, tfar = INFINITY;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const double lo = org[ax];
    const double hi = org[ax] + (double)g.G * g.h;
    if (d[ax] == 0.0) {
      inv[ax] = 0.0;
      if (o[ax] < lo || o[ax] > hi) return 0;
      continue;
    }
    inv[ax] = 1.0 / d[ax];
    const double t0 = (lo - o[ax]) * inv[ax];
    const double t1 = (hi - o[ax]) * inv[ax];
    const double tmin = t0 < t1 ? t0 : t1;
    const double tmax = t0 < t1 ? t1 : t0;
    if (tmin > tnear) tnear = tmin;
    if (tmax < tfar) tfar = tmax;
  }
  if (!(tnear < tfar)) return 0;
  int32_t idx[3], step[3];
  double tn[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const double pa = o[ax] + tnear * d[ax];
    const double f = floor((pa - org[ax]) / g.h);
    idx[ax] = f < 0.0 ? 0 : (f > (double)(g.G - 1) ? g.G - 1 : (int32_t)f);
    step[ax] = d[ax] > 0.0 ? 1 : (d[ax] < 0.0 ? -1 : 0);
  }
#pragma unroll
  for (int ax = 0; ax < 3; ++ax)
    tn[ax] = step[ax] == 0 ? INFINITY : plane_t(org[ax], g.h, o[ax], inv[ax], idx[ax] + (step[ax] > 0 ? 1 : 0));
  int64_t score = 0;
  const int bs = R.brick_shift, NB = R.nbrick, NC = R.ncell;
  int32_t last_brick = -1, last_dist = 0;
  // every iteration crosses at least one plane, and a ray crosses at most 3G
  const int64_t max_steps = 3 * (int64_t)g.G + 3;
  for (int64_t it = 0; it < max_steps; ++it) {
    const int32_t bit = (int32_t)((((uint32_t)idx[2] >> bs) * NB + ((uint32_t)idx[1] >> bs)) * NB +
                                  ((uint32_t)idx[0] >> bs));
    if ((bricks[bit >> 5] >> (bit & 31)) & 1u) {
      // occupied brick: is this voxel in the band?  (4^3 cell mask, rank by popcount)
      const int64_t c = ((int64_t)(idx[2] >> 2) * NC + (idx[1] >> 2)) * NC + (idx[0] >> 2);
      const uint32_t m = (idx[0] & 1) | ((idx[1] & 1) << 1) | ((idx[2] & 1) << 2) | ((idx[0] & 2) << 2) |
                         ((idx[1] & 2) << 3) | ((idx[2] & 2) << 4);
      const unsigned long long mk = cmask[c];
      if ((mk >> m) & 1ull) {
        const int32_t v = cstart[c] + __popcll(mk & ((1ull << m) - 1ull));
        if (R.utility == BF_UTILITY_SUM_VAR) {
          score += q[v];
        } else {
          // expected variance reduction of one new observation at the voxel's depth
          const double x = org[0] + ((double)idx[0] + 0.5) * g.h;
          const double y = org[1] + ((double)idx[1] + 0.5) * g.h;
          const double z = org[2] + ((double)idx[2] + 0.5) * g.h;
          const double dx = x - P[3], dy = y - P[7], dz = z - P[11];
          const double Z = (P[2] * dx + P[6] * dy) + P[10] * dz;
          const double e = Z - R.nz0;
          const double sd = R.na + R.nc * (e * e);
          const double sv = s[v];
          const double term = sv > 0.0 ? (sv * sv) / (sv + sd * sd) : 0.0;
          score += smax > 0.0 ? (int64_t)rint((term / smax) * kScale) : 0;
        }
        if (mu[v] <= 0.0) break;
      }
    } else {
      if (bit != last_brick) {
        last_brick = bit;
        last_dist = bdist[bit];
      }
      if (last_dist >= kJumpMinDist) {
        // bricks within Chebyshev radius r of this one are empty: jump to the
        // last voxel before the walk leaves that cube
        const int r = last_dist - 1;
        int32_t lo[3], hi[3];
        double cut = INFINITY;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const int32_t bb = idx[ax] >> bs;
          lo[ax] = max(0, (bb - r) << bs);
          hi[ax] = min(g.G - 1, ((bb + r + 1) << bs) - 1);
          if (step[ax] != 0) {
            const double te = plane_t(org[ax], g.h, o[ax], inv[ax], step[ax] > 0 ? hi[ax] + 1 : lo[ax]);
            cut = te < cut ? te : cut;
          }
        }
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          if (step[ax] == 0) continue;
          const int32_t sg = step[ax];
          const int32_t p0 = idx[ax] + (sg > 0 ? 1 : 0);
          const int32_t nmax = sg > 0 ? hi[ax] + 1 - p0 : p0 - lo[ax];  // interior planes ahead
          const double u = ((o[ax] + cut * d[ax]) - org[ax]) / g.h;
          double ne = sg > 0 ? floor(u) - (double)p0 + 1.0 : (double)p0 - ceil(u) + 1.0;
          ne = ne < 0.0 ? 0.0 : (ne > (double)nmax ? (double)nmax : ne);
          int32_t n = (int32_t)ne;
          while (n > 0 && plane_t(org[ax], g.h, o[ax], inv[ax], p0 + (n - 1) * sg) >= cut) --n;
          while (n < nmax && plane_t(org[ax], g.h, o[ax], inv[ax], p0 + n * sg) < cut) ++n;
          idx[ax] += n * sg;
          tn[ax] = plane_t(org[ax], g.h, o[ax], inv[ax], p0 + n * sg);
        }
      }
    }
    int ax = 0;
    if (tn[1] < tn[ax]) ax = 1;
    if (tn[2] < tn[ax]) ax = 2;
    idx[ax] += step[ax];
    if (idx[ax] < 0 || idx[ax] >= g.G) break;
    tn[ax] = plane_t(org[ax], g.h, o[ax], inv[ax], idx[ax] + (step[ax] > 0 ? 1 : 0));
  }
  return score;
}

// Persistent grid over (candidate, ray tile) work items; one thread per ray.
// Every workgroup stages the brick bitmap in LDS once.
__global__ __launch_bounds__(256) void k_nbv_rays(ray_k R, const double* __restrict__ cands,
                                                  const unsigned long long* __restrict__ cmask,
                                                  const int32_t* __restrict__ cstart,
                                                  const uint8_t* __restrict__ bdist, const double* __restrict__ mu,
                                                  const double* __restrict__ s, const int64_t* __restrict__ q,
                                                  const double* __restrict__ smax_p,
                                                  const uint32_t* __restrict__ bricks_g,
                                                  unsigned long long* __restrict__ scores) {
  __shared__ uint32_t bricks[kMaxBrickWords];
  __shared__ long long lds[kThreads / 64];
  const int words = (R.nbrick * R.nbrick * R.nbrick + 31) / 32;
  for (int w = threadIdx.x; w < words; w += kThreads) bricks[w] = bricks_g[w];
  __syncthreads();
  const double smax = *smax_p;
  const int64_t npix = (int64_t)R.cam.W * R.cam.H;
  for (int64_t tile = blockIdx.x; tile < R.ntiles; tile += gridDim.x) {
    const int64_t cand = tile / R.tiles_per_cand;
    const int64_t pix = (tile % R.tiles_per_cand) * kThreads + threadIdx.x;
    long long sc = 0;
    if (pix < npix) {
      const int32_t row = (int32_t)(pix / R.cam.W), col = (int32_t)(pix % R.cam.W);
      sc = walk(R, cands + 12 * cand, row, col, cmask, cstart, bdist, mu, s, q, smax, bricks);
    }
    for (int off = 32; off > 0; off >>= 1) sc += __shfl_xor(sc, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = sc;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long t = 0;
      for (int w = 0; w < kThreads / 64; ++w) t += lds[w];
      atomicAdd(&scores[cand], (unsigned long long)t);  // two's complement: exact for signed sums
    }
  }
}

__global__ void k_zero_i64(int64_t* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// Lowest index attaining the maximum score.
__global__ __launch_bounds__(1024) void k_argmax(const int64_t* __restrict__ sc, int n, int32_t* __restrict__ best) {
  __shared__ long long bv[1024];
  __shared__ int bi[1024];
  long long v = LLONG_MIN;
  int idx = 0x7fffffff;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (sc[i] > v) {
      v = sc[i];
      idx = i;
    }
  bv[threadIdx.x] = v;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const long long ov = bv[threadIdx.x + off];
      const int oi = bi[threadIdx.x + off];
      if (ov > bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = ov;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *best = bi[0];
}

}  // namespace

extern "C" bf_status bf_nbv_score(bf_ctx* ctx, const bf_band* band, const double* mu_dev, const double* s_dev,
                                  int32_t n_cand, const double* cand_c2w_dev, const bf_camera* ray_cam,
                                  int32_t utility, const bf_noise* noise, int64_t* scores_dev, int32_t* best_host) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, band && ray_cam && best_host, "bf_nbv_score: NULL argument");
  BF_CHECK(ctx, n_cand >= 0 && n_cand <= 65535, "bf_nbv_score: n_cand=%d outside [0, 65535]", n_cand);
  BF_CHECK(ctx, utility == BF_UTILITY_SUM_VAR || (utility == BF_UTILITY_VAR_REDUCTION && noise),
           "bf_nbv_score: unknown utility or missing noise model");
  BF_CHECK(ctx, ray_cam->width > 0 && ray_cam->height > 0, "bf_nbv_score: bad ray camera");
  *best_host = -1;
  if (n_cand == 0) return BF_OK;
  BF_CHECK(ctx, cand_c2w_dev && scores_dev, "bf_nbv_score: NULL candidates or scores");
  BF_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t N = band->n;
  // workspace: smax | best | q [N]
  const int nbm = (int)std::max<int64_t>(1, std::min<int64_t>(bf_cdiv(N, kThreads), 1024));
  char* ws = nullptr;
  BF_TRY(bf_ws(ctx, bf_ctx::WS_NBV, 256 + N * 8, (void**)&ws));
  double* smax = (double*)ws;
  int32_t* dbest = (int32_t*)(ws + 8);
  int64_t* q = (int64_t*)(ws + 256);
  BF_HIP(ctx, hipMemsetAsync(ws, 0, 16, ctx->stream));
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(256), 0, ctx->stream, scores_dev, n_cand);
  if (N > 0) {
    BF_CHECK(ctx, mu_dev && s_dev, "bf_nbv_score: NULL mu or s");
    hipLaunchKernelGGL(k_max, dim3(nbm), dim3(kThreads), 0, ctx->stream, s_dev, N, (unsigned long long*)smax);
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)bf_cdiv(N, kThreads)), dim3(kThreads), 0, ctx->stream, s_dev, N,
                       smax, q);
    ray_k R{};
    R.g = bf_grid_k{band->G, band->h, band->origin[0], band->origin[1], band->origin[2], band->tau, band->band};
    R.cam = bf_cam_k{ray_cam->width, ray_cam->height, ray_cam->fx, ray_cam->fy, ray_cam->cx, ray_cam->cy};
    R.utility = utility;
    if (noise) {
      R.na = noise->a;
      R.nc = noise->c;
      R.nz0 = noise->z0;
    }
    const int64_t npix = (int64_t)ray_cam->width * ray_cam->height;
    R.brick_shift = band->brick_shift;
    R.nbrick = band->nbrick;
    R.ncell = band->ncell;
    R.tiles_per_cand = bf_cdiv(npix, kThreads);
    R.ntiles = R.tiles_per_cand * n_cand;
    const unsigned grid = (unsigned)std::min<int64_t>(R.ntiles, 16 * (int64_t)ctx->cu_count);
    BF_LAUNCH(ctx, "nbv_rays", k_nbv_rays, dim3(grid), dim3(kThreads), 0, R, cand_c2w_dev,
              (const unsigned long long*)band->cell_mask, band->cell_start, band->brick_dist, mu_dev, s_dev, q, smax,
              band->bricks, (unsigned long long*)scores_dev);
  }
  hipLaunchKernelGGL(k_argmax, dim3(1), dim3(1024), 0, ctx->stream, scores_dev, n_cand, dbest);
  BF_TRY(bf_launch_check(ctx, "nbv"));
  int32_t* pin = nullptr;
  BF_TRY(bf_pinned(ctx, 8, (void**)&pin));
  BF_HIP(ctx, hipMemcpyAsync(pin, dbest, 4, hipMemcpyDeviceToHost, ctx->stream));
  BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *best_host = *pin;
  return BF_OK;
}
