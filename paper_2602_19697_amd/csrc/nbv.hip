// Next-best-view scoring (Sec. 3.8, eq. 13; Algorithm 1 step 8).
//
// Each candidate pose casts one ray per pixel of the ray camera.  A thread
// walks its ray through the voxel grid (Amanatides-Woo, with the next
// boundary on each axis computed directly from the voxel index so the walk is
// reproducible) and sums the quantised variance of the band voxels it crosses
// up to and including the first voxel whose posterior mean is <= 0.  Band
// membership is tested only in occupied bricks (a bitmap in LDS), through the
// 4^3 cell masks; across empty bricks the walk jumps (see Ray).  Variances are quantised to int64
// (q = rint(s / max s * 2^32)) before summation, so the per-candidate
// utility is an exact integer independent of summation order: block sums
// are combined with 64-bit integer atomics.
#include "bf_internal.h"

#include <climits>
#include <cstdlib>

namespace {

constexpr int kThreads = 256;
constexpr double kScale = 4294967296.0;  // 2^32

// max(0, max_v s_v): non-negative doubles order like their bit patterns, so an
// integer atomic max on the bits is exact and order independent.
__global__ __launch_bounds__(256) void k_max(const double* __restrict__ s, int64_t n,
                                             unsigned long long* __restrict__ out_bits) {
  __shared__ double lds[kThreads / 64];
  // four loads in flight per thread; the maximum is exact in any order
  double m = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const double a = s[i], b = s[i + stride], c = s[i + 2 * stride], d = s[i + 3 * stride];
    m = fmax(fmax(m, a), fmax(fmax(b, c), d));
  }
  for (; i < n; i += stride) m = fmax(m, s[i]);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) b = fmax(b, lds[w]);
    atomicMax(out_bits, (unsigned long long)__double_as_longlong(b));
  }
}

// q = rint(s / max s * 2^32), stored as 2q + [mu <= 0]: the low bit says the
// walk stops at this voxel.  q is negative where the estimate s is (eq. 12's
// Hutchinson estimate is unbiased, not positive), and the arithmetic shift
// qs >> 1 gives it back exactly for |q| < 2^62.
__global__ __launch_bounds__(256) void k_quantize(const double* __restrict__ s, const double* __restrict__ mu,
                                                  int64_t n, const double* __restrict__ smax,
                                                  int64_t* __restrict__ qs) {
#pragma clang fp contract(off)
  const int64_t v = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (v >= n) return;
  const double m = *smax;
  const int64_t q = m > 0.0 ? (int64_t)rint((s[v] / m) * kScale) : 0;
  qs[v] = (int64_t)((uint64_t)q << 1) | (mu[v] <= 0.0 ? 1 : 0);
}

struct ray_k {
  bf_grid_k g;
  bf_cam_k cam;
  double inv_h;        // 1/h, only for the jump estimate (corrected exactly after)
  int jump_min;        // jump from empty bricks at least this far (Chebyshev, bricks) from the band
  int jump_batch;      // ... once this many lanes of the wave want to jump (or a quarter of the live ones)
  int refill_batch;    // idle lanes start new rays once this many are idle (or the whole wave)
  double na, nc, nz0;  // sensor model for the variance-reduction utility
  int brick_shift, nbrick, ncell;
  int32_t nbrick3;     // bricks in the grid: offset between octants of the distance table
  int64_t tiles_per_cand, ntiles;
  int32_t tiles_x;     // 16x16-pixel tiles per image row
};

constexpr int kMaxBrickWords = 64 * 64 * 64 / 32;
constexpr int kMaxTable = 256;  // ray cameras up to this many columns and rows use quotient tables
// Defaults of the walk's tuning knobs (see ray_k); BF_NBV_JUMP_MIN,
// BF_NBV_JUMP_BATCH and BF_NBV_REFILL_BATCH override them.  None changes a result.
constexpr int kJumpMinDist = 1;
constexpr int kJumpBatch = 32;
constexpr int kRefillBatch = 24;

// Time at which the ray crosses plane p of one axis (the plane between voxels
// p - 1 and p).  Every step and every jump evaluates plane times with this one
// expression, so a jump lands on exactly the state the voxel steps reach.
__device__ __forceinline__ double plane_t(double org, double h, double o, double inv, int32_t p) {
#pragma clang fp contract(off)
  return ((org + (double)p * h) - o) * inv;
}

// The walk of one ray, as a state advanced one iteration at a time so that a
// lane whose ray has ended can start another while the rest of its wave walks.
//
// The voxel sequence is the Amanatides-Woo walk: each step crosses the
// nearest next plane (lowest axis on ties), with plane times from plane_t.
// Since every plane time depends only on the plane index, the walk is the
// merge, ordered by (time, axis), of the three axes' plane sequences, and
// "every crossing earlier than time c" is a prefix of it.  In an empty brick
// the walk jumps across the box of bricks ahead of the ray that the brick's
// forward-octant distance (for the octant of the ray's direction) proves empty:
// from the current brick to dist - 1 bricks further along each axis the ray
// moves on.  c = the earliest time at which the ray crosses a far face of that
// box, and each axis advances by the number of its planes with time < c
// (estimated from the continuous ray, then corrected with plane_t).  The
// voxels skipped hold no band voxel, so the visited band voxels, the utility
// and the stopping voxel are those of the plain walk.
//
// SUM_VAR reads qs[v]: twice the quantised variance, plus one when the
// voxel's posterior mean is <= 0 (the walk stops there), so one load serves
// both.  VAR_REDUCTION reads mu and s.
struct Ray {
  double d[3], inv[3], tn[3];
  int32_t idx[3], step[3];
  int32_t last_brick, last_dist, iters;
  int32_t steps;  // voxels the plain walk visits (visited here or jumped over)
  int64_t score;
};

// Starts the ray through pixel (row, col) of the candidate camera at o with
// rotation P; false when it misses the grid (utility 0).
// ta, tb (may be null): the quotients (col - cx)/fx and (row - cy)/fy of
// every column and row, the same values computed once per launch.
__device__ __forceinline__ bool ray_init(Ray& r, const ray_k& R, const double* __restrict__ P, const double (&o)[3],
                                         int32_t row, int32_t col, const double* ta = nullptr,
                                         const double* tb = nullptr) {
#pragma clang fp contract(off)
  const bf_grid_k& g = R.g;
  const double a = ta ? ta[col] : ((double)col - R.cam.cx) / R.cam.fx;
  const double b = tb ? tb[row] : ((double)row - R.cam.cy) / R.cam.fy;
  r.d[0] = (P[0] * a + P[1] * b) + P[2];
  r.d[1] = (P[4] * a + P[5] * b) + P[6];
  r.d[2] = (P[8] * a + P[9] * b) + P[10];
  const double org[3] = {g.ox, g.oy, g.oz};
  double tnear = 0.0, tfar = INFINITY;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const double lo = org[ax];
    const double hi = org[ax] + (double)g.G * g.h;
    if (r.d[ax] == 0.0) {
      r.inv[ax] = 0.0;
      if (o[ax] < lo || o[ax] > hi) return false;
      continue;
    }
    r.inv[ax] = 1.0 / r.d[ax];
    const double t0 = (lo - o[ax]) * r.inv[ax];
    const double t1 = (hi - o[ax]) * r.inv[ax];
    const double tmin = t0 < t1 ? t0 : t1;
    const double tmax = t0 < t1 ? t1 : t0;
    if (tmin > tnear) tnear = tmin;
    if (tmax < tfar) tfar = tmax;
  }
  if (!(tnear < tfar)) return false;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const double pa = o[ax] + tnear * r.d[ax];
    const double f = floor((pa - org[ax]) / g.h);
    r.idx[ax] = f < 0.0 ? 0 : (f > (double)(g.G - 1) ? g.G - 1 : (int32_t)f);
    r.step[ax] = r.d[ax] > 0.0 ? 1 : (r.d[ax] < 0.0 ? -1 : 0);
    r.tn[ax] = r.step[ax] == 0 ? INFINITY
                               : plane_t(org[ax], g.h, o[ax], r.inv[ax], r.idx[ax] + (r.step[ax] > 0 ? 1 : 0));
  }
  r.last_brick = -1;
  r.last_dist = 0;
  r.iters = 0;
  r.steps = 0;
  r.score = 0;
  return true;
}

// One iteration: test the current voxel (or jump across empty bricks), then
// step.  Returns false when the ray has ended; r.score then holds its utility.
template <int UTIL>
__device__ __forceinline__ bool ray_advance(Ray& r, const ray_k& R, int nlive, const double* __restrict__ P,
                                            const double (&o)[3], const bf_cell* __restrict__ cells,
                                            const uint8_t* __restrict__ bdist, const double* __restrict__ mu,
                                            const double* __restrict__ s, const int64_t* __restrict__ qs,
                                            double smax, const uint32_t* __restrict__ bricks) {
#pragma clang fp contract(off)
  const bf_grid_k& g = R.g;
  const double org[3] = {g.ox, g.oy, g.oz};
  const int bs = R.brick_shift, NB = R.nbrick, NC = R.ncell;
  // every iteration crosses at least one plane, and a ray crosses at most 3G
  if (++r.iters > 3 * g.G + 3) return false;
  ++r.steps;
  const int32_t bit = (int32_t)((((uint32_t)r.idx[2] >> bs) * NB + ((uint32_t)r.idx[1] >> bs)) * NB +
                                ((uint32_t)r.idx[0] >> bs));
  if ((bricks[bit >> 5] >> (bit & 31)) & 1u) {
    // occupied brick: is this voxel in the band?  (4^3 cell mask, rank by popcount)
    // at most 512^3 cells (G <= 2048): the index fits 32 bits
    const uint32_t c = (((uint32_t)r.idx[2] >> 2) * (uint32_t)NC + ((uint32_t)r.idx[1] >> 2)) * (uint32_t)NC +
                       ((uint32_t)r.idx[0] >> 2);
    const uint32_t m = (r.idx[0] & 1) | ((r.idx[1] & 1) << 1) | ((r.idx[2] & 1) << 2) | ((r.idx[0] & 2) << 2) |
                       ((r.idx[1] & 2) << 3) | ((r.idx[2] & 2) << 4);
    // the cell's mask and start in one 16-byte load: read apart, the start's
    // load would wait for the mask test, one more trip to memory per voxel
    const uint4 cw = *reinterpret_cast<const uint4*>(cells + c);
    int32_t start = (int32_t)cw.z;
    asm volatile("" : "+v"(start));
    const unsigned long long cmask = ((unsigned long long)cw.y << 32) | cw.x;
    if ((cmask >> m) & 1ull) {
      const int32_t v = start + __popcll(cmask & ((1ull << m) - 1ull));
      if constexpr (UTIL == BF_UTILITY_SUM_VAR) {
        const int64_t qv = qs[v];
        r.score += qv >> 1;
        if (qv & 1) return false;
      } else {
        // expected variance reduction of one new observation at the voxel's depth
        const double x = org[0] + ((double)r.idx[0] + 0.5) * g.h;
        const double y = org[1] + ((double)r.idx[1] + 0.5) * g.h;
        const double z = org[2] + ((double)r.idx[2] + 0.5) * g.h;
        const double dx = x - P[3], dy = y - P[7], dz = z - P[11];
        const double Z = (P[2] * dx + P[6] * dy) + P[10] * dz;
        const double e = Z - R.nz0;
        const double sd = R.na + R.nc * (e * e);
        const double sv = s[v];
        const double term = sv > 0.0 ? (sv * sv) / (sv + sd * sd) : 0.0;
        r.score += smax > 0.0 ? (int64_t)rint((term / smax) * kScale) : 0;
        if (mu[v] <= 0.0) return false;
      }
    }
  } else {
    if (bit != r.last_brick) {
      r.last_brick = bit;
      const int32_t oct = (r.step[0] < 0 ? 1 : 0) | (r.step[1] < 0 ? 2 : 0) | (r.step[2] < 0 ? 4 : 0);
      r.last_dist = bdist[oct * R.nbrick3 + bit];
    }
    // The jump costs as much as several voxel steps and the wave executes it for
    // all lanes at once, so it runs only when enough lanes want it; the others
    // (and these, meanwhile) take an ordinary voxel step, which is always exact.
    const bool want = r.last_dist >= R.jump_min;
    const int nwant = __popcll(__ballot(want));
    if (want && (nwant >= R.jump_batch || 4 * nwant >= nlive)) {
      // the bricks from this one to rb further along the ray's octant are
      // empty: jump to the last voxel before the walk leaves that box
      const int rb = r.last_dist - 1;
      int32_t lo[3], hi[3];
      double cut = INFINITY;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const int32_t bb = r.idx[ax] >> bs;
        lo[ax] = r.step[ax] < 0 ? max(0, (bb - rb) << bs) : bb << bs;
        hi[ax] = r.step[ax] < 0 ? ((bb + 1) << bs) - 1 : min(g.G - 1, ((bb + rb + 1) << bs) - 1);
        if (r.step[ax] != 0) {
          const double te = plane_t(org[ax], g.h, o[ax], r.inv[ax], r.step[ax] > 0 ? hi[ax] + 1 : lo[ax]);
          cut = te < cut ? te : cut;
        }
      }
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        if (r.step[ax] == 0) continue;
        const int32_t sg = r.step[ax];
        const int32_t p0 = r.idx[ax] + (sg > 0 ? 1 : 0);
        const int32_t nmax = sg > 0 ? hi[ax] + 1 - p0 : p0 - lo[ax];  // interior planes ahead
        const double u = ((o[ax] + cut * r.d[ax]) - org[ax]) * R.inv_h;
        double ne = sg > 0 ? floor(u) - (double)p0 + 1.0 : (double)p0 - ceil(u) + 1.0;
        ne = ne < 0.0 ? 0.0 : (ne > (double)nmax ? (double)nmax : ne);
        int32_t n = (int32_t)ne;
        // n is right when the last plane taken is earlier than cut and the next
        // one is not; the estimate almost always is, so test that first and
        // walk plane by plane only otherwise
        const double t_last = n > 0 ? plane_t(org[ax], g.h, o[ax], r.inv[ax], p0 + (n - 1) * sg) : -INFINITY;
        double t_next = n < nmax ? plane_t(org[ax], g.h, o[ax], r.inv[ax], p0 + n * sg) : INFINITY;
        if (!(t_last < cut && !(t_next < cut))) {
          while (n > 0 && plane_t(org[ax], g.h, o[ax], r.inv[ax], p0 + (n - 1) * sg) >= cut) --n;
          while (n < nmax && plane_t(org[ax], g.h, o[ax], r.inv[ax], p0 + n * sg) < cut) ++n;
          t_next = plane_t(org[ax], g.h, o[ax], r.inv[ax], p0 + n * sg);
        }
        r.idx[ax] += n * sg;
        r.steps += n;
        r.tn[ax] = n < nmax ? t_next : plane_t(org[ax], g.h, o[ax], r.inv[ax], p0 + n * sg);
      }
    }
  }
  // step across the nearest plane, lowest axis on ties; every array index is a
  // compile-time constant so the ray state stays in registers
  int ax = 0;
  double tm = r.tn[0];
  if (r.tn[1] < tm) {
    ax = 1;
    tm = r.tn[1];
  }
  if (r.tn[2] < tm) ax = 2;
  bool inside = true;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (a == ax) {
      r.idx[a] += r.step[a];
      inside = r.idx[a] >= 0 && r.idx[a] < g.G;
      r.tn[a] = plane_t(org[a], g.h, o[a], r.inv[a], r.idx[a] + (r.step[a] > 0 ? 1 : 0));
    }
  return inside;
}

// Work queue over (candidate, 16x16-pixel tile) taken wave by wave; every
// workgroup stages the brick bitmap in LDS once.  A tile's rays are up to four
// 8x8 pixel blocks (fewer on the image's right and bottom edges), handed out
// block by block, so the 64 rays a wave walks at a time are neighbours in both
// image directions (similar paths: fewer divergent branches, shared cache
// lines).  Rays go to lanes on demand: once enough lanes are idle (refill_batch,
// or the whole wave), they take the tile's next unwalked rays in lane order, so
// no lane is tied to a fixed share of long rays while the others wait.

template <int UTIL>
__global__ __launch_bounds__(256)
void k_nbv_rays(ray_k R, const double* __restrict__ cands, const bf_cell* __restrict__ cells,
                const uint8_t* __restrict__ bdist, const double* __restrict__ mu, const double* __restrict__ s,
                const int64_t* __restrict__ qs, const double* __restrict__ smax_p,
                const uint32_t* __restrict__ bricks_g, unsigned int* __restrict__ queue,
                unsigned long long* __restrict__ walk_steps, unsigned long long* __restrict__ scores) {
  __shared__ uint32_t bricks[kMaxBrickWords];
  __shared__ double tcol[kMaxTable], trow[kMaxTable];
  const int words = (R.nbrick * R.nbrick * R.nbrick + 31) / 32;
  for (int w = threadIdx.x; w < words; w += kThreads) bricks[w] = bricks_g[w];
  // the pixel quotients of ray_init once per workgroup (cameras up to 256 x 256)
  const bool tables = R.cam.W <= kMaxTable && R.cam.H <= kMaxTable;
  if (tables) {
#pragma clang fp contract(off)
    for (int t = threadIdx.x; t < R.cam.W; t += kThreads) tcol[t] = ((double)t - R.cam.cx) / R.cam.fx;
    for (int t = threadIdx.x; t < R.cam.H; t += kThreads) trow[t] = ((double)t - R.cam.cy) / R.cam.fy;
  }
  __syncthreads();
  const double smax = *smax_p;
  const int lane = threadIdx.x & 63;
  for (;;) {
    unsigned int t = 0;
    if (lane == 0) t = atomicAdd(queue, 1u);
    // wave-uniform from here on: the pose and chunk live in scalar registers
    const int64_t tile = (int64_t)(unsigned int)__builtin_amdgcn_readfirstlane((int)__shfl(t, 0, 64));
    if (tile >= R.ntiles) break;
    const int64_t cand = tile / R.tiles_per_cand;
    const int32_t tb = (int32_t)(tile % R.tiles_per_cand);
    const int32_t ty = tb / R.tiles_x, tx = tb % R.tiles_x;
    const double* P = cands + 12 * cand;
    const double o[3] = {P[3], P[7], P[11]};
    const int32_t bxn = min(2, (R.cam.W - tx * 16 + 7) >> 3);  // 8x8 blocks of the tile in the image
    const int32_t byn = min(2, (R.cam.H - ty * 16 + 7) >> 3);
    const int32_t nrays = 64 * bxn * byn;
    int32_t base = 0;  // rays of the tile handed out so far (wave-uniform)
    long long acc = 0;
    unsigned long long nsteps = 0;
    Ray r;
    bool live = false;
    for (;;) {
      const bool want = !live && base < nrays;
      const unsigned long long need = __ballot(want);
      const unsigned long long busy = __ballot(live);
      if (need == 0 && busy == 0) break;  // wave-uniform
      if (need != 0 && (__popcll(need) >= R.refill_batch || busy == 0)) {
        if (want) {
          // ray of the tile: 8x8 block ray / 64, position ray % 64 in it
          const int32_t ray = base + (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
          const int32_t blk = ray >> 6, l = ray & 63;
          const int32_t bx = bxn == 2 ? (blk & 1) : 0, by = bxn == 2 ? (blk >> 1) : blk;
          const int32_t row = ty * 16 + by * 8 + (l >> 3), col = tx * 16 + bx * 8 + (l & 7);
          // re-read the pose here rather than keep its rotation in scalar
          // registers across the whole walk loop (they would spill)
          const double* Pi = P;
          asm volatile("" : "+s"(Pi));
          live = ray < nrays && row < R.cam.H && col < R.cam.W &&
                 ray_init(r, R, Pi, o, row, col, tables ? tcol : nullptr, tables ? trow : nullptr);
        }
        base += __popcll(need);
        continue;
      }
      if (live && !ray_advance<UTIL>(r, R, __popcll(busy), P, o, cells, bdist, mu, s, qs, smax, bricks)) {
        acc += r.score;
        nsteps += (unsigned long long)r.steps;
        live = false;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      acc += __shfl_xor(acc, off, 64);
      nsteps += __shfl_xor(nsteps, off, 64);
    }
    if (lane == 0) {
      atomicAdd(&scores[cand], (unsigned long long)acc);  // two's complement: exact for signed sums
      atomicAdd(walk_steps, nsteps);
    }
  }
}

// The view a sensor with camera R.cam would take from pose P, predicted from
// the mean (the observations a candidate adds, for the post-view variance of
// eq. 13): each pixel's ray is walked voxel by voxel, the walk of
// bf_nbv_score without jumps, to the first band voxel with mu <= 0; the
// pixel's depth is that voxel centre's camera-z depth, rounded to float, and
// 0 (no return) when the ray meets none.  One thread per pixel.
__global__ __launch_bounds__(256) void k_pred_depth(ray_k R, const double* __restrict__ P,
                                                    const bf_cell* __restrict__ cells,
                                                    const double* __restrict__ mu,
                                                    const uint32_t* __restrict__ bricks_g, float* __restrict__ depth) {
#pragma clang fp contract(off)
  __shared__ uint32_t bricks[kMaxBrickWords];
  const int words = (R.nbrick * R.nbrick * R.nbrick + 31) / 32;
  for (int w = threadIdx.x; w < words; w += kThreads) bricks[w] = bricks_g[w];
  __syncthreads();
  const bf_grid_k& g = R.g;
  const double org[3] = {g.ox, g.oy, g.oz};
  const double o[3] = {P[3], P[7], P[11]};
  const int bs = R.brick_shift, NB = R.nbrick, NC = R.ncell;
  const int64_t npix = (int64_t)R.cam.W * R.cam.H;
  for (int64_t p = blockIdx.x * (int64_t)kThreads + threadIdx.x; p < npix; p += (int64_t)gridDim.x * kThreads) {
    const int32_t row = (int32_t)(p / R.cam.W), col = (int32_t)(p % R.cam.W);
    Ray r;
    float z = 0.0f;
    if (ray_init(r, R, P, o, row, col)) {
      for (int32_t it = 0; it < 3 * g.G + 3; ++it) {
        const int32_t bit = (int32_t)((((uint32_t)r.idx[2] >> bs) * NB + ((uint32_t)r.idx[1] >> bs)) * NB +
                                      ((uint32_t)r.idx[0] >> bs));
        if ((bricks[bit >> 5] >> (bit & 31)) & 1u) {
          const uint32_t c = (((uint32_t)r.idx[2] >> 2) * (uint32_t)NC + ((uint32_t)r.idx[1] >> 2)) * (uint32_t)NC +
                             ((uint32_t)r.idx[0] >> 2);
          const uint32_t m = (r.idx[0] & 1) | ((r.idx[1] & 1) << 1) | ((r.idx[2] & 1) << 2) |
                             ((r.idx[0] & 2) << 2) | ((r.idx[1] & 2) << 3) | ((r.idx[2] & 2) << 4);
          const bf_cell cl = cells[c];
          if ((cl.mask >> m) & 1ull) {
            const int32_t v = cl.start + __popcll(cl.mask & ((1ull << m) - 1ull));
            if (mu[v] <= 0.0) {
              const double x = org[0] + ((double)r.idx[0] + 0.5) * g.h;
              const double y = org[1] + ((double)r.idx[1] + 0.5) * g.h;
              const double zc = org[2] + ((double)r.idx[2] + 0.5) * g.h;
              const double dx = x - P[3], dy = y - P[7], dz = zc - P[11];
              z = (float)((P[2] * dx + P[6] * dy) + P[10] * dz);
              break;
            }
          }
        }
        // step across the nearest plane, lowest axis on ties
        int ax = 0;
        double tm = r.tn[0];
        if (r.tn[1] < tm) {
          ax = 1;
          tm = r.tn[1];
        }
        if (r.tn[2] < tm) ax = 2;
        bool inside = true;
#pragma unroll
        for (int a = 0; a < 3; ++a)
          if (a == ax) {
            r.idx[a] += r.step[a];
            inside = r.idx[a] >= 0 && r.idx[a] < g.G;
            r.tn[a] = plane_t(org[a], g.h, o[a], r.inv[a], r.idx[a] + (r.step[a] > 0 ? 1 : 0));
          }
        if (!inside) break;
      }
    }
    depth[p] = z;
  }
}

__global__ void k_zero_f32(float* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

// Clears the scores and the walk's three workspace words (maximum variance,
// best index and hand-out counter, visit count).
__global__ void k_zero_i64(int64_t* p, int n, uint64_t* ws3) {
  if (threadIdx.x < 3) ws3[threadIdx.x] = 0;
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

int env_int(const char* name, int dflt, int lo, int hi) {
  const char* v = getenv(name);
  if (!v) return dflt;
  const int x = atoi(v);
  return x < lo ? lo : (x > hi ? hi : x);
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
  ctx->nbv_walk_steps = 0;
  if (n_cand == 0) return BF_OK;
  BF_CHECK(ctx, cand_c2w_dev && scores_dev, "bf_nbv_score: NULL candidates or scores");
  BF_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t N = band->n;
  // workspace: smax | best | chunk counter | qs [N]
  // few workgroups: each ends in one atomic on the same word, and those serialise
  const int nbm = (int)std::max<int64_t>(1, std::min<int64_t>(bf_cdiv(N, 8 * kThreads), 256));
  char* ws = nullptr;
  BF_TRY(bf_ws(ctx, bf_ctx::WS_NBV, 256 + N * 8, (void**)&ws));
  double* smax = (double*)ws;
  int32_t* dbest = (int32_t*)(ws + 8);
  unsigned int* queue = (unsigned int*)(ws + 12);
  unsigned long long* walk_steps = (unsigned long long*)(ws + 16);
  int64_t* q = (int64_t*)(ws + 256);
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(256), 0, ctx->stream, scores_dev, n_cand, (uint64_t*)ws);
  if (N > 0) {
    BF_CHECK(ctx, mu_dev && s_dev, "bf_nbv_score: NULL mu or s");
    hipLaunchKernelGGL(k_max, dim3(nbm), dim3(kThreads), 0, ctx->stream, s_dev, N, (unsigned long long*)smax);
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)bf_cdiv(N, kThreads)), dim3(kThreads), 0, ctx->stream, s_dev,
                       mu_dev, N, smax, q);
    ray_k R{};
    R.g = bf_grid_k{band->G, band->h, band->origin[0], band->origin[1], band->origin[2], band->tau, band->band};
    R.cam = bf_cam_k{ray_cam->width, ray_cam->height, ray_cam->fx, ray_cam->fy, ray_cam->cx, ray_cam->cy};
    R.inv_h = 1.0 / band->h;
    R.jump_min = env_int("BF_NBV_JUMP_MIN", kJumpMinDist, 1, 256);
    R.jump_batch = env_int("BF_NBV_JUMP_BATCH", kJumpBatch, 1, 64);
    R.refill_batch = env_int("BF_NBV_REFILL_BATCH", kRefillBatch, 1, 64);
    if (noise) {
      R.na = noise->a;
      R.nc = noise->c;
      R.nz0 = noise->z0;
    }
    R.brick_shift = band->brick_shift;
    R.nbrick = band->nbrick;
    R.nbrick3 = band->nbrick * band->nbrick * band->nbrick;
    R.ncell = band->ncell;
    R.tiles_x = (int32_t)bf_cdiv(ray_cam->width, 16);
    R.tiles_per_cand = (int64_t)R.tiles_x * bf_cdiv(ray_cam->height, 16);
    R.ntiles = R.tiles_per_cand * n_cand;
    BF_CHECK(ctx, R.ntiles < (1ll << 31), "bf_nbv_score: too many rays");
    int per_cu = 0;
    BF_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_nbv_rays<BF_UTILITY_SUM_VAR>,
                                                             kThreads, 0));
    const unsigned grid = (unsigned)std::min<int64_t>(R.ntiles, std::max(1, per_cu) * (int64_t)ctx->cu_count);
    if (utility == BF_UTILITY_SUM_VAR)
      BF_LAUNCH(ctx, "nbv_rays", k_nbv_rays<BF_UTILITY_SUM_VAR>, dim3(grid), dim3(kThreads), 0, R, cand_c2w_dev,
                band->cells, band->brick_dist, mu_dev, s_dev, q, smax, band->bricks, queue,
                walk_steps, (unsigned long long*)scores_dev);
    else
      BF_LAUNCH(ctx, "nbv_rays", k_nbv_rays<BF_UTILITY_VAR_REDUCTION>, dim3(grid), dim3(kThreads), 0, R,
                cand_c2w_dev, band->cells, band->brick_dist, mu_dev, s_dev, q, smax, band->bricks, queue,
                walk_steps, (unsigned long long*)scores_dev);
  }
  hipLaunchKernelGGL(k_argmax, dim3(1), dim3(1024), 0, ctx->stream, scores_dev, n_cand, dbest);
  BF_TRY(bf_launch_check(ctx, "nbv"));
  int32_t* pin = nullptr;
  BF_TRY(bf_pinned(ctx, 16, (void**)&pin));
  BF_HIP(ctx, hipMemcpyAsync(pin, dbest, 16, hipMemcpyDeviceToHost, ctx->stream));
  BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *best_host = pin[0];
  ctx->nbv_walk_steps = *(const int64_t*)(pin + 2);
  return BF_OK;
}

extern "C" bf_status bf_predict_depth(bf_ctx* ctx, const bf_band* band, const double* mu_dev,
                                      const double* c2w_dev, const bf_camera* cam, float* depth_dev) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, band && cam && c2w_dev && depth_dev, "bf_predict_depth: NULL argument");
  BF_CHECK(ctx, cam->width > 0 && cam->height > 0 && (int64_t)cam->width * cam->height < (1ll << 31),
           "bf_predict_depth: bad camera");
  BF_CHECK(ctx, band->n == 0 || mu_dev, "bf_predict_depth: NULL mu");
  BF_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t npix = (int64_t)cam->width * cam->height;
  ray_k R{};
  R.g = bf_grid_k{band->G, band->h, band->origin[0], band->origin[1], band->origin[2], band->tau, band->band};
  R.cam = bf_cam_k{cam->width, cam->height, cam->fx, cam->fy, cam->cx, cam->cy};
  R.brick_shift = band->brick_shift;
  R.nbrick = band->nbrick;
  R.nbrick3 = band->nbrick * band->nbrick * band->nbrick;
  R.ncell = band->ncell;
  if (band->n == 0) {  // an empty band: no ray meets a surface
    BF_LAUNCH(ctx, "pred_depth", k_zero_f32, dim3((unsigned)std::min<int64_t>(bf_cdiv(npix, kThreads), 4096)),
              dim3(kThreads), 0, depth_dev, npix);
    return bf_launch_check(ctx, "k_zero_f32");
  }
  const unsigned grid = (unsigned)std::min<int64_t>(bf_cdiv(npix, kThreads), 8 * (int64_t)ctx->cu_count);
  BF_LAUNCH(ctx, "pred_depth", k_pred_depth, dim3(grid), dim3(kThreads), 0, R, c2w_dev, band->cells, mu_dev,
            band->bricks, depth_dev);
  return bf_launch_check(ctx, "k_pred_depth");
}

extern "C" bf_status bf_nbv_walk_steps(bf_ctx* ctx, int64_t* steps) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, steps, "bf_nbv_walk_steps: NULL argument");
  *steps = ctx->nbv_walk_steps;
  return BF_OK;
}
