// Many scenes of uneven band size solved in one persistent launch (the
// Hutchinson block CG of eq. 12, or the mean solve of eq. 11 with one column),
// and the autotuner that picks its schedule.
//
// The work list is the concatenation of every scene's row tiles, ordered by
// the schedule; a grid of co-resident workgroups walks it phase by phase and
// meets at grid barriers between phases:
//   A (stencil + p.q) | alpha | B (updates + dots) | beta / checks |
//   [fold | FP64 residual | decisions]   ... until every column of every
// scene has stopped.
// Per-scene, per-column scalars use the same decisions as the single-system
// solver (block_tiles.h).  Converged scenes drop out of the work list at no
// cost.  Schedules: tile order (scene-major, interleaved, largest scene first)
// and an XCD-aware mapping that keeps contiguous runs of tiles on the blocks of
// one XCD, so stencil gathers of neighbouring rows hit the same L2.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "block_tiles.h"

namespace cg = cooperative_groups;

namespace {

using namespace bt;

struct SceneDev {
  int64_t n;
  int64_t tile0;   // first global tile id
  int32_t ntiles;
  int32_t K;
  const int32_t* nbr;
  const void* diagV;
  const void* dinvV;
  const double* diag64;
  double lam;
  uint64_t seed;
  const double* rhs;  // mean mode: right-hand side (column 0), else null (probes)
  double* x64;
  void* r;
  void* zz;
  void* p0;
  void* p1;
  void* q;
  float* cf;
  double* part;  // [ntiles][3][KC]
  BState* st;
  double* out;   // probes: s = (1/K) sum z u; mean mode: x
};

struct Sched {
  int rows;       // rows per tile
  int xcd;        // 1: XCD-aware block -> tile mapping
  int64_t ntiles;
};

// Work items handled by this block, in order.  With the XCD-aware mapping the
// list is cut into 8 contiguous parts, part x served by blocks b with b % 8 == x
// (workgroups are dispatched to the XCDs round robin).
struct Walker {
  int64_t start, stride, end;
  __device__ Walker(const Sched& s) {
    if (s.xcd && gridDim.x % 8 == 0) {
      const int x = blockIdx.x % 8, loc = blockIdx.x / 8, nloc = gridDim.x / 8;
      const int64_t lo = s.ntiles * x / 8, hi = s.ntiles * (x + 1) / 8;
      start = lo + loc;
      stride = nloc;
      end = hi;
    } else {
      start = blockIdx.x;
      stride = gridDim.x;
      end = s.ntiles;
    }
  }
};

__device__ __forceinline__ int scene_of(const int64_t* __restrict__ tile_start, int S, int64_t gid) {
  int lo = 0, hi = S - 1;
  while (lo < hi) {  // last scene with tile_start <= gid
    const int mid = (lo + hi + 1) / 2;
    if (tile_start[mid] <= gid) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename V, int KC>
__global__ __launch_bounds__(256) void k_batch(const SceneDev* __restrict__ sc, int S,
                                               const int64_t* __restrict__ order, const int64_t* __restrict__ tstart,
                                               Sched sch, int max_iter, int* __restrict__ ctrl) {
  __shared__ double lds[4 * 3 * 64];
  cg::grid_group grid = cg::this_grid();
  const int c = threadIdx.x % KC;
  const Walker wk(sch);

  auto tile_rows = [&](const SceneDev& d, int64_t gid, int64_t& r0, int64_t& r1) {
    const int64_t j = gid - d.tile0;
    r0 = j * sch.rows;
    r1 = std::min<int64_t>(d.n, r0 + sch.rows);
  };

  // ---------------------------------------------------------- residual phase
  auto resid_phase = [&](int mode) {
    for (int64_t w = wk.start; w < wk.end; w += wk.stride) {
      const int64_t gid = order[w];
      const int s = scene_of(tstart, S, gid);
      const SceneDev& d = sc[s];
      BState* st = d.st;
      if (mode == MODE_CHECK && (st->nactive == 0 || !st->any_check)) continue;
      const bool act = mode == MODE_REPORT ? c < d.K
                                           : (st->active[c] != 0 && (mode == MODE_INIT || st->check[c] != 0));
      int64_t r0, r1;
      tile_rows(d, gid, r0, r1);
      double v3[3] = {0.0, 0.0, 0.0};
      if (act) {
        if (d.rhs) {  // mean mode: the right-hand side replaces the probe
          constexpr int RS = kThreads / KC;
          for (int64_t v = r0 + threadIdx.x / KC; v < r1; v += RS) {
            const int64_t e = v * KC + c;
            const double zv = d.rhs[v];
            double res = zv;
            if (mode == MODE_INIT) {
              d.x64[e] = 0.0;
            } else {
              const int32_t* nb = d.nbr + v * 6;
              double acc = 0.0;
#pragma unroll
              for (int t = 0; t < 6; ++t) {
                const int32_t u = nb[t];
                if (u >= 0) acc += d.x64[(int64_t)u * KC + c];
              }
              res = zv - (d.diag64[v] * d.x64[e] - d.lam * acc);
            }
            v3[0] += res * res;
            v3[2] += zv * zv;
            if (mode != MODE_REPORT) {
              const V rv = (V)res;
              const V zzv = rv * ((const V*)d.dinvV)[v];
              ((V*)d.r)[e] = rv;
              ((V*)d.zz)[e] = zzv;
              v3[1] += (double)rv * (double)zzv;
            }
          }
        } else {
          tile_resid<V, KC>(c, mode, splitmix_out(d.seed, (uint64_t)c), d.nbr, d.diag64, d.lam, nullptr, d.x64,
                            (const V*)d.dinvV, (V*)d.r, (V*)d.zz, r0, r1, v3);
        }
      }
      col_block_sum<KC, 3>(v3, lds);
      store_partials<KC, 3>(d.part, gid - d.tile0, v3);
    }
  };
  auto resid_decide = [&](int mode) {
    for (int64_t p = blockIdx.x; p < (int64_t)S * KC; p += gridDim.x) {
      const int s = (int)(p / KC), cc = (int)(p % KC);
      const SceneDev& d = sc[s];
      BState* st = d.st;
      if (mode == MODE_CHECK && !(st->active[cc] && st->check[cc])) continue;
      if (mode == MODE_REPORT && cc >= d.K) continue;
      if (mode == MODE_INIT && !st->active[cc]) continue;
      double tot[3];
      col_partials_sum<KC, 3>(d.part, d.ntiles, cc, tot, lds);
      if (threadIdx.x == 0) decide_R(st, cc, mode, tot, mode == MODE_REPORT ? nullptr : &ctrl[0]);
      __syncthreads();
    }
  };

  resid_phase(MODE_INIT);
  grid.sync();
  resid_decide(MODE_INIT);
  grid.sync();

  for (int it = 0; it < max_iter; ++it) {
    if (ctrl[0] == 0) break;  // every block reads the same value after the barrier
    // A
    for (int64_t w = wk.start; w < wk.end; w += wk.stride) {
      const int64_t gid = order[w];
      const int s = scene_of(tstart, S, gid);
      const SceneDev& d = sc[s];
      BState* st = d.st;
      if (st->nactive == 0) continue;
      const V* pa = (const V*)((it & 1) ? d.p1 : d.p0);
      V* pb = (V*)((it & 1) ? d.p0 : d.p1);
      int64_t r0, r1;
      tile_rows(d, gid, r0, r1);
      double v1[1] = {0.0};
      if (st->active[c])
        tile_A<V, KC>(c, (V)st->beta[c], d.nbr, (const V*)d.diagV, (V)d.lam, (const V*)d.zz, pa, pb, (V*)d.q, r0, r1,
                      v1[0]);
      col_block_sum<KC, 1>(v1, lds);
      store_partials<KC, 1>(d.part, gid - d.tile0, v1);
    }
    grid.sync();
    for (int64_t p = blockIdx.x; p < (int64_t)S * KC; p += gridDim.x) {
      const int s = (int)(p / KC), cc = (int)(p % KC);
      BState* st = sc[s].st;
      if (cc == 0 && threadIdx.x == 0) st->any_check = 0;
      if (blockIdx.x == 0 && p == 0 && threadIdx.x == 0) ctrl[1] = 0;
      if (!st->active[cc]) continue;
      double tot[1];
      col_partials_sum<KC, 1>(sc[s].part, sc[s].ntiles, cc, tot, lds);
      if (threadIdx.x == 0) decide_A(st, cc, tot[0], &ctrl[0]);
      __syncthreads();
    }
    grid.sync();
    // B
    for (int64_t w = wk.start; w < wk.end; w += wk.stride) {
      const int64_t gid = order[w];
      const int s = scene_of(tstart, S, gid);
      const SceneDev& d = sc[s];
      BState* st = d.st;
      if (st->nactive == 0) continue;
      const V* pb = (const V*)((it & 1) ? d.p0 : d.p1);
      V* xin = sizeof(V) == 4 ? (V*)d.cf : (V*)d.x64;
      int64_t r0, r1;
      tile_rows(d, gid, r0, r1);
      double v2[2] = {0.0, 0.0};
      if (st->active[c])
        tile_B<V, KC>(c, (V)st->alpha[c], (const V*)d.dinvV, pb, (const V*)d.q, xin, (V*)d.r, (V*)d.zz, r0, r1, v2[0],
                      v2[1]);
      col_block_sum<KC, 2>(v2, lds);
      store_partials<KC, 2>(d.part, gid - d.tile0, v2);
    }
    grid.sync();
    for (int64_t p = blockIdx.x; p < (int64_t)S * KC; p += gridDim.x) {
      const int s = (int)(p / KC), cc = (int)(p % KC);
      BState* st = sc[s].st;
      if (!st->active[cc]) continue;
      double tot[2];
      col_partials_sum<KC, 2>(sc[s].part, sc[s].ntiles, cc, tot, lds);
      if (threadIdx.x == 0) decide_B(st, cc, tot[0], tot[1], &ctrl[0], &ctrl[1]);
      __syncthreads();
    }
    grid.sync();
    if (ctrl[1]) {  // some column asked for an FP64 residual check
      if (sizeof(V) == 4) {
        for (int64_t w = wk.start; w < wk.end; w += wk.stride) {
          const int64_t gid = order[w];
          const int s = scene_of(tstart, S, gid);
          const SceneDev& d = sc[s];
          BState* st = d.st;
          if (!(st->active[c] && st->check[c])) continue;
          int64_t r0, r1;
          tile_rows(d, gid, r0, r1);
          tile_fold<KC>(c, d.x64, d.cf, r0, r1);
        }
        grid.sync();
      }
      resid_phase(MODE_CHECK);
      grid.sync();
      resid_decide(MODE_CHECK);
      grid.sync();
    }
  }
  // fold the remaining float corrections, outputs, final residuals
  if (sizeof(V) == 4)
    for (int64_t w = wk.start; w < wk.end; w += wk.stride) {
      const int64_t gid = order[w];
      const int s = scene_of(tstart, S, gid);
      const SceneDev& d = sc[s];
      int64_t r0, r1;
      tile_rows(d, gid, r0, r1);
      if (c < d.K) tile_fold<KC>(c, d.x64, d.cf, r0, r1);
    }
  grid.sync();
  for (int64_t w = wk.start; w < wk.end; w += wk.stride) {
    const int64_t gid = order[w];
    const int s = scene_of(tstart, S, gid);
    const SceneDev& d = sc[s];
    int64_t r0, r1;
    tile_rows(d, gid, r0, r1);
    for (int64_t v = r0 + threadIdx.x; v < r1; v += blockDim.x)
      d.out[v] = d.rhs ? d.x64[v * KC] : hutch_row<KC>(d.x64, d.seed, d.K, v);
  }
  resid_phase(MODE_REPORT);
  grid.sync();
  resid_decide(MODE_REPORT);
}

__global__ void k_batch_state_init(BState* st, int S, const int* K, double tol, int32_t max_iter, double inner) {
  for (int s = blockIdx.x; s < S; s += gridDim.x) bt::state_init(st + s, K[s], tol, max_iter, inner);
}

template <typename V>
__global__ __launch_bounds__(256) void k_fill_v(V* __restrict__ p, int64_t n, V val) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}

size_t al(size_t b) { return (b + 255) / 256 * 256; }

// Host side of one batched solve.  mean: rhs of every system, K = 1.
template <typename V, int KC>
bf_status run_batch(bf_ctx* ctx, const bf_system* const* systems, int S, int K, uint64_t seed, double tol,
                    int max_iter, bool mean, const float* const* logvar, double* const* out,
                    const bf_schedule* sched, bf_solve_report* reps, double* seconds) {
  (void)logvar;
  const bool mixed = sizeof(V) == 4;
  const int rows = sched->rows_per_tile;
  // tiles and the schedule's order
  std::vector<int64_t> tstart(S), ntile(S);
  int64_t T = 0;
  for (int s = 0; s < S; ++s) {
    tstart[s] = T;
    ntile[s] = bf_cdiv(systems[s]->n, rows);
    T += ntile[s];
  }
  std::vector<int64_t> order;
  order.reserve(T);
  std::vector<int> sorder(S);
  std::iota(sorder.begin(), sorder.end(), 0);
  if (sched->order == BF_ORDER_LARGEST_FIRST)
    std::stable_sort(sorder.begin(), sorder.end(), [&](int a, int b) { return ntile[a] > ntile[b]; });
  if (sched->order == BF_ORDER_INTERLEAVED) {
    int64_t mx = 0;
    for (int s = 0; s < S; ++s) mx = std::max(mx, ntile[s]);
    for (int64_t j = 0; j < mx; ++j)
      for (int s = 0; s < S; ++s)
        if (j < ntile[s]) order.push_back(tstart[s] + j);
  } else {
    for (int s : sorder)
      for (int64_t j = 0; j < ntile[s]; ++j) order.push_back(tstart[s] + j);
  }
  // device memory: descriptors | states | order | tstart | ctrl | per-scene vectors and partials
  size_t bytes = al(S * sizeof(SceneDev)) + al(S * sizeof(BState)) + al(T * 8) + al(S * 8) + al(64) + al(S * 4);
  std::vector<size_t> off(S);
  for (int s = 0; s < S; ++s) {
    const size_t n = systems[s]->n;
    off[s] = bytes;
    bytes += al(ntile[s] * 3 * KC * 8) + al(n * KC * 8) + 5 * al(n * KC * sizeof(V)) + (mixed ? al(n * KC * 4) : 0);
  }
  char* ws = nullptr;
  BF_TRY(bf_ws(ctx, bf_ctx::WS_BATCH, bytes, (void**)&ws));
  char* p = ws;
  SceneDev* dsc = (SceneDev*)p;
  p += al(S * sizeof(SceneDev));
  BState* dst = (BState*)p;
  p += al(S * sizeof(BState));
  int64_t* dorder = (int64_t*)p;
  p += al(T * 8);
  int64_t* dtstart = (int64_t*)p;
  p += al(S * 8);
  int* ctrl = (int*)p;
  p += al(64);
  int* dK = (int*)p;
  std::vector<SceneDev> hsc(S);
  for (int s = 0; s < S; ++s) {
    const bf_system* sy = systems[s];
    const size_t n = sy->n;
    char* q = ws + off[s];
    SceneDev& d = hsc[s];
    d.n = sy->n;
    d.tile0 = tstart[s];
    d.ntiles = (int32_t)ntile[s];
    d.K = K;
    d.nbr = sy->band->nbr;
    d.diagV = mixed ? (const void*)sy->diag32 : (const void*)sy->diag;
    d.dinvV = mixed ? (const void*)sy->dinv32 : (const void*)sy->dinv;
    d.diag64 = sy->diag;
    d.lam = sy->lambda;
    d.seed = seed;
    d.rhs = mean ? sy->rhs : nullptr;
    d.part = (double*)q;
    q += al(ntile[s] * 3 * KC * 8);
    d.x64 = (double*)q;
    q += al(n * KC * 8);
    d.r = q;
    q += al(n * KC * sizeof(V));
    d.zz = q;
    q += al(n * KC * sizeof(V));
    d.p0 = q;
    q += al(n * KC * sizeof(V));
    d.p1 = q;
    q += al(n * KC * sizeof(V));
    d.q = q;
    q += al(n * KC * sizeof(V));
    d.cf = mixed ? (float*)q : nullptr;
    d.st = dst + s;
    d.out = out[s];
  }
  std::vector<int> hK(S, K);
  int hctrl[2] = {S * K, 0};
  BF_HIP(ctx, hipMemcpyAsync(dsc, hsc.data(), S * sizeof(SceneDev), hipMemcpyHostToDevice, ctx->stream));
  BF_HIP(ctx, hipMemcpyAsync(dorder, order.data(), T * 8, hipMemcpyHostToDevice, ctx->stream));
  BF_HIP(ctx, hipMemcpyAsync(dtstart, tstart.data(), S * 8, hipMemcpyHostToDevice, ctx->stream));
  BF_HIP(ctx, hipMemcpyAsync(dK, hK.data(), S * 4, hipMemcpyHostToDevice, ctx->stream));
  BF_HIP(ctx, hipMemcpyAsync(ctrl, hctrl, sizeof(hctrl), hipMemcpyHostToDevice, ctx->stream));
  hipLaunchKernelGGL(k_batch_state_init, dim3(std::min(S, 1024)), dim3(64), 0, ctx->stream, dst, S, dK, tol, max_iter,
                     mixed ? 1e-6 : 0.0);
  for (int s = 0; s < S; ++s) {
    const int64_t nn = hsc[s].n * KC;
    const int fb = (int)std::min<int64_t>(bf_cdiv(nn, 256), 4096);
    hipLaunchKernelGGL(k_fill_v<V>, dim3(fb), dim3(256), 0, ctx->stream, (V*)hsc[s].p0, nn, (V)0);
    if (mixed) hipLaunchKernelGGL(k_fill_v<float>, dim3(fb), dim3(256), 0, ctx->stream, hsc[s].cf, nn, 0.0f);
  }
  BF_TRY(bf_launch_check(ctx, "batch setup"));

  // co-resident grid
  int per_cu = 0;
  BF_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_batch<V, KC>, 256, 0));
  int grid = sched->blocks_per_cu > 0 ? sched->blocks_per_cu * ctx->cu_count : per_cu * ctx->cu_count;
  grid = std::min(grid, per_cu * ctx->cu_count);
  if (grid < 1) return bf_fail(ctx, BF_ERR_HIP, "batched solve: kernel cannot be resident");
  Sched sch{rows, sched->xcd_aware ? 1 : 0, T};
  void* args[] = {(void*)&dsc, (void*)&S, (void*)&dorder, (void*)&dtstart, (void*)&sch, (void*)&max_iter,
                  (void*)&ctrl};
  hipEvent_t e0, e1;
  BF_HIP(ctx, hipEventCreate(&e0));
  BF_HIP(ctx, hipEventCreate(&e1));
  BF_HIP(ctx, hipEventRecord(e0, ctx->stream));
  hipEvent_t ta = nullptr;
  if (ctx->timing) {
    ta = bf_event_get(ctx);
    (void)hipEventRecord(ta, ctx->stream);
  }
  hipError_t le = hipLaunchCooperativeKernel((const void*)k_batch<V, KC>, dim3(grid), dim3(256), args, 0, ctx->stream);
  if (ctx->timing) bf_timing_stop(ctx, "batch_persistent", ta);
  if (le != hipSuccess) return bf_fail(ctx, BF_ERR_HIP, "cooperative launch failed: %s", hipGetErrorString(le));
  BF_HIP(ctx, hipEventRecord(e1, ctx->stream));
  std::vector<BState> hst(S);
  BF_HIP(ctx, hipMemcpyAsync(hst.data(), dst, S * sizeof(BState), hipMemcpyDeviceToHost, ctx->stream));
  BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (seconds) *seconds = ms * 1e-3;
  bf_status worst = BF_OK;
  for (int s = 0; s < S; ++s) {
    const BState& h = hst[s];
    bf_status st = BF_OK;
    int maxit = 0;
    int64_t sumit = 0;
    double maxres = 0.0;
    for (int k = 0; k < K; ++k) {
      sumit += h.iters[k];
      maxit = std::max(maxit, (int)h.iters[k]);
      if (h.status[k] == BF_ERR_BREAKDOWN) st = BF_ERR_BREAKDOWN;
      else if (h.status[k] == BF_ERR_NOT_CONVERGED && st == BF_OK) st = BF_ERR_NOT_CONVERGED;
      if (h.bnorm2[k] > 0.0) maxres = std::max(maxres, sqrt(h.rr_true[k] / h.bnorm2[k]));
    }
    if (st == BF_OK && h.nactive != 0) st = BF_ERR_NOT_CONVERGED;
    if (reps) {
      reps[s] = bf_solve_report{};
      reps[s].iters = maxit;
      reps[s].status = st;
      reps[s].refinements = h.refinements;
      reps[s].rel_res = maxres;
      reps[s].seconds = ms * 1e-3;
      reps[s].col_iters = sumit;
    }
    if (st == BF_ERR_BREAKDOWN) worst = st;
    else if (st == BF_ERR_NOT_CONVERGED && worst == BF_OK) worst = st;
  }
  if (worst != BF_OK) return bf_fail(ctx, worst, "batched solve: some systems ended with status %d", worst);
  return BF_OK;
}

bf_status dispatch(bf_ctx* ctx, const bf_system* const* systems, int S, int K, uint64_t seed, double tol,
                   int max_iter, int precision, bool mean, double* const* out, const bf_schedule* sched,
                   bf_solve_report* reps, double* seconds) {
  const bool f64 = precision == BF_PREC_FP64;
  if (mean) return f64 ? run_batch<double, 1>(ctx, systems, S, 1, 0, tol, max_iter, true, nullptr, out, sched, reps, seconds)
                       : run_batch<float, 1>(ctx, systems, S, 1, 0, tol, max_iter, true, nullptr, out, sched, reps, seconds);
  if (K <= 16)
    return f64 ? run_batch<double, 16>(ctx, systems, S, K, seed, tol, max_iter, false, nullptr, out, sched, reps, seconds)
               : run_batch<float, 16>(ctx, systems, S, K, seed, tol, max_iter, false, nullptr, out, sched, reps, seconds);
  if (K <= 32)
    return f64 ? run_batch<double, 32>(ctx, systems, S, K, seed, tol, max_iter, false, nullptr, out, sched, reps, seconds)
               : run_batch<float, 32>(ctx, systems, S, K, seed, tol, max_iter, false, nullptr, out, sched, reps, seconds);
  return f64 ? run_batch<double, 64>(ctx, systems, S, K, seed, tol, max_iter, false, nullptr, out, sched, reps, seconds)
             : run_batch<float, 64>(ctx, systems, S, K, seed, tol, max_iter, false, nullptr, out, sched, reps, seconds);
}

bf_status check_batch(bf_ctx* ctx, const bf_system* const* systems, int32_t n_sys, double* const* out,
                      const bf_schedule* sched) {
  BF_CHECK(ctx, systems && out && n_sys >= 1, "batched solve: bad system list");
  for (int s = 0; s < n_sys; ++s) {
    BF_CHECK(ctx, systems[s] && systems[s]->n > 0, "batched solve: system %d is NULL or empty", s);
    BF_CHECK(ctx, out[s], "batched solve: NULL output for system %d", s);
  }
  BF_CHECK(ctx, sched->rows_per_tile >= 16 && sched->rows_per_tile <= 4096, "batched solve: rows_per_tile %d",
           sched->rows_per_tile);
  BF_CHECK(ctx, sched->order >= 0 && sched->order <= 2, "batched solve: unknown order %d", sched->order);
  return BF_OK;
}

const bf_schedule kDefault{256, 0, BF_ORDER_SCENE_MAJOR, 1};

}  // namespace

extern "C" bf_status bf_diag_estimate_batched(bf_ctx* ctx, const bf_system* const* systems, int32_t n_sys,
                                              const bf_probe_opts* opts, const bf_schedule* sched,
                                              double* const* s_dev, bf_solve_report* reps) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, opts, "bf_diag_estimate_batched: NULL options");
  BF_CHECK(ctx, opts->K >= 1 && opts->K <= 64, "bf_diag_estimate_batched: K=%d outside [1, 64]", opts->K);
  const bf_schedule* sc = sched ? sched : &kDefault;
  BF_TRY(check_batch(ctx, systems, n_sys, s_dev, sc));
  BF_HIP(ctx, hipSetDevice(ctx->device));
  return dispatch(ctx, systems, n_sys, opts->K, opts->seed, opts->tol, opts->max_iter, opts->precision, false, s_dev,
                  sc, reps, nullptr);
}

extern "C" bf_status bf_pcg_solve_batched(bf_ctx* ctx, const bf_system* const* systems, int32_t n_sys,
                                          const bf_solve_opts* opts, const bf_schedule* sched, double* const* x_dev,
                                          bf_solve_report* reps) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, opts && !opts->use_x0, "bf_pcg_solve_batched: NULL options or a start (not supported)");
  const bf_schedule* sc = sched ? sched : &kDefault;
  BF_TRY(check_batch(ctx, systems, n_sys, x_dev, sc));
  BF_HIP(ctx, hipSetDevice(ctx->device));
  return dispatch(ctx, systems, n_sys, 1, 0, opts->tol, opts->max_iter, opts->precision, true, x_dev, sc, reps,
                  nullptr);
}

extern "C" bf_status bf_autotune_batch(bf_ctx* ctx, const bf_system* const* systems, int32_t n_sys,
                                       const bf_probe_opts* opts, double* const* s_dev, bf_schedule* best,
                                       char* json, size_t json_len) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, opts && best, "bf_autotune_batch: NULL argument");
  BF_CHECK(ctx, opts->K >= 1 && opts->K <= 64, "bf_autotune_batch: K=%d outside [1, 64]", opts->K);
  BF_TRY(check_batch(ctx, systems, n_sys, s_dev, &kDefault));
  BF_HIP(ctx, hipSetDevice(ctx->device));
  const int rows[] = {64, 128, 256, 512};
  const int bpc[] = {1, 2, 4};
  const int orders[] = {BF_ORDER_SCENE_MAJOR, BF_ORDER_INTERLEAVED, BF_ORDER_LARGEST_FIRST};
  std::string log = "[";
  double best_t = 1e30;
  bool first = true;
  for (int r : rows)
    for (int b : bpc)
      for (int o : orders)
        for (int x = 0; x < 2; ++x) {
          bf_schedule cand{r, b, o, x};
          double t = 0.0;
          // one untimed run to settle allocations, then the timed one
          bf_status st = dispatch(ctx, systems, n_sys, opts->K, opts->seed, opts->tol, opts->max_iter,
                                  opts->precision, false, s_dev, &cand, nullptr, nullptr);
          if (st == BF_OK)
            st = dispatch(ctx, systems, n_sys, opts->K, opts->seed, opts->tol, opts->max_iter, opts->precision, false,
                          s_dev, &cand, nullptr, &t);
          char buf[160];
          snprintf(buf, sizeof(buf), "%s{\"rows\":%d,\"blocks_per_cu\":%d,\"order\":%d,\"xcd\":%d,\"ms\":%.4f,\"ok\":%d}",
                   first ? "" : ",", r, b, o, x, t * 1e3, st == BF_OK ? 1 : 0);
          first = false;
          log += buf;
          if (st == BF_OK && t < best_t) {
            best_t = t;
            *best = cand;
          }
        }
  log += "]";
  if (json && json_len > 0) {
    strncpy(json, log.c_str(), json_len - 1);
    json[json_len - 1] = 0;
  }
  if (best_t >= 1e30) return bf_fail(ctx, BF_ERR_HIP, "bf_autotune_batch: no candidate ran");
  return BF_OK;
}
