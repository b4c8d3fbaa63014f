// Many scenes of uneven band size solved together: the Hutchinson block CG of
// eq. (12) for every scene, the batched mean solve of eq. (11), and the
// autotuner that picks the schedule.
//
// The work list is the concatenation of every scene's row tiles, ordered by
// the schedule.  The CG phases are
//   A (stencil + p.q) | alpha | B (updates + dots) | beta / checks |
//   [fold | FP64 residual | decisions]   ... until every column stops.
// Two launch kinds walk that list:
//  * persistent: one cooperative launch; co-resident workgroups walk the list
//    phase by phase and meet at grid barriers (probe blocks of 16 to 64
//    columns only);
//  * phased: every phase is a launch of its own over the whole list and the
//    host polls the active-column count, so no co-residency is assumed.
// Per-scene, per-column scalars use the decisions of the single-system solver
// (block_tiles.h); converged scenes drop out of the work list.  Schedules:
// tile order (scene-major, interleaved, largest scene first) and an XCD-aware
// mapping that keeps contiguous runs of tiles on the workgroups of one XCD, so
// the stencil gathers of neighbouring rows hit the same L2.
//
// The grid barrier waits a bounded time: a workgroup that waits too long
// raises an abort flag, every workgroup leaves at its next barrier, and the
// call fails with an error instead of hanging.  The one-column (mean) solve
// has no persistent instantiation: it runs phased.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "block_tiles.h"

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
  const double* rhs;  // mean solve: right-hand side (column 0); null for probes
  double* x64;
  void* r;
  void* zz;
  void* p0;
  void* p1;
  void* q;
  float* cf;
  double* part;  // [ntiles][3][KC]
  BState* st;
  double* out;   // probes: s = (1/K) sum z u; mean solve: x
};

struct Sched {
  int rows;       // rows per tile
  int xcd;        // 1: XCD-aware block -> tile mapping
  int64_t ntiles;
};

// ctrl[] words
enum { C_ACTIVE = 0, C_CHECK = 1, C_ARRIVE = 2, C_GEN = 3, C_ABORT = 4, C_WORDS = 5 };

struct Batch {
  const SceneDev* sc;
  int S;
  const int64_t* order;
  const int64_t* tstart;
  Sched sch;
  int* ctrl;  // C_ACTIVE: active columns over all scenes, C_CHECK: a residual check is pending
};

// Work items handled by this block, in order.  With the XCD-aware mapping the
// list is cut into 8 contiguous parts, part x served by blocks b with b % 8 == x
// (workgroups are dispatched to the XCDs round robin).
struct Walker {
  int64_t start, stride, end;
  __device__ Walker(const Sched& s) {
    if (s.xcd && gridDim.x % 8 == 0) {
      const int x = blockIdx.x % 8, loc = blockIdx.x / 8, nloc = gridDim.x / 8;
      start = s.ntiles * x / 8 + loc;
      stride = nloc;
      end = s.ntiles * (x + 1) / 8;
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

__device__ __forceinline__ const SceneDev& item_scene(const Batch& B, int64_t w, int64_t& r0, int64_t& r1,
                                                      int64_t& slot) {
  const int64_t gid = B.order[w];
  const SceneDev& d = B.sc[scene_of(B.tstart, B.S, gid)];
  slot = gid - d.tile0;
  r0 = slot * B.sch.rows;
  r1 = std::min<int64_t>(d.n, r0 + B.sch.rows);
  return d;
}

__device__ __forceinline__ int ctrl_load(int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- work items
// Each item is one row tile of one scene; every thread of the block calls it.
template <typename V, int KC>
__device__ void item_resid(const Batch& B, int64_t w, int mode, double* lds) {
  const int c = threadIdx.x % KC;
  int64_t r0, r1, slot;
  const SceneDev& d = item_scene(B, w, r0, r1, slot);
  const BState* st = d.st;
  if (mode == MODE_CHECK && (st->nactive == 0 || !st->any_check)) return;
  const bool act = mode == MODE_REPORT ? c < d.K : (st->active[c] != 0 && (mode == MODE_INIT || st->check[c] != 0));
  double v3[3] = {0.0, 0.0, 0.0};
  if (act) {
    if (d.rhs) {  // mean solve: the right-hand side replaces the probe
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
  store_partials<KC, 3>(d.part, slot, v3);
}

template <typename V, int KC>
__device__ void item_A(const Batch& B, int64_t w, int it, double* lds) {
  const int c = threadIdx.x % KC;
  int64_t r0, r1, slot;
  const SceneDev& d = item_scene(B, w, r0, r1, slot);
  const BState* st = d.st;
  if (st->nactive == 0) return;
  const V* pa = (const V*)((it & 1) ? d.p1 : d.p0);
  V* pb = (V*)((it & 1) ? d.p0 : d.p1);
  double v1[1] = {0.0};
  if (st->active[c])
    tile_A<V, KC>(c, (V)st->beta[c], false, d.nbr, (const V*)d.diagV, (V)d.lam, (const V*)d.zz, pa, pb, (V*)d.q, r0, r1,
                  v1[0]);
  col_block_sum<KC, 1>(v1, lds);
  store_partials<KC, 1>(d.part, slot, v1);
}

template <typename V, int KC>
__device__ void item_B(const Batch& B, int64_t w, int it, double* lds) {
  const int c = threadIdx.x % KC;
  int64_t r0, r1, slot;
  const SceneDev& d = item_scene(B, w, r0, r1, slot);
  const BState* st = d.st;
  if (st->nactive == 0) return;
  const V* pb = (const V*)((it & 1) ? d.p0 : d.p1);
  V* xin = sizeof(V) == 4 ? (V*)d.cf : (V*)d.x64;
  double v2[2] = {0.0, 0.0};
  if (st->active[c])
    tile_B<V, KC>(c, (V)st->alpha[c], false, false, 0ull, (const V*)d.dinvV, pb, (const V*)d.q, xin, (V*)d.r,
                  (V*)d.zz, r0, r1, v2[0],
                  v2[1]);
  col_block_sum<KC, 2>(v2, lds);
  store_partials<KC, 2>(d.part, slot, v2);
}

// Mixed precision: fold the float correction into x64 (columns being checked,
// or every column at the end).
template <int KC>
__device__ void item_fold(const Batch& B, int64_t w, bool all) {
  const int c = threadIdx.x % KC;
  int64_t r0, r1, slot;
  const SceneDev& d = item_scene(B, w, r0, r1, slot);
  const BState* st = d.st;
  if (all ? c < d.K : (st->active[c] && st->check[c])) tile_fold<KC>(c, d.x64, d.cf, r0, r1);
}

template <int KC>
__device__ void item_out(const Batch& B, int64_t w) {
  int64_t r0, r1, slot;
  const SceneDev& d = item_scene(B, w, r0, r1, slot);
  for (int64_t v = r0 + threadIdx.x; v < r1; v += blockDim.x)
    d.out[v] = d.rhs ? d.x64[v * KC] : hutch_row<KC>(d.x64, d.seed, d.K, v);
}

// ---------------------------------------------------------------- decisions of one (scene, column) pair
// One workgroup per pair: the column's partials summed in a fixed order, then
// thread 0 takes the decision.
enum { DEC_A = 0, DEC_B = 1, DEC_R = 2 };

template <int KC>
__device__ void decide_pair(const Batch& B, int64_t p, int which, int mode, double* lds) {
  const int s = (int)(p / KC), c = (int)(p % KC);
  const SceneDev& d = B.sc[s];
  BState* st = d.st;
  if (which == DEC_A) {
    if (c == 0 && threadIdx.x == 0) st->any_check = 0;  // consumed by the previous check, if any
    if (p == 0 && threadIdx.x == 0) B.ctrl[C_CHECK] = 0;
    if (!st->active[c]) return;
    double tot[1];
    col_partials_sum<KC, 1>(d.part, d.ntiles, c, tot, lds);
    if (threadIdx.x == 0) decide_A(st, c, tot[0], &B.ctrl[C_ACTIVE]);
  } else if (which == DEC_B) {
    if (!st->active[c]) return;
    double tot[2];
    col_partials_sum<KC, 2>(d.part, d.ntiles, c, tot, lds);
    if (threadIdx.x == 0) decide_B(st, c, tot[0], tot[1], &B.ctrl[C_ACTIVE], &B.ctrl[C_CHECK]);
  } else {
    if (mode == MODE_CHECK && !(st->active[c] && st->check[c])) return;
    if (mode == MODE_REPORT && c >= d.K) return;
    if (mode == MODE_INIT && !st->active[c]) return;
    double tot[3];
    col_partials_sum<KC, 3>(d.part, d.ntiles, c, tot, lds);
    if (threadIdx.x == 0) decide_R(st, c, mode, tot, mode == MODE_REPORT ? nullptr : &B.ctrl[C_ACTIVE]);
  }
}

// ---------------------------------------------------------------- persistent kernel
constexpr long kSpinLimit = 1l << 21;  // polls (about 1 us each) before a barrier gives up

// Grid barrier over co-resident workgroups with a bounded wait; returns true
// (in every thread) when the grid must stop because a barrier timed out.
__device__ bool grid_barrier(int* ctrl, int& gen) {
  __shared__ int abort_flag;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ab = __hip_atomic_load(&ctrl[C_ABORT], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!ab) {
      __threadfence();
      const int prev = __hip_atomic_fetch_add(&ctrl[C_ARRIVE], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (prev == (int)gridDim.x - 1) {
        __hip_atomic_store(&ctrl[C_ARRIVE], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctrl[C_GEN], gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        long spins = 0;
        while (__hip_atomic_load(&ctrl[C_GEN], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
          if (__hip_atomic_load(&ctrl[C_ABORT], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            ab = 1;
            break;
          }
          if (++spins > kSpinLimit) {
            __hip_atomic_store(&ctrl[C_ABORT], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ab = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      __threadfence();
    }
    abort_flag = ab;
  }
  ++gen;
  __syncthreads();
  return abort_flag != 0;
}

#define BF_BARRIER()                          \
  do {                                        \
    if (grid_barrier(B.ctrl, gen)) return;    \
  } while (0)

template <typename V, int KC>
__global__ __launch_bounds__(256) void k_batch(Batch B, int max_iter) {
  static_assert(KC >= 16, "the persistent batch kernel serves probe blocks only");
  __shared__ double lds[4 * 3 * 64];
  const Walker wk(B.sch);
  const int64_t npairs = (int64_t)B.S * KC;
  int gen = 0;
  auto decide_all = [&](int which, int mode) {
    for (int64_t p = blockIdx.x; p < npairs; p += gridDim.x) {
      decide_pair<KC>(B, p, which, mode, lds);
      __syncthreads();
    }
  };
  for (int64_t w = wk.start; w < wk.end; w += wk.stride) item_resid<V, KC>(B, w, MODE_INIT, lds);
  BF_BARRIER();
  decide_all(DEC_R, MODE_INIT);
  BF_BARRIER();
  for (int it = 0; it < max_iter; ++it) {
    // every block reads the same value: it only changes between later barriers
    if (ctrl_load(&B.ctrl[C_ACTIVE]) == 0) break;
    for (int64_t w = wk.start; w < wk.end; w += wk.stride) item_A<V, KC>(B, w, it, lds);
    BF_BARRIER();
    decide_all(DEC_A, 0);
    BF_BARRIER();
    for (int64_t w = wk.start; w < wk.end; w += wk.stride) item_B<V, KC>(B, w, it, lds);
    BF_BARRIER();
    decide_all(DEC_B, 0);
    BF_BARRIER();
    if (ctrl_load(&B.ctrl[C_CHECK])) {  // an FP64 residual check was requested
      if (sizeof(V) == 4) {
        for (int64_t w = wk.start; w < wk.end; w += wk.stride) item_fold<KC>(B, w, false);
        BF_BARRIER();
      }
      for (int64_t w = wk.start; w < wk.end; w += wk.stride) item_resid<V, KC>(B, w, MODE_CHECK, lds);
      BF_BARRIER();
      decide_all(DEC_R, MODE_CHECK);
      BF_BARRIER();
    }
  }
  if (sizeof(V) == 4)
    for (int64_t w = wk.start; w < wk.end; w += wk.stride) item_fold<KC>(B, w, true);
  BF_BARRIER();
  for (int64_t w = wk.start; w < wk.end; w += wk.stride) item_out<KC>(B, w);
  for (int64_t w = wk.start; w < wk.end; w += wk.stride) item_resid<V, KC>(B, w, MODE_REPORT, lds);
  BF_BARRIER();
  decide_all(DEC_R, MODE_REPORT);
}

#undef BF_BARRIER

// ---------------------------------------------------------------- phased kernels
enum { PH_RESID = 0, PH_A = 1, PH_B = 2, PH_FOLD = 3, PH_OUT = 4 };

// Phases that only run while columns are active return at once otherwise, so
// the host can queue iterations ahead of its convergence poll.
__device__ __forceinline__ bool phase_idle(const Batch& B, bool needs_active, bool needs_check) {
  if (needs_active && ctrl_load(&B.ctrl[C_ACTIVE]) == 0) return true;
  if (needs_check && ctrl_load(&B.ctrl[C_CHECK]) == 0) return true;
  return false;
}

template <typename V, int KC>
__global__ __launch_bounds__(256) void kp_items(Batch B, int phase, int mode, int it) {
  __shared__ double lds[4 * 3 * 64];
  const bool loop_phase = phase == PH_A || phase == PH_B || mode == MODE_CHECK;
  if (phase_idle(B, loop_phase, mode == MODE_CHECK)) return;
  const Walker wk(B.sch);
  for (int64_t w = wk.start; w < wk.end; w += wk.stride) {
    if (phase == PH_RESID) item_resid<V, KC>(B, w, mode, lds);
    else if (phase == PH_A) item_A<V, KC>(B, w, it, lds);
    else if (phase == PH_B) item_B<V, KC>(B, w, it, lds);
    else if (phase == PH_FOLD) item_fold<KC>(B, w, mode != MODE_CHECK);
    else item_out<KC>(B, w);
  }
}

template <int KC>
__global__ __launch_bounds__(256) void kp_decide(Batch B, int which, int mode) {
  __shared__ double lds[16];
  const bool loop_phase = which != DEC_R || mode == MODE_CHECK;
  if (phase_idle(B, loop_phase, which == DEC_R && mode == MODE_CHECK)) return;
  const int64_t npairs = (int64_t)B.S * KC;
  for (int64_t p = blockIdx.x; p < npairs; p += gridDim.x) {
    decide_pair<KC>(B, p, which, mode, lds);
    __syncthreads();
  }
}

__global__ void k_batch_state_init(BState* st, int S, int K, double tol, int32_t max_iter, double inner,
                                   int32_t replace_every) {
  for (int s = blockIdx.x; s < S; s += gridDim.x) bt::state_init(st + s, K, tol, max_iter, inner, replace_every);
}

template <typename V>
__global__ __launch_bounds__(256) void k_fill_v(V* __restrict__ p, int64_t n, V val) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}

size_t al(size_t b) { return (b + 255) / 256 * 256; }

template <typename V, int KC>
bf_status launch_persistent(bf_ctx* ctx, Batch& B, int max_iter, const bf_schedule* sched, int* ctrl_host) {
  if constexpr (KC >= 16) {
    int per_cu = 0;
    BF_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_batch<V, KC>, 256, 0));
    const int bpc = sched->blocks_per_cu > 0 ? std::min(sched->blocks_per_cu, per_cu) : per_cu;
    const int grid = bpc * ctx->cu_count;
    if (grid < 1) return bf_fail(ctx, BF_ERR_HIP, "batched solve: the persistent kernel cannot be resident");
    void* args[] = {(void*)&B, (void*)&max_iter};
    hipEvent_t ta = nullptr;
    if (ctx->timing) {
      ta = bf_event_get(ctx);
      (void)hipEventRecord(ta, ctx->stream);
    }
    const hipError_t le =
        hipLaunchCooperativeKernel((const void*)k_batch<V, KC>, dim3(grid), dim3(256), args, 0, ctx->stream);
    if (ctx->timing) {
      hipEvent_t tb = bf_event_get(ctx);
      (void)hipEventRecord(tb, ctx->stream);
      bf_timing_add(ctx, "batch_persistent", ta, tb);
    }
    if (le != hipSuccess) return bf_fail(ctx, BF_ERR_HIP, "cooperative launch failed: %s", hipGetErrorString(le));
    BF_HIP(ctx, hipMemcpyAsync(ctrl_host, B.ctrl, C_WORDS * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    return BF_OK;
  } else {
    (void)B, (void)max_iter, (void)sched, (void)ctrl_host;
    return bf_fail(ctx, BF_ERR_INVALID_ARG, "batched solve: the persistent launch serves probe blocks only");
  }
}

template <typename V, int KC>
bf_status launch_phased(bf_ctx* ctx, Batch& B, int S, int64_t T, int max_iter, const bf_schedule* sched,
                        int* ctrl_host) {
  const bool mixed = sizeof(V) == 4;
  const int bpc = sched->blocks_per_cu > 0 ? sched->blocks_per_cu : 4;
  const dim3 grid((unsigned)std::min<int64_t>(T, (int64_t)bpc * ctx->cu_count));
  const dim3 dgrid((unsigned)std::min<int64_t>((int64_t)S * KC, 1024));
  const dim3 blk(256);
  BF_LAUNCH(ctx, "batch_items", (kp_items<V, KC>), grid, blk, 0, B, (int)PH_RESID, (int)MODE_INIT, 0);
  BF_LAUNCH(ctx, "batch_decide", kp_decide<KC>, dgrid, blk, 0, B, (int)DEC_R, (int)MODE_INIT);
  int it = 0, next = 3;
  for (;;) {
    const int upto = std::min(next, max_iter);
    for (; it < upto; ++it) {
      BF_LAUNCH(ctx, "batch_items", (kp_items<V, KC>), grid, blk, 0, B, (int)PH_A, 0, it);
      BF_LAUNCH(ctx, "batch_decide", kp_decide<KC>, dgrid, blk, 0, B, (int)DEC_A, 0);
      BF_LAUNCH(ctx, "batch_items", (kp_items<V, KC>), grid, blk, 0, B, (int)PH_B, 0, it);
      BF_LAUNCH(ctx, "batch_decide", kp_decide<KC>, dgrid, blk, 0, B, (int)DEC_B, 0);
      if (mixed) BF_LAUNCH(ctx, "batch_items", (kp_items<V, KC>), grid, blk, 0, B, (int)PH_FOLD, (int)MODE_CHECK, it);
      BF_LAUNCH(ctx, "batch_items", (kp_items<V, KC>), grid, blk, 0, B, (int)PH_RESID, (int)MODE_CHECK, it);
      BF_LAUNCH(ctx, "batch_decide", kp_decide<KC>, dgrid, blk, 0, B, (int)DEC_R, (int)MODE_CHECK);
    }
    BF_TRY(bf_launch_check(ctx, "phased batch iterations"));
    BF_HIP(ctx, hipMemcpyAsync(ctrl_host, B.ctrl, C_WORDS * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctrl_host[C_ACTIVE] == 0 || it >= max_iter) break;
    next = it + std::max(it, 4);
  }
  if (mixed) BF_LAUNCH(ctx, "batch_items", (kp_items<V, KC>), grid, blk, 0, B, (int)PH_FOLD, (int)MODE_REPORT, 0);
  BF_LAUNCH(ctx, "batch_items", (kp_items<V, KC>), grid, blk, 0, B, (int)PH_OUT, 0, 0);
  BF_LAUNCH(ctx, "batch_items", (kp_items<V, KC>), grid, blk, 0, B, (int)PH_RESID, (int)MODE_REPORT, 0);
  BF_LAUNCH(ctx, "batch_decide", kp_decide<KC>, dgrid, blk, 0, B, (int)DEC_R, (int)MODE_REPORT);
  BF_TRY(bf_launch_check(ctx, "phased batch tail"));
  return BF_OK;
}

// Host side of one batched solve.  mean: every system's rhs, one column.
template <typename V, int KC>
bf_status run_batch(bf_ctx* ctx, const bf_system* const* systems, int S, int K, uint64_t seed, double tol,
                    int max_iter, bool mean, double* const* out, const bf_schedule* sched, bf_solve_report* reps,
                    double* seconds) {
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
  // device memory: descriptors | states | order | tstart | ctrl | per-scene partials and vectors
  size_t bytes = al(S * sizeof(SceneDev)) + al(S * sizeof(BState)) + al(T * 8) + al(S * 8) + al(C_WORDS * 4);
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
  int* hc = nullptr;
  BF_TRY(bf_pinned(ctx, 64, (void**)&hc));
  const int hinit[C_WORDS] = {S * K, 0, 0, 0, 0};
  BF_HIP(ctx, hipMemcpyAsync(dsc, hsc.data(), S * sizeof(SceneDev), hipMemcpyHostToDevice, ctx->stream));
  BF_HIP(ctx, hipMemcpyAsync(dorder, order.data(), T * 8, hipMemcpyHostToDevice, ctx->stream));
  BF_HIP(ctx, hipMemcpyAsync(dtstart, tstart.data(), S * 8, hipMemcpyHostToDevice, ctx->stream));
  BF_HIP(ctx, hipMemcpyAsync(ctrl, hinit, sizeof(hinit), hipMemcpyHostToDevice, ctx->stream));
  hipLaunchKernelGGL(k_batch_state_init, dim3(std::min(S, 1024)), dim3(64), 0, ctx->stream, dst, S, K, tol, max_iter,
                     mixed ? 1e-6 : 0.0, mixed ? bf_mixed_restart() : 0);
  for (int s = 0; s < S; ++s) {
    const int64_t nn = hsc[s].n * KC;
    const int fb = (int)std::min<int64_t>(bf_cdiv(nn, 256), 4096);
    hipLaunchKernelGGL(k_fill_v<V>, dim3(fb), dim3(256), 0, ctx->stream, (V*)hsc[s].p0, nn, (V)0);
    if (mixed) hipLaunchKernelGGL(k_fill_v<float>, dim3(fb), dim3(256), 0, ctx->stream, hsc[s].cf, nn, 0.0f);
  }
  BF_TRY(bf_launch_check(ctx, "batch setup"));
  // the descriptors above come from pageable host memory: let their copies finish
  // before the timed region starts
  BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  Batch B{dsc, S, dorder, dtstart, Sched{rows, sched->xcd_aware ? 1 : 0, T}, ctrl};

  // solve-time events from the context's pool (no create / destroy per call)
  hipEvent_t e0 = bf_event_get(ctx), e1 = bf_event_get(ctx);
  if (!e0 || !e1) return bf_fail(ctx, BF_ERR_HIP, "event creation failed");
  BF_HIP(ctx, hipEventRecord(e0, ctx->stream));
  bf_status ls = sched->persistent ? launch_persistent<V, KC>(ctx, B, max_iter, sched, hc)
                                   : launch_phased<V, KC>(ctx, B, S, T, max_iter, sched, hc);
  if (ls != BF_OK) {
    (void)hipStreamSynchronize(ctx->stream);
    ctx->pool.push_back(e0);
    ctx->pool.push_back(e1);
    return ls;
  }
  BF_HIP(ctx, hipEventRecord(e1, ctx->stream));
  std::vector<BState> hst(S);
  BF_HIP(ctx, hipMemcpyAsync(hst.data(), dst, S * sizeof(BState), hipMemcpyDeviceToHost, ctx->stream));
  BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  ctx->pool.push_back(e0);
  ctx->pool.push_back(e1);
  if (seconds) *seconds = ms * 1e-3;
  if (sched->persistent && hc[C_ABORT])
    return bf_fail(ctx, BF_ERR_HIP, "persistent batch: a grid barrier timed out (workgroups not co-resident)");
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
  if (mean)
    return f64 ? run_batch<double, 1>(ctx, systems, S, 1, 0, tol, max_iter, true, out, sched, reps, seconds)
               : run_batch<float, 1>(ctx, systems, S, 1, 0, tol, max_iter, true, out, sched, reps, seconds);
  if (K <= 16)
    return f64 ? run_batch<double, 16>(ctx, systems, S, K, seed, tol, max_iter, false, out, sched, reps, seconds)
               : run_batch<float, 16>(ctx, systems, S, K, seed, tol, max_iter, false, out, sched, reps, seconds);
  if (K <= 32)
    return f64 ? run_batch<double, 32>(ctx, systems, S, K, seed, tol, max_iter, false, out, sched, reps, seconds)
               : run_batch<float, 32>(ctx, systems, S, K, seed, tol, max_iter, false, out, sched, reps, seconds);
  return f64 ? run_batch<double, 64>(ctx, systems, S, K, seed, tol, max_iter, false, out, sched, reps, seconds)
             : run_batch<float, 64>(ctx, systems, S, K, seed, tol, max_iter, false, out, sched, reps, seconds);
}

bf_status check_batch(bf_ctx* ctx, const bf_system* const* systems, int32_t n_sys, double* const* out,
                      const bf_schedule* sched) {
  BF_CHECK(ctx, systems && out && n_sys >= 1, "batched solve: bad system list");
  for (int s = 0; s < n_sys; ++s) {
    BF_CHECK(ctx, systems[s] && systems[s]->n > 0, "batched solve: system %d is NULL or empty", s);
    BF_CHECK(ctx, systems[s]->kind == BF_SYSTEM_VOXEL, "batched solve: system %d has trilinear rows", s);
    BF_CHECK(ctx, out[s], "batched solve: NULL output for system %d", s);
  }
  BF_CHECK(ctx, sched->rows_per_tile >= 16 && sched->rows_per_tile <= 4096, "batched solve: rows_per_tile %d",
           sched->rows_per_tile);
  BF_CHECK(ctx, sched->order >= 0 && sched->order <= 2, "batched solve: unknown order %d", sched->order);
  BF_CHECK(ctx, sched->blocks_per_cu >= 0 && sched->blocks_per_cu <= 16, "batched solve: blocks_per_cu %d",
           sched->blocks_per_cu);
  BF_CHECK(ctx, sched->persistent == 0 || sched->persistent == 1, "batched solve: persistent must be 0 or 1");
  return BF_OK;
}

const bf_schedule kProbeDefault{256, 0, BF_ORDER_SCENE_MAJOR, 1, 1};
const bf_schedule kMeanDefault{256, 4, BF_ORDER_SCENE_MAJOR, 1, 0};

}  // namespace

extern "C" bf_status bf_diag_estimate_batched(bf_ctx* ctx, const bf_system* const* systems, int32_t n_sys,
                                              const bf_probe_opts* opts, const bf_schedule* sched,
                                              double* const* s_dev, bf_solve_report* reps) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, opts, "bf_diag_estimate_batched: NULL options");
  BF_CHECK(ctx, opts->K >= 1 && opts->K <= 64, "bf_diag_estimate_batched: K=%d outside [1, 64]", opts->K);
  BF_CHECK(ctx, opts->tol >= 0.0 && opts->max_iter >= 0, "bf_diag_estimate_batched: tol and max_iter must be >= 0");
  const bf_schedule* sc = sched ? sched : &kProbeDefault;
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
  BF_CHECK(ctx, opts->tol >= 0.0 && opts->max_iter >= 0, "bf_pcg_solve_batched: tol and max_iter must be >= 0");
  const bf_schedule* sc = sched ? sched : &kMeanDefault;
  BF_CHECK(ctx, !sc->persistent, "bf_pcg_solve_batched: the mean solve runs phased (persistent = 0) only");
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
  BF_TRY(check_batch(ctx, systems, n_sys, s_dev, &kProbeDefault));
  BF_HIP(ctx, hipSetDevice(ctx->device));
  const int rows[] = {64, 128, 256, 512};
  const int bpc[] = {1, 2, 4};
  const int orders[] = {BF_ORDER_SCENE_MAJOR, BF_ORDER_INTERLEAVED, BF_ORDER_LARGEST_FIRST};
  std::string log = "[";
  double best_t = 1e30;
  bool first = true;
  for (int pers = 0; pers < 2; ++pers)
    for (int r : rows)
      for (int b : bpc)
        for (int o : orders)
          for (int x = 0; x < 2; ++x) {
            const bf_schedule cand{r, b, o, x, pers};
            double t = 0.0;
            // one untimed run to settle allocations, then the timed one
            bf_status st = dispatch(ctx, systems, n_sys, opts->K, opts->seed, opts->tol, opts->max_iter,
                                    opts->precision, false, s_dev, &cand, nullptr, nullptr);
            if (st == BF_OK)
              st = dispatch(ctx, systems, n_sys, opts->K, opts->seed, opts->tol, opts->max_iter, opts->precision,
                            false, s_dev, &cand, nullptr, &t);
            char buf[192];
            snprintf(buf, sizeof(buf),
                     "%s{\"persistent\":%d,\"rows\":%d,\"blocks_per_cu\":%d,\"order\":%d,\"xcd\":%d,\"ms\":%.4f,"
                     "\"ok\":%d}",
                     first ? "" : ",", pers, r, b, o, x, t * 1e3, st == BF_OK ? 1 : 0);
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
