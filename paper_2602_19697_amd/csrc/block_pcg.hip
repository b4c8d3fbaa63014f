// Hutchinson estimate of diag(Q^-1) (Sec. 3.7, eq. 12; Algorithm 1 step 6)
// with all K probe solves run as one block CG.
//
// Layout: block vectors are row-major [N][KC] (KC = K rounded up to 16, 32 or
// 64), so one band voxel's K values are contiguous: the stencil gathers of a
// neighbour row are coalesced and the neighbour table and diagonal are read
// once per row for all K columns.  A thread owns one column, a workgroup a
// tile of rows; every column keeps its own FP64 alpha, beta and stopping test
// (independent CGs sharing each matrix pass).  Probes z_k are never stored:
// the SplitMix64 counter hash regenerates them in registers wherever the
// right-hand side is needed.  Precision as in the single right-hand-side
// solver: FP64, or float vectors with FP64 scalars, FP64 folds/residuals and
// restarted float solves (mixed-precision iterative refinement).
#include "bf_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kRowsPerTile = 64;
constexpr int kMaxK = 64;

struct BState {
  double rho[kMaxK], alpha[kMaxK], beta[kMaxK], tol2b[kMaxK], rr_true[kMaxK], bnorm2[kMaxK], rr_ref[kMaxK];
  double inner2;
  int32_t active[kMaxK], check[kMaxK], last[kMaxK], iters[kMaxK], status[kMaxK];
  int32_t nactive, any_check, max_iter, replace_every, K, refinements;
  int32_t pad_[2];
};

enum { MODE_INIT = 0, MODE_CHECK = 1, MODE_REPORT = 2 };

// SplitMix64 output n (0-based) of the generator started at `start`.
__device__ __forceinline__ uint64_t splitmix_out(uint64_t start, uint64_t n) {
  uint64_t z = start + (n + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double probe(uint64_t col_seed, int64_t i) {
  return (splitmix_out(col_seed, (uint64_t)i) >> 63) ? -1.0 : 1.0;
}

__global__ void k_bstate_init(BState* st, int K, double tol, int32_t max_iter, int32_t replace_every,
                              double inner) {
  const int c = threadIdx.x;
  if (c < kMaxK) {
    st->rho[c] = st->alpha[c] = st->beta[c] = st->rr_true[c] = st->bnorm2[c] = st->rr_ref[c] = 0.0;
    st->tol2b[c] = tol * tol;
    st->active[c] = c < K ? 1 : 0;
    st->check[c] = st->last[c] = st->iters[c] = st->status[c] = 0;
  }
  if (c == 0) {
    st->inner2 = inner * inner;
    st->nactive = K;
    st->any_check = 0;
    st->max_iter = max_iter;
    st->replace_every = replace_every;
    st->K = K;
    st->refinements = 0;
  }
}

// Per-column block reduction of NQ quantities; afterwards threads c < KC hold
// the block's column sums in out[q] (fixed order).
template <int KC, int NQ>
__device__ __forceinline__ void col_block_sum(double (&v)[NQ], double* lds /*[4][NQ][64]*/) {
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int off = KC; off < 64; off <<= 1) v[q] += __shfl_xor(v[q], off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane < KC)
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds[(wid * NQ + q) * 64 + lane] = v[q];
  __syncthreads();
  if (threadIdx.x < KC)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double s = 0.0;
      for (int w = 0; w < kThreads / 64; ++w) s += lds[(w * NQ + q) * 64 + threadIdx.x];
      v[q] = s;
    }
}

// Column c's sums over all block partials part[nb][NQ][KC], computed by one
// workgroup per column in a fixed order; the result is returned to every
// thread of the workgroup.
template <int KC, int NQ>
__device__ __forceinline__ void col_partials_sum(const double* __restrict__ part, int nb, int c, double (&tot)[NQ],
                                                 double* lds) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += part[((size_t)b * NQ + q) * KC + c];
    tot[q] = bf_block_sum(acc, lds);
  }
}

template <int KC, int NQ>
__device__ __forceinline__ void store_partials(double* __restrict__ part, double (&v)[NQ]) {
  if (threadIdx.x < KC)
#pragma unroll
    for (int q = 0; q < NQ; ++q) part[((size_t)blockIdx.x * NQ + q) * KC + threadIdx.x] = v[q];
}

// A: p = zz + beta p_old (with neighbours on the fly), q = Q p, partial p.q.
template <typename V, int KC>
__global__ __launch_bounds__(256) void k_bA(BState* __restrict__ st, const int32_t* __restrict__ nbr,
                                            const V* __restrict__ diag, V lam, const V* __restrict__ zz,
                                            const V* __restrict__ p_old, V* __restrict__ p_new, V* __restrict__ q,
                                            int64_t n, double* __restrict__ part) {
  __shared__ double lds[4 * 3 * 64];
  if (st->nactive == 0) return;
  const int c = threadIdx.x % KC, rsub = threadIdx.x / KC;
  constexpr int RS = kThreads / KC;
  const bool act = st->active[c] != 0;
  const V beta = (V)st->beta[c];
  double v1[1] = {0.0};
  if (act) {
    for (int64_t tile = blockIdx.x; tile * kRowsPerTile < n; tile += gridDim.x) {
      for (int s = rsub; s < kRowsPerTile; s += RS) {
        const int64_t v = tile * kRowsPerTile + s;
        if (v >= n) break;
        const int32_t* nb = nbr + v * 6;
        V acc = 0;
#pragma unroll
        for (int t = 0; t < 6; ++t) {
          const int32_t u = nb[t];
          if (u >= 0) acc += zz[(int64_t)u * KC + c] + beta * p_old[(int64_t)u * KC + c];
        }
        const int64_t e = v * KC + c;
        const V pv = zz[e] + beta * p_old[e];
        const V qv = diag[v] * pv - lam * acc;
        p_new[e] = pv;
        q[e] = qv;
        v1[0] += (double)pv * (double)qv;
      }
    }
  }
  col_block_sum<KC, 1>(v1, lds);
  store_partials<KC, 1>(part, v1);
}

// Per-column alpha from A's block partials (one workgroup per column).
template <int KC>
__global__ __launch_bounds__(256) void k_bscal_A(BState* __restrict__ st, const double* __restrict__ part, int nb) {
  __shared__ double lds[16];
  const int c = blockIdx.x;
  if (c == 0 && threadIdx.x == 0) st->any_check = 0;  // consumed by the previous check, if any
  if (!st->active[c]) return;
  double tot[1];
  col_partials_sum<KC, 1>(part, nb, c, tot, lds);
  if (threadIdx.x == 0) {
    if (!(tot[0] > 0.0) || !isfinite(tot[0])) {
      st->status[c] = BF_ERR_BREAKDOWN;
      st->active[c] = 0;
      atomicSub(&st->nactive, 1);
    } else {
      st->alpha[c] = st->rho[c] / tot[0];
    }
  }
}

// B: x += alpha p, r -= alpha q, zz = r / diag, partials r.zz and r.r.
template <typename V, int KC>
__global__ __launch_bounds__(256) void k_bB(BState* __restrict__ st, const V* __restrict__ dinv,
                                            const V* __restrict__ p, const V* __restrict__ q, V* __restrict__ x,
                                            V* __restrict__ r, V* __restrict__ zz, int64_t n,
                                            double* __restrict__ part) {
  __shared__ double lds[4 * 3 * 64];
  if (st->nactive == 0) return;
  const int c = threadIdx.x % KC, rsub = threadIdx.x / KC;
  constexpr int RS = kThreads / KC;
  const bool act = st->active[c] != 0;
  const V alpha = (V)st->alpha[c];
  double v2[2] = {0.0, 0.0};
  if (act) {
    for (int64_t tile = blockIdx.x; tile * kRowsPerTile < n; tile += gridDim.x) {
      for (int s = rsub; s < kRowsPerTile; s += RS) {
        const int64_t v = tile * kRowsPerTile + s;
        if (v >= n) break;
        const int64_t e = v * KC + c;
        x[e] = x[e] + alpha * p[e];
        const V rv = r[e] - alpha * q[e];
        const V zv = rv * dinv[v];
        r[e] = rv;
        zz[e] = zv;
        v2[0] += (double)rv * (double)zv;
        v2[1] += (double)rv * (double)rv;
      }
    }
  }
  col_block_sum<KC, 2>(v2, lds);
  store_partials<KC, 2>(part, v2);
}

// Per-column beta or residual-check request from B's block partials.
template <int KC>
__global__ __launch_bounds__(256) void k_bscal_B(BState* __restrict__ st, const double* __restrict__ part, int nb) {
  __shared__ double lds[16];
  const int c = blockIdx.x;
  if (!st->active[c]) return;
  double tot[2];
  col_partials_sum<KC, 2>(part, nb, c, tot, lds);
  if (threadIdx.x == 0) {
    const int it = st->iters[c] + 1;
    st->iters[c] = it;
    const bool at_max = it >= st->max_iter;
    const bool periodic = st->replace_every > 0 && (it % st->replace_every) == 0;
    if (!isfinite(tot[0]) || !isfinite(tot[1])) {
      st->status[c] = BF_ERR_BREAKDOWN;
      st->active[c] = 0;
      atomicSub(&st->nactive, 1);
    } else if (tot[1] <= fmax(st->tol2b[c], st->inner2 * st->rr_ref[c]) || at_max || periodic) {
      st->check[c] = 1;
      st->last[c] = at_max ? 1 : 0;
      atomicOr(&st->any_check, 1);
    } else {
      st->beta[c] = tot[0] / st->rho[c];
      st->rho[c] = tot[0];
    }
  }
}

// Mixed precision: fold the float corrections of checked columns into x64.
template <int KC>
__global__ __launch_bounds__(256) void k_bfold(const BState* __restrict__ st, int force, double* __restrict__ x64,
                                               float* __restrict__ cc, int64_t n) {
  if (!force && (st->nactive == 0 || !st->any_check)) return;
  const int c = threadIdx.x % KC, rsub = threadIdx.x / KC;
  constexpr int RS = kThreads / KC;
  if (!force && !(st->active[c] && st->check[c])) return;
  for (int64_t tile = blockIdx.x; tile * kRowsPerTile < n; tile += gridDim.x)
    for (int s = rsub; s < kRowsPerTile; s += RS) {
      const int64_t v = tile * kRowsPerTile + s;
      if (v >= n) break;
      const int64_t e = v * KC + c;
      x64[e] = x64[e] + (double)cc[e];
      cc[e] = 0.0f;
    }
}

// True residual r = z - Q x in FP64 for the checked columns (INIT: every
// active column, optionally from the warm start u0 = exp(logvar) z / diag,
// which is written to x64).
template <typename V, int KC>
__global__ __launch_bounds__(256) void k_bresid(BState* __restrict__ st, int mode, const int32_t* __restrict__ nbr,
                                                const double* __restrict__ diag, double lam,
                                                const float* __restrict__ logvar, uint64_t seed,
                                                double* __restrict__ x64, const V* __restrict__ dinv,
                                                V* __restrict__ r, V* __restrict__ zz, int64_t n,
                                                double* __restrict__ part) {
  __shared__ double lds[4 * 3 * 64];
  if (mode == MODE_CHECK && (st->nactive == 0 || !st->any_check)) return;
  const int c = threadIdx.x % KC, rsub = threadIdx.x / KC;
  constexpr int RS = kThreads / KC;
  const bool act = mode == MODE_REPORT ? c < st->K :
                   (st->active[c] != 0 && (mode == MODE_INIT || st->check[c] != 0));
  const uint64_t cs = splitmix_out(seed, (uint64_t)c);
  double v3[3] = {0.0, 0.0, 0.0};
  if (act) {
    for (int64_t tile = blockIdx.x; tile * kRowsPerTile < n; tile += gridDim.x) {
      for (int s = rsub; s < kRowsPerTile; s += RS) {
        const int64_t v = tile * kRowsPerTile + s;
        if (v >= n) break;
        const int64_t e = v * KC + c;
        const double zv = probe(cs, v);
        double res = zv;
        if (mode == MODE_INIT) {
          if (logvar) {
            const int32_t* nb = nbr + v * 6;
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < 6; ++t) {
              const int32_t u = nb[t];
              if (u >= 0) acc += exp((double)logvar[u]) * probe(cs, u) / diag[u];
            }
            const double x0 = exp((double)logvar[v]) * zv / diag[v];
            x64[e] = x0;
            res = zv - (diag[v] * x0 - lam * acc);
          } else {
            x64[e] = 0.0;
          }
        } else {
          const int32_t* nb = nbr + v * 6;
          double acc = 0.0;
#pragma unroll
          for (int t = 0; t < 6; ++t) {
            const int32_t u = nb[t];
            if (u >= 0) acc += x64[(int64_t)u * KC + c];
          }
          res = zv - (diag[v] * x64[e] - lam * acc);
        }
        v3[0] += res * res;
        v3[2] += zv * zv;
        if (mode != MODE_REPORT) {
          const V rv = (V)res;
          const V zzv = rv * dinv[v];
          r[e] = rv;
          zz[e] = zzv;
          v3[1] += (double)rv * (double)zzv;
        }
      }
    }
  }
  col_block_sum<KC, 3>(v3, lds);
  store_partials<KC, 3>(part, v3);
}

// Per-column decisions after an FP64 residual (one workgroup per column).
template <int KC>
__global__ __launch_bounds__(256) void k_bscal_R(BState* __restrict__ st, int mode, const double* __restrict__ part,
                                                 int nb) {
  __shared__ double lds[16];
  const int cc = blockIdx.x;
  if (mode == MODE_CHECK && !(st->active[cc] && st->check[cc])) return;
  if (mode == MODE_REPORT && cc >= st->K) return;
  if (mode == MODE_INIT && !st->active[cc]) return;
  double tot[3];
  col_partials_sum<KC, 3>(part, nb, cc, tot, lds);
  if (threadIdx.x != 0) return;
  if (mode == MODE_REPORT) {
    st->rr_true[cc] = tot[0];
  } else if (mode == MODE_INIT) {
    st->bnorm2[cc] = tot[2];
    st->tol2b[cc] *= tot[2];
    st->rr_true[cc] = tot[0];
    if (tot[2] == 0.0 || tot[0] <= st->tol2b[cc] || st->max_iter <= 0) {
      if (!(tot[2] == 0.0 || tot[0] <= st->tol2b[cc])) st->status[cc] = BF_ERR_NOT_CONVERGED;
      st->active[cc] = 0;
      atomicSub(&st->nactive, 1);
    } else {
      st->rho[cc] = tot[1];
      st->beta[cc] = 0.0;
      st->rr_ref[cc] = tot[0];
    }
  } else {
    st->rr_true[cc] = tot[0];
    atomicAdd(&st->refinements, 1);
    if (!isfinite(tot[0]) || !isfinite(tot[1])) {
      st->status[cc] = BF_ERR_BREAKDOWN;
      st->active[cc] = 0;
      atomicSub(&st->nactive, 1);
    } else if (tot[0] <= st->tol2b[cc]) {
      st->active[cc] = 0;
      atomicSub(&st->nactive, 1);
    } else if (st->last[cc]) {
      st->status[cc] = BF_ERR_NOT_CONVERGED;
      st->active[cc] = 0;
      atomicSub(&st->nactive, 1);
    } else {
      // FP64 continues CG from the replaced residual; mixed restarts the
      // float solve on the FP64 residual (iterative refinement).
      st->beta[cc] = st->inner2 > 0.0 ? 0.0 : tot[1] / st->rho[cc];
      st->rho[cc] = tot[1];
      st->rr_ref[cc] = tot[0];
    }
    st->check[cc] = 0;
  }
}

// s_v = (1/K) sum_k z_k[v] u_k[v], columns in ascending order.
template <int KC>
__global__ __launch_bounds__(256) void k_hutch_final(const double* __restrict__ x64, uint64_t seed, int K,
                                                     int64_t n, double* __restrict__ s_out) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  double s = 0.0;
  for (int k = 0; k < K; ++k) s += probe(splitmix_out(seed, (uint64_t)k), v) * x64[v * KC + k];
  s_out[v] = s / (double)K;
}

template <typename V>
__global__ __launch_bounds__(256) void k_bfill(V* __restrict__ p, int64_t n, V val) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}

template <typename V, int KC>
bf_status run_block(bf_ctx* ctx, const bf_system* sys, const bf_probe_opts* o, const float* logvar,
                    double* s_out, bf_solve_report* rep) {
  const int64_t N = sys->n;
  const bool mixed = sizeof(V) == 4;
  const int64_t ntiles = bf_cdiv(N, kRowsPerTile);
  const int nb = (int)std::min<int64_t>(ntiles, 4 * (int64_t)ctx->cu_count);
  const size_t st_bytes = (sizeof(BState) + 255) / 256 * 256;
  const size_t part_bytes = ((size_t)nb * 3 * KC * 8 + 255) / 256 * 256;
  const size_t vec = ((size_t)N * KC * sizeof(V) + 255) / 256 * 256;
  const size_t vec64 = ((size_t)N * KC * 8 + 255) / 256 * 256;
  // state | partials | x64 | r zz p0 p1 q (V) | c (float, mixed)
  char* ws = nullptr;
  BF_TRY(bf_ws(ctx, bf_ctx::WS_PROBE, st_bytes + part_bytes + vec64 + 5 * vec + (mixed ? vec : 0), (void**)&ws));
  BState* st = (BState*)ws;
  double* part = (double*)(ws + st_bytes);
  double* x64 = (double*)(ws + st_bytes + part_bytes);
  V* r = (V*)((char*)x64 + vec64);
  V* zz = (V*)((char*)r + vec);
  V* p0 = (V*)((char*)zz + vec);
  V* p1 = (V*)((char*)p0 + vec);
  V* q = (V*)((char*)p1 + vec);
  float* cc = mixed ? (float*)((char*)q + vec) : nullptr;
  V* xin = mixed ? (V*)cc : (V*)x64;
  const V* diagV = mixed ? (const V*)sys->diag32 : (const V*)sys->diag;
  const V* dinvV = mixed ? (const V*)sys->dinv32 : (const V*)sys->dinv;
  const V lamV = (V)sys->lambda;
  const int fb = (int)std::min<int64_t>(bf_cdiv(N * KC, 256), 8192);

  hipEvent_t e0, e1;
  BF_HIP(ctx, hipEventCreate(&e0));
  BF_HIP(ctx, hipEventCreate(&e1));
  BF_HIP(ctx, hipEventRecord(e0, ctx->stream));
  hipLaunchKernelGGL(k_bstate_init, dim3(1), dim3(64), 0, ctx->stream, st, o->K, o->tol, o->max_iter, 0,
                     mixed ? 1e-6 : 0.0);
  hipLaunchKernelGGL(k_bfill<V>, dim3(fb), dim3(256), 0, ctx->stream, p0, N * KC, (V)0);
  if (mixed) hipLaunchKernelGGL(k_bfill<float>, dim3(fb), dim3(256), 0, ctx->stream, cc, N * KC, 0.0f);
  BF_LAUNCH(ctx, "block_residual", (k_bresid<V, KC>), dim3(nb), dim3(kThreads), 0, st, (int)MODE_INIT, sys->band->nbr,
                     sys->diag, sys->lambda, logvar, o->seed, x64, dinvV, r, zz, N, part);
  BF_LAUNCH(ctx, "block_scalars", k_bscal_R<KC>, dim3(KC), dim3(256), 0, st, (int)MODE_INIT, part, nb);
  BF_TRY(bf_launch_check(ctx, "block pcg init"));
  BState* hs = nullptr;
  BF_TRY(bf_pinned(ctx, sizeof(BState), (void**)&hs));
  int it = 0, next = 3;
  V* pa = p0;
  V* pb = p1;
  for (;;) {
    const int upto = std::min(next, o->max_iter);
    for (; it < upto; ++it) {
      BF_LAUNCH(ctx, "block_A", (k_bA<V, KC>), dim3(nb), dim3(kThreads), 0, st, sys->band->nbr, diagV, lamV,
                         zz, pa, pb, q, N, part);
      BF_LAUNCH(ctx, "block_scalars", k_bscal_A<KC>, dim3(KC), dim3(256), 0, st, part, nb);
      BF_LAUNCH(ctx, "block_B", (k_bB<V, KC>), dim3(nb), dim3(kThreads), 0, st, dinvV, pb, q, xin, r, zz, N,
                         part);
      BF_LAUNCH(ctx, "block_scalars", k_bscal_B<KC>, dim3(KC), dim3(256), 0, st, part, nb);
      if (mixed) BF_LAUNCH(ctx, "block_fold", k_bfold<KC>, dim3(nb), dim3(kThreads), 0, st, 0, x64, cc, N);
      BF_LAUNCH(ctx, "block_residual", (k_bresid<V, KC>), dim3(nb), dim3(kThreads), 0, st, (int)MODE_CHECK,
                         sys->band->nbr, sys->diag, sys->lambda, nullptr, o->seed, x64, dinvV, r, zz, N, part);
      BF_LAUNCH(ctx, "block_scalars", k_bscal_R<KC>, dim3(KC), dim3(256), 0, st, (int)MODE_CHECK, part, nb);
      std::swap(pa, pb);
    }
    BF_TRY(bf_launch_check(ctx, "block pcg iteration"));
    BF_HIP(ctx, hipMemcpyAsync(hs, st, sizeof(BState), hipMemcpyDeviceToHost, ctx->stream));
    BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (hs->nactive == 0 || it >= o->max_iter) break;
    next = it + std::max(it, 4);
  }
  if (mixed) BF_LAUNCH(ctx, "block_fold", k_bfold<KC>, dim3(nb), dim3(kThreads), 0, st, 1, x64, cc, N);
  BF_LAUNCH(ctx, "hutch_final", k_hutch_final<KC>, dim3((unsigned)bf_cdiv(N, 256)), dim3(256), 0, x64, o->seed,
                     o->K, N, s_out);
  BF_HIP(ctx, hipEventRecord(e1, ctx->stream));
  // final FP64 residual of every probe column for the report
  BF_LAUNCH(ctx, "block_residual", (k_bresid<V, KC>), dim3(nb), dim3(kThreads), 0, st, (int)MODE_REPORT,
                     sys->band->nbr, sys->diag, sys->lambda, nullptr, o->seed, x64, dinvV, r, zz, N, part);
  BF_LAUNCH(ctx, "block_scalars", k_bscal_R<KC>, dim3(KC), dim3(256), 0, st, (int)MODE_REPORT, part, nb);
  BF_HIP(ctx, hipMemcpyAsync(hs, st, sizeof(BState), hipMemcpyDeviceToHost, ctx->stream));
  BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  bf_status status = BF_OK;
  int maxit = 0;
  int64_t sumit = 0;
  double maxres = 0.0;
  for (int k = 0; k < o->K; ++k) {
    sumit += hs->iters[k];
    if (hs->status[k] == BF_ERR_BREAKDOWN) status = BF_ERR_BREAKDOWN;
    else if (hs->status[k] == BF_ERR_NOT_CONVERGED && status == BF_OK) status = BF_ERR_NOT_CONVERGED;
    maxit = std::max(maxit, (int)hs->iters[k]);
    if (hs->bnorm2[k] > 0.0) maxres = std::max(maxres, sqrt(hs->rr_true[k] / hs->bnorm2[k]));
  }
  if (status == BF_OK && hs->nactive != 0) status = BF_ERR_NOT_CONVERGED;
  if (rep) {
    rep->iters = maxit;
    rep->status = status;
    rep->refinements = hs->refinements;
    rep->used_warm_start = logvar ? 1 : 0;
    rep->rel_res = maxres;
    rep->seconds = ms * 1e-3;
    rep->col_iters = sumit;
  }
  if (status != BF_OK) return bf_fail(ctx, status, "bf_diag_estimate: probe solves ended with status %d", status);
  return BF_OK;
}

template <typename V>
bf_status dispatch_k(bf_ctx* ctx, const bf_system* sys, const bf_probe_opts* o, const float* logvar, double* s,
                     bf_solve_report* rep) {
  if (o->K <= 16) return run_block<V, 16>(ctx, sys, o, logvar, s, rep);
  if (o->K <= 32) return run_block<V, 32>(ctx, sys, o, logvar, s, rep);
  return run_block<V, 64>(ctx, sys, o, logvar, s, rep);
}

}  // namespace

extern "C" bf_status bf_diag_estimate(bf_ctx* ctx, const bf_system* sys, const bf_probe_opts* opts,
                                      const float* logvar_dev, double* s_dev, bf_solve_report* rep) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, sys && opts, "bf_diag_estimate: NULL argument");
  BF_CHECK(ctx, opts->K >= 1 && opts->K <= kMaxK, "bf_diag_estimate: K=%d outside [1, 64]", opts->K);
  BF_CHECK(ctx, opts->tol >= 0.0 && opts->max_iter >= 0, "bf_diag_estimate: tol and max_iter must be >= 0");
  BF_CHECK(ctx, opts->precision == BF_PREC_FP64 || opts->precision == BF_PREC_MIXED,
           "bf_diag_estimate: unknown precision %d", opts->precision);
  if (rep) *rep = bf_solve_report{};
  if (sys->n == 0) return BF_OK;
  BF_CHECK(ctx, s_dev, "bf_diag_estimate: NULL output");
  BF_HIP(ctx, hipSetDevice(ctx->device));
  if (opts->precision == BF_PREC_FP64) return dispatch_k<double>(ctx, sys, opts, logvar_dev, s_dev, rep);
  return dispatch_k<float>(ctx, sys, opts, logvar_dev, s_dev, rep);
}
