// Jacobi-preconditioned conjugate gradients for the posterior mean
// (Sec. 3.6, eq. 11; Algorithm 1 step 5).
//
// Q = diag(Q) - lambda * adjacency(band) is never assembled: the product is a
// 7-point stencil through the neighbour table.  Each iteration is two
// streaming kernels whose last-arriving block turns the block partials into
// the CG scalars on the device, so the host never waits inside an iteration:
//   A: p = z + beta p_old (own row and, on the fly, each neighbour), q = Q p,
//      partial p.q  ->  alpha = rho / p.q (breakdown check)
//   B: x += alpha p, r -= alpha q, z = r / diag, partials r.z and r.r
//      -> beta, or a request for an FP64 true-residual check
// Precision V = double runs everything in FP64.  V = float (mixed) keeps the
// vectors and the stencil in float while the dot products, alpha/beta and the
// residual test stay FP64; its correction c is folded into the FP64 solution
// and the residual recomputed in FP64 whenever the float residual has fallen
// 1e6-fold (or below the tolerance); the float solve then restarts on the FP64
// residual (mixed-precision iterative refinement).
// Reductions are deterministic: fixed-order wave butterflies, a fixed block
// tree and a fixed-order sum of the block partials.  The scalar step runs in
// its own one-workgroup kernel: a "last block done" epilogue would need a
// device-scope release fence in every workgroup, which on this chip writes
// back the XCD's L2 each time.
#include "bf_internal.h"

#include <chrono>
#include <mutex>

namespace {

constexpr int kThreads = 256;

struct PcgState {
  double rho, alpha, beta, tol2b, bnorm2, rr, rr_true, rho_new, inner2, rr_ref;
  int32_t iters, done, check, status, last, refinements, max_iter, replace_every;
  int32_t guard;    // a start was supplied: drop it if ||rhs - Q x0|| >= ||rhs||
  int32_t dropped;  // ... and it was: the solve restarts from x = 0
  int32_t closed;   // done was decided by a true-residual pass, so x is folded and rr_true is its residual
};

// GUARD: after INIT with a supplied start that was dropped, INIT again from x = 0.
enum { MODE_INIT = 0, MODE_CHECK = 1, MODE_REPORT = 2, MODE_GUARD = 3 };

__global__ void k_state_init(PcgState* st, double tol, int32_t max_iter, int32_t replace_every, double inner,
                             int32_t guard) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    PcgState s{};
    s.tol2b = tol * tol;  // scaled by ||rhs||^2 once known
    s.max_iter = max_iter;
    s.replace_every = replace_every;
    s.inner2 = inner * inner;
    s.guard = guard;
    *st = s;
  }
}

// x = 0 where the supplied start was dropped.
__global__ __launch_bounds__(256) void k_zero_if_dropped(const PcgState* __restrict__ st, double* __restrict__ x,
                                                         int64_t n) {
  if (!st->dropped) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

template <typename V>
__global__ __launch_bounds__(256) void k_fill(V* __restrict__ p, int64_t n, V v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Sum the per-block partials [nb][W] in a fixed order, in the one workgroup
// of a scalar kernel (1024 threads: the partials of one workgroup per 256
// rows, 8.9k at 512^3, are read 9 per thread instead of 35).
template <int W>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int nb, double* out,
                                                double* lds) {
  double acc[W];
#pragma unroll
  for (int w = 0; w < W; ++w) acc[w] = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] += part[b * W + w];
#pragma unroll
  for (int w = 0; w < W; ++w) out[w] = bf_block_sum(acc[w], lds);
}

// The 6 neighbour indices of row v (24 B, 8-byte aligned: the band's arrays
// start on 256-byte boundaries) as three 8-byte loads.
__device__ __forceinline__ void nbr6(const int32_t* __restrict__ nbr, int64_t v, int32_t (&nb)[6]) {
  const int2* q = reinterpret_cast<const int2*>(nbr + v * 6);
  const int2 a = q[0], b = q[1], c = q[2];
  nb[0] = a.x;
  nb[1] = a.y;
  nb[2] = b.x;
  nb[3] = b.y;
  nb[4] = c.x;
  nb[5] = c.y;
}

// A: direction update fused with the stencil product and p.q.
template <typename V>
__global__ __launch_bounds__(256) void k_pcg_A(PcgState* __restrict__ st, const int32_t* __restrict__ nbr,
                                               const V* __restrict__ diag, V lam, const V* __restrict__ z,
                                               const V* __restrict__ p_old, V* __restrict__ p_new,
                                               V* __restrict__ q, int64_t n, double* __restrict__ part) {
  __shared__ double lds[16];
  if (st->done) return;
  const V beta = (V)st->beta;
  const int64_t v = bf_xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  double pq = 0.0;
  if (v < n) {
    int32_t nb[6];
    nbr6(nbr, v, nb);
    V s = 0;
#pragma unroll
    for (int t = 0; t < 6; ++t) {  // unconditional loads: an absent neighbour reads the row itself
      const int64_t u = nb[t] >= 0 ? (int64_t)nb[t] : v;
      const V a = z[u] + beta * p_old[u];
      s = fma(a, nb[t] >= 0 ? (V)1 : (V)0, s);  // an absent neighbour adds +-0 (a is finite)
    }
    const V pv = z[v] + beta * p_old[v];
    const V qv = diag[v] * pv - lam * s;
    p_new[v] = pv;
    q[v] = qv;
    pq = (double)pv * (double)qv;
  }
  pq = bf_block_sum(pq, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = pq;
}

// A for a trilinear system: q = diag p + sum over the 26 stored couplings
// (ascending slot; slot-major [26][N]) of off * p_u, with p = z + beta p_old
// formed on the fly.
template <typename V>
__global__ __launch_bounds__(256) void k_pcg_A27(PcgState* __restrict__ st, const int32_t* __restrict__ nb26,
                                                 const V* __restrict__ off, const V* __restrict__ diag,
                                                 const V* __restrict__ z, const V* __restrict__ p_old,
                                                 V* __restrict__ p_new, V* __restrict__ q, int64_t n,
                                                 double* __restrict__ part) {
  __shared__ double lds[16];
  if (st->done) return;
  const V beta = (V)st->beta;
  const int64_t v = bf_xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  double pq = 0.0;
  if (v < n) {
    V s = 0;
#pragma unroll
    for (int t = 0; t < 26; ++t) {  // unconditional loads: an absent voxel reads the row itself
      const int32_t nbt = nb26[t * n + v];
      const int64_t u = nbt >= 0 ? (int64_t)nbt : v;
      const V a = z[u] + beta * p_old[u];
      if (nbt >= 0) s += off[t * n + v] * a;
    }
    const V pv = z[v] + beta * p_old[v];
    const V qv = diag[v] * pv + s;
    p_new[v] = pv;
    q[v] = qv;
    pq = (double)pv * (double)qv;
  }
  pq = bf_block_sum(pq, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = pq;
}

// alpha = rho / p.q from A's block partials (one workgroup, fixed order).
__global__ __launch_bounds__(1024) void k_pcg_alpha(PcgState* __restrict__ st, const double* __restrict__ part,
                                                   int nb) {
  __shared__ double lds[16];
  if (st->done) return;
  double tot;
  reduce_partials<1>(part, nb, &tot, lds);
  if (threadIdx.x == 0) {
    if (!(tot > 0.0) || !isfinite(tot)) {
      st->status = BF_ERR_BREAKDOWN;
      st->done = 1;
    } else {
      st->alpha = st->rho / tot;
    }
  }
}

// B: solution/residual update, preconditioned residual and the two dots.
template <typename V>
__global__ __launch_bounds__(256) void k_pcg_B(PcgState* __restrict__ st, const V* __restrict__ dinv,
                                               const V* __restrict__ p, const V* __restrict__ q,
                                               V* __restrict__ x, V* __restrict__ r, V* __restrict__ z,
                                               int64_t n, double* __restrict__ part) {
  __shared__ double lds[16];
  if (st->done) return;
  const V alpha = (V)st->alpha;
  const int64_t v = bf_xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (v < n) {
    x[v] = x[v] + alpha * p[v];
    const V rv = r[v] - alpha * q[v];
    const V zv = rv * dinv[v];
    r[v] = rv;
    z[v] = zv;
    rz = (double)rv * (double)zv;
    rr = (double)rv * (double)rv;
  }
  rz = bf_block_sum(rz, lds);
  rr = bf_block_sum(rr, lds);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = rz;
    part[2 * blockIdx.x + 1] = rr;
  }
}

// beta, or a request for an FP64 residual check, from B's block partials.
__global__ __launch_bounds__(1024) void k_pcg_beta(PcgState* __restrict__ st, const double* __restrict__ part,
                                                  int nb) {
  __shared__ double lds[16];
  if (st->done) return;
  double tot[2];
  reduce_partials<2>(part, nb, tot, lds);
  if (threadIdx.x == 0) {
    st->iters += 1;
    st->rr = tot[1];
    const bool at_max = st->iters >= st->max_iter;
    const bool periodic = st->replace_every > 0 && (st->iters % st->replace_every) == 0;
    if (!isfinite(tot[0]) || !isfinite(tot[1])) {
      st->status = BF_ERR_BREAKDOWN;
      st->done = 1;
    } else if (tot[1] <= fmax(st->tol2b, st->inner2 * st->rr_ref) || at_max || periodic) {
      st->check = 1;
      st->last = at_max ? 1 : 0;
      st->rho_new = tot[0];
    } else {
      st->beta = tot[0] / st->rho;
      st->rho = tot[0];
    }
  }
}

// Mixed precision: fold the float correction into the FP64 solution.
__global__ __launch_bounds__(256) void k_fold(const PcgState* __restrict__ st, int force, double* __restrict__ x64,
                                              float* __restrict__ c, int64_t n) {
  if (!force && (st->done || !st->check)) return;
  const int64_t v = bf_xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  if (v < n) {
    x64[v] = x64[v] + (double)c[v];
    c[v] = 0.0f;
  }
}

// True residual r = rhs - Q x in FP64 (INIT: start of the solve; CHECK:
// confirm convergence / replace the recursive residual; REPORT: norm only).
template <typename V>
__global__ __launch_bounds__(256) void k_residual(PcgState* __restrict__ st, int mode,
                                                  const int32_t* __restrict__ nbr,
                                                  const double* __restrict__ diag, double lam,
                                                  const double* __restrict__ rhs,
                                                  const double* __restrict__ x, const V* __restrict__ dinv,
                                                  V* __restrict__ r, V* __restrict__ z, int64_t n,
                                                  double* __restrict__ part) {
  __shared__ double lds[16];
  if (mode == MODE_CHECK && (st->done || !st->check)) return;
  if (mode == MODE_GUARD && !st->dropped) return;
  const int64_t v = bf_xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  double rr = 0.0, rz = 0.0, bb = 0.0;
  if (v < n) {
    const double hv = rhs[v];
    double res = hv;
    if (x) {
      int32_t nb[6];
      nbr6(nbr, v, nb);
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int64_t u = nb[t] >= 0 ? (int64_t)nb[t] : v;
        const double xu = x[u];
        s = fma(xu, nb[t] >= 0 ? 1.0 : 0.0, s);  // an absent neighbour adds +-0
      }
      res = hv - (diag[v] * x[v] - lam * s);
    }
    rr = res * res;
    bb = hv * hv;
    if (mode != MODE_REPORT) {
      const V rv = (V)res;
      const V zv = rv * dinv[v];
      r[v] = rv;
      z[v] = zv;
      rz = (double)rv * (double)zv;
    }
  }
  rr = bf_block_sum(rr, lds);
  rz = bf_block_sum(rz, lds);
  bb = bf_block_sum(bb, lds);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = rr;
    part[3 * blockIdx.x + 1] = rz;
    part[3 * blockIdx.x + 2] = bb;
  }
}

// True FP64 residual of a trilinear system (modes as in k_residual).
template <typename V>
__global__ __launch_bounds__(256) void k_residual27(PcgState* __restrict__ st, int mode,
                                                    const int32_t* __restrict__ nb26, const double* __restrict__ off,
                                                    const double* __restrict__ diag, const double* __restrict__ rhs,
                                                    const double* __restrict__ x, const V* __restrict__ dinv,
                                                    V* __restrict__ r, V* __restrict__ z, int64_t n,
                                                    double* __restrict__ part) {
  __shared__ double lds[16];
  if (mode == MODE_CHECK && (st->done || !st->check)) return;
  if (mode == MODE_GUARD && !st->dropped) return;
  const int64_t v = bf_xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  double rr = 0.0, rz = 0.0, bb = 0.0;
  if (v < n) {
    const double hv = rhs[v];
    double res = hv;
    if (x) {
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < 26; ++t) {
        const int32_t nbt = nb26[t * n + v];
        const int64_t u = nbt >= 0 ? (int64_t)nbt : v;
        const double xu = x[u];
        if (nbt >= 0) s += off[t * n + v] * xu;
      }
      res = hv - (diag[v] * x[v] + s);
    }
    rr = res * res;
    bb = hv * hv;
    if (mode != MODE_REPORT) {
      const V rv = (V)res;
      const V zv = rv * dinv[v];
      r[v] = rv;
      z[v] = zv;
      rz = (double)rv * (double)zv;
    }
  }
  rr = bf_block_sum(rr, lds);
  rz = bf_block_sum(rz, lds);
  bb = bf_block_sum(bb, lds);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = rr;
    part[3 * blockIdx.x + 1] = rz;
    part[3 * blockIdx.x + 2] = bb;
  }
}

// Decisions after an FP64 residual: stop, or continue / restart from it.
__global__ __launch_bounds__(1024) void k_residual_scalars(PcgState* __restrict__ st, int mode,
                                                          const double* __restrict__ part, int nb) {
  __shared__ double lds[16];
  if (mode == MODE_CHECK && (st->done || !st->check)) return;
  if (mode == MODE_GUARD && !st->dropped) return;
  double tot[3];
  reduce_partials<3>(part, nb, tot, lds);
  if (threadIdx.x != 0) return;
  if (mode == MODE_INIT && st->guard && tot[2] > 0.0 && !(tot[0] < tot[2])) {
    // the supplied start is no better than zero: drop it (GUARD restarts from x = 0)
    st->dropped = 1;
    st->bnorm2 = tot[2];
    st->tol2b = st->tol2b * tot[2];
    return;
  }
  st->rr_true = tot[0];
  if (mode == MODE_REPORT) return;
  if (mode == MODE_INIT || mode == MODE_GUARD) {
    if (mode == MODE_INIT) {
      st->bnorm2 = tot[2];
      st->tol2b = st->tol2b * tot[2];
    }
    if (tot[2] == 0.0 || tot[0] <= st->tol2b) {
      st->done = 1;
      st->closed = 1;
      return;
    }
    st->rho = tot[1];
    st->beta = 0.0;
    st->rr_ref = tot[0];
    if (st->max_iter <= 0) {
      st->status = BF_ERR_NOT_CONVERGED;
      st->done = 1;
      st->closed = 1;
    }
    return;
  }
  st->refinements += 1;
  if (!isfinite(tot[0]) || !isfinite(tot[1])) {
    st->status = BF_ERR_BREAKDOWN;
    st->done = 1;
    st->closed = 1;
  } else if (tot[0] <= st->tol2b) {
    st->done = 1;
    st->closed = 1;
  } else if (st->last) {
    st->status = BF_ERR_NOT_CONVERGED;
    st->done = 1;
    st->closed = 1;
  } else {
    // FP64: continue CG from the replaced residual.  Mixed: the float
    // correction has been folded; restart the inner solve on the new residual
    // (iterative refinement), since float drift breaks the conjugacy.
    st->beta = st->inner2 > 0.0 ? 0.0 : tot[1] / st->rho;
    st->rho = tot[1];
    st->rr_ref = tot[0];
    st->check = 0;
  }
}

// Workspace of one solve of N rows: state | partials [nb][3] | r z p0 p1 q (V)
// | c (float, mixed precision only).
size_t pcg_ws_bytes(int64_t N, bool mixed) {
  const int nb = (int)bf_round8(bf_cdiv(N, kThreads));
  const size_t vsz = mixed ? 4 : 8;
  return 256 + ((size_t)nb * 3 * 8 + 255) / 256 * 256 + 5 * (((size_t)N * vsz + 255) / 256 * 256) +
         (mixed ? ((size_t)N * 4 + 255) / 256 * 256 : 0);
}

// The workspace of bf_pcg_solve_noalloc: one array per GPU, loaded with the
// code object and kept until the process ends.  Host code never names it
// directly: its device address comes from hipGetSymbolAddress (per device,
// in bf_create) and is passed to the kernels like any workspace.
constexpr size_t kNoallocBytes = (size_t)BF_PCG_NOALLOC_BYTES;
__device__ __align__(256) char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Disables per-kernel timing records for one call (they would allocate
// events) and restores the setting on every return path.
struct TimingOff {
  bf_ctx* ctx;
  int saved;
  explicit TimingOff(bf_ctx* c) : ctx(c), saved(c->timing) { c->timing = 0; }
  ~TimingOff() { ctx->timing = saved; }
};

// fixed_ws == nullptr: the context's workspace, pinned host staging and
// pooled events (the allocating path of bf_pcg_solve).  Otherwise every
// temporary lives in fixed_ws (pcg_ws_bytes of it), the state comes back
// through a stack copy and the solve time is taken on the host.
template <typename V>
bf_status run_pcg(bf_ctx* ctx, const bf_system* sys, const bf_solve_opts* o, const double* rhs, double* x,
                  bf_solve_report* rep, char* fixed_ws = nullptr) {
  const int64_t N = sys->n;
  // one workgroup per 256 rows, a multiple of 8 workgroups (XCD-contiguous row ranges)
  const int nb = (int)bf_round8(bf_cdiv(N, kThreads));
  const bool mixed = sizeof(V) == 4;
  const bool noalloc = fixed_ws != nullptr;
  const size_t st_bytes = 256;
  const size_t part_bytes = ((size_t)nb * 3 * 8 + 255) / 256 * 256;
  const size_t vec_bytes = ((size_t)N * sizeof(V) + 255) / 256 * 256;
  char* ws = fixed_ws;
  if (!noalloc) BF_TRY(bf_ws(ctx, bf_ctx::WS_PCG, pcg_ws_bytes(N, mixed), (void**)&ws));
  PcgState* st = (PcgState*)ws;
  double* part = (double*)(ws + st_bytes);
  V* r = (V*)(ws + st_bytes + part_bytes);
  V* z = (V*)((char*)r + vec_bytes);
  V* p0 = (V*)((char*)z + vec_bytes);
  V* p1 = (V*)((char*)p0 + vec_bytes);
  V* q = (V*)((char*)p1 + vec_bytes);
  float* c = mixed ? (float*)((char*)q + vec_bytes) : nullptr;
  const V* diagV = mixed ? (const V*)sys->diag32 : (const V*)sys->diag;
  const V* dinvV = mixed ? (const V*)sys->dinv32 : (const V*)sys->dinv;
  V* xin = mixed ? (V*)c : (V*)x;
  const int replace_every = mixed ? bf_mixed_restart() : 0;
  // Mixed: each inner float solve reduces its residual 1e6-fold (or runs
  // replace_every iterations) before an FP64 check.
  const double inner = mixed ? 1e-6 : 0.0;
  const int fb = std::min(nb, 4096);

  // solve-time events from the context's pool (no create / destroy per call)
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  if (!noalloc) {
    e0 = bf_event_get(ctx);
    e1 = bf_event_get(ctx);
    if (!e0 || !e1) return bf_fail(ctx, BF_ERR_HIP, "event creation failed");
    BF_HIP(ctx, hipEventRecord(e0, ctx->stream));
  }
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, ctx->stream, st, o->tol, o->max_iter, replace_every,
                     inner, o->use_x0 ? 1 : 0);
  if (!o->use_x0) hipLaunchKernelGGL(k_fill<double>, dim3(fb), dim3(256), 0, ctx->stream, x, N, 0.0);
  hipLaunchKernelGGL(k_fill<V>, dim3(fb), dim3(256), 0, ctx->stream, p0, N, (V)0);
  if (mixed) hipLaunchKernelGGL(k_fill<float>, dim3(fb), dim3(256), 0, ctx->stream, c, N, 0.0f);
  const bool tri = sys->kind == BF_SYSTEM_TRILINEAR;
  const V* offV = mixed ? (const V*)sys->off32 : (const V*)sys->off;
  // FP64 true residual r = rhs - Q x (x == nullptr: x = 0)
  auto residual = [&](int mode, const double* xr) {
    if (tri)
      BF_LAUNCH(ctx, "pcg_residual", k_residual27<V>, dim3(nb), dim3(kThreads), 0, st, mode, sys->nb26, sys->off,
                sys->diag, rhs, xr, dinvV, r, z, N, part);
    else
      BF_LAUNCH(ctx, "pcg_residual", k_residual<V>, dim3(nb), dim3(kThreads), 0, st, mode, sys->band->nbr,
                sys->diag, sys->lambda, rhs, xr, dinvV, r, z, N, part);
  };
  residual((int)MODE_INIT, o->use_x0 ? (const double*)x : nullptr);
  BF_LAUNCH(ctx, "pcg_scalars", k_residual_scalars, dim3(1), dim3(1024), 0, st, (int)MODE_INIT, part, nb);
  if (o->use_x0) {  // a start no better than zero is dropped: x = 0 and INIT again
    hipLaunchKernelGGL(k_zero_if_dropped, dim3(fb), dim3(256), 0, ctx->stream, st, x, N);
    residual((int)MODE_GUARD, nullptr);
    BF_LAUNCH(ctx, "pcg_scalars", k_residual_scalars, dim3(1), dim3(1024), 0, st, (int)MODE_GUARD, part, nb);
  }
  BF_TRY(bf_launch_check(ctx, "pcg init"));

  PcgState hs_local;
  PcgState* hs = &hs_local;
  if (!noalloc) BF_TRY(bf_pinned(ctx, sizeof(PcgState), (void**)&hs));
  int it = 0;
  // iterations queued before the first poll: one from a supplied start (a
  // learned start often meets the tolerance at once), else three; then the
  // batches grow (3, 7, 14, ...)
  int next = o->check_every > 0 ? o->check_every : (o->use_x0 ? 1 : 3);
  V* pa = p0;
  V* pb = p1;
  const V lamV = (V)sys->lambda;
  std::vector<size_t> iter_rec;  // timing record count at the start of each iteration
  size_t fin_rec = 0;  // timing record of the last queued report pass (FP64)
  for (;;) {
    const int upto = std::min(next, o->max_iter);
    for (; it < upto; ++it) {
      if (ctx->timing) iter_rec.push_back(ctx->recs.size());
      if (tri)
        BF_LAUNCH(ctx, "pcg_A", k_pcg_A27<V>, dim3(nb), dim3(kThreads), 0, st, sys->nb26, offV, diagV, z, pa, pb, q,
                  N, part);
      else
        BF_LAUNCH(ctx, "pcg_A", k_pcg_A<V>, dim3(nb), dim3(kThreads), 0, st, sys->band->nbr, diagV, lamV, z, pa, pb,
                  q, N, part);
      BF_LAUNCH(ctx, "pcg_scalars", k_pcg_alpha, dim3(1), dim3(1024), 0, st, part, nb);
      BF_LAUNCH(ctx, "pcg_B", k_pcg_B<V>, dim3(nb), dim3(kThreads), 0, st, dinvV, pb, q, xin, r, z, N,
                         part);
      BF_LAUNCH(ctx, "pcg_scalars", k_pcg_beta, dim3(1), dim3(1024), 0, st, part, nb);
      if (mixed)
        BF_LAUNCH(ctx, "pcg_fold", k_fold, dim3(nb), dim3(kThreads), 0, st, 0, x, c, N);
      residual((int)MODE_CHECK, (const double*)x);
      BF_LAUNCH(ctx, "pcg_scalars", k_residual_scalars, dim3(1), dim3(1024), 0, st, (int)MODE_CHECK, part, nb);
      std::swap(pa, pb);
    }
    BF_TRY(bf_launch_check(ctx, "pcg iteration"));
    // FP64: the report's residual is queued behind every batch, so the poll
    // that finds the solve done has it already.  It reads x and sets only the
    // reported residual, which every later check overwrites, so a batch that
    // is not the last one loses nothing but the pass.
    if (!mixed) {
      fin_rec = ctx->recs.size();
      residual((int)MODE_REPORT, (const double*)x);
      BF_LAUNCH(ctx, "pcg_scalars", k_residual_scalars, dim3(1), dim3(1024), 0, st, (int)MODE_REPORT, part, nb);
    }
    // the solve's end, if this poll finds it done (mixed: unless a closing pass follows)
    if (e1) BF_HIP(ctx, hipEventRecord(e1, ctx->stream));
    BF_HIP(ctx, hipMemcpyAsync(hs, st, sizeof(PcgState), hipMemcpyDeviceToHost, ctx->stream));
    BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (hs->done || it >= o->max_iter) break;
    next = o->check_every > 0 ? it + o->check_every : (it < 3 ? 3 : it + std::max(it, 4));
  }
  const size_t loop_rec_end = mixed ? ctx->recs.size() : fin_rec;
  // Mixed: unless the solve ended at a true-residual pass (its x folded, its
  // residual the reported one), fold what is left and take the residual.
  if (mixed && !(hs->done && hs->closed)) {
    BF_LAUNCH(ctx, "pcg_fold", k_fold, dim3(nb), dim3(kThreads), 0, st, 1, x, c, N);
    residual((int)MODE_REPORT, (const double*)x);
    BF_LAUNCH(ctx, "pcg_scalars", k_residual_scalars, dim3(1), dim3(1024), 0, st, (int)MODE_REPORT, part, nb);
    if (e1) BF_HIP(ctx, hipEventRecord(e1, ctx->stream));
    BF_HIP(ctx, hipMemcpyAsync(hs, st, sizeof(PcgState), hipMemcpyDeviceToHost, ctx->stream));
    BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  float ms = 0.0f;
  if (noalloc) {
    ms = (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  } else {
    (void)hipEventElapsedTime(&ms, e0, e1);
    ctx->pool.push_back(e0);
    ctx->pool.push_back(e1);
  }
  if (ctx->timing && hs->iters >= 0 && (size_t)hs->iters < iter_rec.size())
    bf_timing_mark_idle(ctx, iter_rec[hs->iters], loop_rec_end);
  bf_status status = (bf_status)hs->status;
  if (status == BF_OK && !hs->done) status = BF_ERR_NOT_CONVERGED;
  if (hs->bnorm2 == 0.0) {  // Q x = 0 has the solution x = 0
    hipLaunchKernelGGL(k_fill<double>, dim3(fb), dim3(256), 0, ctx->stream, x, N, 0.0);
    BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  if (rep) {
    rep->iters = hs->iters;
    rep->status = status;
    rep->refinements = mixed ? hs->refinements : 0;
    rep->used_warm_start = (o->use_x0 && !hs->dropped) ? 1 : 0;
    rep->rel_res = hs->bnorm2 > 0.0 ? sqrt(hs->rr_true / hs->bnorm2) : 0.0;
    rep->seconds = ms * 1e-3;
    rep->col_iters = hs->iters;
  }
  if (status == BF_ERR_BREAKDOWN) return bf_fail(ctx, status, "bf_pcg_solve: breakdown (p.Qp <= 0 or non-finite)");
  if (status == BF_ERR_NOT_CONVERGED)
    return bf_fail(ctx, status, "bf_pcg_solve: not converged after %d iterations", hs->iters);
  return BF_OK;
}

}  // namespace

// Called by bf_create with ctx->device current: the device address of this
// GPU's copy of `scratch`, looked up once per device.
bf_status bf_pcg_scratch_init(bf_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return bf_fail(ctx, BF_ERR_INVALID_ARG, "device %d beyond the %d the library tracks", ctx->device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    void* p = nullptr;
    BF_HIP(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return bf_fail(ctx, BF_ERR_HIP, "hipGetSymbolAddress returned no address for the solver scratch");
    g_scratch_ptr[ctx->device] = p;
  }
  ctx->pcg_scratch = g_scratch_ptr[ctx->device];
  return BF_OK;
}

extern "C" bf_status bf_pcg_solve_noalloc(bf_ctx* ctx, const bf_system* sys, const bf_solve_opts* opts,
                                          const double* rhs_dev, double* x_dev, bf_solve_report* rep) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, sys && opts, "bf_pcg_solve_noalloc: NULL argument");
  BF_CHECK(ctx, opts->tol >= 0.0 && opts->max_iter >= 0, "bf_pcg_solve_noalloc: tol and max_iter must be >= 0");
  BF_CHECK(ctx, opts->precision == BF_PREC_FP64 || opts->precision == BF_PREC_MIXED,
           "bf_pcg_solve_noalloc: unknown precision %d", opts->precision);
  if (rep) *rep = bf_solve_report{};
  if (sys->n == 0) return BF_OK;
  BF_CHECK(ctx, x_dev, "bf_pcg_solve_noalloc: NULL x");
  const bool mixed = opts->precision == BF_PREC_MIXED;
  const size_t need = pcg_ws_bytes(sys->n, mixed);
  if (need > kNoallocBytes)
    return bf_fail(ctx, BF_ERR_CAPACITY,
                   "bf_pcg_solve_noalloc: %lld band voxels need %zu bytes of solver scratch in %s precision; "
                   "the static scratch holds %zu (at most %lld voxels in FP64, %lld mixed)",
                   (long long)sys->n, need, mixed ? "mixed" : "FP64", kNoallocBytes,
                   (long long)bf_pcg_noalloc_max_n(BF_PREC_FP64), (long long)bf_pcg_noalloc_max_n(BF_PREC_MIXED));
  if (!ctx->pcg_scratch) return bf_fail(ctx, BF_ERR_HIP, "bf_pcg_solve_noalloc: solver scratch not initialised");
  BF_HIP(ctx, hipSetDevice(ctx->device));
  TimingOff no_records(ctx);
  const double* rhs = rhs_dev ? rhs_dev : sys->rhs;
  char* ws = (char*)ctx->pcg_scratch;
  if (!mixed) return run_pcg<double>(ctx, sys, opts, rhs, x_dev, rep, ws);
  return run_pcg<float>(ctx, sys, opts, rhs, x_dev, rep, ws);
}

extern "C" int64_t bf_pcg_noalloc_max_n(int32_t precision) {
  const bool mixed = precision == BF_PREC_MIXED;
  int64_t lo = 0, hi = (int64_t)(kNoallocBytes / (mixed ? 24 : 40)) + 1;
  while (lo < hi) {  // largest N whose workspace fits
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (pcg_ws_bytes(mid, mixed) <= kNoallocBytes) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

extern "C" bf_status bf_pcg_solve(bf_ctx* ctx, const bf_system* sys, const bf_solve_opts* opts,
                                  const double* rhs_dev, double* x_dev, bf_solve_report* rep) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, sys && opts, "bf_pcg_solve: NULL argument");
  BF_CHECK(ctx, opts->tol >= 0.0 && opts->max_iter >= 0, "bf_pcg_solve: tol and max_iter must be >= 0");
  BF_CHECK(ctx, opts->precision == BF_PREC_FP64 || opts->precision == BF_PREC_MIXED,
           "bf_pcg_solve: unknown precision %d", opts->precision);
  if (rep) *rep = bf_solve_report{};
  if (sys->n == 0) return BF_OK;
  BF_CHECK(ctx, x_dev, "bf_pcg_solve: NULL x");
  BF_HIP(ctx, hipSetDevice(ctx->device));
  const double* rhs = rhs_dev ? rhs_dev : sys->rhs;
  if (opts->precision == BF_PREC_FP64) return run_pcg<double>(ctx, sys, opts, rhs, x_dev, rep);
  return run_pcg<float>(ctx, sys, opts, rhs, x_dev, rep);
}
