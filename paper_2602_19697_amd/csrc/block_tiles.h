// Building blocks of the K-column block CG for the Hutchinson probes
// (Sec. 3.7, eq. 12), shared by the single-system kernels and the persistent
// multi-scene kernel: per-column solver state, the in-register Rademacher
// probes, the per-tile work of each CG phase and the per-column decisions.
//
// Block vectors are row-major [N][KC] (KC = 1, 16, 32 or 64 >= K).  A thread owns
// one column c = threadIdx.x % KC and rows rsub, rsub + 256/KC, ... of a tile,
// so each row's KC values and each neighbour row's KC values are read as one
// coalesced segment while the neighbour table and diagonal are read once per
// row for all columns.
#pragma once

#include "bf_internal.h"

namespace bt {

constexpr int kThreads = 256;
constexpr int kMaxK = 64;

// VERIFY: residual norms of the columns whose recurrence residual met the
// tolerance (check == 2), with no stores; CHECK: the residual, stored, of the
// columns to continue or restart from it (check == 1).
// GUARD: after INIT with a supplied start, the columns whose start was no
// better than zero (dropped) restart from x = 0.
enum { MODE_INIT = 0, MODE_CHECK = 1, MODE_REPORT = 2, MODE_VERIFY = 3, MODE_GUARD = 4 };

struct BState {
  double rho[kMaxK], alpha[kMaxK], beta[kMaxK], tol2b[kMaxK], rr_true[kMaxK], bnorm2[kMaxK], rr_ref[kMaxK];
  double inner2;
  int32_t active[kMaxK], check[kMaxK], last[kMaxK], iters[kMaxK], status[kMaxK];
  int32_t nactive, any_check, max_iter, replace_every, K, refinements;
  int32_t pending;  // columns with check == 1 (a stored residual is due)
  int32_t guard;    // a start was supplied: drop it where ||z - Q u0|| >= ||z||
  int32_t dropped[kMaxK];
  // Mixed precision, 7-point path: where column c's FP64 part x64 lives.
  // 0: stored; 1: the warm start +-w[v] by the sign of probe c at row v,
  // regenerated where it is read; 2: the zero start.  A column is stored (0)
  // from its first fold on.
  int32_t xbase[kMaxK];
  int32_t ndropped;
  // 1 while the estimate s was formed by a VERIFY pass that covered every
  // column and every column passed it (the closing estimate pass is then
  // skipped); a failed column clears it
  int32_t s_fused;
};

// SplitMix64 output n (0-based) of the generator started at `start`.
__device__ __forceinline__ uint64_t splitmix_out(uint64_t start, uint64_t n) {
  uint64_t z = start + (n + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// z_k[i] = -1 if the top bit of output i of the generator started at u_k is set.
__device__ __forceinline__ double probe(uint64_t col_seed, int64_t i) {
  return (splitmix_out(col_seed, (uint64_t)i) >> 63) ? -1.0 : 1.0;
}

__device__ __forceinline__ void state_init(BState* st, int K, double tol, int32_t max_iter, double inner,
                                           int32_t replace_every) {
  const int c = threadIdx.x;
  if (c < kMaxK) {
    st->rho[c] = st->alpha[c] = st->beta[c] = st->rr_true[c] = st->bnorm2[c] = st->rr_ref[c] = 0.0;
    st->tol2b[c] = tol * tol;
    st->active[c] = c < K ? 1 : 0;
    st->check[c] = st->last[c] = st->iters[c] = st->status[c] = st->dropped[c] = st->xbase[c] = 0;
  }
  if (c == 0) {
    st->guard = 0;
    st->ndropped = 0;
    st->s_fused = 0;
    st->inner2 = inner * inner;
    st->nactive = K;
    st->any_check = 0;
    st->max_iter = max_iter;
    st->replace_every = replace_every;
    st->K = K;
    st->refinements = 0;
    st->pending = 0;
  }
}

// Per-column sum over the workgroup in a fixed order; threads c < KC end with
// the column totals.  lds holds >= 4*NQ*64 doubles.
template <int KC, int NQ>
__device__ __forceinline__ void col_block_sum(double (&v)[NQ], double* lds) {
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

template <int KC, int NQ>
__device__ __forceinline__ void store_partials(double* __restrict__ part, int64_t slot, double (&v)[NQ]) {
  if (threadIdx.x < KC)
#pragma unroll
    for (int q = 0; q < NQ; ++q) part[((size_t)slot * NQ + q) * KC + threadIdx.x] = v[q];
}

// Column c's sums over `nb` partial slots, by one whole workgroup in a fixed
// order; every thread receives the totals.
template <int KC, int NQ>
__device__ __forceinline__ void col_partials_sum(const double* __restrict__ part, int64_t nb, int c,
                                                 double (&tot)[NQ], double* lds) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) acc += part[((size_t)b * NQ + q) * KC + c];
    tot[q] = bf_block_sum(acc, lds);
  }
}

// Tiles [start, end) with stride of this workgroup in a grid-strided loop
// over ntiles: with a grid that is a multiple of 8, each XCD's workgroups
// (b % 8 == x, dispatched round robin) walk one contiguous eighth of the tiles.
struct TileWalk {
  int64_t start, stride, end;
  __device__ explicit TileWalk(int64_t ntiles) {
    const int64_t g = gridDim.x, b = blockIdx.x;
    if ((g & 7) == 0) {
      const int64_t x = b & 7;
      start = ntiles * x / 8 + (b >> 3);
      stride = g >> 3;
      end = ntiles * (x + 1) / 8;
    } else {
      start = b;
      stride = g;
      end = ntiles;
    }
  }
};

// ---------------------------------------------------------------- tile work
// A: p = zz + beta p_old (neighbours on the fly), q = Q p; acc += p.q.
// Each thread keeps kRowsInFlight rows' gathers in flight: the neighbour
// indices of all of them are loaded first, and absent neighbours (-1) read the
// row itself and add nothing, so every gather is an unconditional load that the
// compiler can issue back to back.
constexpr int kRowsInFlight = 4;

// The 6 neighbour indices of row v (24 B, 8-byte aligned: the band's arrays
// start on 256-byte boundaries) as three 8-byte loads instead of six.
__device__ __forceinline__ void load_nbr6(const int32_t* __restrict__ nbr, int64_t v, int32_t* nb) {
  const int2* q = reinterpret_cast<const int2*>(nbr + v * 6);
  const int2 a = q[0], b = q[1], c = q[2];
  nb[0] = a.x;
  nb[1] = a.y;
  nb[2] = b.x;
  nb[3] = b.y;
  nb[4] = c.x;
  nb[5] = c.y;
}

// store_p: write p_new (the first iteration's direction p = zz can stay
// where zz is instead).
template <typename V, int KC>
__device__ __forceinline__ void tile_A(int c, V beta, bool first, const int32_t* __restrict__ nbr,
                                       const V* __restrict__ diag, V lam, const V* __restrict__ zz,
                                       const V* __restrict__ p_old, V* __restrict__ p_new, V* __restrict__ q,
                                       int64_t r0, int64_t r1, double& acc1, bool store_p = true) {
  constexpr int RS = kThreads / KC;
  constexpr int U = kRowsInFlight;
  for (int64_t v0 = r0 + threadIdx.x / KC; v0 < r1; v0 += U * RS) {
    int64_t vr[U];
    int32_t nb[U][6];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t v = v0 + j * RS;
      vr[j] = v < r1 ? v : r0;
      load_nbr6(nbr, vr[j], nb[j]);
    }
    V s[U], pv[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      s[j] = 0;
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int64_t u = nb[j][t] >= 0 ? (int64_t)nb[j][t] : vr[j];
        const V a = zz[u * KC + c] + beta * (first ? (V)0 : p_old[u * KC + c]);
        s[j] = fma(a, nb[j][t] >= 0 ? (V)1 : (V)0, s[j]);  // an absent neighbour adds +-0 (a is finite)
      }
      const int64_t e = vr[j] * KC + c;
      pv[j] = zz[e] + beta * (first ? (V)0 : p_old[e]);
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (v0 + j * RS >= r1) break;
      const int64_t e = vr[j] * KC + c;
      const V qv = diag[vr[j]] * pv[j] - lam * s[j];
      if (store_p) p_new[e] = pv[j];
      q[e] = qv;
      acc1 += (double)pv[j] * (double)qv;
    }
  }
}

// B: x += alpha p, r -= alpha q, zz = r / diag; acc += r.zz, r.r.
template <typename V, int KC>
// first: x still holds its zero start, taken as the literal 0 (not read).
// gen: r still holds the probe z (not stored), regenerated from the column's
// generator cs.
__device__ __forceinline__ void tile_B(int c, V alpha, bool first, bool gen, uint64_t cs,
                                       const V* __restrict__ dinv, const V* __restrict__ p, const V* __restrict__ q,
                                       V* __restrict__ x, V* __restrict__ r, V* __restrict__ zz, int64_t r0,
                                       int64_t r1, double& rz, double& rr) {
  constexpr int RS = kThreads / KC;
  for (int64_t v = r0 + threadIdx.x / KC; v < r1; v += RS) {
    const int64_t e = v * KC + c;
    x[e] = (first ? (V)0 : x[e]) + alpha * p[e];
    const V rv = (gen ? (V)probe(cs, v) : r[e]) - alpha * q[e];
    const V zv = rv * dinv[v];
    r[e] = rv;
    zz[e] = zv;
    rz += (double)rv * (double)zv;
    rr += (double)rv * (double)rv;
  }
}

// Mixed precision: x64 += c (float correction), c = 0.
template <int KC>
__device__ __forceinline__ void tile_fold(int c, double* __restrict__ x64, float* __restrict__ cf, int64_t r0,
                                          int64_t r1) {
  constexpr int RS = kThreads / KC;
  for (int64_t v = r0 + threadIdx.x / KC; v < r1; v += RS) {
    const int64_t e = v * KC + c;
    x64[e] = x64[e] + (double)cf[e];
    cf[e] = 0.0f;
  }
}

// FP64 residual r = z - Q x (INIT: x = 0 or the warm start exp(logvar) z / diag,
// written to x64).  acc: r.r, r.zz (stored precision), z.z.  The gathers of
// x64 are unconditional loads, kRowsInFlight rows at a time, as in tile_A.
template <typename V, int KC>
__device__ __forceinline__ void tile_resid(int c, int mode, uint64_t cs, const int32_t* __restrict__ nbr,
                                           const double* __restrict__ diag, double lam,
                                           const float* __restrict__ logvar, double* __restrict__ x64,
                                           const V* __restrict__ dinv, V* __restrict__ r, V* __restrict__ zz,
                                           int64_t r0, int64_t r1, double (&v3)[3], bool write_x0 = true,
                                           bool store_r = true) {
  constexpr int RS = kThreads / KC;
  constexpr int U = kRowsInFlight;
  for (int64_t v0 = r0 + threadIdx.x / KC; v0 < r1; v0 += U * RS) {
    double res[U], zv[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t v = v0 + j * RS < r1 ? v0 + j * RS : r0;
      zv[j] = probe(cs, v);
      res[j] = zv[j];
    }
    if (mode == MODE_INIT) {
#pragma unroll
      for (int j = 0; j < U; ++j) {
        if (v0 + j * RS >= r1) break;
        const int64_t v = v0 + j * RS, e = v * KC + c;
        if (logvar) {
          const int32_t* nb = nbr + v * 6;
          double acc = 0.0;
#pragma unroll
          for (int t = 0; t < 6; ++t) {
            const int32_t u = nb[t];
            if (u >= 0) acc += exp((double)logvar[u]) * probe(cs, u) / diag[u];
          }
          const double x0 = exp((double)logvar[v]) * zv[j] / diag[v];
          x64[e] = x0;
          res[j] = zv[j] - (diag[v] * x0 - lam * acc);
        } else if (write_x0) {
          x64[e] = 0.0;
        }
      }
    } else {
      int64_t vr[U];
      int32_t nb[U][6];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        vr[j] = v0 + j * RS < r1 ? v0 + j * RS : r0;
        load_nbr6(nbr, vr[j], nb[j]);
      }
#pragma unroll
      for (int j = 0; j < U; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < 6; ++t) {
          const int64_t u = nb[j][t] >= 0 ? (int64_t)nb[j][t] : vr[j];
          const double xu = x64[u * KC + c];
          if (nb[j][t] >= 0) acc += xu;
        }
        res[j] = zv[j] - (diag[vr[j]] * x64[vr[j] * KC + c] - lam * acc);
      }
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (v0 + j * RS >= r1) break;
      const int64_t v = v0 + j * RS, e = v * KC + c;
      v3[0] += res[j] * res[j];
      v3[2] += zv[j] * zv[j];
      if (mode == MODE_VERIFY) {
        const V rv = (V)res[j];
        v3[1] += (double)rv * (double)(rv * dinv[v]);
      } else if (mode != MODE_REPORT) {
        const V rv = (V)res[j];
        const V zzv = rv * dinv[v];
        if (store_r || mode != MODE_INIT) r[e] = rv;
        zz[e] = zzv;
        v3[1] += (double)rv * (double)zzv;
      }
    }
  }
}

// ---------------------------------------------------------------- decisions
// Executed by one thread per column; *nactive_all (may be null) mirrors the
// count of active columns across all systems of a batch.
__device__ __forceinline__ void deactivate(BState* st, int c, int status, int* nactive_all) {
  if (status) st->status[c] = status;
  st->active[c] = 0;
  atomicSub(&st->nactive, 1);
  if (nactive_all) atomicSub(nactive_all, 1);
}

__device__ __forceinline__ void decide_A(BState* st, int c, double pq, int* nactive_all) {
  if (!(pq > 0.0) || !isfinite(pq)) deactivate(st, c, BF_ERR_BREAKDOWN, nactive_all);
  else st->alpha[c] = st->rho[c] / pq;
}

__device__ __forceinline__ void decide_B(BState* st, int c, double rz, double rr, int* nactive_all, int* any_all) {
  const int it = st->iters[c] + 1;
  st->iters[c] = it;
  const bool at_max = it >= st->max_iter;
  const bool periodic = st->replace_every > 0 && (it % st->replace_every) == 0;
  if (!isfinite(rz) || !isfinite(rr)) {
    deactivate(st, c, BF_ERR_BREAKDOWN, nactive_all);
  } else if (rr <= fmax(st->tol2b[c], st->inner2 * st->rr_ref[c]) || at_max || periodic) {
    // 2: the recurrence says converged, so a store-free FP64 residual decides
    // first; 1: the column continues or restarts from a stored FP64 residual
    st->check[c] = rr <= st->tol2b[c] ? 2 : 1;
    if (st->check[c] == 1) atomicAdd(&st->pending, 1);
    st->last[c] = at_max ? 1 : 0;
    atomicOr(&st->any_check, 1);
    if (any_all) atomicOr(any_all, 1);
  } else {
    st->beta[c] = rz / st->rho[c];
    st->rho[c] = rz;
  }
}

// After a VERIFY pass: a column whose FP64 residual meets the tolerance stops
// (as it would after a CHECK); any other one is handed to the CHECK pass,
// which recomputes the same residual and stores it.
__device__ __forceinline__ void decide_V(BState* st, int c, const double (&tot)[3], int* nactive_all) {
  st->rr_true[c] = tot[0];
  if (isfinite(tot[0]) && isfinite(tot[1]) && tot[0] <= st->tol2b[c]) {
    atomicAdd(&st->refinements, 1);
    deactivate(st, c, 0, nactive_all);
    st->check[c] = 0;
  } else {
    st->check[c] = 1;
    atomicAdd(&st->pending, 1);
    st->s_fused = 0;  // this column goes on: its estimate rows are not final
  }
}

__device__ __forceinline__ void decide_R(BState* st, int c, int mode, const double (&tot)[3], int* nactive_all) {
  if (mode == MODE_REPORT) {
    st->rr_true[c] = tot[0];
  } else if (mode == MODE_INIT || mode == MODE_GUARD) {
    if (mode == MODE_INIT) {
      st->bnorm2[c] = tot[2];
      st->tol2b[c] *= tot[2];
      // a supplied start no better than zero is dropped; GUARD redoes INIT from x = 0
      if (st->guard && tot[2] > 0.0 && !(tot[0] < tot[2])) {
        st->dropped[c] = 1;
        if (st->xbase[c] == 1) st->xbase[c] = 2;  // its x64 is the zero start now
        atomicAdd(&st->ndropped, 1);
        return;
      }
    }
    st->rr_true[c] = tot[0];
    if (tot[2] == 0.0 || tot[0] <= st->tol2b[c]) {
      deactivate(st, c, 0, nactive_all);
    } else if (st->max_iter <= 0) {
      deactivate(st, c, BF_ERR_NOT_CONVERGED, nactive_all);
    } else {
      st->rho[c] = tot[1];
      st->beta[c] = 0.0;
      st->rr_ref[c] = tot[0];
    }
  } else {
    st->rr_true[c] = tot[0];
    atomicAdd(&st->refinements, 1);
    if (!isfinite(tot[0]) || !isfinite(tot[1])) {
      deactivate(st, c, BF_ERR_BREAKDOWN, nactive_all);
    } else if (tot[0] <= st->tol2b[c]) {
      deactivate(st, c, 0, nactive_all);
    } else if (st->last[c]) {
      deactivate(st, c, BF_ERR_NOT_CONVERGED, nactive_all);
    } else {
      // FP64 continues CG from the replaced residual; mixed restarts the
      // float solve on the FP64 residual (iterative refinement).
      st->beta[c] = st->inner2 > 0.0 ? 0.0 : tot[1] / st->rho[c];
      st->rho[c] = tot[1];
      st->rr_ref[c] = tot[0];
    }
    if (st->check[c] == 1) atomicSub(&st->pending, 1);
    st->check[c] = 0;
    st->xbase[c] = 0;  // the check's fold stored x64
  }
}

// s_v = (1/K) sum_k z_k[v] u_k[v], columns in ascending order.
template <int KC>
__device__ __forceinline__ double hutch_row(const double* __restrict__ x64, uint64_t seed, int K, int64_t v) {
  double s = 0.0;
  for (int k = 0; k < K; ++k) s += probe(splitmix_out(seed, (uint64_t)k), v) * x64[v * KC + k];
  return s / (double)K;
}

}  // namespace bt
