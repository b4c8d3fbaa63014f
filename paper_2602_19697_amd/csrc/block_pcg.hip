// Hutchinson estimate of diag(Q^-1) (Sec. 3.7, eq. 12; Algorithm 1 step 6)
// with all K probe solves run as one block CG.
//
// Layout: block vectors are row-major [N][KC] (KC = 1 for a single probe,
// else K rounded up to 16, 32 or 64), so one band voxel's K values are contiguous: the stencil gathers of a
// neighbour row are coalesced and the neighbour table and diagonal are read
// once per row for all K columns.  Every column keeps its own FP64 alpha, beta
// and stopping test (independent CGs sharing each matrix pass).  Probes z_k
// come from the SplitMix64 counter hash; for the 7-point system their signs
// are hashed once per solve and kept packed, one bit per column (KC/32 words
// per row), and every pass that needs z reads those bits.  Precision as in the single
// right-hand-side solver: FP64, or float vectors with FP64 scalars, FP64
// folds/residuals and restarted float solves (mixed-precision iterative
// refinement).  The per-tile work and the per-column decisions live in
// block_tiles.h and are shared with the persistent multi-scene solver.
#include <cstdlib>

#include "block_tiles.h"

namespace {

using namespace bt;
// rows per tile: 4 (one column) to 16 (64 columns) values per thread
template <int KC>
constexpr int kRowsPerTile = KC == 1 ? 1024 : 64;

__global__ void k_bstate_init(BState* st, int K, double tol, int32_t max_iter, double inner, int32_t replace_every,
                              int32_t guard, int32_t xbase) {
  state_init(st, K, tol, max_iter, inner, replace_every);
  if (threadIdx.x == 0) st->guard = guard;
  if (threadIdx.x < K) st->xbase[threadIdx.x] = xbase;
}


// A: p = zz + beta p_old, q = Q p, per-column partial p.q.
//
// The tile's own rows of p are formed once and staged in LDS (32 KB: 64 to 512
// rows, by column count and precision); neighbour rows inside the tile are
// read from there, the others (Morton order keeps most neighbours within a few
// hundred rows) from global memory as zz + beta p_old.  Every sum runs in the
// same order as the plain tile, so the results are the same bits.
template <typename V, int KC, int LDSKB>
constexpr int kStencilRows = KC == 1 ? 1024 : LDSKB * 1024 / (KC * (int)sizeof(V));

// CPL adjacent columns of a row, loaded and stored as one element (8 bytes
// for two floats).
template <typename V, int CPL>
struct Cols {
  V v[CPL];
};
template <typename V, int CPL>
__device__ __forceinline__ Cols<V, CPL> ldc(const V* __restrict__ p) {
  Cols<V, CPL> r;
  if constexpr (CPL == 2) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    r.v[0] = t.x;
    r.v[1] = t.y;
  } else {
    r.v[0] = *p;
  }
  return r;
}
template <typename V, int CPL>
__device__ __forceinline__ void stc(V* __restrict__ p, const Cols<V, CPL>& c) {
  if constexpr (CPL == 2) *reinterpret_cast<float2*>(p) = make_float2(c.v[0], c.v[1]);
  else *p = c.v[0];
}
// Columns per thread of the stencil pass: two in single precision (the row's
// neighbour indices, tests and addresses then serve two values), one in FP64
// (pairs of doubles held the pass to fewer waves and ran slower).
template <typename V>
constexpr int kStencilCols = sizeof(V) == 4 ? 2 : 1;

// The sums and stores of stencil rows [r0, r1), the tile's p staged in pt
// (LDS): neighbour rows inside the tile come from there, the others from
// global memory as zz + beta p_old.  A thread takes the CPL adjacent columns
// from cc; each column's sums are those of a thread with one column.
template <typename V, int KC, int CPL, bool FIRST>
__device__ __forceinline__ void stencil_sums(int cc, const V (&beta)[CPL], V lam, const int32_t* __restrict__ nbr,
                                             const V* __restrict__ diag, const V* __restrict__ zz,
                                             const V* __restrict__ p_old, V* __restrict__ p_new, V* __restrict__ q,
                                             const V* __restrict__ pt, int64_t r0, int64_t r1,
                                             double (&acc)[CPL]) {
  typedef Cols<V, CPL> C;
  constexpr int RS = kThreads / (KC / CPL);
  constexpr bool first = FIRST;
  // the gathers of neighbours outside the tile are all issued before the
  // sums use them.  No branch guards them: a lane with nothing to gather
  // (neighbour absent or inside the tile) loads row 0, a line every wave
  // reads, and takes 0, so an absent neighbour adds +0.0, which leaves the
  // sum unchanged (it starts at +0.0, so it is never -0.0).  Row indices
  // fit 31 bits (checked by the host).
  constexpr int U = 2;
  const uint32_t span = (uint32_t)(r1 - r0);
  for (int64_t v0 = r0 + threadIdx.x / (KC / CPL); v0 < r1; v0 += U * RS) {
    int64_t vr[U];
    int32_t nb[U][6];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      vr[j] = v0 + j * RS < r1 ? v0 + j * RS : r0;
      load_nbr6(nbr, vr[j], nb[j]);
    }
    C gz[U][6], gp[U][6];
#pragma unroll
    for (int j = 0; j < U; ++j)
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int32_t u = nb[j][t];
        const bool in = (uint32_t)(u - (int32_t)r0) < span;
        const bool out = u >= 0 && !in;
        if constexpr (sizeof(V) == 8) {
          // FP64: the gathers under a branch (faster there: a row's lanes
          // read 256 bytes per load)
#pragma unroll
          for (int h = 0; h < CPL; ++h) gz[j][t].v[h] = gp[j][t].v[h] = 0;
          if (out) {
            const size_t e = (size_t)u * KC + cc;
            gz[j][t] = ldc<V, CPL>(zz + e);
            if constexpr (!first) gp[j][t] = ldc<V, CPL>(p_old + e);
          }
        } else {
          const size_t e = (size_t)(out ? (uint32_t)u : 0u) * KC + cc;
          const C za = ldc<V, CPL>(zz + e);
          C pa;
          if constexpr (!first) pa = ldc<V, CPL>(p_old + e);
#pragma unroll
          for (int h = 0; h < CPL; ++h) {
            gz[j][t].v[h] = out ? za.v[h] : (V)0;
            gp[j][t].v[h] = first ? (V)0 : (out ? pa.v[h] : (V)0);
          }
        }
      }
    C sacc[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
#pragma unroll
      for (int h = 0; h < CPL; ++h) sacc[j].v[h] = 0;
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int32_t u = nb[j][t];
        const bool in = (uint32_t)(u - (int32_t)r0) < span;
        const C lv = ldc<V, CPL>(pt + (in ? u - (int32_t)r0 : 0) * KC + cc);
#pragma unroll
        for (int h = 0; h < CPL; ++h) {
          const V gv = gz[j][t].v[h] + beta[h] * gp[j][t].v[h];
          sacc[j].v[h] += in ? lv.v[h] : gv;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (v0 + j * RS >= r1) break;
      const int64_t e = vr[j] * KC + cc;
      const C pv = ldc<V, CPL>(pt + (vr[j] - r0) * KC + cc);
      const V d = diag[vr[j]];
      C qv;
#pragma unroll
      for (int h = 0; h < CPL; ++h) qv.v[h] = d * pv.v[h] - lam * sacc[j].v[h];
      if constexpr (!FIRST) stc<V, CPL>(p_new + e, pv);
      stc<V, CPL>(q + e, qv);
#pragma unroll
      for (int h = 0; h < CPL; ++h) acc[h] += (double)pv.v[h] * (double)qv.v[h];
    }
  }
}

// The pass over the band (see stencil_sums); k_bA and k_bA4 launch it.
template <typename V, int KC, int LDSKB, bool FIRST>
__device__ __forceinline__ void bA_pass(BState* __restrict__ st, const int32_t* __restrict__ nbr,
                                        const V* __restrict__ diag, V lam, const V* __restrict__ zz,
                                        const V* __restrict__ p_old, V* __restrict__ p_new, V* __restrict__ q,
                                        int64_t n, double* __restrict__ part, double* lds, V* pt) {
  constexpr int R = kStencilRows<V, KC, LDSKB>;
  if (st->nactive == 0) return;
  const TileWalk tw(bf_cdiv(n, R));
  // FIRST (the first iteration's launch; every active column starts there):
  // the direction is z (beta = 0) and p_old is not read, as if it held zeros
  // (z + 0 * 0, the same value), so it needs no clearing; nor is p written:
  // it equals z, which stays where it is and serves as this iteration's p.
  // A separate instantiation, so the later launches carry no switch around
  // their loads.
  constexpr bool first = FIRST;
  if constexpr (KC == 1) {
    double v1[1] = {0.0};
    const bool act = st->active[0] != 0;
    const V beta = (V)st->beta[0];
    for (int64_t tile = tw.start; tile < tw.end; tile += tw.stride)
      if (act)
        tile_A<V, KC>(0, beta, first, nbr, diag, lam, zz, p_old, p_new, q, tile * R,
                      std::min<int64_t>(n, (tile + 1) * R), v1[0], !first);
    col_block_sum<KC, 1>(v1, lds);
    store_partials<KC, 1>(part, blockIdx.x, v1);
  } else {
    // a thread's columns: cc .. cc + CPL - 1 (a column that has stopped is
    // computed along with the others; its sums are not used)
    constexpr int CPL = kStencilCols<V>;
    typedef Cols<V, CPL> C;
    constexpr int KH = KC / CPL;
    constexpr int RS = kThreads / KH;
    constexpr int SJ = R / RS;  // rows of a tile per thread
    const int cc = CPL * (threadIdx.x % KH);
    bool act = false;
    V beta[CPL];
#pragma unroll
    for (int h = 0; h < CPL; ++h) {
      act = act || st->active[cc + h] != 0;
      beta[h] = (V)st->beta[cc + h];
    }
    double acc[CPL];
#pragma unroll
    for (int h = 0; h < CPL; ++h) acc[h] = 0.0;
    if constexpr (FIRST) {
      // p = z: the next tile's rows of z are loaded into registers while the
      // current tile's sums run, so staging a tile waits on no load
      C za[SJ];
      auto fetch = [&](int64_t tile) {
        const int64_t r0 = tile * R, r1 = std::min<int64_t>(n, r0 + R);
#pragma unroll
        for (int j = 0; j < SJ; ++j) {
          const int64_t v = r0 + threadIdx.x / KH + (int64_t)j * RS;
          if (v < r1) za[j] = ldc<V, CPL>(zz + v * KC + cc);
        }
      };
      if (act && tw.start < tw.end) fetch(tw.start);
      for (int64_t tile = tw.start; tile < tw.end; tile += tw.stride) {
        const int64_t r0 = tile * R, r1 = std::min<int64_t>(n, r0 + R);
        __syncthreads();  // the previous tile's readers are done
        if (act) {
#pragma unroll
          for (int j = 0; j < SJ; ++j) {
            const int64_t v = r0 + threadIdx.x / KH + (int64_t)j * RS;
            if (v < r1) {
              C pv;
#pragma unroll
              for (int h = 0; h < CPL; ++h) pv.v[h] = za[j].v[h] + beta[h] * (V)0;
              stc<V, CPL>(pt + (v - r0) * KC + cc, pv);
            }
          }
        }
        __syncthreads();
        if (act && tile + tw.stride < tw.end) fetch(tile + tw.stride);
        if (act) stencil_sums<V, KC, CPL, FIRST>(cc, beta, lam, nbr, diag, zz, p_old, p_new, q, pt, r0, r1, acc);
      }
    } else {
      for (int64_t tile = tw.start; tile < tw.end; tile += tw.stride) {
        const int64_t r0 = tile * R, r1 = std::min<int64_t>(n, r0 + R);
        __syncthreads();  // the previous tile's readers are done
        if (act) {
          // every load of a batch of rows is issued before the first LDS store
          constexpr int SB = SJ < 8 ? SJ : 8;
          static_assert(SJ % SB == 0, "staging batches must tile the rows of a thread");
          for (int j0 = 0; j0 < SJ; j0 += SB) {
            C za[SB], pa[SB];
#pragma unroll
            for (int j = 0; j < SB; ++j) {
              const int64_t v = r0 + threadIdx.x / KH + (int64_t)(j0 + j) * RS;
              if (v < r1) {
                za[j] = ldc<V, CPL>(zz + v * KC + cc);
                pa[j] = ldc<V, CPL>(p_old + v * KC + cc);
              }
            }
#pragma unroll
            for (int j = 0; j < SB; ++j) {
              const int64_t v = r0 + threadIdx.x / KH + (int64_t)(j0 + j) * RS;
              if (v < r1) {
                C pv;
#pragma unroll
                for (int h = 0; h < CPL; ++h) pv.v[h] = za[j].v[h] + beta[h] * pa[j].v[h];
                stc<V, CPL>(pt + (v - r0) * KC + cc, pv);
              }
            }
          }
        }
        __syncthreads();
        if (act) stencil_sums<V, KC, CPL, FIRST>(cc, beta, lam, nbr, diag, zz, p_old, p_new, q, pt, r0, r1, acc);
      }
    }
    // column totals: the lanes of a column group add up, then the waves
    col_block_sum<KH, CPL>(acc, lds);
    if (threadIdx.x < KH)
#pragma unroll
      for (int h = 0; h < CPL; ++h) part[(size_t)blockIdx.x * KC + CPL * threadIdx.x + h] = acc[h];
  }
}

template <typename V, int KC, int LDSKB, bool FIRST>
__global__ __launch_bounds__(256) void k_bA(BState* __restrict__ st, const int32_t* __restrict__ nbr,
                                            const V* __restrict__ diag, V lam, const V* __restrict__ zz,
                                            const V* __restrict__ p_old, V* __restrict__ p_new, V* __restrict__ q,
                                            int64_t n, double* __restrict__ part) {
  __shared__ double lds[4 * 3 * 64];
  __shared__ V pt[KC == 1 ? 1 : kStencilRows<V, KC, LDSKB> * KC];
  bA_pass<V, KC, LDSKB, FIRST>(st, nbr, diag, lam, zz, p_old, p_new, q, n, part, lds, pt);
}

// The pass over 32 KB tiles with the register budget of four waves per
// SIMD, which the tiles allow (measured faster than the compiler's choice).
template <typename V, int KC, bool FIRST>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_bA4(
    BState* __restrict__ st, const int32_t* __restrict__ nbr, const V* __restrict__ diag, V lam,
    const V* __restrict__ zz, const V* __restrict__ p_old, V* __restrict__ p_new, V* __restrict__ q, int64_t n,
    double* __restrict__ part) {
  __shared__ double lds[4 * 3 * 64];
  __shared__ V pt[KC == 1 ? 1 : kStencilRows<V, KC, 32> * KC];
  bA_pass<V, KC, 32, FIRST>(st, nbr, diag, lam, zz, p_old, p_new, q, n, part, lds, pt);
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
  if (threadIdx.x == 0) decide_A(st, c, tot[0], nullptr);
}

// B: x += alpha p, r -= alpha q, zz = r / diag, per-column partials r.zz, r.r.
template <typename V, int KC, bool ZX, bool GR>
__global__ __launch_bounds__(256) void k_bB(BState* __restrict__ st, const V* __restrict__ dinv,
                                            const V* __restrict__ p, const V* __restrict__ q, V* __restrict__ x,
                                            V* __restrict__ r, V* __restrict__ zz, int64_t n,
                                            double* __restrict__ part, uint64_t seed) {
  __shared__ double lds[4 * 3 * 64];
  if (st->nactive == 0) return;
  const int c = threadIdx.x % KC;
  const TileWalk tw(bf_cdiv(n, kRowsPerTile<KC>));
  double v2[2] = {0.0, 0.0};
  // first launch only (every active column starts there), as instantiations of
  // their own: ZX, x is still its (unwritten) zero start; GR, r is still the
  // (unstored) probe z
  constexpr bool first = ZX, gen = GR;
  const uint64_t cs = splitmix_out(seed, (uint64_t)c);
  if (st->active[c])
    for (int64_t tile = tw.start; tile < tw.end; tile += tw.stride)
      tile_B<V, KC>(c, (V)st->alpha[c], first, gen, cs, dinv, p, q, x, r, zz, tile * kRowsPerTile<KC>,
                    std::min<int64_t>(n, (tile + 1) * kRowsPerTile<KC>), v2[0], v2[1]);
  col_block_sum<KC, 2>(v2, lds);
  store_partials<KC, 2>(part, blockIdx.x, v2);
}

// Per-column beta or residual-check request from B's block partials.
template <int KC>
__global__ __launch_bounds__(256) void k_bscal_B(BState* __restrict__ st, const double* __restrict__ part, int nb) {
  __shared__ double lds[16];
  const int c = blockIdx.x;
  if (!st->active[c]) return;
  double tot[2];
  col_partials_sum<KC, 2>(part, nb, c, tot, lds);
  if (threadIdx.x == 0) decide_B(st, c, tot[0], tot[1], nullptr, nullptr);
}

// Mixed precision: fold the float corrections of checked columns into x64.
template <int KC>
__global__ __launch_bounds__(256) void k_bfold(const BState* __restrict__ st, int force, double* __restrict__ x64,
                                               float* __restrict__ cf, int64_t n) {
  if (!force && (st->nactive == 0 || !st->any_check)) return;
  const int c = threadIdx.x % KC;
  if (!force && !(st->active[c] && st->check[c])) return;
  const TileWalk tw(bf_cdiv(n, kRowsPerTile<KC>));
  for (int64_t tile = tw.start; tile < tw.end; tile += tw.stride)
    tile_fold<KC>(c, x64, cf, tile * kRowsPerTile<KC>, std::min<int64_t>(n, (tile + 1) * kRowsPerTile<KC>));
}

// ---------------------------------------------------------------- 7-point probe path
// Words of packed probe signs per row.
template <int KC>
constexpr int kZWords = KC > 32 ? KC / 32 : 1;

// z_c[v] from the packed signs: bit c % 32 of word c / 32 set means -1.
template <int KC>
__device__ __forceinline__ double zsign(const uint32_t* __restrict__ zb, int64_t v, int c) {
  const uint32_t w = zb[v * kZWords<KC> + (KC > 32 ? (c >> 5) : 0)];
  return ((w >> (c & 31)) & 1u) ? -1.0 : 1.0;
}

// A double from lane l ^ m of the lane's group (the permutation CTRL of a DPP
// move, applied to both halves).  Every permutation used here stays within a
// 16-lane row and a row's lanes are active together, so no lane keeps its old
// value: the move takes none (no register to clear first).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Sum of p over the first NL lanes of each group of NL (lane l's group:
// l / NL), the group's first lane's value being the one used: the quad's
// pairs (DPP quad permutations), then the other quad of 8, the other 8 of 16
// (DPP mirrors), the other 16 of 32 (an LDS swizzle with lane XOR 16) and the
// other 32 (a lane shuffle).  The estimate's one summation order over the
// column pairs of a row, in k_hutch_bits and in the VERIFY pass that forms it.
template <int NL>
__device__ __forceinline__ double row_sum(double p) {
  static_assert(NL == 1 || NL == 8 || NL == 16 || NL == 32, "groups of 1, 8, 16 or 32 lanes");
  if constexpr (NL >= 8) {
    p += dpp_move<0xB1>(p);   // quad_perm [1, 0, 3, 2]
    p += dpp_move<0x4E>(p);   // quad_perm [2, 3, 0, 1]
    p += dpp_move<0x141>(p);  // row_half_mirror: lane 7 - l of 8
  }
  if constexpr (NL >= 16) p += dpp_move<0x140>(p);  // row_mirror: lane 15 - l of 16
  if constexpr (NL >= 32)
    p += __hiloint2double(__builtin_amdgcn_ds_swizzle(__double2hiint(p), 0x401F),
                          __builtin_amdgcn_ds_swizzle(__double2loint(p), 0x401F));
  return p;
}

// Element (u, c) of the FP64 part of a mixed-precision 7-point solve (see
// BState::xbase): stored at xc[u * KC], or the warm start +-w[u] by probe c's
// sign bit (bit sh of packed word wd), or zero.
template <int KC>
__device__ __forceinline__ double x_base(int xb, const double* __restrict__ xc, const double* __restrict__ w,
                                         const uint32_t* __restrict__ zb, uint32_t u, int sh, int wd) {
  if (xb == 0) return xc[u * (uint32_t)KC];
  if (xb == 1) return ((zb[(size_t)u * kZWords<KC> + wd] >> sh) & 1u) ? -w[u] : w[u];
  return 0.0;
}

// The start of x at one element under BState::xbase kind k: the stored x64
// value, the warm start +-w by the probe's sign, or zero.  sgn holds the sign
// in bit 31 (the rest zero), so the negation is one XOR on the high word;
// wp[wi] is read only for k == 1 (w is null without a warm start).
__device__ __forceinline__ double xbase_at(int k, const double* __restrict__ xc, uint32_t e, uint32_t sgn,
                                           const double* __restrict__ wp, uint32_t wi) {
  if (k == 0) return xc[e];
  if (k == 1) {
    const double v = wp[wi];
    return __hiloint2double(__double2hiint(v) ^ (int)sgn, __double2loint(v));
  }
  return 0.0;
}

// Bit sh of word moved to bit 31: the sign of probe sh in a packed-sign word.
__device__ __forceinline__ uint32_t sign_bit(uint32_t word, int sh) { return (word << (31 - sh)) & 0x80000000u; }

// Packs the signs of the K probes (eq. 12's Rademacher vectors, SplitMix64 as
// in the header) of every row: one hash per (row, column), gathered with a
// wave ballot.  Columns c >= K get +1 (they never run).
template <int KC>
__global__ __launch_bounds__(256) void k_bzbits(uint64_t seed, int K, uint32_t* __restrict__ zb, int64_t n) {
  constexpr int RS = kThreads / KC;
  const int c = threadIdx.x % KC;
  const int lane = threadIdx.x & 63;
  const uint64_t cs = splitmix_out(seed, (uint64_t)c);
  for (int64_t base = (int64_t)blockIdx.x * RS; base < n; base += (int64_t)gridDim.x * RS) {
    const int64_t v = base + threadIdx.x / KC;  // the rows of a wave are whole (KC divides 64)
    const bool neg = v < n && c < K && (splitmix_out(cs, (uint64_t)v) >> 63) != 0;
    const unsigned long long m = __ballot(neg);
    if (v >= n) continue;
    const unsigned long long row = m >> (lane - c);
    if constexpr (KC == 64) {
      if (c < 2) zb[v * 2 + c] = (uint32_t)(row >> (32 * c));
    } else {
      if (c == 0) zb[v] = (uint32_t)(row & ((1ull << KC) - 1ull));
    }
  }
}

// Warm start of the probe columns, x = exp(logvar) z / diag: one weight
// w = exp(logvar) / diag per row.  For z = +-1, (exp z) / diag and z (exp /
// diag) are the same double, so x = +-w.
__global__ __launch_bounds__(256) void k_bweight(const float* __restrict__ logvar, const double* __restrict__ diag,
                                                 double* __restrict__ w, int64_t n) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    w[v] = exp((double)logvar[v]) / diag[v];
}

// Per-row data of one tile of R rows, staged in LDS by R threads so that the
// KC column threads of a row read it as LDS broadcasts instead of each
// loading it (row-uniform loads from every column lane had made the L1
// request rate the limit of these passes).  nb: the 6 neighbours (-1: absent);
// zs: the row's packed-sign word of the thread's 32-column group; d, di: diag,
// 1/diag.
template <typename V, int KC, int R>
struct RowTile {
  int32_t nb[6][R];
  uint32_t zs[kZWords<KC>][R];
  double d[R];
  V di[R];
  __device__ void stage(const int32_t* __restrict__ nbr, const double* __restrict__ diag, const V* __restrict__ dinv,
                        const uint32_t* __restrict__ zb, int64_t r0, int64_t r1) {
    for (int t = threadIdx.x; t < R; t += kThreads) {
      const int64_t v = r0 + t < r1 ? r0 + t : r0;
      int32_t nv[6];
      load_nbr6(nbr, v, nv);
#pragma unroll
      for (int a = 0; a < 6; ++a) nb[a][t] = r0 + t < r1 ? nv[a] : -1;
#pragma unroll
      for (int wd = 0; wd < kZWords<KC>; ++wd) zs[wd][t] = zb[v * kZWords<KC> + wd];
      d[t] = diag[v];
      di[t] = dinv[v];
    }
  }
};

// INIT from the warm start: x = +-w is written, and r = z - Q x is formed
// from the neighbours' weights and packed signs (per row, staged in LDS with
// the rest of the tile's row data) instead of gathering x back from memory.
// The sums and stores are those of k_bres INIT with x gathered.
template <typename V, int KC>
__global__ __launch_bounds__(256) void k_bstart_res(BState* __restrict__ st, const int32_t* __restrict__ nbr,
                                                    const double* __restrict__ diag, double lam,
                                                    const uint32_t* __restrict__ zb, const double* __restrict__ w,
                                                    double* __restrict__ x64, const V* __restrict__ dinv,
                                                    V* __restrict__ r, V* __restrict__ zz, int64_t n,
                                                    double* __restrict__ part, int store_x) {
  // one column: every lane is its own row, so the row data is read directly;
  // otherwise one row per thread is staged (as in k_bres)
  constexpr bool kStage = KC > 1;
  constexpr int R = kStage ? kThreads : kRowsPerTile<KC>;
  constexpr int RT = kStage ? R : 1;
  __shared__ double lds[4 * 3 * 64];
  __shared__ RowTile<V, KC, RT> rt;
  __shared__ double wn[7][RT];                 // weights of the row (0) and its neighbours (1..6)
  __shared__ uint32_t zn[7][kZWords<KC>][RT];  // their packed signs
  const TileWalk tw(bf_cdiv(n, R));
  if constexpr (!kStage) {
    double v3[3] = {0.0, 0.0, 0.0};
    if (st->active[0] != 0)
      for (int64_t v = blockIdx.x * (int64_t)kThreads + threadIdx.x; v < n; v += (int64_t)gridDim.x * kThreads) {
        const bool neg = zb[v] & 1u;
        const double zv = neg ? -1.0 : 1.0;
        const double xs = neg ? -w[v] : w[v];
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < 6; ++a) {
          const int32_t u = nbr[v * 6 + a];
          if (u >= 0) acc += (zb[u] & 1u) ? -w[u] : w[u];
        }
        const double res = zv - (diag[v] * xs - lam * acc);
        if (store_x) x64[v] = xs;
        v3[0] += res * res;
        v3[2] += zv * zv;
        const V rv = (V)res;
        const V zzv = rv * dinv[v];
        r[v] = rv;
        zz[v] = zzv;
        v3[1] += (double)rv * (double)zzv;
      }
    col_block_sum<KC, 3>(v3, lds);
    store_partials<KC, 3>(part, blockIdx.x, v3);
    return;
  }
  // a thread takes the column pair cc, cc + 1 of its rows (their bits sh,
  // sh + 1 of the same packed-sign word), so a row's staged data serves both
  constexpr int KH = KC > 1 ? KC / 2 : 1, RS2 = kThreads / KH;
  const int cc = 2 * (threadIdx.x % KH);
  const int sh = cc & 31, wd = KC > 32 ? (cc >> 5) : 0;
  const bool any = st->active[cc] != 0 || st->active[cc + 1] != 0;
  double v[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  for (int64_t tile = tw.start; tile < tw.end; tile += tw.stride) {
    const int64_t r0 = tile * R, r1 = std::min<int64_t>(n, r0 + R);
    __syncthreads();  // the previous tile's readers are done
    rt.stage(nbr, diag, dinv, zb, r0, r1);
    for (int t = threadIdx.x; t < R; t += kThreads) {
      const int64_t v = r0 + t < r1 ? r0 + t : r0;
      wn[0][t] = w[v];
#pragma unroll
      for (int g = 0; g < kZWords<KC>; ++g) zn[0][g][t] = zb[v * kZWords<KC> + g];
#pragma unroll
      for (int a = 0; a < 6; ++a) {  // an absent neighbour reads the row itself (its term is not added)
        const int32_t u0 = rt.nb[a][t];  // staged by this thread just above
        const int64_t u = u0 >= 0 ? (int64_t)u0 : v;
        wn[1 + a][t] = w[u];
#pragma unroll
        for (int g = 0; g < kZWords<KC>; ++g) zn[1 + a][g][t] = zb[u * kZWords<KC> + g];
      }
    }
    __syncthreads();
    if (!any) continue;
    for (int j = threadIdx.x / KH; j < R && r0 + j < r1; j += RS2) {
      const int64_t e = (r0 + j) * KC + cc;
      const uint32_t zw = zn[0][wd][j];
      double zv[2], xs[2], acc[2] = {0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        zv[q] = ((zw >> (sh + q)) & 1u) ? -1.0 : 1.0;
        xs[q] = xbase_at(1, nullptr, 0u, sign_bit(zw, sh + q), wn[0], (uint32_t)j);
      }
      // no branch per neighbour: an absent one adds +0.0, which leaves the sum
      // unchanged (a sum of nonzero terms that starts at +0.0 is never -0.0)
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        const double m = rt.nb[a][j] >= 0 ? 1.0 : 0.0;  // (as in bverify_rows)
        const uint32_t zw1 = zn[1 + a][wd][j];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const double t = xbase_at(1, nullptr, 0u, sign_bit(zw1, sh + q), wn[1 + a], (uint32_t)j);
          acc[q] = fma(t, m, acc[q]);
        }
      }
      V rv[2], zzv[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const double res = zv[q] - (rt.d[j] * xs[q] - lam * acc[q]);
        v[q][0] += res * res;
        v[q][2] += zv[q] * zv[q];
        rv[q] = (V)res;
        zzv[q] = rv[q] * rt.di[j];
        v[q][1] += (double)rv[q] * (double)zzv[q];
      }
      if (store_x) *reinterpret_cast<double2*>(x64 + e) = make_double2(xs[0], xs[1]);
      if constexpr (sizeof(V) == 4) {
        *reinterpret_cast<float2*>(r + e) = make_float2(rv[0], rv[1]);
        *reinterpret_cast<float2*>(zz + e) = make_float2(zzv[0], zzv[1]);
      } else {
        *reinterpret_cast<double2*>(r + e) = make_double2(rv[0], rv[1]);
        *reinterpret_cast<double2*>(zz + e) = make_double2(zzv[0], zzv[1]);
      }
    }
  }
  // per-column totals, the pair's two columns in turn
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    col_block_sum<KH, 3>(v[q], lds);
    if (threadIdx.x < KH)
#pragma unroll
      for (int i = 0; i < 3; ++i) part[((size_t)blockIdx.x * 3 + i) * KC + 2 * threadIdx.x + q] = v[q][i];
  }
}

// The rows of one tile of k_bres (see there).  XBK: the start kind of x in
// mixed precision when it is the same for every column of the wave (then the
// choice is made at compile time), or -1 (each lane reads its column's).
template <typename V, int KC, int MODE, bool GATHER, bool XC, int XBK, int R, int RT, int RW>
__device__ __forceinline__ void bres_rows(int c, int xbl, const RowTile<V, KC, RT>& rt, const double (&wn)[7][RW],
                                          const uint32_t (&zn)[7][kZWords<KC>][RW],
                                          const int32_t* __restrict__ nbr, const double* __restrict__ diag,
                                          double lam, const uint32_t* __restrict__ zb, double* __restrict__ x64,
                                          const float* __restrict__ cf, const double* __restrict__ w,
                                          const V* __restrict__ dinv, V* __restrict__ r, V* __restrict__ zz,
                                          int64_t r0, int64_t r1, int write_x0, int store_r, double (&v3)[3]) {
  constexpr bool kStage = KC > 1;
  constexpr bool kStageW = XC && kStage;
  constexpr int RS = kThreads / KC;
  const int sh = c & 31, wd = KC > 32 ? (c >> 5) : 0;
  // element (u, c) at xc[u * KC] with u * KC < 2^32 (checked by the host)
  const double* xc = x64 + c;
  const float* cc = XC ? cf + c : nullptr;
  // two rows in flight: their gathers are issued before they are summed
  for (int j0 = threadIdx.x / KC; j0 < R && r0 + j0 < r1; j0 += 2 * RS) {
    int jr[2];
    int32_t nb[2][6];
    double dg[2];
    V di[2];
    uint32_t zw[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      jr[h] = (j0 + h * RS < R && r0 + j0 + h * RS < r1) ? j0 + h * RS : j0;
      const int64_t v = r0 + jr[h];
      if constexpr (kStage) {
#pragma unroll
        for (int a = 0; a < 6; ++a) nb[h][a] = rt.nb[a][jr[h]];
        zw[h] = rt.zs[wd][jr[h]];
        dg[h] = rt.d[jr[h]];
        di[h] = rt.di[jr[h]];
      } else {
#pragma unroll
        for (int a = 0; a < 6; ++a) nb[h][a] = nbr[v * 6 + a];
        zw[h] = zb[v * kZWords<KC> + wd];
        dg[h] = diag[v];
        di[h] = dinv[v];
      }
    }
    double res[2], zv[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      zv[h] = ((zw[h] >> sh) & 1u) ? -1.0 : 1.0;
      res[h] = zv[h];
    }
    if constexpr (GATHER) {
      const int k = XBK >= 0 ? XBK : xbl;
      double xs[2], xn[2][6];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t vs = (uint32_t)(r0 + jr[h]), es = vs * (uint32_t)KC;
        if constexpr (XC) {
          const uint32_t sg = sign_bit(zw[h], sh);
          xs[h] = (kStageW ? xbase_at(k, xc, es, sg, wn[0], (uint32_t)jr[h]) : xbase_at(k, xc, es, sg, w, vs)) +
                  (double)cc[es];
        } else {
          xs[h] = xc[es];
        }
#pragma unroll
        for (int a = 0; a < 6; ++a) {  // an absent neighbour reads the row itself and adds nothing
          const uint32_t vu = (uint32_t)(nb[h][a] >= 0 ? nb[h][a] : (int32_t)vs), u = vu * (uint32_t)KC;
          if constexpr (kStageW) {
            xn[h][a] = xbase_at(k, xc, u, sign_bit(zn[1 + a][wd][jr[h]], sh), wn[1 + a], (uint32_t)jr[h]) +
                       (double)cc[u];
          } else {
            xn[h][a] = XC ? x_base<KC>(k, xc, w, zb, vu, sh, wd) + (double)cc[u] : xc[u];
          }
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < 6; ++a)
          acc = fma(xn[h][a], nb[h][a] >= 0 ? 1.0 : 0.0, acc);  // an absent neighbour adds +-0.0
        res[h] = zv[h] - (dg[h] * xs[h] - lam * acc);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 1 && jr[1] == j0) break;  // no second row
      const int64_t e = (r0 + jr[h]) * KC + c;
      if constexpr (!GATHER)
        if (write_x0) x64[e] = 0.0;
      v3[0] += res[h] * res[h];
      v3[2] += zv[h] * zv[h];
      const V rv = (V)res[h];
      if constexpr (MODE == MODE_VERIFY) {
        v3[1] += (double)rv * (double)(rv * di[h]);
      } else {
        const V zzv = rv * di[h];
        if (store_r) r[e] = rv;
        zz[e] = zzv;
        v3[1] += (double)rv * (double)zzv;
      }
    }
  }
}

// FP64 residual r = z - Q x of the selected columns (one pass over the band):
//   INIT   every active column; GATHER: x from x64 (a supplied start), else
//          x = 0 (written to x64 when write_x0);
//   GUARD  the columns whose supplied start was dropped, from x = 0;
//   VERIFY the columns whose recurrence residual met the tolerance (check ==
//          2), norms only;
//   CHECK  the columns that continue or restart from it (check == 1).
// XC (mixed precision, VERIFY): x = x64 + the float correction cf, the value a
// fold would store, without storing it; x64 per BState::xbase (w: the start
// weights).  Sums: r.r, r.zz (stored precision),
// z.z.  kRowsInFlight rows' gathers are issued before they are summed.
template <typename V, int KC, int MODE, bool GATHER, bool XC>
__global__ __launch_bounds__(256) void k_bres(BState* __restrict__ st, const int32_t* __restrict__ nbr,
                                              const double* __restrict__ diag, double lam,
                                              const uint32_t* __restrict__ zb, double* __restrict__ x64,
                                              const float* __restrict__ cf, const double* __restrict__ w,
                                              const V* __restrict__ dinv, V* __restrict__ r, V* __restrict__ zz,
                                              int64_t n, double* __restrict__ part, int write_x0, int store_r) {
  // one column: every lane is its own row and nothing is shared, so the row
  // data is read directly; otherwise it is staged per tile in LDS, one row per
  // thread (a dependent chain of loads: neighbour indices, then the
  // neighbours' start weights and signs), amortised over the tile's rows
  constexpr bool kStage = KC > 1;
  constexpr int R = kStage ? kThreads : kRowsPerTile<KC>;
  constexpr int RT = kStage ? R : 1;
  // mixed VERIFY from a warm start: the start weights and packed signs of each
  // row and its neighbours are staged with the row data, so a column lane
  // regenerates +-w from LDS and gathers only its float correction
  constexpr bool kStageW = XC && kStage;
  constexpr int RW = kStageW ? R : 1;
  __shared__ double lds[4 * 3 * 64];
  __shared__ RowTile<V, KC, RT> rt;
  __shared__ double wn[7][RW];
  __shared__ uint32_t zn[7][kZWords<KC>][RW];
  if constexpr (MODE == MODE_CHECK || MODE == MODE_VERIFY)
    if (st->nactive == 0 || !st->any_check) return;
  if constexpr (MODE == MODE_CHECK)
    if (st->pending == 0) return;
  if constexpr (MODE == MODE_GUARD)
    if (st->ndropped == 0) return;
  const int c = threadIdx.x % KC;
  bool act;
  if constexpr (MODE == MODE_GUARD) act = st->dropped[c] != 0;
  else if constexpr (MODE == MODE_INIT) act = st->active[c] != 0;
  else act = st->active[c] != 0 && st->check[c] == (MODE == MODE_VERIFY ? 2 : 1);
  const TileWalk tw(bf_cdiv(n, R));
  // the start kind of x per column, and the wave's common one (-1: they
  // differ), a scalar that selects the rows' code once per tile
  const int xbl = XC ? st->xbase[c] : 0;
  const int xbf = __builtin_amdgcn_readfirstlane(xbl);
  const int xbw = __builtin_amdgcn_readfirstlane(__ballot(act && xbl != xbf) == 0 ? xbf : -1);
  double v3[3] = {0.0, 0.0, 0.0};
  for (int64_t tile = tw.start; tile < tw.end; tile += tw.stride) {
    const int64_t r0 = tile * R, r1 = std::min<int64_t>(n, r0 + R);
    if constexpr (kStage) {
      __syncthreads();  // the previous tile's readers are done
      rt.stage(nbr, diag, dinv, zb, r0, r1);
      if constexpr (kStageW)
        if (w)
          for (int t = threadIdx.x; t < R; t += kThreads) {
            const int64_t v = r0 + t < r1 ? r0 + t : r0;
            wn[0][t] = w[v];
#pragma unroll
            for (int a = 0; a < 6; ++a) {  // an absent neighbour stages the row itself (never added)
              const int32_t u0 = rt.nb[a][t];  // staged by this thread just above
              const int64_t u = u0 >= 0 ? (int64_t)u0 : v;
              wn[1 + a][t] = w[u];
#pragma unroll
              for (int g = 0; g < kZWords<KC>; ++g) zn[1 + a][g][t] = zb[u * kZWords<KC> + g];
            }
          }
      __syncthreads();
    }
    if (!act) continue;
#define BF_BRES_ROWS(K)                                                                                        \
  bres_rows<V, KC, MODE, GATHER, XC, K, R, RT, RW>(c, xbl, rt, wn, zn, nbr, diag, lam, zb, x64, cf, w, dinv, r, \
                                                    zz, r0, r1, write_x0, store_r, v3)
    if constexpr (XC && GATHER) {
      if (xbw == 1) BF_BRES_ROWS(1);
      else if (xbw == 0) BF_BRES_ROWS(0);
      else if (xbw == 2) BF_BRES_ROWS(2);
      else BF_BRES_ROWS(-1);
    } else {
      BF_BRES_ROWS(0);
    }
#undef BF_BRES_ROWS
  }
  col_block_sum<KC, 3>(v3, lds);
  store_partials<KC, 3>(part, blockIdx.x, v3);
}

// The rows of one tile of k_bverify2 (see there) for the start kind XBK of
// every column of the wave, or -1 (each column's own, xbl).  One row at a
// time: with two columns per thread, its gathers are as many as two rows'
// were with one.
template <int KC, int XBK>
__device__ __forceinline__ void bverify_rows(int cc, const int (&xbl)[2], const RowTile<float, KC, kThreads>& rt,
                                             const double (&wn)[7][kThreads],
                                             const uint32_t (&zn)[7][kZWords<KC>][kThreads], double lam,
                                             const double* __restrict__ x64, const float* __restrict__ cf,
                                             int64_t r0, int64_t r1, double (&v)[2][3],
                                             double* __restrict__ s_out) {
  constexpr int KH = KC / 2;
  constexpr int R = kThreads, RS = kThreads / KH;
  const int sh = cc & 31, wd = KC > 32 ? (cc >> 5) : 0;  // cc + 1: bit sh + 1 of the same word
  for (int j = threadIdx.x / KH; j < R && r0 + j < r1; j += RS) {
    double xs[2], xn[6][2], zv[2];
    const uint32_t vs = (uint32_t)(r0 + j), es = vs * (uint32_t)KC + (uint32_t)cc;
    const uint32_t zw = rt.zs[wd][j];
    const float2 co = *reinterpret_cast<const float2*>(cf + es);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int k = XBK >= 0 ? XBK : xbl[q];
      zv[q] = ((zw >> (sh + q)) & 1u) ? -1.0 : 1.0;
      xs[q] = xbase_at(k, x64 + q, es, sign_bit(zw, sh + q), wn[0], (uint32_t)j) + (double)(q ? co.y : co.x);
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) {  // an absent neighbour reads the row itself and adds nothing
      const int32_t u0 = rt.nb[a][j];
      const uint32_t u = (uint32_t)(u0 >= 0 ? u0 : (int32_t)vs) * (uint32_t)KC + (uint32_t)cc;
      const float2 cn = *reinterpret_cast<const float2*>(cf + u);
      const uint32_t zw1 = zn[1 + a][wd][j];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = XBK >= 0 ? XBK : xbl[q];
        xn[a][q] = xbase_at(k, x64 + q, u, sign_bit(zw1, sh + q), wn[1 + a], (uint32_t)j) + (double)(q ? cn.y : cn.x);
      }
    }
    const double dg = rt.d[j];
    const float di = rt.di[j];
    // an absent neighbour's term times 0.0: x is finite, so it adds +-0.0,
    // which leaves the sum unchanged (one fma per column instead of a select)
    double m[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) m[a] = rt.nb[a][j] >= 0 ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < 6; ++a) acc = fma(xn[a][q], m[a], acc);
      const double res = zv[q] - (dg * xs[q] - lam * acc);
      v[q][0] += res * res;
      v[q][2] += zv[q] * zv[q];
      const float rv = (float)res;
      v[q][1] += (double)rv * (double)(rv * di);
    }
    if (s_out) {  // the estimate's row, as k_hutch_bits forms it (a row's lanes agree on j)
      double p = zv[0] * xs[0];
      p += zv[1] * xs[1];
      const double sum = row_sum<KH>(p);
      if (cc == 0) s_out[r0 + j] = sum / (double)KC;
    }
  }
}

// VERIFY of the mixed-precision 7-point solve over column pairs: the FP64
// residual norms of the columns whose recurrence residual met the tolerance
// (check == 2), x = x64 (per BState::xbase) + the float correction cf, as
// k_bres VERIFY computes them column by column; a thread takes the columns
// cc, cc + 1 of its rows, so a row's staged data, neighbour indices and
// addresses serve both.  When every column is verified here (K = KC, all at
// check 2: they met the tolerance at the same iteration), the pass also forms
// the estimate s from the x it reads; it is final unless a column fails the
// check (BState::s_fused).
template <int KC>
__device__ __forceinline__ void bverify_pass(BState* __restrict__ st, const int32_t* __restrict__ nbr,
                                             const double* __restrict__ diag, double lam,
                                             const uint32_t* __restrict__ zb, const double* __restrict__ x64,
                                             const float* __restrict__ cf, const double* __restrict__ w,
                                             const float* __restrict__ dinv, int64_t n, double* __restrict__ part,
                                             double* __restrict__ s_fuse) {
  static_assert(KC >= 16, "column pairs of a 16- to 64-column block");
  constexpr int KH = KC / 2;
  constexpr int R = kThreads;
  __shared__ double lds[4 * 3 * 64];
  __shared__ RowTile<float, KC, R> rt;
  __shared__ double wn[7][R];
  __shared__ uint32_t zn[7][kZWords<KC>][R];
  if (st->nactive == 0 || !st->any_check) return;
  const int cc = 2 * (threadIdx.x % KH);
  bool act[2];
  int xbl[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    act[q] = st->active[cc + q] != 0 && st->check[cc + q] == 2;
    xbl[q] = st->xbase[cc + q];
  }
  const bool any = act[0] || act[1];
  // the start kind shared by every active column of the wave (-1: they differ)
  const int xbf = __builtin_amdgcn_readfirstlane(xbl[0]);
  const int xbw = __builtin_amdgcn_readfirstlane(
      __ballot((act[0] && xbl[0] != xbf) || (act[1] && xbl[1] != xbf)) == 0 ? xbf : -1);
  double* s_out = nullptr;
  if (s_fuse && st->K == KC) {
    bool all = true;
    for (int k = 0; k < KC; ++k) all = all && st->active[k] && st->check[k] == 2;
    if (all) {
      s_out = s_fuse;
      if (blockIdx.x == 0 && threadIdx.x == 0) st->s_fused = 1;
    }
  }
  const TileWalk tw(bf_cdiv(n, R));
  double v[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  for (int64_t tile = tw.start; tile < tw.end; tile += tw.stride) {
    const int64_t r0 = tile * R, r1 = std::min<int64_t>(n, r0 + R);
    __syncthreads();  // the previous tile's readers are done
    rt.stage(nbr, diag, dinv, zb, r0, r1);
    if (w)
      for (int t = threadIdx.x; t < R; t += kThreads) {
        const int64_t vv = r0 + t < r1 ? r0 + t : r0;
        wn[0][t] = w[vv];
#pragma unroll
        for (int a = 0; a < 6; ++a) {  // an absent neighbour stages the row itself (never added)
          const int32_t u0 = rt.nb[a][t];  // staged by this thread just above
          const int64_t u = u0 >= 0 ? (int64_t)u0 : vv;
          wn[1 + a][t] = w[u];
#pragma unroll
          for (int g = 0; g < kZWords<KC>; ++g) zn[1 + a][g][t] = zb[u * kZWords<KC> + g];
        }
      }
    __syncthreads();
    if (!any) continue;
    if (xbw == 1) bverify_rows<KC, 1>(cc, xbl, rt, wn, zn, lam, x64, cf, r0, r1, v, s_out);
    else if (xbw == 0) bverify_rows<KC, 0>(cc, xbl, rt, wn, zn, lam, x64, cf, r0, r1, v, s_out);
    else if (xbw == 2) bverify_rows<KC, 2>(cc, xbl, rt, wn, zn, lam, x64, cf, r0, r1, v, s_out);
    else bverify_rows<KC, -1>(cc, xbl, rt, wn, zn, lam, x64, cf, r0, r1, v, s_out);
  }
  // per-column totals, the pair's two columns in turn
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    col_block_sum<KH, 3>(v[q], lds);
    if (threadIdx.x < KH)
#pragma unroll
      for (int i = 0; i < 3; ++i) part[((size_t)blockIdx.x * 3 + i) * KC + 2 * threadIdx.x + q] = v[q][i];
  }
}

// 16 and 32 columns: the register budget of four waves per SIMD, which their
// LDS allows (faster than the compiler's choice of three).
template <int KC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_bverify2(
    BState* __restrict__ st, const int32_t* __restrict__ nbr, const double* __restrict__ diag, double lam,
    const uint32_t* __restrict__ zb, const double* __restrict__ x64, const float* __restrict__ cf,
    const double* __restrict__ w, const float* __restrict__ dinv, int64_t n, double* __restrict__ part,
    double* __restrict__ s_fuse) {
  bverify_pass<KC>(st, nbr, diag, lam, zb, x64, cf, w, dinv, n, part, s_fuse);
}
// 64 columns: twice the packed-sign words in LDS, at most three workgroups per CU
__global__ __launch_bounds__(256) void k_bverify2_64(BState* __restrict__ st, const int32_t* __restrict__ nbr,
                                                     const double* __restrict__ diag, double lam,
                                                     const uint32_t* __restrict__ zb, const double* __restrict__ x64,
                                                     const float* __restrict__ cf, const double* __restrict__ w,
                                                     const float* __restrict__ dinv, int64_t n,
                                                     double* __restrict__ part, double* __restrict__ s_fuse) {
  bverify_pass<64>(st, nbr, diag, lam, zb, x64, cf, w, dinv, n, part, s_fuse);
}

// B of the 7-point path's first iteration from x = 0 with r = z unstored:
// x = alpha p, r = z - alpha q (z from the packed signs), zz = r / diag.
template <typename V, int KC>
__global__ __launch_bounds__(256) void k_bB_gen(BState* __restrict__ st, const V* __restrict__ dinv,
                                                const V* __restrict__ p, const V* __restrict__ q, V* __restrict__ x,
                                                V* __restrict__ r, V* __restrict__ zz, int64_t n,
                                                double* __restrict__ part, const uint32_t* __restrict__ zb) {
  __shared__ double lds[4 * 3 * 64];
  if (st->nactive == 0) return;
  constexpr int RS = kThreads / KC;
  const int c = threadIdx.x % KC;
  const TileWalk tw(bf_cdiv(n, kRowsPerTile<KC>));
  double v2[2] = {0.0, 0.0};
  if (st->active[c]) {
    const V alpha = (V)st->alpha[c];
    for (int64_t tile = tw.start; tile < tw.end; tile += tw.stride) {
      const int64_t r0 = tile * kRowsPerTile<KC>, r1 = std::min<int64_t>(n, r0 + kRowsPerTile<KC>);
      for (int64_t v = r0 + threadIdx.x / KC; v < r1; v += RS) {
        const int64_t e = v * KC + c;
        x[e] = (V)0 + alpha * p[e];
        const V rv = (V)zsign<KC>(zb, v, c) - alpha * q[e];
        const V zv = rv * dinv[v];
        r[e] = rv;
        zz[e] = zv;
        v2[0] += (double)rv * (double)zv;
        v2[1] += (double)rv * (double)rv;
      }
    }
  }
  col_block_sum<KC, 2>(v2, lds);
  store_partials<KC, 2>(part, blockIdx.x, v2);
}

// Mixed precision, 7-point path: fold the float correction of the columns
// that go on from a stored FP64 residual (check == 1) into x64, storing x64
// (x64 = base + cf, cf = 0; the base per BState::xbase, w: the start weights).
template <int KC>
__global__ __launch_bounds__(256) void k_bfold_check(const BState* __restrict__ st, double* __restrict__ x64,
                                                     float* __restrict__ cf, const double* __restrict__ w,
                                                     const uint32_t* __restrict__ zb, int64_t n) {
  if (st->nactive == 0 || st->pending == 0) return;
  constexpr int RS = kThreads / KC;
  const int c = threadIdx.x % KC;
  if (!(st->active[c] && st->check[c] == 1)) return;
  const int xb = st->xbase[c], sh = c & 31, wd = KC > 32 ? (c >> 5) : 0;
  const TileWalk tw(bf_cdiv(n, kRowsPerTile<KC>));
  for (int64_t tile = tw.start; tile < tw.end; tile += tw.stride) {
    const int64_t r1 = std::min<int64_t>(n, (tile + 1) * kRowsPerTile<KC>);
    for (int64_t v = tile * kRowsPerTile<KC> + threadIdx.x / KC; v < r1; v += RS) {
      const int64_t e = v * KC + c;
      x64[e] = x_base<KC>(xb, x64 + c, w, zb, (uint32_t)v, sh, wd) + (double)cf[e];
      cf[e] = 0.0f;
    }
  }
}

// s_v = (1/K) sum_k z_k[v] u_k[v] of the 7-point path, u = x64 (+ cf, mixed
// precision: the corrections of columns that stopped after a store-free check
// are not folded).  FP64, zero_start: a column that never iterated still has
// its unwritten zero start.  Mixed: x64 per BState::xbase (w: the start
// weights), and a column that never iterated has no correction (cf unwritten).
// A thread takes the column pair (cc, cc + 1) of its rows (one column for
// KC = 1): the pair's products are added, then the row's pair sums with
// row_sum.  U rows' loads are issued before their sums.  Nothing to do when
// the last VERIFY pass formed the estimate (BState::s_fused).
template <int KC, bool XC>
__global__ __launch_bounds__(256) void k_hutch_bits(const BState* __restrict__ st, int zero_start,
                                                    const double* __restrict__ x64, const float* __restrict__ cf,
                                                    const double* __restrict__ w, const uint32_t* __restrict__ zb,
                                                    int K, int64_t n, double* __restrict__ s_out) {
  if (st->s_fused) return;
  constexpr int CP = KC > 1 ? 2 : 1;  // columns per thread
  constexpr int KH = KC / CP;
  constexpr int RS = kThreads / KH;
  constexpr int U = KC > 1 ? 8 : 4;
  const int cc = CP * (threadIdx.x % KH);
  bool in[CP], zero[CP], nocf[CP];
  int xb[CP];
#pragma unroll
  for (int h = 0; h < CP; ++h) {
    in[h] = cc + h < K;
    zero[h] = in[h] && zero_start && st->iters[cc + h] == 0;
    nocf[h] = in[h] && st->iters[cc + h] == 0;
    xb[h] = XC && in[h] ? st->xbase[cc + h] : 0;
  }
  const int wd = KC > 32 ? (cc >> 5) : 0;
  for (int64_t r0 = blockIdx.x * (int64_t)(U * RS); r0 < n; r0 += (int64_t)gridDim.x * U * RS) {
    double xv[U][CP];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t v = r0 + j * RS + threadIdx.x / KH;
#pragma unroll
      for (int h = 0; h < CP; ++h) {
        const int c = cc + h;
        const int64_t e = v * KC + c;
        if constexpr (XC)
          xv[j][h] = (v < n && in[h]) ? x_base<KC>(xb[h], x64 + c, w, zb, (uint32_t)v, c & 31, wd) +
                                            (nocf[h] ? 0.0 : (double)cf[e])
                                      : 0.0;
        else
          xv[j][h] = (v < n && in[h] && !zero[h]) ? x64[e] : 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t v = r0 + j * RS + threadIdx.x / KH;
      // the rows of a wave are whole (KH divides 64), so a row's lanes agree on v < n
      if (v < n) {
        double p = in[0] ? zsign<KC>(zb, v, cc) * xv[j][0] : 0.0;
        if constexpr (CP == 2) p += in[1] ? zsign<KC>(zb, v, cc + 1) * xv[j][1] : 0.0;
        const double acc = row_sum<KH>(p);
        if (cc == 0) s_out[v] = acc / (double)K;
      }
    }
  }
}

// Couplings and neighbour indices of rows [r0, r1) of one tile, staged in LDS
// as [26][R] from the slot-major arrays (each slot's rows are contiguous, so
// the loads are coalesced); all K column threads of a row then share them.
template <typename W, int R>
__device__ __forceinline__ void stage27(const W* __restrict__ off, const int32_t* __restrict__ nb26, int64_t n,
                                        int64_t r0, int64_t r1, W* __restrict__ soff, int32_t* __restrict__ snb) {
  for (int e = threadIdx.x; e < 26 * R; e += kThreads) {
    const int t = e / R;
    const int64_t v = r0 + (e % R);
    const bool in = v < r1;
    soff[e] = in ? off[t * n + v] : (W)0;
    snb[e] = in ? nb26[t * n + v] : -1;
  }
}

// Trilinear systems: A and the FP64 residual with the 26 stored couplings per
// row (ascending slot; slot-major [26][N], staged per tile in LDS for K > 1),
// rows of a tile spread over the workgroup as in tile_B.  An absent voxel
// reads the row itself and adds nothing.
template <typename V, int KC>
__global__ __launch_bounds__(256) void k_bA27(BState* __restrict__ st, const int32_t* __restrict__ nb26,
                                              const V* __restrict__ off, const V* __restrict__ diag,
                                              const V* __restrict__ zz, const V* __restrict__ p_old,
                                              V* __restrict__ p_new, V* __restrict__ q, int64_t n,
                                              double* __restrict__ part) {
  constexpr int R = kRowsPerTile<KC>;
  constexpr int RS = kThreads / KC;
  constexpr bool kStage = KC > 1;
  __shared__ double lds[4 * 3 * 64];
  __shared__ V soff[kStage ? 26 * R : 1];
  __shared__ int32_t snb[kStage ? 26 * R : 1];
  if (st->nactive == 0) return;
  const int c = threadIdx.x % KC;
  const TileWalk tw(bf_cdiv(n, R));
  double v1[1] = {0.0};
  const V beta = (V)st->beta[c];
  const bool act = st->active[c] != 0;
  for (int64_t tile = tw.start; tile < tw.end; tile += tw.stride) {
    const int64_t r0 = tile * R, r1 = std::min<int64_t>(n, r0 + R);
    if constexpr (kStage) {
      __syncthreads();  // the previous tile's readers are done
      stage27<V, R>(off, nb26, n, r0, r1, soff, snb);
      __syncthreads();
    }
    if (!act) continue;
    for (int64_t v = r0 + threadIdx.x / KC; v < r1; v += RS) {
      V s = 0;
#pragma unroll
      for (int t = 0; t < 26; ++t) {
        const int32_t nbt = kStage ? snb[t * R + (v - r0)] : nb26[t * n + v];
        const V o = kStage ? soff[t * R + (v - r0)] : off[t * n + v];
        const int64_t u = nbt >= 0 ? (int64_t)nbt : v;
        const V a = zz[u * KC + c] + beta * p_old[u * KC + c];
        if (nbt >= 0) s += o * a;
      }
      const int64_t e = v * KC + c;
      const V pv = zz[e] + beta * p_old[e];
      const V qv = diag[v] * pv + s;
      p_new[e] = pv;
      q[e] = qv;
      v1[0] += (double)pv * (double)qv;
    }
  }
  col_block_sum<KC, 1>(v1, lds);
  store_partials<KC, 1>(part, blockIdx.x, v1);
}

template <typename V, int KC>
__global__ __launch_bounds__(256) void k_bresid27(BState* __restrict__ st, int mode, const int32_t* __restrict__ nb26,
                                                  const double* __restrict__ off, const double* __restrict__ diag,
                                                  uint64_t seed, double* __restrict__ x64,
                                                  const V* __restrict__ dinv, V* __restrict__ r, V* __restrict__ zz,
                                                  int64_t n, double* __restrict__ part) {
  constexpr int R = kRowsPerTile<KC>;
  constexpr int RS = kThreads / KC;
  constexpr bool kStage = KC > 1;
  __shared__ double lds[4 * 3 * 64];
  __shared__ double soff[kStage ? 26 * R : 1];
  __shared__ int32_t snb[kStage ? 26 * R : 1];
  if ((mode == MODE_CHECK || mode == MODE_VERIFY) && (st->nactive == 0 || !st->any_check)) return;
  if (mode == MODE_CHECK && st->pending == 0) return;
  const int c = threadIdx.x % KC;
  const bool act = mode == MODE_REPORT ? c < st->K
                                       : (st->active[c] != 0 &&
                                          (mode == MODE_INIT || st->check[c] == (mode == MODE_VERIFY ? 2 : 1)));
  const uint64_t cs = splitmix_out(seed, (uint64_t)c);
  const TileWalk tw(bf_cdiv(n, R));
  double v3[3] = {0.0, 0.0, 0.0};
  for (int64_t tile = tw.start; tile < tw.end; tile += tw.stride) {
    const int64_t r0 = tile * R, r1 = std::min<int64_t>(n, r0 + R);
    if constexpr (kStage) {
      if (mode != MODE_INIT) {  // uniform across the workgroup
        __syncthreads();
        stage27<double, R>(off, nb26, n, r0, r1, soff, snb);
        __syncthreads();
      }
    }
    if (!act) continue;
    for (int64_t v = r0 + threadIdx.x / KC; v < r1; v += RS) {
      const int64_t e = v * KC + c;
      const double zv = probe(cs, v);
      double res = zv;
      if (mode == MODE_INIT) {
        x64[e] = 0.0;
      } else {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < 26; ++t) {
          const int32_t nbt = kStage ? snb[t * R + (v - r0)] : nb26[t * n + v];
          const double o = kStage ? soff[t * R + (v - r0)] : off[t * n + v];
          const int64_t u = nbt >= 0 ? (int64_t)nbt : v;
          const double xu = x64[u * KC + c];
          if (nbt >= 0) s += o * xu;
        }
        res = zv - (diag[v] * x64[e] + s);
      }
      v3[0] += res * res;
      v3[2] += zv * zv;
      if (mode == MODE_VERIFY) {
        const V rv = (V)res;
        v3[1] += (double)rv * (double)(rv * dinv[v]);
      } else if (mode != MODE_REPORT) {
        const V rv = (V)res;
        const V zzv = rv * dinv[v];
        r[e] = rv;
        zz[e] = zzv;
        v3[1] += (double)rv * (double)zzv;
      }
    }
  }
  col_block_sum<KC, 3>(v3, lds);
  store_partials<KC, 3>(part, blockIdx.x, v3);
}

// Per-column decisions after an FP64 residual (one workgroup per column).
template <int KC>
__global__ __launch_bounds__(256) void k_bscal_R(BState* __restrict__ st, int mode, const double* __restrict__ part,
                                                 int nb) {
  __shared__ double lds[16];
  const int c = blockIdx.x;
  if (mode == MODE_CHECK && !(st->active[c] && st->check[c] == 1)) return;
  if (mode == MODE_VERIFY && !(st->active[c] && st->check[c] == 2)) return;
  if (mode == MODE_REPORT && c >= st->K) return;
  if (mode == MODE_INIT && !st->active[c]) return;
  if (mode == MODE_GUARD && !st->dropped[c]) return;
  double tot[3];
  col_partials_sum<KC, 3>(part, nb, c, tot, lds);
  if (threadIdx.x == 0) {
    if (mode == MODE_VERIFY)
      decide_V(st, c, tot, nullptr);
    else
      decide_R(st, c, mode, tot, nullptr);
  }
}

// s_v = (1/K) sum_k z_k[v] u_k[v].  Lanes run along the columns of a row
// (coalesced reads of the [N][KC] block), the products go through LDS, and
// one thread per row sums them in ascending k, the order of hutch_row.
template <int KC>
// zero_start: a column that never iterated still has its zero start, which
// was not written.
__global__ __launch_bounds__(256) void k_hutch_final(const BState* __restrict__ st, int zero_start,
                                                     const double* __restrict__ x64, uint64_t seed, int K,
                                                     int64_t n, double* __restrict__ s_out) {
  constexpr int RS = kThreads / KC;
  __shared__ double prod[kThreads];
  const int c = threadIdx.x % KC;
  const uint64_t cs = splitmix_out(seed, (uint64_t)c);
  const bool zero = c < K && zero_start && st->iters[c] == 0;
  for (int64_t r0 = blockIdx.x * (int64_t)RS; r0 < n; r0 += (int64_t)gridDim.x * RS) {
    const int64_t v = r0 + threadIdx.x / KC;
    prod[threadIdx.x] = (v < n && c < K) ? probe(cs, v) * (zero ? 0.0 : x64[v * KC + c]) : 0.0;
    __syncthreads();
    if (threadIdx.x < RS && r0 + threadIdx.x < n) {
      double acc = 0.0;
      for (int k = 0; k < K; ++k) acc += prod[threadIdx.x * KC + k];
      s_out[r0 + threadIdx.x] = acc / (double)K;
    }
    __syncthreads();
  }
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
  const bool tri = sys->kind == BF_SYSTEM_TRILINEAR;
  const int64_t ntiles = bf_cdiv(N, kRowsPerTile<KC>);
  // a multiple of 8 workgroups so that each XCD walks a contiguous eighth of the tiles
  const int nb = (int)bf_round8(std::min<int64_t>(ntiles, 4 * (int64_t)ctx->cu_count));
  const size_t st_bytes = (sizeof(BState) + 255) / 256 * 256;
  const size_t part_bytes = ((size_t)nb * 3 * KC * 8 + 255) / 256 * 256;
  const size_t vec = ((size_t)N * KC * sizeof(V) + 255) / 256 * 256;
  const size_t vec64 = ((size_t)N * KC * 8 + 255) / 256 * 256;
  const size_t zb_bytes = tri ? 0 : ((size_t)N * kZWords<KC> * 4 + 255) / 256 * 256;
  const size_t w_bytes = (tri || !logvar) ? 0 : ((size_t)N * 8 + 255) / 256 * 256;
  // state | partials | x64 | r zz p0 p1 q (V) | c (float, mixed) | packed probe signs (7-point)
  // | start weights (7-point, warm start)
  char* ws = nullptr;
  BF_TRY(bf_ws(ctx, bf_ctx::WS_PROBE,
               st_bytes + part_bytes + vec64 + 5 * vec + (mixed ? vec : 0) + zb_bytes + w_bytes, (void**)&ws));
  BState* st = (BState*)ws;
  double* part = (double*)(ws + st_bytes);
  double* x64 = (double*)(ws + st_bytes + part_bytes);
  V* r = (V*)((char*)x64 + vec64);
  V* zz = (V*)((char*)r + vec);
  V* p0 = (V*)((char*)zz + vec);
  V* p1 = (V*)((char*)p0 + vec);
  V* q = (V*)((char*)p1 + vec);
  float* cf = mixed ? (float*)((char*)q + vec) : nullptr;
  uint32_t* zb = tri ? nullptr : (uint32_t*)((char*)q + vec + (mixed ? vec : 0));
  double* wst = w_bytes ? (double*)((char*)zb + zb_bytes) : nullptr;
  V* xin = mixed ? (V*)cf : (V*)x64;
  const V* diagV = mixed ? (const V*)sys->diag32 : (const V*)sys->diag;
  const V* dinvV = mixed ? (const V*)sys->dinv32 : (const V*)sys->dinv;
  const V lamV = (V)sys->lambda;
  const int fb = (int)std::min<int64_t>(bf_cdiv(N * KC, 256), 8192);
  const unsigned rows_grid = (unsigned)std::min<int64_t>(bf_cdiv(N, kThreads), 8 * (int64_t)ctx->cu_count);

  // solve-time events from the context's pool (no create / destroy per call)
  hipEvent_t e0 = bf_event_get(ctx), e1 = bf_event_get(ctx);
  if (!e0 || !e1) return bf_fail(ctx, BF_ERR_HIP, "event creation failed");
  BF_HIP(ctx, hipEventRecord(e0, ctx->stream));
  // Mixed precision on the 7-point system keeps the FP64 part of each column
  // implicit until its first fold: the warm start +-w (from the weights and
  // packed signs) or zero, regenerated where it is read, so the start is never
  // written and read back; the float correction starts unwritten (the first B
  // pass takes it as 0, a column that never iterated has none).
  const bool mixed7 = mixed && !tri;
  hipLaunchKernelGGL(k_bstate_init, dim3(1), dim3(64), 0, ctx->stream, st, o->K, o->tol, o->max_iter,
                     mixed ? 1e-6 : 0.0, mixed ? bf_mixed_restart() : 0, logvar ? 1 : 0,
                     mixed7 ? (logvar ? 1 : 2) : 0);
  // FP64 from x = 0: the zero start is not written; the first B pass takes x
  // as 0 and the estimate takes a column that never iterated as 0.  (The
  // trilinear mixed path folds its float corrections into x64, which must
  // hold zeros.)
  const int zero_start = (!mixed && !logvar) ? 1 : 0;
  // ... and the initial residual r = z is not stored either: the first B pass
  // regenerates it from the probe (the 7-point system's initial pass)
  const int gen_start = (zero_start && !tri) ? 1 : 0;
  // the 27-point A reads the first p_old (all zeros); the 7-point one does not
  if (tri) hipLaunchKernelGGL(k_bfill<V>, dim3(fb), dim3(256), 0, ctx->stream, p0, N * KC, (V)0);
  if (mixed && tri) hipLaunchKernelGGL(k_bfill<float>, dim3(fb), dim3(256), 0, ctx->stream, cf, N * KC, 0.0f);
  const V* offV = mixed ? (const V*)sys->off32 : (const V*)sys->off;
  if (tri) {
    BF_LAUNCH(ctx, "block_residual", (k_bresid27<V, KC>), dim3(nb), dim3(kThreads), 0, st, (int)MODE_INIT, sys->nb26,
              sys->off, sys->diag, o->seed, x64, dinvV, r, zz, N, part);
  } else {
    BF_LAUNCH(ctx, "block_probes", k_bzbits<KC>,
              dim3((unsigned)std::min<int64_t>(bf_cdiv(N, kThreads / KC), 16 * (int64_t)ctx->cu_count)),
              dim3(kThreads), 0, o->seed, o->K, zb, N);
    if (logvar) {
      BF_LAUNCH(ctx, "block_start", k_bweight, dim3(rows_grid), dim3(kThreads), 0, logvar, sys->diag, wst, N);
      BF_LAUNCH(ctx, "block_start_res", (k_bstart_res<V, KC>), dim3(nb), dim3(kThreads), 0, st, sys->band->nbr,
                sys->diag, sys->lambda, zb, wst, x64, dinvV, r, zz, N, part, mixed7 ? 0 : 1);
    } else {
      BF_LAUNCH(ctx, "block_residual", (k_bres<V, KC, MODE_INIT, false, false>), dim3(nb), dim3(kThreads), 0, st,
                sys->band->nbr, sys->diag, sys->lambda, zb, x64, cf, wst, dinvV, r, zz, N, part,
                (zero_start || mixed7) ? 0 : 1, gen_start ? 0 : 1);
    }
  }
  BF_LAUNCH(ctx, "block_scalars", k_bscal_R<KC>, dim3(KC), dim3(256), 0, st, (int)MODE_INIT, part, nb);
  if (logvar) {  // columns whose start was no better than zero restart from x = 0
    BF_LAUNCH(ctx, "block_guard", (k_bres<V, KC, MODE_GUARD, false, false>), dim3(nb), dim3(kThreads), 0, st,
              sys->band->nbr, sys->diag, sys->lambda, zb, x64, cf, wst, dinvV, r, zz, N, part, mixed7 ? 0 : 1, 1);
    BF_LAUNCH(ctx, "block_scalars", k_bscal_R<KC>, dim3(KC), dim3(256), 0, st, (int)MODE_GUARD, part, nb);
  }
  BF_TRY(bf_launch_check(ctx, "block pcg init"));
  BState* hs = nullptr;
  BF_TRY(bf_pinned(ctx, sizeof(BState), (void**)&hs));
  // LDS per workgroup for the stencil tile (KB): 32 measured best on the 256^3 and 512^3 bands
  // (8: -12%, 16: -5%, 64: -34% at two workgroups per CU); BF_STENCIL_LDS_KB in {16, 32, 64} overrides
  const char* skb = getenv("BF_STENCIL_LDS_KB");
  const int stencil_kb = skb ? atoi(skb) : 32;
  // iterations queued before the first poll: one from the log-variance start
  // (a learned start often meets the tolerance at once), else three; then the
  // batches grow (3, 7, 14, ...)
  int it = 0, next = logvar ? 1 : 3;
  size_t fin_rec = 0;  // timing record of the last queued estimate pass (FP64)
  const unsigned hutch_grid =
      (unsigned)std::min<int64_t>(bf_cdiv(N, (KC > 1 ? 8 : 4) * (kThreads / (KC > 1 ? KC / 2 : 1))),
                                  8 * (int64_t)ctx->cu_count);
  V* pa = p0;
  V* pb = p1;
  // the buffer holding the current zz.  The 7-point path's first iteration
  // uses p_0 = zz_0 in place (its A does not copy it), so its B writes zz_1 to
  // pa's buffer, and zz_0's buffer becomes the next iteration's p_old.
  V* zc = zz;
  std::vector<size_t> iter_rec;  // timing record count at the start of each iteration
  // the 7-point estimate: u = x64 (+ the float corrections, which this path folds
  // only for columns that restart from a stored residual)
  auto hutch = [&]() {
    if (tri)
      BF_LAUNCH(ctx, "hutch_final", k_hutch_final<KC>, dim3(hutch_grid), dim3(kThreads), 0, st, zero_start, x64,
                o->seed, o->K, N, s_out);
    else if (mixed)
      BF_LAUNCH(ctx, "hutch_final", (k_hutch_bits<KC, true>), dim3(hutch_grid), dim3(kThreads), 0, st, zero_start,
                x64, cf, wst, zb, o->K, N, s_out);
    else
      BF_LAUNCH(ctx, "hutch_final", (k_hutch_bits<KC, false>), dim3(hutch_grid), dim3(kThreads), 0, st, zero_start,
                x64, cf, wst, zb, o->K, N, s_out);
  };
  for (;;) {
    const int upto = std::min(next, o->max_iter);
    for (; it < upto; ++it) {
      if (ctx->timing) iter_rec.push_back(ctx->recs.size());
      // the first iteration's A and B move fewer bytes (no p_old, x or r reads)
      // and are timed under names of their own
      if (tri) {
        BF_LAUNCH(ctx, "block_A", (k_bA27<V, KC>), dim3(nb), dim3(kThreads), 0, st, sys->nb26, offV, diagV, zz, pa,
                  pb, q, N, part);
      } else switch (stencil_kb) {
        case 16:
          if (it == 0)
            BF_LAUNCH(ctx, "block_A_first", (k_bA<V, KC, 16, true>), dim3(nb), dim3(kThreads), 0, st, sys->band->nbr,
                      diagV, lamV, zc, pa, pb, q, N, part);
          else
            BF_LAUNCH(ctx, "block_A", (k_bA<V, KC, 16, false>), dim3(nb), dim3(kThreads), 0, st, sys->band->nbr,
                      diagV, lamV, zc, pa, pb, q, N, part);
          break;
        case 64:
          if (it == 0)
            BF_LAUNCH(ctx, "block_A_first", (k_bA<V, KC, 64, true>), dim3(nb), dim3(kThreads), 0, st, sys->band->nbr,
                      diagV, lamV, zc, pa, pb, q, N, part);
          else
            BF_LAUNCH(ctx, "block_A", (k_bA<V, KC, 64, false>), dim3(nb), dim3(kThreads), 0, st, sys->band->nbr,
                      diagV, lamV, zc, pa, pb, q, N, part);
          break;
        default:
          if constexpr (KC > 1) {
            if (it == 0)
              BF_LAUNCH(ctx, "block_A_first", (k_bA4<V, KC, true>), dim3(nb), dim3(kThreads), 0, st, sys->band->nbr,
                        diagV, lamV, zc, pa, pb, q, N, part);
            else
              BF_LAUNCH(ctx, "block_A", (k_bA4<V, KC, false>), dim3(nb), dim3(kThreads), 0, st, sys->band->nbr,
                        diagV, lamV, zc, pa, pb, q, N, part);
          } else {
            if (it == 0)
              BF_LAUNCH(ctx, "block_A_first", (k_bA<V, KC, 32, true>), dim3(nb), dim3(kThreads), 0, st,
                        sys->band->nbr, diagV, lamV, zc, pa, pb, q, N, part);
            else
              BF_LAUNCH(ctx, "block_A", (k_bA<V, KC, 32, false>), dim3(nb), dim3(kThreads), 0, st, sys->band->nbr,
                        diagV, lamV, zc, pa, pb, q, N, part);
          }
      }
      BF_LAUNCH(ctx, "block_scalars", k_bscal_A<KC>, dim3(KC), dim3(256), 0, st, part, nb);
      const bool moved = it == 0 && !tri;  // p_0 in zz_0's buffer, zz_1 to pa's
      V* bp = moved ? zc : pb;
      V* bz = moved ? pa : zc;
      if (it == 0 && gen_start)
        BF_LAUNCH(ctx, "block_B_first", (k_bB_gen<V, KC>), dim3(nb), dim3(kThreads), 0, st, dinvV, bp, q, xin, r, bz,
                  N, part, (const uint32_t*)zb);
      else if (it == 0 && (zero_start || mixed7))
        BF_LAUNCH(ctx, "block_B_first", (k_bB<V, KC, true, false>), dim3(nb), dim3(kThreads), 0, st, dinvV, bp, q,
                  xin, r, bz, N, part, o->seed);
      else
        BF_LAUNCH(ctx, "block_B", (k_bB<V, KC, false, false>), dim3(nb), dim3(kThreads), 0, st, dinvV, bp, q, xin,
                  r, bz, N, part, o->seed);
      BF_LAUNCH(ctx, "block_scalars", k_bscal_B<KC>, dim3(KC), dim3(256), 0, st, part, nb);
      if (moved) {
        pa = zc;  // p_0, the next iteration's p_old
        zc = bz;
      }
      if (tri) {
        if (mixed) BF_LAUNCH(ctx, "block_fold", k_bfold<KC>, dim3(nb), dim3(kThreads), 0, st, 0, x64, cf, N);
        // columns the recurrence calls converged: FP64 residual norms without
        // stores; then the stored FP64 residual of the columns to go on from it
        for (const int mode : {(int)MODE_VERIFY, (int)MODE_CHECK}) {
          BF_LAUNCH(ctx, mode == MODE_VERIFY ? "block_verify" : "block_residual", (k_bresid27<V, KC>), dim3(nb),
                    dim3(kThreads), 0, st, mode, sys->nb26, sys->off, sys->diag, o->seed, x64, dinvV, r, zz, N, part);
          BF_LAUNCH(ctx, "block_scalars", k_bscal_R<KC>, dim3(KC), dim3(256), 0, st, mode, part, nb);
        }
      } else {
        // store-free FP64 residual norms of the columns the recurrence calls
        // converged (mixed: of x64 + the float correction, unfolded); then the
        // columns to go on from a stored FP64 residual fold (mixed) and store it
        if constexpr (sizeof(V) == 4 && KC == 64)
          BF_LAUNCH(ctx, "block_verify", k_bverify2_64, dim3(nb), dim3(kThreads), 0, st, sys->band->nbr, sys->diag,
                    sys->lambda, zb, x64, cf, wst, dinvV, N, part, s_out);
        else if constexpr (sizeof(V) == 4 && KC > 1)
          BF_LAUNCH(ctx, "block_verify", k_bverify2<KC>, dim3(nb), dim3(kThreads), 0, st, sys->band->nbr, sys->diag,
                    sys->lambda, zb, x64, cf, wst, dinvV, N, part, s_out);
        else if (mixed)
          BF_LAUNCH(ctx, "block_verify", (k_bres<V, KC, MODE_VERIFY, true, true>), dim3(nb), dim3(kThreads), 0, st,
                    sys->band->nbr, sys->diag, sys->lambda, zb, x64, cf, wst, dinvV, r, zc, N, part, 0, 0);
        else
          BF_LAUNCH(ctx, "block_verify", (k_bres<V, KC, MODE_VERIFY, true, false>), dim3(nb), dim3(kThreads), 0, st,
                    sys->band->nbr, sys->diag, sys->lambda, zb, x64, cf, wst, dinvV, r, zc, N, part, 0, 0);
        BF_LAUNCH(ctx, "block_scalars", k_bscal_R<KC>, dim3(KC), dim3(256), 0, st, (int)MODE_VERIFY, part, nb);
        if (mixed)
          BF_LAUNCH(ctx, "block_fold", k_bfold_check<KC>, dim3(nb), dim3(kThreads), 0, st, x64, cf, wst,
                    (const uint32_t*)zb, N);
        BF_LAUNCH(ctx, "block_residual", (k_bres<V, KC, MODE_CHECK, true, false>), dim3(nb), dim3(kThreads), 0, st,
                  sys->band->nbr, sys->diag, sys->lambda, zb, x64, cf, wst, dinvV, r, zc, N, part, 0, 1);
        BF_LAUNCH(ctx, "block_scalars", k_bscal_R<KC>, dim3(KC), dim3(256), 0, st, (int)MODE_CHECK, part, nb);
      }
      if (!moved) std::swap(pa, pb);
    }
    BF_TRY(bf_launch_check(ctx, "block pcg iteration"));
    // FP64: the estimate is formed behind every batch, so the poll that finds
    // every column done has it already; it reads the solutions only, and a
    // later batch's pass overwrites it.
    if (!mixed) {
      fin_rec = ctx->recs.size();
      hutch();
    }
    // the solve's end, if this poll finds it done (mixed: unless a closing pass follows)
    BF_HIP(ctx, hipEventRecord(e1, ctx->stream));
    BF_HIP(ctx, hipMemcpyAsync(hs, st, sizeof(BState), hipMemcpyDeviceToHost, ctx->stream));
    BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (hs->nactive == 0 || it >= o->max_iter) break;
    next = it < 3 ? 3 : it + std::max(it, 4);
  }
  const size_t loop_rec_end = mixed ? ctx->recs.size() : fin_rec;
  // The report's residual of each column is the FP64 one of its last check:
  // a column stops only after such a check (or at INIT, or on a breakdown),
  // and its solution does not change afterwards, so no further pass is needed.
  // timing record of the last queued estimate pass (none: mixed, until one is queued below)
  size_t hutch_rec = mixed ? SIZE_MAX : fin_rec;
  // Mixed: the estimate pass, unless every column stopped at a VERIFY pass
  // that formed it (then the last poll has the final state already)
  if (mixed && !(hs->nactive == 0 && hs->s_fused)) {
    if (tri) BF_LAUNCH(ctx, "block_fold", k_bfold<KC>, dim3(nb), dim3(kThreads), 0, st, 1, x64, cf, N);
    hutch_rec = ctx->recs.size();
    hutch();
    BF_HIP(ctx, hipEventRecord(e1, ctx->stream));
    BF_HIP(ctx, hipMemcpyAsync(hs, st, sizeof(BState), hipMemcpyDeviceToHost, ctx->stream));
    BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  ctx->pool.push_back(e0);
  ctx->pool.push_back(e1);
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
  if (ctx->timing && (size_t)maxit < iter_rec.size()) bf_timing_mark_idle(ctx, iter_rec[maxit], loop_rec_end);
  // a VERIFY pass formed the estimate: the closing estimate pass found nothing to do
  if (ctx->timing && hs->s_fused && hutch_rec != SIZE_MAX) bf_timing_mark_idle(ctx, hutch_rec, hutch_rec + 1);
  if (rep) {
    rep->iters = maxit;
    rep->status = status;
    rep->refinements = hs->refinements;
    rep->used_warm_start = (logvar && hs->ndropped == 0) ? 1 : 0;
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
  if (o->K == 1) return run_block<V, 1>(ctx, sys, o, logvar, s, rep);
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
  BF_CHECK(ctx, !(sys->kind == BF_SYSTEM_TRILINEAR && logvar_dev),
           "bf_diag_estimate: no log-variance start for trilinear systems");
  if (sys->n == 0) return BF_OK;
  BF_CHECK(ctx, s_dev, "bf_diag_estimate: NULL output");
  BF_CHECK(ctx, sys->n <= (int64_t)(0xffffffffll / 64), "bf_diag_estimate: %lld band voxels exceed the %lld a probe "
           "block indexes", (long long)sys->n, (long long)(0xffffffffll / 64));
  BF_HIP(ctx, hipSetDevice(ctx->device));
  if (opts->precision == BF_PREC_FP64) return dispatch_k<double>(ctx, sys, opts, logvar_dev, s_dev, rep);
  return dispatch_k<float>(ctx, sys, opts, logvar_dev, s_dev, rep);
}
