// Learned warm start: a per-voxel MLP 12 -> 64 -> 64 -> 64 -> 2 (SiLU) on the
// gfx950 matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32
// accumulation), its backward pass, Adam, and the warm start it feeds the
// solvers.  The paper lists learned priors as future work (Sec. 6-7); here the
// network only proposes starting points: CG to the same tolerance decides the
// answer.
//
// MFMA conventions (16x16x32, per lane l, g = l / 16, n = l % 16):
//   A (16 x 32): lane holds A[n][8g .. 8g+7];  B (32 x 16): B[8g .. 8g+7][n];
//   D (16 x 16): D[4g .. 4g+3][n].
// Layers are computed transposed, H^T = W * A^T: the MFMA M dimension is the
// layer's output units, N is 16 voxels.  A lane's D values are units
// 16*mt + 4g + j of voxel n.  Numbering the next layer's K positions by
//   kappa = 32c + 8g + e  ->  unit 16*(2c + e/4) + 4g + e%4
// makes those D registers exactly the next layer's B operand, so activations
// never move between lanes; the weights are permuted once when packed.
#include "bf_internal.h"
#include "bf_features.h"

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

namespace {

constexpr int NIN = 12, NH = 64, NOUT = 2;
constexpr int N_TRAIN = 9282;  // trainable values; 28 fixed scaling values follow
constexpr int oW1 = 0, ob1 = 768, oW2 = 832, ob2 = 4928, oW3 = 4992, ob3 = 9088, oW4 = 9152, ob4 = 9280;
constexpr int oInMean = 9282, oInStd = 9294, oOutMean = 9306, oOutStd = 9308;
// packed operand tiles (64 lanes x 8 bf16): forward L1..L4, backward W4^T, W3^T, W2^T
constexpr int T_L1 = 0, T_L2 = 4, T_L3 = 12, T_L4 = 20, T_B4 = 22, T_B3 = 26, T_B2 = 34, NTILES = 42;
constexpr int NFWD = 22;
constexpr int NBIAS = 3 * NH + NOUT;  // 194

__device__ __forceinline__ int unit_of(int kappa) {
  const int c = kappa >> 5, r = kappa & 31, g = r >> 3, e = r & 7;
  return 16 * (2 * c + (e >> 2)) + 4 * g + (e & 3);
}

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// SiLU z sigmoid(z) with the hardware base-2 exponential and reciprocal
// (about 1 ulp each in float): its value is rounded to bfloat16 (8 bits) right
// away, so the full-precision expf and division (about 25 instructions, most of
// the forward pass's issue time at 192 activations per voxel) buy nothing.
// Large |z| saturates correctly: exp2 -> inf gives 0, exp2 -> 0 gives z.
__device__ __forceinline__ float silu(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z * -1.4426950408889634f));
}
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// FP32 master parameters -> BF16 MFMA operand tiles (weights permuted as above).
__global__ __launch_bounds__(256) void k_mlp_pack(const float* __restrict__ prm, __bf16* __restrict__ wt) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= NTILES * 64 * 8) return;
  const int t = idx / 512, l = (idx / 8) % 64, e = idx % 8;
  const int n = l & 15, g = l >> 4;
  float v = 0.0f;
  if (t < T_L2) {  // layer 1: rows = units, K = raw input features
    const int m = 16 * t + n, k = 8 * g + e;
    v = k < NIN ? prm[oW1 + m * NIN + k] : 0.0f;
  } else if (t < T_L4) {  // layers 2, 3
    const int base = t < T_L3 ? oW2 : oW3;
    const int i = t - (t < T_L3 ? T_L2 : T_L3);
    const int mt = i >> 1, c = i & 1;
    const int m = 16 * mt + n, kappa = 32 * c + 8 * g + e;
    v = prm[base + m * NH + unit_of(kappa)];
  } else if (t < T_B4) {  // layer 4: rows 0, 1 real
    const int c = t - T_L4, m = n, kappa = 32 * c + 8 * g + e;
    v = m < NOUT ? prm[oW4 + m * NH + unit_of(kappa)] : 0.0f;
  } else if (t < T_B3) {  // W4^T: rows = layer-3 units, K = outputs
    const int m = 16 * (t - T_B4) + n, k = 8 * g + e;
    v = k < NOUT ? prm[oW4 + k * NH + m] : 0.0f;
  } else {  // W3^T, W2^T: rows = layer-(l-1) units, K = layer-l units (permuted)
    const int base = t < T_B2 ? oW3 : oW2;
    const int i = t - (t < T_B2 ? T_B3 : T_B2);
    const int mt = i >> 1, c = i & 1;
    const int m = 16 * mt + n, kappa = 32 * c + 8 * g + e;
    v = prm[base + unit_of(kappa) * NH + m];
  }
  wt[idx] = (__bf16)v;
}

struct lane_consts {
  float imean[8], iinv[8];
  float bias[3][16];
  float b4[2], omean[2], ostd[2];
};

__device__ __forceinline__ void load_consts(const float* __restrict__ prm, int g, lane_consts& k) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int f = 8 * g + e;
    k.imean[e] = f < NIN ? prm[oInMean + f] : 0.0f;
    k.iinv[e] = f < NIN ? 1.0f / prm[oInStd + f] : 0.0f;
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int u = 16 * mt + 4 * g + j;
      k.bias[0][mt * 4 + j] = prm[ob1 + u];
      k.bias[1][mt * 4 + j] = prm[ob2 + u];
      k.bias[2][mt * 4 + j] = prm[ob3 + u];
    }
  k.b4[0] = prm[ob4];
  k.b4[1] = prm[ob4 + 1];
  k.omean[0] = prm[oOutMean];
  k.omean[1] = prm[oOutMean + 1];
  k.ostd[0] = prm[oOutStd];
  k.ostd[1] = prm[oOutStd + 1];
}

// Standardised input features 8g..8g+7 of voxel v as a B operand.
__device__ __forceinline__ bf16x8 load_input(const float* __restrict__ feat, int64_t v, bool valid, int g,
                                             const lane_consts& k, float* xs) {
  bf16x8 b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int f = 8 * g + e;
    float x = 0.0f;
    if (valid && f < NIN) x = (feat[v * NIN + f] - k.imean[e]) * k.iinv[e];
    xs[e] = x;
    b[e] = (__bf16)x;
  }
  return b;
}

// One hidden layer's activation: D (+bias) -> SiLU -> next B operands.
__device__ __forceinline__ void activate(const f32x4 (&acc)[4], const float* bias, float (&z)[16], bf16x8 (&B)[2]) {
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float zz = acc[mt][j] + bias[mt * 4 + j];
      z[mt * 4 + j] = zz;
      B[mt >> 1][(mt & 1) * 4 + j] = (__bf16)silu(zz);
    }
}

__device__ __forceinline__ void layer(const bf16x8* __restrict__ sw, int tbase, int lane, const bf16x8 (&B)[2],
                                      f32x4 (&acc)[4]) {
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 a = {0.f, 0.f, 0.f, 0.f};
    a = mfma(sw[(tbase + mt * 2 + 0) * 64 + lane], B[0], a);
    a = mfma(sw[(tbase + mt * 2 + 1) * 64 + lane], B[1], a);
    acc[mt] = a;
  }
}

// Inference: physical outputs [n][2]; optionally the warm start
// x0 = rhs/diag + h*o0 and logvar = o1.  The weight tiles, biases and the
// input and output scalings sit in LDS (the same values load_consts gives a
// lane) and are read there in every iteration: kept in registers across the
// loop they held the kernel to two waves per SIMD, too few to overlap the
// chains of dependent MFMAs.
// FUSED: the input features are computed here from the band and the system
// (src) instead of read from feat, the values the features kernel writes:
// lanes 0-15 of a wave compute features 0-7 of their voxels, lanes 16-31
// features 8-11 (bf_features.h), the operand values those lanes hold.  (Spreading
// the features over all four lane groups and exchanging them through LDS was
// no faster: the pass waits on the feature loads, not on lanes.)
constexpr int kFeatPitch = 15;  // floats per voxel in the fused pass's LDS: 12 features, 2 outputs (odd: no bank conflicts)
template <bool FUSED>
__global__ __launch_bounds__(256) void k_mlp_forward(const bf16x8* __restrict__ wt, const float* __restrict__ prm,
                                                     const float* __restrict__ feat, bf_feat_in src, int64_t n,
                                                     float* __restrict__ out, const double* __restrict__ rhs,
                                                     const double* __restrict__ diag, double h,
                                                     double* __restrict__ x0, float* __restrict__ logvar) {
  __shared__ bf16x8 sw[NFWD * 64];
  __shared__ float sb[3 * NH], sim[16], sii[16], so[6];
  __shared__ float sfeat[FUSED ? 4 : 1][FUSED ? 64 * kFeatPitch : 1];  // per wave: 64 voxels' features
  for (int i = threadIdx.x; i < NFWD * 64; i += blockDim.x) sw[i] = wt[i];
  for (int i = threadIdx.x; i < 3 * NH; i += blockDim.x) {
    const int l = i / NH, u = i % NH;
    sb[i] = prm[(l == 0 ? ob1 : (l == 1 ? ob2 : ob3)) + u];
  }
  if (threadIdx.x < 16) {
    const int f = threadIdx.x;
    sim[f] = f < NIN ? prm[oInMean + f] : 0.0f;
    sii[f] = f < NIN ? 1.0f / prm[oInStd + f] : 0.0f;
  }
  if (threadIdx.x == 0) {
    so[0] = prm[ob4];
    so[1] = prm[ob4 + 1];
    so[2] = prm[oOutMean];
    so[3] = prm[oOutMean + 1];
    so[4] = prm[oOutStd];
    so[5] = prm[oOutStd + 1];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, col = lane & 15;
  // one 16-voxel tile: features (f(voxel, feature index)) -> network ->
  // outputs (sink(voxel, p0, p1) on the lanes of the first 16)
  auto run_tile = [&](int64_t t, auto&& feature, auto&& sink) {
    // an offset of zero the compiler cannot see through: the weight reads
    // below stay in the loop instead of being hoisted into registers
    int z0;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z0));
    const bf16x8* swl = sw + z0 + lane;
    const int64_t v = t * 16 + col;
    const bool valid = v < n;
    bf16x8 B0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int f = 8 * g + e;
      float x = 0.0f;
      if (valid && f < NIN) x = (feature(v, f) - sim[f]) * sii[f];
      B0[e] = (__bf16)x;
    }
    f32x4 acc[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 a = {0.f, 0.f, 0.f, 0.f};
      acc[mt] = mfma(swl[(T_L1 + mt) * 64], B0, a);
    }
    bf16x8 B[2];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      // D (+bias) -> SiLU -> the next B operands (see activate)
      const float* bl = sb + l * NH + 4 * g;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) B[mt >> 1][(mt & 1) * 4 + j] = (__bf16)silu(acc[mt][j] + bl[16 * mt + j]);
      if (l < 2) layer(swl - lane, l == 0 ? T_L2 : T_L3, lane, B, acc);
    }
    f32x4 o = {0.f, 0.f, 0.f, 0.f};
    o = mfma(swl[(T_L4 + 0) * 64], B[0], o);
    o = mfma(swl[(T_L4 + 1) * 64], B[1], o);
    if (g == 0 && valid) sink(v, (o[0] + so[0]) * so[4] + so[2], (o[1] + so[1]) * so[5] + so[3]);
  };
  auto write = [&](int64_t v, float p0, float p1) {
    if (out) {
      out[2 * v] = p0;
      out[2 * v + 1] = p1;
    }
    if (x0) x0[v] = rhs[v] / diag[v] + h * (double)p0;
    if (logvar) logvar[v] = p1;
  };
  if constexpr (FUSED) {
    // every lane computes all the features of one voxel of a group of 64 (the
    // four tiles a wave then runs), so the FP64 feature work uses the whole
    // wave instead of a quarter of it; they pass through the wave's LDS slice
    const int64_t ngrp = (n + 63) / 64;
    float* fs = sfeat[wave];
    for (int64_t gi = (int64_t)blockIdx.x * 4 + wave; gi < ngrp; gi += (int64_t)gridDim.x * 4) {
      float fv[NIN];
#pragma unroll
      for (int e = 0; e < NIN; ++e) fv[e] = 0.0f;
      const int64_t vl = gi * 64 + lane;
      if (vl < n) {
        bf_features_0_7(vl, src, fv);
        bf_features_8_11(vl, src, fv + 8);
      }
#pragma unroll
      for (int e = 0; e < NIN; ++e) fs[lane * kFeatPitch + e] = fv[e];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // the wave's LDS writes are done
      // the network's two outputs of each voxel go back to its LDS row, and
      // every lane then writes its own voxel's results
#pragma unroll 1
      for (int sub = 0; sub < 4; ++sub)
        run_tile(
            gi * 4 + sub, [&](int64_t v, int f) { return fs[(int)(v - gi * 64) * kFeatPitch + f]; },
            [&](int64_t v, float p0, float p1) {
              fs[(int)(v - gi * 64) * kFeatPitch + NIN] = p0;
              fs[(int)(v - gi * 64) * kFeatPitch + NIN + 1] = p1;
            });
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      if (vl < n) write(vl, fs[lane * kFeatPitch + NIN], fs[lane * kFeatPitch + NIN + 1]);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // read before the next group overwrites
    }
  } else {
    const int64_t ntile = (n + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < ntile; t += (int64_t)gridDim.x * 4)
      run_tile(t, [&](int64_t v, int f) { return feat[v * NIN + f]; }, write);
  }
}

// Training pass over one batch (rows idx[0..M) of feat/target): forward,
// loss, backward to every pre-activation gradient.  Writes the BF16 layer
// inputs A_l and pre-activation gradients dZ_l in [unit][voxel] layout for the
// weight-gradient products, plus per-wave bias-gradient and loss partials.
__global__ __launch_bounds__(256) void k_mlp_train(const bf16x8* __restrict__ wt, const float* __restrict__ prm,
                                                   const float* __restrict__ feat, const float* __restrict__ tgt,
                                                   const int32_t* __restrict__ idx, int64_t nrows, int64_t M,
                                                   int64_t Mpad,
                                                   __bf16* __restrict__ A0, __bf16* __restrict__ A1,
                                                   __bf16* __restrict__ A2, __bf16* __restrict__ A3,
                                                   __bf16* __restrict__ dZ1, __bf16* __restrict__ dZ2,
                                                   __bf16* __restrict__ dZ3, __bf16* __restrict__ dZ4,
                                                   float* __restrict__ bias_part, float* __restrict__ loss_part) {
  __shared__ bf16x8 sw[NTILES * 64];
  for (int i = threadIdx.x; i < NTILES * 64; i += blockDim.x) sw[i] = wt[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, col = lane & 15;
  lane_consts k;
  load_consts(prm, g, k);
  const float invM = 1.0f / (float)M;
  float bsum[3][16], b4sum[2] = {0.f, 0.f}, lsum = 0.f;
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int i = 0; i < 16; ++i) bsum[l][i] = 0.f;
  const int64_t ntile = Mpad / 16;
  for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < ntile; t += (int64_t)gridDim.x * 4) {
    const int64_t v = t * 16 + col;
    int64_t row = v < M ? (int64_t)idx[v] : -1;
    const bool valid = row >= 0 && row < nrows;  // out-of-range rows are skipped
    if (!valid) row = 0;
    float xs[8];
    const bf16x8 B0 = load_input(feat, row, valid, g, k, xs);
    if (g < 2)
#pragma unroll
      for (int e = 0; e < 8; ++e) A0[(8 * g + e) * Mpad + v] = B0[e];
    f32x4 acc[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 a = {0.f, 0.f, 0.f, 0.f};
      acc[mt] = mfma(sw[(T_L1 + mt) * 64 + lane], B0, a);
    }
    float z1[16], z2[16], z3[16];
    bf16x8 B1[2], B2[2], B3[2];
    activate(acc, k.bias[0], z1, B1);
    layer(sw, T_L2, lane, B1, acc);
    activate(acc, k.bias[1], z2, B2);
    layer(sw, T_L3, lane, B2, acc);
    activate(acc, k.bias[2], z3, B3);
    f32x4 o = {0.f, 0.f, 0.f, 0.f};
    o = mfma(sw[(T_L4 + 0) * 64 + lane], B3[0], o);
    o = mfma(sw[(T_L4 + 1) * 64 + lane], B3[1], o);
    // store the BF16 layer inputs A1..A3 (units 16mt + 4g + j, voxel v)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int u = 16 * mt + 4 * g + j;
        A1[u * Mpad + v] = B1[mt >> 1][(mt & 1) * 4 + j];
        A2[u * Mpad + v] = B2[mt >> 1][(mt & 1) * 4 + j];
        A3[u * Mpad + v] = B3[mt >> 1][(mt & 1) * 4 + j];
      }
    // output gradient (standardised units), rows 0, 1 in lane group 0
    float d0 = 0.f, d1 = 0.f;
    if (g == 0 && valid) {
      const float t0 = (tgt[2 * row] - k.omean[0]) / k.ostd[0];
      const float t1 = (tgt[2 * row + 1] - k.omean[1]) / k.ostd[1];
      const float e0 = (o[0] + k.b4[0]) - t0, e1 = (o[1] + k.b4[1]) - t1;
      lsum += 0.5f * (e0 * e0 + e1 * e1) * invM;
      d0 = e0 * invM;
      d1 = e1 * invM;
    }
    b4sum[0] += d0;
    b4sum[1] += d1;
    bf16x8 Bd;
#pragma unroll
    for (int e = 0; e < 8; ++e) Bd[e] = (__bf16)0.0f;
    if (g == 0) {
      Bd[0] = (__bf16)d0;
      Bd[1] = (__bf16)d1;
      dZ4[0 * Mpad + v] = Bd[0];
      dZ4[1 * Mpad + v] = Bd[1];
    }
    // dA3 = W4^T dO, dZ3 = dA3 * silu'(z3)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 a = {0.f, 0.f, 0.f, 0.f};
      acc[mt] = mfma(sw[(T_B4 + mt) * 64 + lane], Bd, a);
    }
    bf16x8 Bz[2];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float dz = acc[mt][j] * dsilu(z3[mt * 4 + j]);
        bsum[2][mt * 4 + j] += dz;
        const __bf16 bz = (__bf16)dz;
        Bz[mt >> 1][(mt & 1) * 4 + j] = bz;
        dZ3[(16 * mt + 4 * g + j) * Mpad + v] = bz;
      }
    // dA2 = W3^T dZ3
    layer(sw, T_B3, lane, Bz, acc);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float dz = acc[mt][j] * dsilu(z2[mt * 4 + j]);
        bsum[1][mt * 4 + j] += dz;
        const __bf16 bz = (__bf16)dz;
        Bz[mt >> 1][(mt & 1) * 4 + j] = bz;
        dZ2[(16 * mt + 4 * g + j) * Mpad + v] = bz;
      }
    // dA1 = W2^T dZ2
    layer(sw, T_B2, lane, Bz, acc);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float dz = acc[mt][j] * dsilu(z1[mt * 4 + j]);
        bsum[0][mt * 4 + j] += dz;
        dZ1[(16 * mt + 4 * g + j) * Mpad + v] = (__bf16)dz;
      }
  }
  // per-wave partials: reduce over the 16 voxel lanes of each lane group
  const int64_t wg = (int64_t)blockIdx.x * 4 + wave;
  float* bp = bias_part + wg * NBIAS;
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      float s = bsum[l][i];
      for (int off = 1; off < 16; off <<= 1) s += __shfl_xor(s, off, 64);
      if (col == 0) bp[l * NH + 16 * (i >> 2) + 4 * g + (i & 3)] = s;
    }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    float s = b4sum[r];
    for (int off = 1; off < 64; off <<= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) bp[3 * NH + r] = s;
  }
  for (int off = 1; off < 64; off <<= 1) lsum += __shfl_xor(lsum, off, 64);
  if (lane == 0) loss_part[wg] = lsum;
}

// Weight gradients dW_l = dZ_l A_{l-1}^T with the batch as the K dimension.
// 40 output tiles of 16x16 (layer 1: 4, layers 2-3: 16 each, layer 4: 4); a
// wave owns one tile over one K slice; partials [ks][tile][64 lanes][4].
__global__ __launch_bounds__(256) void k_mlp_dw(const __bf16* __restrict__ A0, const __bf16* __restrict__ A1,
                                                const __bf16* __restrict__ A2, const __bf16* __restrict__ A3,
                                                const __bf16* __restrict__ dZ1, const __bf16* __restrict__ dZ2,
                                                const __bf16* __restrict__ dZ3, const __bf16* __restrict__ dZ4,
                                                int64_t Mpad, int ksplit, float* __restrict__ dw_part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tile = blockIdx.x * 4 + wave;
  if (tile >= 40) return;
  const int ks = blockIdx.y;
  const int g = lane >> 4, col = lane & 15;
  const __bf16 *Am, *Bm;
  int mt, nt;
  if (tile < 4) {
    Am = dZ1; Bm = A0; mt = tile; nt = 0;
  } else if (tile < 20) {
    Am = dZ2; Bm = A1; mt = (tile - 4) >> 2; nt = (tile - 4) & 3;
  } else if (tile < 36) {
    Am = dZ3; Bm = A2; mt = (tile - 20) >> 2; nt = (tile - 20) & 3;
  } else {
    Am = dZ4; Bm = A3; mt = 0; nt = tile - 36;
  }
  const int64_t nchunk = Mpad / 32;
  const int64_t c0 = nchunk * ks / ksplit, c1 = nchunk * (ks + 1) / ksplit;
  const bf16x8* ap = (const bf16x8*)(Am + (int64_t)(16 * mt + col) * Mpad + 8 * g);
  const bf16x8* bp = (const bf16x8*)(Bm + (int64_t)(16 * nt + col) * Mpad + 8 * g);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int64_t c = c0; c < c1; ++c) acc = mfma(ap[c * 4], bp[c * 4], acc);
  ((f32x4*)dw_part)[((int64_t)ks * 40 + tile) * 64 + lane] = acc;
}

// Gradient vector in parameter order: fixed-order sums of the partials.
__global__ __launch_bounds__(256) void k_mlp_grad_reduce(const float* __restrict__ dw_part, int ksplit,
                                                         const float* __restrict__ bias_part, int nwaves,
                                                         const float* __restrict__ loss_part, float* __restrict__ grad,
                                                         float* __restrict__ loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p == 0 && loss) {
    float s = 0.f;
    for (int w = 0; w < nwaves; ++w) s += loss_part[w];
    *loss = s;
  }
  if (p >= N_TRAIN) return;
  int tile = -1, m = 0, nn = 0, b = -1;
  if (p < ob1) {
    m = p / NIN; nn = p % NIN; tile = m / 16;
  } else if (p < oW2) {
    b = p - ob1;
  } else if (p < ob2) {
    const int q = p - oW2; m = q / NH; nn = q % NH; tile = 4 + (m / 16) * 4 + nn / 16;
  } else if (p < oW3) {
    b = NH + p - ob2;
  } else if (p < ob3) {
    const int q = p - oW3; m = q / NH; nn = q % NH; tile = 20 + (m / 16) * 4 + nn / 16;
  } else if (p < oW4) {
    b = 2 * NH + p - ob3;
  } else if (p < ob4) {
    const int q = p - oW4; m = q / NH; nn = q % NH; tile = 36 + nn / 16;
  } else {
    b = 3 * NH + p - ob4;
  }
  float s = 0.f;
  if (tile >= 0) {
    const int mi = m % 16, ni = nn % 16;
    const int lane = ni + 16 * (mi >> 2), j = mi & 3;
    for (int ks = 0; ks < ksplit; ++ks) s += dw_part[(((int64_t)ks * 40 + tile) * 64 + lane) * 4 + j];
  } else {
    for (int w = 0; w < nwaves; ++w) s += bias_part[(int64_t)w * NBIAS + b];
  }
  grad[p] = s;
}

// Adam (Kingma & Ba 2015) on the trainable parameters, FP32 master weights.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ prm, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ grad, int step, float lr, float b1, float b2,
                                              float eps) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= N_TRAIN) return;
  const float gr = grad[p];
  const float mm = b1 * m[p] + (1.0f - b1) * gr;
  const float vv = b2 * v[p] + (1.0f - b2) * gr * gr;
  m[p] = mm;
  v[p] = vv;
  const float mh = mm / (1.0f - powf(b1, (float)step));
  const float vh = vv / (1.0f - powf(b2, (float)step));
  prm[p] = prm[p] - lr * mh / (sqrtf(vh) + eps);
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero(T* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (T)0;
}

// Training targets of one band voxel from the method's own solves:
// o0 = (mu - rhs/diag) / h, o1 = log(clamp(s * diag, lo, hi)), as float.
__global__ __launch_bounds__(256) void k_targets(const double* __restrict__ mu, const double* __restrict__ s,
                                                 const double* __restrict__ rhs, const double* __restrict__ diag,
                                                 double h, double lo, double hi, int64_t n, float* __restrict__ tgt) {
#pragma clang fp contract(off)
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double d = diag[v];
  const double t0 = (mu[v] - rhs[v] / d) / h;
  const double sd = s[v] * d;
  const double t1 = log(sd < lo ? lo : (sd > hi ? hi : sd));
  tgt[2 * v] = (float)t0;
  tgt[2 * v + 1] = (float)t1;
}

bf_status pack(bf_ctx* ctx, const float* params, __bf16** wt) {
  BF_TRY(bf_ws(ctx, bf_ctx::WS_MLP, NTILES * 64 * 16, (void**)wt));
  BF_LAUNCH(ctx, "mlp_pack", k_mlp_pack, dim3((NTILES * 512 + 255) / 256), dim3(256), 0, params, *wt);
  return bf_launch_check(ctx, "k_mlp_pack");
}

}  // namespace

extern "C" bf_status bf_mlp_forward(bf_ctx* ctx, const float* params_dev, const float* feat_dev, int64_t n,
                                    float* out_dev) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, n >= 0, "bf_mlp_forward: n < 0");
  if (n == 0) return BF_OK;
  BF_CHECK(ctx, params_dev && feat_dev && out_dev, "bf_mlp_forward: NULL argument");
  BF_HIP(ctx, hipSetDevice(ctx->device));
  __bf16* wt = nullptr;
  BF_TRY(pack(ctx, params_dev, &wt));
  const unsigned grid = (unsigned)std::min<int64_t>(bf_cdiv(bf_cdiv(n, 16), 4), 8 * (int64_t)ctx->cu_count);
  BF_LAUNCH(ctx, "mlp_forward", k_mlp_forward<false>, dim3(grid), dim3(256), 0, (const bf16x8*)wt, params_dev,
            feat_dev, bf_feat_in{}, n, out_dev, (const double*)nullptr, (const double*)nullptr, 0.0, (double*)nullptr,
            (float*)nullptr);
  return bf_launch_check(ctx, "k_mlp_forward");
}

extern "C" bf_status bf_warm_start(bf_ctx* ctx, const bf_system* sys, const float* params_dev,
                                   const float* feat_dev, double* x0_dev, float* logvar_dev) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, sys && params_dev, "bf_warm_start: NULL argument");
  BF_CHECK(ctx, sys->kind == BF_SYSTEM_VOXEL, "bf_warm_start: the network was trained on voxel-centric rows");
  if (sys->n == 0) return BF_OK;
  BF_CHECK(ctx, x0_dev || logvar_dev, "bf_warm_start: no output requested");
  BF_HIP(ctx, hipSetDevice(ctx->device));
  __bf16* wt = nullptr;
  BF_TRY(pack(ctx, params_dev, &wt));
  const int64_t n = sys->n;
  const unsigned grid = (unsigned)std::min<int64_t>(bf_cdiv(bf_cdiv(n, 16), 4), 8 * (int64_t)ctx->cu_count);
  if (feat_dev) {
    BF_LAUNCH(ctx, "mlp_forward", k_mlp_forward<false>, dim3(grid), dim3(256), 0, (const bf16x8*)wt, params_dev,
              feat_dev, bf_feat_in{}, n, (float*)nullptr, (const double*)sys->rhs, (const double*)sys->diag,
              sys->band->h, x0_dev, logvar_dev);
  } else {  // features computed in the same pass
    const bf_band* b = sys->band;
    const bf_feat_in src = bf_feat_make(b->tsdf, sys->Lambda, sys->acc, b->w, b->nbr, b->deg, sys->T, b->h);
    BF_LAUNCH(ctx, "mlp_fused", k_mlp_forward<true>, dim3(grid), dim3(256), 0, (const bf16x8*)wt, params_dev,
              (const float*)nullptr, src, n, (float*)nullptr, (const double*)sys->rhs, (const double*)sys->diag,
              b->h, x0_dev, logvar_dev);
  }
  return bf_launch_check(ctx, "k_mlp_forward");
}

extern "C" bf_status bf_warm_start_targets(bf_ctx* ctx, const bf_system* sys, const double* mu_dev,
                                           const double* s_dev, double clamp_lo, double clamp_hi,
                                           float* target_dev) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, sys && mu_dev && s_dev && target_dev, "bf_warm_start_targets: NULL argument");
  BF_CHECK(ctx, sys->kind == BF_SYSTEM_VOXEL, "bf_warm_start_targets: voxel-centric systems only");
  BF_CHECK(ctx, clamp_lo > 0.0 && clamp_lo <= clamp_hi, "bf_warm_start_targets: need 0 < clamp_lo <= clamp_hi");
  if (sys->n == 0) return BF_OK;
  BF_HIP(ctx, hipSetDevice(ctx->device));
  BF_LAUNCH(ctx, "mlp_targets", k_targets, dim3((unsigned)bf_cdiv(sys->n, 256)), dim3(256), 0, mu_dev, s_dev,
            (const double*)sys->rhs, (const double*)sys->diag, sys->band->h, clamp_lo, clamp_hi, sys->n, target_dev);
  return bf_launch_check(ctx, "k_targets");
}

extern "C" bf_status bf_mlp_grad(bf_ctx* ctx, const float* params_dev, const float* feat_dev,
                                 const float* target_dev, int64_t nrows, const int32_t* idx_dev, int64_t M,
                                 float* grad_dev, float* loss_dev) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, M > 0 && M <= (1ll << 26), "bf_mlp_grad: batch size %lld outside [1, 2^26]", (long long)M);
  BF_CHECK(ctx, params_dev && feat_dev && target_dev && idx_dev && grad_dev, "bf_mlp_grad: NULL argument");
  BF_HIP(ctx, hipSetDevice(ctx->device));
  __bf16* wt = nullptr;
  BF_TRY(pack(ctx, params_dev, &wt));
  const int64_t Mpad = bf_cdiv(M, 32) * 32;
  const unsigned grid = (unsigned)std::min<int64_t>(bf_cdiv(Mpad / 16, 4), 4 * (int64_t)ctx->cu_count);
  const int nwaves = (int)grid * 4;
  const int ksplit = (int)std::max<int64_t>(1, std::min<int64_t>(Mpad / 32 / 64, 256));
  // workspace: A0 dZ4 [16][Mpad], A1-3, dZ1-3 [64][Mpad] (bf16) | bias partials | loss partials | dW partials
  const size_t mat16 = (size_t)16 * Mpad * 2, mat64 = (size_t)64 * Mpad * 2;
  const size_t bias_b = (size_t)nwaves * NBIAS * 4, loss_b = (size_t)nwaves * 4;
  const size_t dw_b = (size_t)ksplit * 40 * 64 * 16;
  const size_t total = 2 * mat16 + 6 * mat64 + bias_b + loss_b + dw_b + 1024;
  char* ws = nullptr;
  BF_TRY(bf_ws(ctx, bf_ctx::WS_BATCH, total, (void**)&ws));
  __bf16* A0 = (__bf16*)ws;
  __bf16* dZ4 = (__bf16*)(ws + mat16);
  __bf16* A1 = (__bf16*)(ws + 2 * mat16);
  __bf16* A2 = (__bf16*)((char*)A1 + mat64);
  __bf16* A3 = (__bf16*)((char*)A2 + mat64);
  __bf16* dZ1 = (__bf16*)((char*)A3 + mat64);
  __bf16* dZ2 = (__bf16*)((char*)dZ1 + mat64);
  __bf16* dZ3 = (__bf16*)((char*)dZ2 + mat64);
  float* bias_part = (float*)((char*)dZ3 + mat64);
  float* loss_part = (float*)((char*)bias_part + bias_b);
  float* dw_part = (float*)(((uintptr_t)((char*)loss_part + loss_b) + 255) & ~(uintptr_t)255);
  // rows that no lane writes (A0 rows 12-15 are written as zeros; dZ4 rows 2-15 are not)
  BF_LAUNCH(ctx, "mlp_zero", k_zero<__bf16>, dim3(1024), dim3(256), 0, dZ4, (int64_t)16 * Mpad);
  BF_LAUNCH(ctx, "mlp_train", k_mlp_train, dim3(grid), dim3(256), 0, (const bf16x8*)wt, params_dev, feat_dev,
            target_dev, idx_dev, nrows, M, Mpad, A0, A1, A2, A3, dZ1, dZ2, dZ3, dZ4, bias_part, loss_part);
  BF_LAUNCH(ctx, "mlp_dw", k_mlp_dw, dim3(10, ksplit), dim3(256), 0, A0, A1, A2, A3, dZ1, dZ2, dZ3, dZ4, Mpad,
            ksplit, dw_part);
  BF_LAUNCH(ctx, "mlp_grad_reduce", k_mlp_grad_reduce, dim3((N_TRAIN + 255) / 256), dim3(256), 0, dw_part, ksplit,
            bias_part, nwaves, loss_part, grad_dev, loss_dev);
  return bf_launch_check(ctx, "bf_mlp_grad");
}

extern "C" bf_status bf_adam_step(bf_ctx* ctx, float* params_dev, float* m_dev, float* v_dev, const float* grad_dev,
                                  int32_t step, float lr, float beta1, float beta2, float eps) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, params_dev && m_dev && v_dev && grad_dev && step >= 1, "bf_adam_step: bad argument");
  BF_HIP(ctx, hipSetDevice(ctx->device));
  BF_LAUNCH(ctx, "adam", k_adam, dim3((N_TRAIN + 255) / 256), dim3(256), 0, params_dev, m_dev, v_dev, grad_dev, step,
            lr, beta1, beta2, eps);
  return bf_launch_check(ctx, "k_adam");
}
