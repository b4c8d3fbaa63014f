// Observation assembly and posterior precision (Sec. 3.5-3.6, eqs. 3-5 and
// 8-11; Algorithm 1 steps 3-4), the explicit Q p product, and the per-voxel
// features of the learned warm start.
//
// Observation rows are voxel-centric (a_i = e_v): every band voxel receives
// one observation per view that sees it, so A^T W A is the diagonal Lambda and
// A^T W y the vector b.  One thread per band voxel walks the views in order;
// the FP64 operation order is fixed so Lambda, b and diag(Q) are reproducible
// bit for bit.
#include "bf_internal.h"
#include "bf_features.h"

#include <vector>

namespace {

struct noise_k {
  double a, c, z0, model;
  const double* pose;  // [T] or null
};

// A band voxel's running sums over the views that observe it, in view order.
struct obs_sums {
  double L = 0.0, B = 0.0, cnt = 0.0, sy = 0.0, syy = 0.0, ss = 0.0, smin = INFINITY;
};

// One view's observation of voxel (i, j, k), eqs. (3)-(5): accepted when the
// projective distance d = D - Z is >= -tau, y = min(d, tau), weight 1/sigma^2.
__device__ __forceinline__ void add_view(obs_sums& a, const bf_grid_k& g, const bf_cam_k& c,
                                         const float* __restrict__ depth_t, const double* __restrict__ pose_t,
                                         double pose_var, const noise_k& nz, int32_t i, int32_t j, int32_t k) {
#pragma clang fp contract(off)
  double D, Z;
  if (!bf_observe(g, c, depth_t, pose_t, i, j, k, D, Z)) return;
  const double d = D - Z;
  if (d < -g.tau) return;
  const double y = d < g.tau ? d : g.tau;
  const double e = D - nz.z0;
  const double sd = nz.a + nz.c * (e * e);
  double var = sd * sd + pose_var;
  var = var + nz.model;
  // a positive normal variance (every realistic sensor model) takes the
  // reciprocal sequence; anything else the plain division
  const double w = (var >= 1e-300 && var <= 1e300) ? bf_recip(var) : 1.0 / var;
  a.L = a.L + w;
  a.B = a.B + w * y;
  a.cnt = a.cnt + 1.0;
  a.sy = a.sy + y;
  a.syy = a.syy + y * y;
  a.ss = a.ss + sd;
  a.smin = sd < a.smin ? sd : a.smin;
}

// Lambda, b, the anchored right-hand side, diag(Q) (eqs. 7, 10-11) and the
// feature statistics of voxel v from its sums.
__device__ __forceinline__ void finish_voxel(const obs_sums& a, int64_t v, int32_t dg, double tsdf_v, double lam,
                                             double eps, double lam_b, double* __restrict__ Lambda,
                                             double* __restrict__ b, double* __restrict__ rhs,
                                             double* __restrict__ diag, double* __restrict__ dinv,
                                             float* __restrict__ diag32, float* __restrict__ dinv32,
                                             double* __restrict__ acc) {
#pragma clang fp contract(off)
  double dq = a.L + lam * (double)dg;
  dq = dq + eps;
  double h = a.B;
  if (lam_b != 0.0 && dg < 6) {
    dq = dq + lam_b;
    h = h + lam_b * tsdf_v;
  }
  Lambda[v] = a.L;
  b[v] = a.B;
  rhs[v] = h;
  diag[v] = dq;
  const double inv = 1.0 / dq;
  dinv[v] = inv;
  diag32[v] = (float)dq;
  dinv32[v] = (float)inv;
  double* o = acc + v * 5;
  o[0] = a.cnt;
  o[1] = a.sy;
  o[2] = a.syy;
  o[3] = a.ss;
  o[4] = a.cnt > 0.0 ? a.smin : 0.0;
}

__global__ __launch_bounds__(256) void k_assemble(bf_grid_k g, bf_cam_k c, int32_t T,
                                                  const float* __restrict__ depth,
                                                  const double* __restrict__ poses, noise_k nz,
                                                  const uint64_t* __restrict__ keys,
                                                  const double* __restrict__ tsdf,
                                                  const int32_t* __restrict__ deg, int64_t n,
                                                  double lam, double eps, double lam_b,
                                                  double* __restrict__ Lambda, double* __restrict__ b,
                                                  double* __restrict__ rhs, double* __restrict__ diag,
                                                  double* __restrict__ dinv, float* __restrict__ diag32,
                                                  float* __restrict__ dinv32, double* __restrict__ acc,
                                                  const uint32_t* __restrict__ vmask, int vw) {
#pragma clang fp contract(off)
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool valid = v < n;  // every lane takes part in the wave's view loop
  const uint64_t key = valid ? keys[v] : 0;
  const int32_t i = (int32_t)bf_compact3(key), j = (int32_t)bf_compact3(key >> 1),
                k = (int32_t)bf_compact3(key >> 2);
  const int64_t plane = (int64_t)c.W * c.H;
  obs_sums a;
  int32_t t0 = 0;
  if (vmask) {
    // the band's screen proved that a view with a clear bit observes no voxel
    // of this voxel's cell: only the set bits are visited, in view order, so
    // every sum is the one over all views.  The wave walks the union of its
    // lanes' bits (a wave spans a few cells with similar masks), so the view,
    // its pose and its depth map are the same for every lane
    for (int q = 0; q < vw; ++q) {
      const uint32_t bits = valid ? vmask[v * vw + q] : 0u;
      uint32_t un = bits;
      for (int off = 32; off > 0; off >>= 1) un |= (uint32_t)__shfl_xor((int)un, off, 64);
      un = (uint32_t)__builtin_amdgcn_readfirstlane((int)un);
      while (un) {
        const int32_t t = 32 * q + __builtin_ctz(un);
        un &= un - 1u;
        if ((bits >> (t & 31)) & 1u)
          add_view(a, g, c, depth + t * plane, poses + 12 * t, nz.pose ? nz.pose[t] : 0.0, nz, i, j, k);
      }
    }
    t0 = 32 * vw < T ? 32 * vw : T;  // views past the masked ones
  }
  if (!valid) return;
  for (int32_t t = t0; t < T; ++t)
    add_view(a, g, c, depth + t * plane, poses + 12 * t, nz.pose ? nz.pose[t] : 0.0, nz, i, j, k);
  const int32_t dg = deg[v];
  finish_voxel(a, v, dg, (lam_b != 0.0 && dg < 6) ? tsdf[v] : 0.0, lam, eps, lam_b, Lambda, b, rhs, diag, dinv,
               diag32, dinv32, acc);
}

// Set bits of the band's per-voxel view masks, per workgroup (for the
// assembly's voxel-view count; integer sums, any order is exact).
__global__ __launch_bounds__(256) void k_popc_sum(const uint32_t* __restrict__ w, int64_t n,
                                                  unsigned long long* __restrict__ part) {
  __shared__ unsigned long long lds[4];
  unsigned long long c = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c += (unsigned long long)__popc(w[i]);
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = lds[0] + lds[1] + lds[2] + lds[3];
}

// More views appended to an assembled system: the sums of the first views
// come back from Lambda, b and the statistics (the running minimum of sigma
// is "none yet" for a voxel no view observed), and the new views continue
// them in order, so the result is that of assembling all views at once.
__global__ __launch_bounds__(256) void k_assemble_more(bf_grid_k g, bf_cam_k c, int32_t T,
                                                       const float* __restrict__ depth,
                                                       const double* __restrict__ poses, noise_k nz,
                                                       const uint64_t* __restrict__ keys,
                                                       const double* __restrict__ tsdf,
                                                       const int32_t* __restrict__ deg, int64_t n, double lam,
                                                       double eps, double lam_b, const double* __restrict__ L0,
                                                       const double* __restrict__ b0,
                                                       const double* __restrict__ acc0,
                                                       double* __restrict__ Lambda, double* __restrict__ b,
                                                       double* __restrict__ rhs, double* __restrict__ diag,
                                                       double* __restrict__ dinv, float* __restrict__ diag32,
                                                       float* __restrict__ dinv32, double* __restrict__ acc) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint64_t key = keys[v];
  const int32_t i = (int32_t)bf_compact3(key), j = (int32_t)bf_compact3(key >> 1),
                k = (int32_t)bf_compact3(key >> 2);
  const int64_t plane = (int64_t)c.W * c.H;
  const double* a0 = acc0 + v * 5;
  obs_sums a;
  a.L = L0[v];
  a.B = b0[v];
  a.cnt = a0[0];
  a.sy = a0[1];
  a.syy = a0[2];
  a.ss = a0[3];
  a.smin = a0[0] > 0.0 ? a0[4] : INFINITY;
  for (int32_t t = 0; t < T; ++t)
    add_view(a, g, c, depth + t * plane, poses + 12 * t, nz.pose ? nz.pose[t] : 0.0, nz, i, j, k);
  const int32_t dg = deg[v];
  finish_voxel(a, v, dg, (lam_b != 0.0 && dg < 6) ? tsdf[v] : 0.0, lam, eps, lam_b, Lambda, b, rhs, diag, dinv,
               diag32, dinv32, acc);
}

__global__ __launch_bounds__(256) void k_apply_Q(const int32_t* __restrict__ nbr,
                                                 const double* __restrict__ diag, double lam,
                                                 const double* __restrict__ p, double* __restrict__ q,
                                                 int64_t n) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t* nb = nbr + v * 6;
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    const int32_t u = nb[t];
    if (u >= 0) s += p[u];
  }
  q[v] = diag[v] * p[v] - lam * s;
}

// q = Q p for a trilinear system: diag p plus the 26 couplings (slot-major
// [26][N]) in slot order.
__global__ __launch_bounds__(256) void k_apply_Q27(const int32_t* __restrict__ nb26, const double* __restrict__ off,
                                                   const double* __restrict__ diag, const double* __restrict__ p,
                                                   double* __restrict__ q, int64_t n) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < 26; ++t) {
    const int32_t u = nb26[t * n + v];
    if (u >= 0) s += off[t * n + v] * p[u];
  }
  q[v] = diag[v] * p[v] + s;
}

// Features of the learned warm start, lengths in units of h (bf_features.h).
__global__ __launch_bounds__(256) void k_features(int64_t n, bf_feat_in in, float* __restrict__ feat) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  float f[12];
  bf_features_0_7(v, in, f);
  bf_features_8_11(v, in, f + 8);
  float* o = feat + v * 12;
#pragma unroll
  for (int q = 0; q < 12; ++q) o[q] = f[q];
}

}  // namespace

extern "C" bf_status bf_assemble(bf_ctx* ctx, const bf_band* band, const bf_camera* cam, int32_t T,
                                 const float* depth_dev, const double* c2w_dev, const bf_noise* noise,
                                 const bf_prior* prior, bf_system** out) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, band && cam && noise && prior && out, "bf_assemble: NULL argument");
  *out = nullptr;
  BF_CHECK(ctx, T >= 0, "bf_assemble: T < 0");
  BF_CHECK(ctx, T == 0 || band->n == 0 || (depth_dev && c2w_dev && cam->width > 0 && cam->height > 0),
           "bf_assemble: bad camera or NULL depth/poses");
  BF_CHECK(ctx, prior->lambda >= 0.0 && prior->eps >= 0.0 && prior->lambda_b >= 0.0,
           "bf_assemble: lambda, eps and lambda_b must be >= 0");
  BF_HIP(ctx, hipSetDevice(ctx->device));
  bf_system* sys = new (std::nothrow) bf_system();
  if (!sys) return bf_fail(ctx, BF_ERR_OOM, "bf_assemble: host allocation");
  sys->n = band->n;
  sys->band = band;
  sys->lambda = prior->lambda;
  sys->eps = prior->eps;
  sys->lambda_b = prior->lambda_b;
  sys->T = T;
  sys->masked = 0;
  const int64_t N = band->n;
  auto fail = [&](bf_status st) {
    bf_system_free(ctx, sys);
    return st;
  };
  if (N > 0) {
    if (bf_status s = bf_obj_alloc_parts(ctx, &sys->block,
                                         {{(void**)&sys->Lambda, (size_t)N * 8}, {(void**)&sys->b, (size_t)N * 8},
                                          {(void**)&sys->rhs, (size_t)N * 8}, {(void**)&sys->diag, (size_t)N * 8},
                                          {(void**)&sys->dinv, (size_t)N * 8}, {(void**)&sys->diag32, (size_t)N * 4},
                                          {(void**)&sys->dinv32, (size_t)N * 4}, {(void**)&sys->acc, (size_t)N * 40}}))
      return fail(s);
    bf_grid_k gk{band->G, band->h, band->origin[0], band->origin[1], band->origin[2], band->tau, band->band};
    bf_cam_k ck{cam->width, cam->height, cam->fx, cam->fy, cam->cx, cam->cy};
    noise_k nz{noise->a, noise->c, noise->z0, noise->sigma2_model, noise->sigma2_pose_dev};
    // the band's view masks hold for the depth maps and poses it was built from
    const bool masks = band->vmask && depth_dev == band->view_depth && c2w_dev == band->view_poses &&
                       T == band->view_T && cam->width == band->view_W && cam->height == band->view_H &&
                       cam->fx == band->view_f[0] && cam->fy == band->view_f[1] && cam->cx == band->view_f[2] &&
                       cam->cy == band->view_f[3];
    BF_LAUNCH(ctx, "assemble", k_assemble, dim3((unsigned)bf_cdiv(N, 256)), dim3(256), 0, gk, ck, T,
                       depth_dev, c2w_dev, nz, band->keys, band->tsdf, band->deg, N, prior->lambda,
                       prior->eps, prior->lambda_b, sys->Lambda, sys->b, sys->rhs, sys->diag, sys->dinv,
                       sys->diag32, sys->dinv32, sys->acc, masks ? band->vmask : nullptr,
                       masks ? band->vmask_words : 0);
    sys->masked = masks ? 1 : 0;
    if (bf_status s = bf_launch_check(ctx, "k_assemble")) return fail(s);
  }
  *out = sys;
  return BF_OK;
}

extern "C" bf_status bf_system_assembly_views(bf_ctx* ctx, const bf_system* sys, int64_t* out) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, sys && out, "bf_system_assembly_views: NULL argument");
  *out = 0;
  BF_CHECK(ctx, sys->masked >= 0, "bf_system_assembly_views: the system was not made by bf_assemble");
  const int64_t N = sys->n;
  if (N == 0 || sys->T == 0) return BF_OK;
  if (!sys->masked) {
    *out = N * (int64_t)sys->T;
    return BF_OK;
  }
  // every view past the masked ones, plus the masks' set bits
  const bf_band* band = sys->band;
  const int vw = band->vmask_words;
  const int64_t words = N * vw;
  const int nb = (int)std::min<int64_t>(bf_cdiv(words, 256), 1024);
  void* ws = nullptr;
  BF_TRY(bf_ws(ctx, bf_ctx::WS_POST, (size_t)nb * 8, &ws));
  BF_HIP(ctx, hipSetDevice(ctx->device));
  hipLaunchKernelGGL(k_popc_sum, dim3(nb), dim3(256), 0, ctx->stream, band->vmask, words,
                     (unsigned long long*)ws);
  BF_TRY(bf_launch_check(ctx, "k_popc_sum"));
  std::vector<unsigned long long> h((size_t)nb);
  BF_HIP(ctx, hipMemcpyAsync(h.data(), ws, h.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
  BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  int64_t t = 0;
  for (const unsigned long long c : h) t += (int64_t)c;
  *out = t + N * (int64_t)(sys->T - std::min<int32_t>(sys->T, 32 * vw));
  return BF_OK;
}

// The system `in` with T more views appended, into out's arrays (Lambda, b,
// rhs, diag, dinv, diag32, dinv32, acc; they may not alias in's).
bf_status bf_assemble_more_into(bf_ctx* ctx, const bf_system* in, const bf_camera* cam, int32_t T,
                                const float* depth_dev, const double* c2w_dev, const bf_noise* noise,
                                bf_system* out) {
  const bf_band* band = in->band;
  const int64_t N = in->n;
  out->n = N;
  out->band = band;
  out->lambda = in->lambda;
  out->eps = in->eps;
  out->lambda_b = in->lambda_b;
  out->T = in->T + T;
  out->kind = BF_SYSTEM_VOXEL;
  if (N == 0) return BF_OK;
  bf_grid_k gk{band->G, band->h, band->origin[0], band->origin[1], band->origin[2], band->tau, band->band};
  bf_cam_k ck{cam->width, cam->height, cam->fx, cam->fy, cam->cx, cam->cy};
  noise_k nz{noise->a, noise->c, noise->z0, noise->sigma2_model, noise->sigma2_pose_dev};
  BF_LAUNCH(ctx, "assemble_more", k_assemble_more, dim3((unsigned)bf_cdiv(N, 256)), dim3(256), 0, gk, ck, T,
            depth_dev, c2w_dev, nz, band->keys, band->tsdf, band->deg, N, in->lambda, in->eps, in->lambda_b,
            in->Lambda, in->b, in->acc, out->Lambda, out->b, out->rhs, out->diag, out->dinv, out->diag32,
            out->dinv32, out->acc);
  return bf_launch_check(ctx, "k_assemble_more");
}

extern "C" bf_status bf_assemble_more(bf_ctx* ctx, const bf_system* sys, const bf_camera* cam, int32_t T,
                                      const float* depth_dev, const double* c2w_dev, const bf_noise* noise,
                                      bf_system** out) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, sys && cam && noise && out, "bf_assemble_more: NULL argument");
  *out = nullptr;
  BF_CHECK(ctx, sys->kind == BF_SYSTEM_VOXEL, "bf_assemble_more: voxel-centric systems only");
  BF_CHECK(ctx, T >= 0, "bf_assemble_more: T < 0");
  BF_CHECK(ctx, T == 0 || sys->n == 0 || (depth_dev && c2w_dev && cam->width > 0 && cam->height > 0),
           "bf_assemble_more: bad camera or NULL depth/poses");
  BF_HIP(ctx, hipSetDevice(ctx->device));
  bf_system* ns = new (std::nothrow) bf_system();
  if (!ns) return bf_fail(ctx, BF_ERR_OOM, "bf_assemble_more: host allocation");
  const int64_t N = sys->n;
  if (N > 0) {
    if (bf_status s = bf_obj_alloc_parts(ctx, &ns->block,
                                         {{(void**)&ns->Lambda, (size_t)N * 8}, {(void**)&ns->b, (size_t)N * 8},
                                          {(void**)&ns->rhs, (size_t)N * 8}, {(void**)&ns->diag, (size_t)N * 8},
                                          {(void**)&ns->dinv, (size_t)N * 8}, {(void**)&ns->diag32, (size_t)N * 4},
                                          {(void**)&ns->dinv32, (size_t)N * 4}, {(void**)&ns->acc, (size_t)N * 40}})) {
      bf_system_free(ctx, ns);
      return s;
    }
  }
  if (bf_status s = bf_assemble_more_into(ctx, sys, cam, T, depth_dev, c2w_dev, noise, ns)) {
    bf_system_free(ctx, ns);
    return s;
  }
  *out = ns;
  return BF_OK;
}

extern "C" bf_status bf_apply_Q(bf_ctx* ctx, const bf_system* sys, const double* p_dev, double* q_dev) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, sys, "bf_apply_Q: NULL system");
  if (sys->n == 0) return BF_OK;
  BF_CHECK(ctx, p_dev && q_dev && p_dev != q_dev, "bf_apply_Q: bad vectors");
  if (sys->kind == BF_SYSTEM_TRILINEAR) {
    hipLaunchKernelGGL(k_apply_Q27, dim3((unsigned)bf_cdiv(sys->n, 256)), dim3(256), 0, ctx->stream, sys->nb26,
                       sys->off, sys->diag, p_dev, q_dev, sys->n);
    return bf_launch_check(ctx, "k_apply_Q27");
  }
  hipLaunchKernelGGL(k_apply_Q, dim3((unsigned)bf_cdiv(sys->n, 256)), dim3(256), 0, ctx->stream,
                     sys->band->nbr, sys->diag, sys->lambda, p_dev, q_dev, sys->n);
  return bf_launch_check(ctx, "k_apply_Q");
}

extern "C" bf_status bf_features(bf_ctx* ctx, const bf_system* sys, float* feat_dev) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, sys, "bf_features: NULL system");
  BF_CHECK(ctx, sys->kind == BF_SYSTEM_VOXEL, "bf_features: the features need voxel-centric rows");
  if (sys->n == 0) return BF_OK;
  BF_CHECK(ctx, feat_dev && sys->T > 0, "bf_features: NULL output or system without views");
  const bf_band* band = sys->band;
  BF_LAUNCH(ctx, "features", k_features, dim3((unsigned)bf_cdiv(sys->n, 256)), dim3(256), 0, sys->n,
            bf_feat_make(band->tsdf, sys->Lambda, sys->acc, band->w, band->nbr, band->deg, sys->T, band->h),
            feat_dev);
  return bf_launch_check(ctx, "k_features");
}
