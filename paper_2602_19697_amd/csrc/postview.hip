// Next-best-view utility with the post-view variance (Sec. 3.8, eq. 13):
// U(v) = sum over the voxels of Omega_eps of (s_i - s'_i), where s' is the
// marginal variance once the view from candidate v has been fused.  The view
// is predicted from the current mean (bf_predict_depth), appended to the
// assembled system as one more view (bf_assemble_more's arithmetic, so the
// post-view system is the one assembled from all views at once), and s' is
// estimated with the same Hutchinson block solve as s (bf_diag_estimate, the
// caller's probe seed, so the difference shares the probes' noise).
#include "bf_internal.h"

namespace {

constexpr int kThreads = 256;

// Start of the post-view probe solves: log(s diag') clamped to [1e-3, 1e3],
// i.e. u0 = z s (the pre-view variance as a diagonal guess of the new one).
__global__ __launch_bounds__(256) void k_post_logvar(const double* __restrict__ s, const double* __restrict__ diag,
                                                     float* __restrict__ lv, int64_t n) {
  for (int64_t v = blockIdx.x * (int64_t)kThreads + threadIdx.x; v < n; v += (int64_t)gridDim.x * kThreads) {
    double r = s[v] * diag[v];
    r = r < 1e-3 ? 1e-3 : (r > 1e3 ? 1e3 : r);
    lv[v] = (float)log(r);
  }
}

// Per-workgroup partial sums of (s - s') over the voxels with |mu| <= eps:
// each thread in ascending index, then a fixed tree; the host adds the
// partials in workgroup order, so the sum does not change between runs.
__global__ __launch_bounds__(256) void k_post_util(const double* __restrict__ mu, const double* __restrict__ s,
                                                   const double* __restrict__ s_post, double eps, int64_t n,
                                                   double* __restrict__ part) {
  __shared__ double red[kThreads];
  double acc = 0.0;
  for (int64_t v = blockIdx.x * (int64_t)kThreads + threadIdx.x; v < n; v += (int64_t)gridDim.x * kThreads)
    if (fabs(mu[v]) <= eps) acc += s[v] - s_post[v];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace

extern "C" bf_status bf_nbv_postview(bf_ctx* ctx, const bf_system* sys, const double* mu_dev, const double* s_dev,
                                     int32_t n_cand, const double* cand_c2w_dev, int32_t n_sel,
                                     const int32_t* cand_idx_host, const bf_camera* cam, const bf_noise* noise,
                                     const bf_probe_opts* opts, double eps_band, int32_t warm, double* util_host,
                                     int32_t* best_host, double* s_post_dev, bf_solve_report* reps_host) {
  if (!ctx) return BF_ERR_INVALID_ARG;
  BF_CHECK(ctx, sys && cam && noise && opts && util_host && best_host, "bf_nbv_postview: NULL argument");
  BF_CHECK(ctx, sys->kind == BF_SYSTEM_VOXEL, "bf_nbv_postview: voxel-centric systems only");
  BF_CHECK(ctx, n_sel >= 0 && n_sel <= n_cand && (n_sel == 0 || (cand_idx_host && cand_c2w_dev)),
           "bf_nbv_postview: bad candidate selection");
  BF_CHECK(ctx, eps_band >= 0.0, "bf_nbv_postview: eps_band < 0");
  BF_CHECK(ctx, cam->width > 0 && cam->height > 0, "bf_nbv_postview: bad camera");
  for (int32_t i = 0; i < n_sel; ++i)
    BF_CHECK(ctx, cand_idx_host[i] >= 0 && cand_idx_host[i] < n_cand,
             "bf_nbv_postview: candidate index %d outside [0, %d)", cand_idx_host[i], n_cand);
  *best_host = -1;
  if (n_sel == 0) return BF_OK;
  const int64_t N = sys->n;
  BF_CHECK(ctx, N == 0 || (mu_dev && s_dev), "bf_nbv_postview: NULL mu or s");
  BF_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t npix = (int64_t)cam->width * cam->height;
  const int nparts = (int)std::max<int64_t>(1, std::min<int64_t>(bf_cdiv(N, kThreads), 1024));
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  // post-view system arrays | predicted depth | start | s' (unless the caller's) | partials
  const size_t sys_bytes = al(N * 8) * 5 + al(N * 4) * 2 + al(N * 40);
  const size_t bytes = sys_bytes + al(npix * 4) + al(N * 4) + (s_post_dev ? 0 : al(N * 8)) + al(nparts * 8);
  char* ws = nullptr;
  BF_TRY(bf_ws(ctx, bf_ctx::WS_POST, bytes, (void**)&ws));
  bf_system post;
  char* p = ws;
  auto take = [&](size_t b) {
    char* r = p;
    p += al(b);
    return r;
  };
  post.Lambda = (double*)take(N * 8);
  post.b = (double*)take(N * 8);
  post.rhs = (double*)take(N * 8);
  post.diag = (double*)take(N * 8);
  post.dinv = (double*)take(N * 8);
  post.diag32 = (float*)take(N * 4);
  post.dinv32 = (float*)take(N * 4);
  post.acc = (double*)take(N * 40);
  float* depth = (float*)take(npix * 4);
  float* lv = (float*)take(N * 4);
  double* s_own = s_post_dev ? nullptr : (double*)take(N * 8);
  double* part = (double*)take(nparts * 8);
  // the predicted view's pose is taken as exact: no pose variance for it
  bf_noise nz = *noise;
  nz.sigma2_pose_dev = nullptr;
  for (int32_t i = 0; i < n_sel; ++i) {
    const double* pose = cand_c2w_dev + 12 * (int64_t)cand_idx_host[i];
    double* sp = s_post_dev ? s_post_dev + (int64_t)i * N : s_own;
    BF_TRY(bf_predict_depth(ctx, sys->band, mu_dev, pose, cam, depth));
    BF_TRY(bf_assemble_more_into(ctx, sys, cam, 1, depth, pose, &nz, &post));
    if (warm && N > 0)
      BF_LAUNCH(ctx, "post_start", k_post_logvar, dim3((unsigned)std::min<int64_t>(bf_cdiv(N, kThreads), 4096)),
                dim3(kThreads), 0, s_dev, post.diag, lv, N);
    bf_solve_report rep{};
    BF_TRY(bf_diag_estimate(ctx, &post, opts, (warm && N > 0) ? lv : nullptr, sp, &rep));
    if (reps_host) reps_host[i] = rep;
    double u = 0.0;
    if (N > 0) {
      BF_LAUNCH(ctx, "post_util", k_post_util, dim3(nparts), dim3(kThreads), 0, mu_dev, s_dev, sp, eps_band, N, part);
      BF_TRY(bf_launch_check(ctx, "k_post_util"));
      // the context's pinned buffer is shared with the solve: take it afresh
      double* parts_host = nullptr;
      BF_TRY(bf_pinned(ctx, (size_t)nparts * 8, (void**)&parts_host));
      BF_HIP(ctx, hipMemcpyAsync(parts_host, part, (size_t)nparts * 8, hipMemcpyDeviceToHost, ctx->stream));
      BF_HIP(ctx, hipStreamSynchronize(ctx->stream));
      for (int b = 0; b < nparts; ++b) u += parts_host[b];
    }
    util_host[i] = u;
    if (*best_host < 0 || u > util_host[*best_host]) *best_host = i;
  }
  *best_host = cand_idx_host[*best_host];
  return BF_OK;
}
