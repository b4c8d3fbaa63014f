// Per-voxel input features of the learned warm start (not in the paper; the
// paper names learned priors as future work, Sec. 6-7), lengths in units of
// the voxel edge h.  Shared by k_features and the fused warm start so both
// give the same floats:
//   0 TSDF/h   1 log(1+W)   2 deg/6   3 n_obs/T   4 mean y/h   5 var y/h^2
//   6 mean sigma/h   7 min sigma/h   8 log(1 + Lambda h^2)
//   9-11 central difference of the TSDF along x, y, z over 2h, using the
//        voxel's own value where a band neighbour is absent.
#pragma once

struct bf_feat_in {
  const double *tsdf, *Lambda, *acc;
  const int32_t *w, *nbr, *deg;
  int32_t T;
  double h;
  // 1/h, 1/h^2, 1/(2h), 1/T: the divisions by these become products (a
  // double-level difference that the features' rounding to float absorbs)
  double ih, ih2, i2h, iT;
};

inline bf_feat_in bf_feat_make(const double* tsdf, const double* Lambda, const double* acc, const int32_t* w,
                               const int32_t* nbr, const int32_t* deg, int32_t T, double h) {
  return bf_feat_in{tsdf, Lambda, acc, w, nbr, deg, T, h, 1.0 / h, 1.0 / (h * h), 1.0 / (2.0 * h),
                    T > 0 ? 1.0 / (double)T : 0.0};
}

// Features 0..7 of band voxel v into f[0..7].
__device__ __forceinline__ void bf_features_0_7(int64_t v, const bf_feat_in& s, float* f) {
#pragma clang fp contract(off)
  const double* a = s.acc + v * 5;
  const double cnt = a[0];
  const double rc = cnt > 0.0 ? 1.0 / cnt : 0.0;
  const double my = a[1] * rc;
  const double vy = cnt > 0.0 ? a[2] * rc - my * my : 0.0;
  const double ms = a[3] * rc;
  f[0] = (float)(s.tsdf[v] * s.ih);
  f[1] = (float)log(1.0 + (double)s.w[v]);
  f[2] = (float)((double)s.deg[v] * (1.0 / 6.0));
  f[3] = (float)(cnt * s.iT);
  f[4] = (float)(my * s.ih);
  f[5] = (float)(vy * s.ih2);
  f[6] = (float)(ms * s.ih);
  f[7] = (float)(a[4] * s.ih);
}

// Features 8..11 of band voxel v into f[0..3].
__device__ __forceinline__ void bf_features_8_11(int64_t v, const bf_feat_in& s, float* f) {
#pragma clang fp contract(off)
  const double h = s.h;
  f[0] = (float)log(s.Lambda[v] * (h * h) + 1.0);
  const double tv = s.tsdf[v];
  const int32_t* nb = s.nbr + v * 6;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const int32_t m = nb[2 * ax], p = nb[2 * ax + 1];
    const double tm = m >= 0 ? s.tsdf[m] : tv;
    const double tp = p >= 0 ? s.tsdf[p] : tv;
    f[1 + ax] = (float)((tp - tm) * s.i2h);
  }
}
