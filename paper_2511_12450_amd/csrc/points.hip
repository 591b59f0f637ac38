// Point sources in the layered medium: boundary values of the layered
// Green's function (Sec. 3.1, eq. layeredGreensfun) at the collocation
// points.  G(r | s) is the field at r of a unit point source at s; it
// satisfies the transmission conditions at every interface and radiates, so
// with s inside a scatterer its boundary values are the data of an exterior
// problem whose solution is G(. | s) itself (the manufactured solution of
// Sec. 5, Example 1), and with s outside, -G(. | s) on the boundary is the
// data of a point-source incident field.
#include "lm_internal.hpp"
#include "sommerfeld.hpp"

// g[r][i] = G(c_i | s_r) = delta_{l_i l_r} (i/4) H_0(k |c_i - s_r|) + G^r(c_i | s_r),
// the reaction part by direct Sommerfeld quadrature.  Grid (ceil(N / 128), R).
__global__ void __launch_bounds__(128) k_point_rhs(MediumDev m, int N, const double* __restrict__ sx,
                                                   const double* __restrict__ sy, const int* __restrict__ sl,
                                                   const double* __restrict__ cx, const double* __restrict__ cy,
                                                   const int* __restrict__ lay, double2* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= N) return;
  const int li = lay[i], ls = sl[r];
  const double dx = cx[i] - sx[r], dy = cy[i] - sy[r];
  zd v = lmq::reaction_direct(m, li, ls, fabs(dx), cy[i], sy[r]);
  if (li == ls) {
    const double kr = m.k[li] * sqrt(dx * dx + dy * dy);
    v += zd(-0.25 * y0(kr), 0.25 * j0(kr));
  }
  g[(int64_t)r * N + i] = make_double2(v.re, v.im);
}

extern "C" lm_status lm_point_source_rhs(lm_geom g, int n_src, const double* src_xy, void* g_dev, void* hip_stream) {
  LM_CHECK(g, LM_EINVAL, "geom is NULL");
  LM_CHECK(n_src >= 1 && src_xy && g_dev, LM_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<double> x(n_src), y(n_src);
  std::vector<int32_t> l(n_src);
  for (int r = 0; r < n_src; ++r) {
    x[r] = src_xy[2 * r];
    y[r] = src_xy[2 * r + 1];
    LM_CHECK(std::isfinite(x[r]) && std::isfinite(y[r]), LM_EINVAL, "non-finite source position");
    l[r] = layer_of(g->m, y[r]);
    for (int64_t i = 0; i < g->N; ++i)
      LM_CHECK(g->cx[i] != x[r] || g->cy[i] != y[r], LM_EINVAL, "source %d coincides with collocation point %lld", r,
               (long long)i);
  }
  DevBuf dx, dy, dl;
  LM_TRY(upload(dx, x.data(), n_src * sizeof(double), s));
  LM_TRY(upload(dy, y.data(), n_src * sizeof(double), s));
  LM_TRY(upload(dl, l.data(), n_src * sizeof(int32_t), s));
  const int N = (int)g->N;
  hipLaunchKernelGGL(k_point_rhs, dim3(div_up(N, 128), n_src), dim3(128), 0, s, g->m, N, dx.as<double>(),
                     dy.as<double>(), dl.as<int>(), g->d_cx.as<double>(), g->d_cy.as<double>(), g->d_layer.as<int>(),
                     (double2*)g_dev);
  LM_TRY_HIP(hipGetLastError());
  LM_TRY_HIP(hipStreamSynchronize(s));  // temporaries are freed on return
  return LM_OK;
}

extern "C" lm_status lm_point_far_field(lm_layers layers, int n_src, const double* src_xy, int n_obs,
                                        const double* obs, void* out_dev, void* hip_stream) {
  LM_CHECK(layers, LM_EINVAL, "layers is NULL");
  LM_CHECK(n_src >= 1 && n_obs >= 1 && src_xy && obs && out_dev, LM_EINVAL, "bad arguments");
  for (int r = 0; r < 2 * n_src; ++r) LM_CHECK(std::isfinite(src_xy[r]), LM_EINVAL, "non-finite source position");
  for (int j = 0; j < n_obs; ++j)
    LM_CHECK(std::isfinite(obs[j]) && std::fabs(std::sin(obs[j])) > 1e-12, LM_EINVAL,
             "observation angles must be finite and not horizontal");
  return point_far_field_launch(layers->m, n_src, src_xy, n_obs, obs, out_dev, (hipStream_t)hip_stream);
}
