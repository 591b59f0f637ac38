// Right-hand side (incident + background field) and far-field patterns.
#include <algorithm>
#include <cstring>

#include "lm_internal.hpp"

// ------------------------------------------------------------------- rhs --
// Sec. 2.2: u^b = A_l e^{i(kx x + k_{l,y} y)} + B_l e^{i(kx x - k_{l,y} y)} with
// A_0 = R~_{01} e^{2 i k_{0,y} d_0}, A_l = R~_{l,l+1} T~_{0l} e^{2 i k_{l,y} d_l},
// B_l = T~_{0l} (B_0 = 0, A_L = 0), all at lam = kx = k_0 cos(theta).
struct BgAmp {
  double kx;
  zd ky[LM_MAXL], A[LM_MAXL], B[LM_MAXL];
};

__global__ void k_background(MediumDev m, int R, const double* __restrict__ theta, BgAmp* __restrict__ amp) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const double kx = m.k[0] * cos(theta[r]);
  StackAt st;
  stack_at(m, zd(kx, 0.0), st);
  BgAmp a;
  a.kx = kx;
  for (int l = 0; l <= m.L; ++l) {
    a.ky[l] = st.ky[l];
    a.A[l] = a.B[l] = zd(0.0, 0.0);
  }
  a.A[0] = st.Rdn[0] * zexp(zd(0.0, 2.0 * m.d[0]) * st.ky[0]);
  for (int l = 1; l <= m.L; ++l) {
    zd T = gen_transmission(m, st, 0, l);
    a.B[l] = T;
    if (l < m.L) a.A[l] = st.Rdn[l] * T * zexp(zd(0.0, 2.0 * m.d[l]) * st.ky[l]);
  }
  amp[r] = a;
}

__global__ void k_rhs(int N, int R, const BgAmp* __restrict__ amp, const double* __restrict__ cx,
                      const double* __restrict__ cy, const int* __restrict__ lay, const double* __restrict__ theta,
                      const MediumDev m, double2* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= N) return;
  const BgAmp& a = amp[r];
  const int l = lay[i];
  const double x = cx[i], y = cy[i];
  const zd ex = zexp(zd(0.0, a.kx * x));
  zd u = a.A[l] * zexp(zd(0.0, y) * a.ky[l]) + a.B[l] * zexp(zd(0.0, -y) * a.ky[l]);
  if (l == 0) u += zexp(zd(0.0, -m.k[0] * sin(theta[r]) * y));
  u = -(u * ex);
  g[(int64_t)r * N + i] = make_double2(u.re, u.im);
}

// Sound-hard / impedance scatterers: g = -(d_n + i beta)(u^inc + u^b), with
// d/dx = i kx and d/dy = +-i k_{l,y} on the up / down-going terms.
__global__ void k_rhs_bc(int N, int R, const BgAmp* __restrict__ amp, const double* __restrict__ cx,
                         const double* __restrict__ cy, const double* __restrict__ nx, const double* __restrict__ ny,
                         const int* __restrict__ lay, const double* __restrict__ theta, const MediumDev m, double beta,
                         double2* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= N) return;
  const BgAmp& a = amp[r];
  const int l = lay[i];
  const double x = cx[i], y = cy[i];
  const zd ex = zexp(zd(0.0, a.kx * x));
  const zd up = a.A[l] * zexp(zd(0.0, y) * a.ky[l]), dn = a.B[l] * zexp(zd(0.0, -y) * a.ky[l]);
  zd u = up + dn;
  zd uy = (up - dn) * (zd(0.0, 1.0) * a.ky[l]);
  if (l == 0) {
    const double k0y = m.k[0] * sin(theta[r]);
    const zd ui = zexp(zd(0.0, -k0y * y));
    u += ui;
    uy += ui * zd(0.0, -k0y);
  }
  u = u * ex;
  uy = uy * ex;
  const zd ux = u * zd(0.0, a.kx);
  const zd v = -(ux * nx[i] + uy * ny[i] + u * zd(0.0, beta));
  g[(int64_t)r * N + i] = make_double2(v.re, v.im);
}

size_t rhs_scratch_bytes(int R) { return (size_t)std::max(R, 1) * sizeof(BgAmp); }

lm_status rhs_launch_dev(lm_geom_s* g, int R, const double* theta_dev, void* scratch, void* g_dev, hipStream_t s) {
  BgAmp* amp = static_cast<BgAmp*>(scratch);
  hipLaunchKernelGGL(k_background, dim3(div_up(R, 64)), dim3(64), 0, s, g->m, R, theta_dev, amp);
  LM_TRY_HIP(hipGetLastError());
  const int N = (int)g->N;
  if (g->bc == LM_BC_DIRICHLET)
    hipLaunchKernelGGL(k_rhs, dim3(div_up(N, 256), R), dim3(256), 0, s, N, R, amp, g->d_cx.as<double>(),
                       g->d_cy.as<double>(), g->d_layer.as<int>(), theta_dev, g->m, (double2*)g_dev);
  else
    hipLaunchKernelGGL(k_rhs_bc, dim3(div_up(N, 256), R), dim3(256), 0, s, N, R, amp, g->d_cx.as<double>(),
                       g->d_cy.as<double>(), g->d_nx.as<double>(), g->d_ny.as<double>(), g->d_layer.as<int>(),
                       theta_dev, g->m, g->robin_beta, (double2*)g_dev);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

lm_status rhs_launch(lm_geom_s* g, int R, const double* theta_host, void* g_dev, hipStream_t s) {
  DevBuf th, amp;
  LM_TRY(upload(th, theta_host, R * sizeof(double), s));
  LM_TRY(amp.alloc(rhs_scratch_bytes(R)));
  LM_TRY(rhs_launch_dev(g, R, th.as<double>(), amp.p, g_dev, s));
  LM_TRY_HIP(hipStreamSynchronize(s));  // temporaries are freed on return
  return LM_OK;
}

// ------------------------------------------------------ values by value --
// Up to PUT_F64 doubles travel in the kernel arguments, so the copy reads no
// host memory after the launch call returns (no staging buffer to keep alive).
constexpr int PUT_F64 = 128;
struct F64Chunk {
  double v[PUT_F64];
};

__global__ void __launch_bounds__(PUT_F64) k_put_f64(F64Chunk a, int n, double* __restrict__ dst) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = a.v[i];
}

lm_status put_f64_async(const double* host, int n, double* dev, hipStream_t s) {
  for (int o = 0; o < n; o += PUT_F64) {
    F64Chunk a;
    const int k = std::min(PUT_F64, n - o);
    std::memcpy(a.v, host + o, (size_t)k * sizeof(double));
    hipLaunchKernelGGL(k_put_f64, dim3(1), dim3(PUT_F64), 0, s, a, k, dev + o);
    LM_TRY_HIP(hipGetLastError());
  }
  return LM_OK;
}

// -------------------------------------------------------------- far field --
// Stationary phase of the single-layer representation (eq. integralrep) in
// side form: for an observation direction in the top layer the target side is
// B of layer 0 (h_t = y + d_0), so u^s ~ e^{i k_0 R}/sqrt(R) u_inf with
//   u_inf = e^{-i pi/4} sqrt(k_0/2pi) |sin t| sum_e |Gamma_e| phi_e e^{-i lam x_e} a_e,
//   a_e = [l_e = 0] i/(2 k_{0,y}) e^{-i k_{0,y} y_e}
//       + e^{i k_{0,y} d_0} sum_s S^{(B,s)}_{0 l_e}(lam) e^{i k_{l_e,y} h_s(y_e)},
// lam = k_0 cos t; the bottom layer mirrors this with side T of layer L.
// One workgroup: an angle, FF_RB right-hand sides (the amplitudes a_e are
// evaluated once for all of them) and a chunk of elements; with several
// chunks (grid z) each writes its partial sums to out + z R n_obs and
// k_far_field_sum adds them in chunk order.  16 right-hand sides per
// workgroup (64k elements, 682 angles: 2.61 -> 2.24 ms at R = 21 and
// 7.42 -> 5.86 ms at R = 64 against 8; 12 was no better).
constexpr int FF_RB = 16;

__global__ void __launch_bounds__(256) k_far_field(MediumDev m, int N, int R, const double* __restrict__ obs,
                                                   const double* __restrict__ cx, const double* __restrict__ cy,
                                                   const double* __restrict__ w, const int* __restrict__ lay,
                                                   const double2* __restrict__ phi, double2* __restrict__ out,
                                                   int n_obs, int chunk) {
  const int o = blockIdx.x;
  const int r0 = blockIdx.y * FF_RB;
  const int nr = min(FF_RB, R - r0);
  const int e0 = blockIdx.z * chunk, e1 = min(N, e0 + chunk);
  out += (int64_t)blockIdx.z * R * n_obs;
  const double th = obs[o];
  const bool top = sin(th) > 0.0;
  const int lt = top ? 0 : m.L;
  const int tside = top ? SIDE_B : SIDE_T;
  const double kk = m.k[lt];
  const double lam = kk * cos(th);
  __shared__ double2 Ssh[LM_MAXL][2];  // S^{(tside, s)}_{lt, ls}, premultiplied by the target constant
  __shared__ double2 kysh[LM_MAXL];
  if (threadIdx.x <= (unsigned)m.L) {
    const int ls = threadIdx.x;
    StackAt st;
    stack_at(m, zd(lam, 0.0), st);
    zd S[4];
    for (int c = 0; c < 4; ++c) S[c] = zd(0.0, 0.0);
    side_densities(m, st, lt, ls, 0xFu, S);
    const zd tc = top ? zexp(zd(0.0, m.d[0]) * st.ky[0]) : zexp(zd(0.0, -m.d[m.L - 1]) * st.ky[m.L]);
    for (int s = 0; s < 2; ++s) {
      const int c = tside + 2 * s;
      const zd v = (side_exists(m, lt, tside) && side_exists(m, ls, s)) ? S[c] * tc : zd(0.0, 0.0);
      Ssh[ls][s] = make_double2(v.re, v.im);
    }
    kysh[ls] = make_double2(st.ky[ls].re, st.ky[ls].im);
  }
  __syncthreads();
  zd acc[FF_RB];
  for (int e = e0 + (int)threadIdx.x; e < e1; e += blockDim.x) {
    const int l = lay[e];
    const double y = cy[e];
    zd a(0.0, 0.0);
    const zd kyl(kysh[l].x, kysh[l].y);
    if (l == lt) a += (zd(0.0, 0.5) / kyl) * zexp(zd(0.0, top ? -y : y) * kyl);
    for (int s = 0; s < 2; ++s) {
      if (!side_exists(m, l, s)) continue;
      a += zd(Ssh[l][s].x, Ssh[l][s].y) * zexp(zd(0.0, side_h(m, l, s, y)) * kyl);
    }
    a = a * zexp(zd(0.0, -lam * cx[e])) * w[e];
    for (int q = 0; q < FF_RB; ++q) {
      if (q < nr) {
        const double2 p = phi[(int64_t)(r0 + q) * N + e];
        acc[q] += a * zd(p.x, p.y);
      }
    }
  }
  __shared__ double red[2][FF_RB][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int q = 0; q < FF_RB; ++q) {
    double a = acc[q].re, b = acc[q].im;
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_down(a, off, 64);
      b += __shfl_down(b, off, 64);
    }
    if (lane == 0) {
      red[0][q][wv] = a;
      red[1][q][wv] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < (unsigned)nr) {
    const int q = threadIdx.x;
    zd v(red[0][q][0] + red[0][q][1] + red[0][q][2] + red[0][q][3],
         red[1][q][0] + red[1][q][1] + red[1][q][2] + red[1][q][3]);
    const zd pre = zexp(zd(0.0, -0.25 * M_PI)) * (sqrt(kk / (2.0 * M_PI)) * fabs(sin(th)));
    v = v * pre;
    out[(int64_t)(r0 + q) * n_obs + o] = make_double2(v.re, v.im);
  }
}

// out[i] = sum over z of part[z n + i], z = 0..nz-1 in order.
__global__ void __launch_bounds__(256) k_far_field_sum(int64_t n, int nz, const double2* __restrict__ part,
                                                       double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double2 v = part[i];
  for (int z = 1; z < nz; ++z) {
    const double2 p = part[(int64_t)z * n + i];
    v.x += p.x;
    v.y += p.y;
  }
  out[i] = v;
}

namespace {
// Element chunks of a far-field launch: enough workgroups to fill the GPU
// (about 2048), chunks of at least 4096 elements, at most FF_MAXZ of them.
constexpr int FF_MAXZ = 8;
int ff_chunks(int N, int R, int n_obs) {
  const int64_t wg = (int64_t)n_obs * div_up(R, FF_RB);
  const int want = (int)std::min<int64_t>(FF_MAXZ, std::max<int64_t>(1, div_up(2048, std::max<int64_t>(wg, 1))));
  return std::max(1, std::min(want, (int)div_up(N, 4096)));
}
}  // namespace

size_t farfield_work_bytes(lm_geom_s* g, int R, int n_obs) {
  const int nz = ff_chunks((int)g->N, R, n_obs);
  return nz > 1 ? (size_t)nz * R * n_obs * sizeof(double2) : 0;
}

lm_status farfield_launch_dev(lm_geom_s* g, int R, const void* phi, int n_obs, const double* obs_dev, void* out,
                              void* work, hipStream_t s) {
  const int N = (int)g->N;
  const int nz = ff_chunks(N, R, n_obs);
  const int chunk = (int)div_up(div_up(N, nz), 256) * 256;
  double2* dst = nz > 1 ? (double2*)work : (double2*)out;
  LM_CHECK(nz == 1 || work, LM_EINVAL, "far field: a work buffer is needed");
  hipLaunchKernelGGL(k_far_field, dim3(n_obs, div_up(R, FF_RB), nz), dim3(256), 0, s, g->m, N, R, obs_dev,
                     g->d_cx.as<double>(), g->d_cy.as<double>(), g->d_w.as<double>(), g->d_layer.as<int>(),
                     (const double2*)phi, dst, n_obs, chunk);
  LM_TRY_HIP(hipGetLastError());
  if (nz > 1) {
    const int64_t n = (int64_t)R * n_obs;
    hipLaunchKernelGGL(k_far_field_sum, dim3(div_up(n, 256)), dim3(256), 0, s, n, nz, (const double2*)work,
                       (double2*)out);
    LM_TRY_HIP(hipGetLastError());
  }
  return LM_OK;
}

lm_status farfield_launch(lm_geom_s* g, int R, const void* phi, int n_obs, const double* obs_host, void* out,
                          hipStream_t s) {
  DevBuf ob, wk;
  LM_TRY(upload(ob, obs_host, n_obs * sizeof(double), s));
  LM_TRY(wk.alloc(farfield_work_bytes(g, R, n_obs)));
  LM_TRY(farfield_launch_dev(g, R, phi, n_obs, ob.as<double>(), out, wk.p, s));
  LM_TRY_HIP(hipStreamSynchronize(s));  // before ob and wk are freed
  return LM_OK;
}

// Far-field patterns of unit point sources: the same sum with one term per
// source (weight 1, density 1): source r is "element" r and the density of
// right-hand side r is the r-th unit vector.
lm_status point_far_field_launch(const MediumDev& m, int R, const double* src_xy_host, int n_obs,
                                 const double* obs_host, void* out, hipStream_t s) {
  std::vector<double> x(R), y(R), w(R, 1.0);
  std::vector<int32_t> lay(R);
  std::vector<double2> eye((size_t)R * R, make_double2(0.0, 0.0));
  for (int r = 0; r < R; ++r) {
    x[r] = src_xy_host[2 * r];
    y[r] = src_xy_host[2 * r + 1];
    lay[r] = layer_of(m, y[r]);
    eye[(size_t)r * R + r] = make_double2(1.0, 0.0);
  }
  DevBuf ob, dx, dy, dw, dl, dphi;
  LM_TRY(upload(ob, obs_host, n_obs * sizeof(double), s));
  LM_TRY(upload(dx, x.data(), R * sizeof(double), s));
  LM_TRY(upload(dy, y.data(), R * sizeof(double), s));
  LM_TRY(upload(dw, w.data(), R * sizeof(double), s));
  LM_TRY(upload(dl, lay.data(), R * sizeof(int32_t), s));
  LM_TRY(upload(dphi, eye.data(), eye.size() * sizeof(double2), s));
  hipLaunchKernelGGL(k_far_field, dim3(n_obs, div_up(R, FF_RB), 1), dim3(256), 0, s, m, R, R, ob.as<double>(),
                     dx.as<double>(), dy.as<double>(), dw.as<double>(), dl.as<int>(), dphi.as<double2>(),
                     (double2*)out, n_obs, R);
  LM_TRY_HIP(hipGetLastError());
  LM_TRY_HIP(hipStreamSynchronize(s));  // temporaries are freed on return
  return LM_OK;
}
