// Device-resident restarted GMRES for K phi = g with n_rhs right-hand sides
// advanced in lockstep (Sec. 3.3 and Sec. 5: GMRES, relative tolerance).
//
// x0 = 0; right preconditioning (the monitored residual is the true one);
// classical Gram-Schmidt with a second pass (CGS2) -- both passes are one
// batched dot-product kernel and one update kernel over the basis, so the
// basis is streamed from HBM twice per pass instead of once per vector as in
// modified Gram-Schmidt.  Arnoldi coefficients, norms and Givens rotations are
// FP64 for both precisions; with LM_MIXED only the matvec runs in FP32.  The
// (j+1) x n_rhs Hessenberg column comes back to the host each iteration and
// the rotations are applied there.
#include <algorithm>
#include <cmath>
#include <complex>

#include "lm_internal.hpp"

// h[r][i] = sum_n conj(V[i][r][n]) w[r][n], i = 0..j  (grid: (j+1) x R)
__global__ void __launch_bounds__(256) k_dots(int N, int R, const double2* __restrict__ V,
                                              const double2* __restrict__ w, double2* __restrict__ h, int ldh) {
  const int i = blockIdx.x, r = blockIdx.y;
  const double2* v = V + ((int64_t)i * R + r) * N;
  const double2* x = w + (int64_t)r * N;
  double a = 0, b = 0;
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    const double2 p = v[n], q = x[n];
    a += p.x * q.x + p.y * q.y;
    b += p.x * q.y - p.y * q.x;
  }
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  __shared__ double red[2][4];
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) h[(int64_t)r * ldh + i] = make_double2(red[0][0] + red[0][1] + red[0][2] + red[0][3],
                                                             red[1][0] + red[1][1] + red[1][2] + red[1][3]);
}

// w[r] -= sum_{i<=j} V[i][r] h[r][i]
__global__ void k_update(int N, int R, int j, const double2* __restrict__ V, double2* __restrict__ w,
                         const double2* __restrict__ h, int ldh) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (n >= N) return;
  double2 acc = w[(int64_t)r * N + n];
  for (int i = 0; i <= j; ++i) {
    const double2 c = h[(int64_t)r * ldh + i];
    const double2 v = V[((int64_t)i * R + r) * N + n];
    acc.x -= c.x * v.x - c.y * v.y;
    acc.y -= c.x * v.y + c.y * v.x;
  }
  w[(int64_t)r * N + n] = acc;
}

// nrm[r] = ||w_r||^2
__global__ void __launch_bounds__(256) k_norm2(int N, const double2* __restrict__ w, double* __restrict__ nrm) {
  const int r = blockIdx.x;
  const double2* x = w + (int64_t)r * N;
  double a = 0;
  for (int n = threadIdx.x; n < N; n += blockDim.x) a += x[n].x * x[n].x + x[n].y * x[n].y;
  for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) nrm[r] = red[0] + red[1] + red[2] + red[3];
}

// out[r] = in[r] * scale[r]
__global__ void k_scale(int N, const double2* __restrict__ in, const double* __restrict__ scale,
                        double2* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (n >= N) return;
  const double s = scale[r];
  const double2 v = in[(int64_t)r * N + n];
  out[(int64_t)r * N + n] = make_double2(v.x * s, v.y * s);
}

// z[r] = sum_{i < cnt} V[i][r] y[r][i]
__global__ void k_lincomb(int N, int R, int cnt, const double2* __restrict__ V, const double2* __restrict__ y,
                          int ldy, double2* __restrict__ z) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (n >= N) return;
  double2 acc = make_double2(0, 0);
  for (int i = 0; i < cnt; ++i) {
    const double2 c = y[(int64_t)r * ldy + i];
    const double2 v = V[((int64_t)i * R + r) * N + n];
    acc.x += c.x * v.x - c.y * v.y;
    acc.y += c.x * v.y + c.y * v.x;
  }
  z[(int64_t)r * N + n] = acc;
}

// out = a + sa * b (elementwise over R*N)
__global__ void k_axpby(int64_t n, const double2* __restrict__ a, double sa, const double2* __restrict__ b,
                        double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = make_double2(a[i].x + sa * b[i].x, a[i].y + sa * b[i].y);
}

__global__ void k_c128_to_c64(int64_t n, const double2* __restrict__ a, float2* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}
__global__ void k_c64_to_c128(int64_t n, const float2* __restrict__ a, double2* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = make_double2((double)a[i].x, (double)a[i].y);
}

namespace {

struct Work {
  DevBuf V, w, z, h, y, nrm, scale, x32, y32, mz;
  std::vector<double2> hh;
};

// y = K M x in FP64 storage; the matvec itself runs in the requested precision.
lm_status apply_KM(lm_geom_s* g, int precision, int R, const double2* x, double2* y, bool use_pre, Work& wk,
                   hipStream_t s) {
  const int64_t N = g->N, n = (int64_t)R * N;
  const double2* xin = x;
  if (use_pre) {
    LM_TRY(precond_apply(g, R, x, wk.mz.p, s));
    xin = wk.mz.as<double2>();
  }
  if (precision == LM_FP64) return geom_matvec(g, precision, R, xin, y, s);
  hipLaunchKernelGGL(k_c128_to_c64, dim3(div_up(n, 256)), dim3(256), 0, s, n, xin, wk.x32.as<float2>());
  LM_TRY(geom_matvec(g, precision, R, wk.x32.p, wk.y32.p, s));
  hipLaunchKernelGGL(k_c64_to_c128, dim3(div_up(n, 256)), dim3(256), 0, s, n, wk.y32.as<float2>(), y);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

}  // namespace

lm_status gmres_run(lm_geom_s* g, int precision, int R, const void* g_dev, const lm_gmres_opts* o, void* phi_dev,
                    lm_solve_report* rep, hipStream_t s) {
  const int64_t N = g->N, n = (int64_t)R * N;
  const int m = std::max(1, std::min(o->restart, o->max_iter));
  const bool use_pre = o->precond && g->pre;
  const double2* gv = (const double2*)g_dev;
  double2* phi = (double2*)phi_dev;
  Work wk;
  LM_TRY(wk.V.alloc((size_t)(m + 1) * n * sizeof(double2)));
  LM_TRY(wk.w.alloc(n * sizeof(double2)));
  LM_TRY(wk.z.alloc(n * sizeof(double2)));
  LM_TRY(wk.h.alloc((size_t)2 * R * (m + 1) * sizeof(double2)));
  LM_TRY(wk.y.alloc((size_t)R * (m + 1) * sizeof(double2)));
  LM_TRY(wk.nrm.alloc(R * sizeof(double)));
  LM_TRY(wk.scale.alloc(R * sizeof(double)));
  if (precision == LM_MIXED) {
    LM_TRY(wk.x32.alloc(n * sizeof(float2)));
    LM_TRY(wk.y32.alloc(n * sizeof(float2)));
  }
  if (use_pre) LM_TRY(wk.mz.alloc(n * sizeof(double2)));
  double2* V = wk.V.as<double2>();
  double2* w = wk.w.as<double2>();
  double2* h1 = wk.h.as<double2>();
  double2* h2 = h1 + (size_t)R * (m + 1);
  const int ldh = m + 1;
  const dim3 gN(div_up(N, 256), R), b256(256);

  LM_TRY_HIP(hipMemsetAsync(phi, 0, n * sizeof(double2), s));
  // ||g_r||
  std::vector<double> gnorm(R), nrm_h(R), scale_h(R);
  hipLaunchKernelGGL(k_norm2, dim3(R), b256, 0, s, (int)N, gv, wk.nrm.as<double>());
  LM_TRY_HIP(hipMemcpyAsync(gnorm.data(), wk.nrm.p, R * sizeof(double), hipMemcpyDeviceToHost, s));
  LM_TRY_HIP(hipStreamSynchronize(s));
  for (auto& v : gnorm) v = std::sqrt(v);

  std::vector<int> its(R, 0);
  std::vector<char> done(R, 0);
  std::vector<double> res(R, 1.0);
  for (int r = 0; r < R; ++r)
    if (gnorm[r] == 0.0) {
      done[r] = 1;
      res[r] = 0.0;
    }
  typedef std::complex<double> C;
  std::vector<C> H((size_t)R * (m + 1) * m), cs((size_t)R * m), sn((size_t)R * m), e1((size_t)R * (m + 1));
  std::vector<int> cols(R, 0);
  std::vector<double2> hbuf((size_t)2 * R * (m + 1)), ybuf((size_t)R * (m + 1));
  int total = 0;
  bool first = true;
  while (true) {
    // residual r0 = g - K M phi  (phi = 0 on the first cycle)
    if (first) {
      LM_TRY_HIP(hipMemcpyAsync(w, gv, n * sizeof(double2), hipMemcpyDeviceToDevice, s));
    } else {
      LM_TRY(apply_KM(g, precision, R, wk.z.as<double2>(), w, use_pre, wk, s));  // z holds phi_hat (see below)
      hipLaunchKernelGGL(k_axpby, dim3(div_up(n, 256)), b256, 0, s, n, gv, -1.0, w, w);
    }
    hipLaunchKernelGGL(k_norm2, dim3(R), b256, 0, s, (int)N, w, wk.nrm.as<double>());
    LM_TRY_HIP(hipMemcpyAsync(nrm_h.data(), wk.nrm.p, R * sizeof(double), hipMemcpyDeviceToHost, s));
    LM_TRY_HIP(hipStreamSynchronize(s));
    std::vector<double> beta(R);
    for (int r = 0; r < R; ++r) {
      beta[r] = std::sqrt(nrm_h[r]);
      scale_h[r] = beta[r] > 0 ? 1.0 / beta[r] : 0.0;
      if (!done[r]) res[r] = beta[r] / gnorm[r];
      if (!done[r] && res[r] <= o->tol) done[r] = 1;
      cols[r] = 0;
      for (int i = 0; i <= m; ++i) e1[(size_t)r * (m + 1) + i] = 0.0;
      e1[(size_t)r * (m + 1)] = beta[r];
    }
    LM_TRY_HIP(hipMemcpyAsync(wk.scale.p, scale_h.data(), R * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_scale, gN, b256, 0, s, (int)N, w, wk.scale.as<double>(), V);
    bool all_done = std::all_of(done.begin(), done.end(), [](char c) { return c != 0; });
    std::vector<char> active(R);
    for (int r = 0; r < R; ++r) active[r] = !done[r];
    int j = 0;
    for (; j < m && !all_done && total < o->max_iter; ++j) {
      double2* Vj = V + (size_t)j * n;
      LM_TRY(apply_KM(g, precision, R, Vj, w, use_pre, wk, s));
      // CGS2
      hipLaunchKernelGGL(k_dots, dim3(j + 1, R), b256, 0, s, (int)N, R, V, w, h1, ldh);
      hipLaunchKernelGGL(k_update, gN, b256, 0, s, (int)N, R, j, V, w, h1, ldh);
      hipLaunchKernelGGL(k_dots, dim3(j + 1, R), b256, 0, s, (int)N, R, V, w, h2, ldh);
      hipLaunchKernelGGL(k_update, gN, b256, 0, s, (int)N, R, j, V, w, h2, ldh);
      hipLaunchKernelGGL(k_norm2, dim3(R), b256, 0, s, (int)N, w, wk.nrm.as<double>());
      LM_TRY_HIP(hipGetLastError());
      LM_TRY_HIP(hipMemcpyAsync(hbuf.data(), h1, (size_t)2 * R * (m + 1) * sizeof(double2), hipMemcpyDeviceToHost, s));
      LM_TRY_HIP(hipMemcpyAsync(nrm_h.data(), wk.nrm.p, R * sizeof(double), hipMemcpyDeviceToHost, s));
      LM_TRY_HIP(hipStreamSynchronize(s));
      ++total;
      for (int r = 0; r < R; ++r) {
        const double hn = std::sqrt(nrm_h[r]);
        scale_h[r] = hn > 1e-300 ? 1.0 / hn : 0.0;
        if (!active[r]) continue;
        C* Hc = &H[((size_t)r * m + j) * (m + 1)];  // column j of r
        for (int i = 0; i <= j; ++i) {
          const double2 a = hbuf[(size_t)r * ldh + i], b = hbuf[(size_t)R * ldh + (size_t)r * ldh + i];
          Hc[i] = C(a.x + b.x, a.y + b.y);
        }
        Hc[j + 1] = hn;
        C* csr = &cs[(size_t)r * m];
        C* snr = &sn[(size_t)r * m];
        for (int i = 0; i < j; ++i) {
          const C a = Hc[i], b = Hc[i + 1];
          Hc[i] = std::conj(csr[i]) * a + std::conj(snr[i]) * b;
          Hc[i + 1] = -snr[i] * a + csr[i] * b;
        }
        const C a = Hc[j], b = Hc[j + 1];
        const double rr = std::hypot(std::abs(a), std::abs(b));
        csr[j] = rr > 0 ? a / rr : C(1.0);
        snr[j] = rr > 0 ? b / rr : C(0.0);
        Hc[j] = std::conj(csr[j]) * a + std::conj(snr[j]) * b;
        Hc[j + 1] = 0.0;
        C* er = &e1[(size_t)r * (m + 1)];
        er[j + 1] = -snr[j] * er[j];
        er[j] = std::conj(csr[j]) * er[j];
        cols[r] = j + 1;
        its[r] += 1;
        res[r] = std::abs(er[j + 1]) / gnorm[r];
        if (res[r] <= o->tol || hn <= 1e-300) {
          done[r] = 1;
          active[r] = 0;
        }
      }
      all_done = std::all_of(done.begin(), done.end(), [](char c) { return c != 0; });
      if (!all_done && j + 1 < m && total < o->max_iter) {
        LM_TRY_HIP(hipMemcpyAsync(wk.scale.p, scale_h.data(), R * sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_scale, gN, b256, 0, s, (int)N, w, wk.scale.as<double>(), V + (size_t)(j + 1) * n);
      }
    }
    // y_r = H_r^{-1} e1_r; phi_hat += V y (phi = M phi_hat at the end)
    int maxc = 0;
    for (int r = 0; r < R; ++r) {
      const int c = cols[r];
      maxc = std::max(maxc, c);
      std::vector<C> yv(c);
      for (int i = c - 1; i >= 0; --i) {
        C acc = e1[(size_t)r * (m + 1) + i];
        for (int k2 = i + 1; k2 < c; ++k2) acc -= H[((size_t)r * m + k2) * (m + 1) + i] * yv[k2];
        yv[i] = acc / H[((size_t)r * m + i) * (m + 1) + i];
      }
      for (int i = 0; i <= m; ++i) {
        const C v = i < c ? yv[i] : C(0.0);
        ybuf[(size_t)r * (m + 1) + i] = make_double2(v.real(), v.imag());
      }
    }
    if (maxc > 0) {
      LM_TRY_HIP(hipMemcpyAsync(wk.y.p, ybuf.data(), (size_t)R * (m + 1) * sizeof(double2), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_lincomb, gN, b256, 0, s, (int)N, R, maxc, V, wk.y.as<double2>(), m + 1, w);
      // z accumulates phi_hat across restarts (phi = M z)
      if (first) {
        LM_TRY_HIP(hipMemcpyAsync(wk.z.p, w, n * sizeof(double2), hipMemcpyDeviceToDevice, s));
      } else {
        hipLaunchKernelGGL(k_axpby, dim3(div_up(n, 256)), b256, 0, s, n, wk.z.as<double2>(), 1.0, w,
                           wk.z.as<double2>());
      }
    } else if (first) {
      LM_TRY_HIP(hipMemsetAsync(wk.z.p, 0, n * sizeof(double2), s));
    }
    LM_TRY_HIP(hipGetLastError());
    first = false;
    if (all_done || total >= o->max_iter) break;
  }
  // phi = M z
  if (use_pre) {
    LM_TRY(precond_apply(g, R, wk.z.p, phi, s));
  } else {
    LM_TRY_HIP(hipMemcpyAsync(phi, wk.z.p, n * sizeof(double2), hipMemcpyDeviceToDevice, s));
  }
  // true residual
  LM_TRY(apply_KM(g, precision, R, wk.z.as<double2>(), w, use_pre, wk, s));
  hipLaunchKernelGGL(k_axpby, dim3(div_up(n, 256)), b256, 0, s, n, gv, -1.0, w, w);
  hipLaunchKernelGGL(k_norm2, dim3(R), b256, 0, s, (int)N, w, wk.nrm.as<double>());
  LM_TRY_HIP(hipMemcpyAsync(nrm_h.data(), wk.nrm.p, R * sizeof(double), hipMemcpyDeviceToHost, s));
  LM_TRY_HIP(hipStreamSynchronize(s));
  bool ok = true;
  for (int r = 0; r < R; ++r) {
    rep[r].iterations = its[r];
    rep[r].rel_residual = gnorm[r] > 0 ? std::sqrt(nrm_h[r]) / gnorm[r] : 0.0;
    if (!done[r]) ok = false;
  }
  return ok ? LM_OK : LM_NOT_CONVERGED;
}
