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

// Gram-Schmidt passes stream the basis V[i][r][n] from HBM: every kernel is
// element-parallel over n (grid (ceil(N / GS_SLICE), R)), keeps GS_UNROLL
// basis loads in flight per lane and leaves one partial sum per wavefront;
// a small second kernel adds the partials.
constexpr int GS_UNROLL = 8;
constexpr int GS_EPT = 4;                 // elements per thread in the dot kernel
constexpr int GS_SLICE = 256 * GS_EPT;    // elements per workgroup in the dot kernel

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// part[(r ldh + i) nw + wave] = sum over the wave's elements of conj(V[i][r][n]) w[r][n]
// Basis vectors [GS_IBLK z, GS_IBLK (z + 1)) for grid index z.
constexpr int GS_IBLK = 64;
__global__ void __launch_bounds__(256) k_dots_part(int N, int R, int cnt, const double2* __restrict__ V,
                                                   const double2* __restrict__ w, double2* __restrict__ part,
                                                   int ldh, int nw) {
  const int r = blockIdx.y;
  const int ib = blockIdx.z * GS_IBLK;
  cnt = min(cnt, ib + GS_IBLK);
  const int wv = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t stride = (int64_t)R * N;
  double2 x[GS_EPT];
  int64_t off[GS_EPT];
  bool ok[GS_EPT];
#pragma unroll
  for (int e = 0; e < GS_EPT; ++e) {
    const int n = blockIdx.x * GS_SLICE + threadIdx.x + 256 * e;
    ok[e] = n < N;
    off[e] = (int64_t)r * N + (ok[e] ? n : 0);
    x[e] = ok[e] ? w[off[e]] : make_double2(0.0, 0.0);
  }
  for (int i0 = ib; i0 < cnt; i0 += GS_UNROLL) {
    double re[GS_UNROLL], im[GS_UNROLL];
#pragma unroll
    for (int u = 0; u < GS_UNROLL; ++u) re[u] = im[u] = 0.0;
#pragma unroll
    for (int e = 0; e < GS_EPT; ++e) {
      double2 a[GS_UNROLL];
#pragma unroll
      for (int u = 0; u < GS_UNROLL; ++u)
        a[u] = (i0 + u < cnt) ? V[(int64_t)(i0 + u) * stride + off[e]] : make_double2(0.0, 0.0);
#pragma unroll
      for (int u = 0; u < GS_UNROLL; ++u) {
        const double2 b = ok[e] ? a[u] : make_double2(0.0, 0.0);
        re[u] = fma(b.x, x[e].x, re[u]);
        re[u] = fma(b.y, x[e].y, re[u]);
        im[u] = fma(b.x, x[e].y, im[u]);
        im[u] = fma(-b.y, x[e].x, im[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < GS_UNROLL; ++u) {
      re[u] = wave_sum(re[u]);
      im[u] = wave_sum(im[u]);
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int u = 0; u < GS_UNROLL; ++u)
        if (i0 + u < cnt) part[((int64_t)r * ldh + i0 + u) * nw + wv] = make_double2(re[u], im[u]);
    }
  }
}

// h[r ldh + i] = sum_k part[(r ldh + i) nw + k]   (grid (cnt, R), one wavefront each)
__global__ void __launch_bounds__(64) k_dots_final(int nw, const double2* __restrict__ part, int ldh,
                                                   double2* __restrict__ h) {
  const int64_t row = (int64_t)blockIdx.y * ldh + blockIdx.x;
  double re = 0.0, im = 0.0;
  for (int k = threadIdx.x; k < nw; k += 64) {
    const double2 v = part[row * nw + k];
    re += v.x;
    im += v.y;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (threadIdx.x == 0) h[row] = make_double2(re, im);
}

// w[r] -= sum_{i < cnt} V[i][r] h[r][i]; with nrm_part, also the wave partials of |w[r]|^2.
__global__ void __launch_bounds__(256) k_update(int N, int R, int cnt, const double2* __restrict__ V,
                                                double2* __restrict__ w, const double2* __restrict__ h, int ldh,
                                                double* __restrict__ nrm_part, int nw) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  const bool ok = n < N;
  const int64_t o = (int64_t)r * N + (ok ? n : 0);
  const int64_t stride = (int64_t)R * N;
  const double2* hr = h + (int64_t)r * ldh;
  double2 acc = ok ? w[o] : make_double2(0.0, 0.0);
  for (int i0 = 0; i0 < cnt; i0 += GS_UNROLL) {
    double2 v[GS_UNROLL];
#pragma unroll
    for (int u = 0; u < GS_UNROLL; ++u) v[u] = (i0 + u < cnt) ? V[(int64_t)(i0 + u) * stride + o] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < GS_UNROLL; ++u) {
      if (i0 + u < cnt) {
        const double2 c = hr[i0 + u];
        acc.x = fma(-c.x, v[u].x, acc.x);
        acc.x = fma(c.y, v[u].y, acc.x);
        acc.y = fma(-c.x, v[u].y, acc.y);
        acc.y = fma(-c.y, v[u].x, acc.y);
      }
    }
  }
  if (ok) w[o] = acc;
  if (nrm_part) {
    const double q = wave_sum(ok ? acc.x * acc.x + acc.y * acc.y : 0.0);
    if ((threadIdx.x & 63) == 0) nrm_part[(int64_t)r * nw + blockIdx.x * 4 + (threadIdx.x >> 6)] = q;
  }
}

// Wave partials of |w[r]|^2 (grid (ceil(N / 256), R)).
__global__ void __launch_bounds__(256) k_norm_part(int N, const double2* __restrict__ w, double* __restrict__ part,
                                                   int nw) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  double q = 0.0;
  if (n < N) {
    const double2 v = w[(int64_t)r * N + n];
    q = v.x * v.x + v.y * v.y;
  }
  q = wave_sum(q);
  if ((threadIdx.x & 63) == 0) part[(int64_t)r * nw + blockIdx.x * 4 + (threadIdx.x >> 6)] = q;
}

// nrm[r] = sum_k part[r nw + k]   (grid R, one wavefront each)
__global__ void __launch_bounds__(64) k_norm_final(int nw, const double* __restrict__ part, double* __restrict__ nrm) {
  double q = 0.0;
  for (int k = threadIdx.x; k < nw; k += 64) q += part[(int64_t)blockIdx.x * nw + k];
  q = wave_sum(q);
  if (threadIdx.x == 0) nrm[blockIdx.x] = q;
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

// y = K M x in FP64 storage (M = the preconditioner when use_pre); the matvec
// itself runs in the requested precision.  Work buffers grow on demand.
lm_status apply_km(lm_geom_s* g, int precision, int R, const double2* x, double2* y, bool use_pre, KmBufs& b,
                   hipStream_t s) {
  const int64_t N = g->N, n = (int64_t)R * N;
  const double2* xin = x;
  if (use_pre) {
    if (b.mz.bytes < (size_t)n * sizeof(double2)) LM_TRY(b.mz.alloc(n * sizeof(double2)));
    LM_TRY(precond_apply(g, b.pre_precision < 0 ? precision : b.pre_precision, R, x, b.mz.p, s));
    xin = b.mz.as<double2>();
  }
  if (precision == LM_FP64) return geom_matvec(g, precision, R, xin, y, s, b.stage_ev);
  if (b.x32.bytes < (size_t)n * sizeof(float2)) {
    LM_TRY(b.x32.alloc(n * sizeof(float2)));
    LM_TRY(b.y32.alloc(n * sizeof(float2)));
  }
  hipLaunchKernelGGL(k_c128_to_c64, dim3(div_up(n, 256)), dim3(256), 0, s, n, xin, b.x32.as<float2>());
  LM_TRY(geom_matvec(g, precision, R, b.x32.p, b.y32.p, s, b.stage_ev));
  hipLaunchKernelGGL(k_c64_to_c128, dim3(div_up(n, 256)), dim3(256), 0, s, n, b.y32.as<float2>(), y);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

namespace {

struct Work {
  DevBuf V, w, z, h, y, nrm, scale, dpart, npart;
  KmBufs km;
};

lm_status apply_KM(lm_geom_s* g, int precision, int R, const double2* x, double2* y, bool use_pre, Work& wk,
                   hipStream_t s) {
  return apply_km(g, precision, R, x, y, use_pre, wk.km, s);
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
  double2* V = wk.V.as<double2>();
  const int nw_d = 4 * (int)div_up(N, GS_SLICE), nw_u = 4 * (int)div_up(N, 256);
  LM_TRY(wk.dpart.alloc((size_t)R * (m + 1) * nw_d * sizeof(double2)));
  LM_TRY(wk.npart.alloc((size_t)R * nw_u * sizeof(double)));
  const dim3 gD(div_up(N, GS_SLICE), R);
  auto norm2 = [&](const double2* v) {
    hipLaunchKernelGGL(k_norm_part, dim3(div_up(N, 256), R), dim3(256), 0, s, (int)N, v, wk.npart.as<double>(), nw_u);
    hipLaunchKernelGGL(k_norm_final, dim3(R), dim3(64), 0, s, nw_u, wk.npart.as<double>(), wk.nrm.as<double>());
  };
  double2* w = wk.w.as<double2>();
  double2* h1 = wk.h.as<double2>();
  double2* h2 = h1 + (size_t)R * (m + 1);
  const int ldh = m + 1;
  const dim3 gN(div_up(N, 256), R), b256(256);
  auto gs_pass = [&](int cnt, double2* h, bool with_norm) {
    hipLaunchKernelGGL(k_dots_part, dim3(gD.x, R, div_up(cnt, GS_IBLK)), b256, 0, s, (int)N, R, cnt, V, w,
                       wk.dpart.as<double2>(), ldh, nw_d);
    hipLaunchKernelGGL(k_dots_final, dim3(cnt, R), dim3(64), 0, s, nw_d, wk.dpart.as<double2>(), ldh, h);
    hipLaunchKernelGGL(k_update, gN, b256, 0, s, (int)N, R, cnt, V, w, h, ldh,
                       with_norm ? wk.npart.as<double>() : nullptr, nw_u);
    if (with_norm)
      hipLaunchKernelGGL(k_norm_final, dim3(R), dim3(64), 0, s, nw_u, wk.npart.as<double>(), wk.nrm.as<double>());
  };

  LM_TRY_HIP(hipMemsetAsync(phi, 0, n * sizeof(double2), s));
  // ||g_r||
  std::vector<double> gnorm(R), nrm_h(R), scale_h(R);
  norm2(gv);
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
    norm2(w);
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
      gs_pass(j + 1, h1, false);
      gs_pass(j + 1, h2, true);
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
    LM_TRY(precond_apply(g, precision, R, wk.z.p, phi, s));
  } else {
    LM_TRY_HIP(hipMemcpyAsync(phi, wk.z.p, n * sizeof(double2), hipMemcpyDeviceToDevice, s));
  }
  // true residual
  LM_TRY(apply_KM(g, precision, R, wk.z.as<double2>(), w, use_pre, wk, s));
  hipLaunchKernelGGL(k_axpby, dim3(div_up(n, 256)), b256, 0, s, n, gv, -1.0, w, w);
  norm2(w);
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
