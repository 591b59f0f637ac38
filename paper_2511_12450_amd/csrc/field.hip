// Scattered field at points off the boundary (eq. integralrep):
//   u^s(p) = sum_e |Gamma_e| phi_e G(p | c_e),
// the same single-layer sum as the matrix rows, at receivers instead of
// collocation points.
//
// Free-space part (receivers and sources in the same layer): a direct sum of
// (i/4) H_0(k |p - c_e|), one workgroup per receiver.
//
// Reaction part, by the spectral form of every component (see the matvec):
// with the horizontal part of the kernel folded onto lam >= 0 and the
// receiver's and the source's factors separated,
//   u^r(p) = (1/2pi) int_C sum_{l', t, s} S^{(t,s)}_{l_p l'}(lam) e^{i k_{l_p,y} h_t(p)}
//            [e^{i lam x_p} B+_{l's}(lam) + e^{-i lam x_p} B-_{l's}(lam)] dlam,
//   B-+_{l's}(lam) = sum_{e in layer l'} |Gamma_e| phi_e e^{-+i lam x_e} e^{i k_{l',y} h_s(e)},
// so the sources enter through the source spectra B at the quadrature nodes
// (O(N Q)) and each receiver through one pass over the nodes (O(Q)).  C is the
// contour of the direct quadrature (below the branch points and guided-mode
// poles up to T = k_max + 1.5, then the real axis), extended along the real
// axis until e^{-lam h} is negligible for the receivers' smallest distance h
// to the interface their arriving waves come from; receivers are binned by
// that distance (powers of two) so that each bin has its own node set.
// Horizontal positions are taken relative to the centre of the sources and
// receivers, which bounds the growth of e^{-+i lam x} on the deformed part.
#include <algorithm>
#include <cmath>
#include <map>

#include "lm_internal.hpp"
#include "sommerfeld.hpp"

namespace {

constexpr int FD_RC = 4;  // right-hand sides per launch of the spectral kernels

struct FieldSrc {
  DevBuf x, y, w, lay, perm;  // sources sorted by layer: perm[k] = element index
  std::vector<int> lptr;      // sources of layer l: perm[lptr[l] .. lptr[l+1])
  int N = 0;
};

// Free-space part: out[r][p] = sum_{e in layer(p)} q_e[r] (i/4) H_0(k |p - c_e|).
__global__ void __launch_bounds__(256) k_field_free(MediumDev m, int R, int Ntot, const double* __restrict__ px,
                                                    const double* __restrict__ py, const int* __restrict__ pl,
                                                    const int* __restrict__ lptr, const int* __restrict__ perm,
                                                    const double* __restrict__ sx, const double* __restrict__ sy,
                                                    const double* __restrict__ sw, const double2* __restrict__ phi,
                                                    int r0, double2* __restrict__ out, int n_pts) {
  const int p = blockIdx.x;
  const int l = pl[p];
  const double x = px[p], y = py[p], k = m.k[l];
  zd acc[FD_RC];
  const int nr = min(FD_RC, R - r0);
  for (int kk = lptr[l] + threadIdx.x; kk < lptr[l + 1]; kk += blockDim.x) {
    const int e = perm[kk];
    const double kr = k * hypot(x - sx[e], y - sy[e]);
    const zd g = zd(-0.25 * y0(kr), 0.25 * j0(kr)) * sw[e];
#pragma unroll
    for (int q = 0; q < FD_RC; ++q)
      if (q < nr) {
        const double2 v = phi[(int64_t)(r0 + q) * Ntot + e];
        acc[q] += g * zd(v.x, v.y);
      }
  }
  __shared__ double red[2][FD_RC][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < FD_RC; ++q) {
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
    out[(int64_t)(r0 + q) * n_pts + p] =
        make_double2(red[0][q][0] + red[0][q][1] + red[0][q][2] + red[0][q][3],
                     red[1][q][0] + red[1][q][1] + red[1][q][2] + red[1][q][3]);
  }
}

// Node tables: ky[q][l] and S[q][lt][ls][c] (c = t + 2 s).
__global__ void k_field_tables(MediumDev m, int Q, const double2* __restrict__ lam, double2* __restrict__ ky,
                               double2* __restrict__ S) {
  const int nl = m.L + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= Q * nl * nl) return;
  const int q = idx / (nl * nl), lt = (idx / nl) % nl, ls = idx % nl;
  StackAt st;
  stack_at(m, zd(lam[q].x, lam[q].y), st);
  zd s4[4];
  for (int c = 0; c < 4; ++c) s4[c] = zd(0.0, 0.0);
  side_densities(m, st, lt, ls, 0xFu, s4);
  for (int c = 0; c < 4; ++c) S[(((int64_t)q * nl + lt) * nl + ls) * 4 + c] = make_double2(s4[c].re, s4[c].im);
  if (ls == 0) ky[(int64_t)q * nl + lt] = make_double2(st.ky[lt].re, st.ky[lt].im);
}

// Source spectra B[ls][s][sign][q][r] for right-hand sides r0 .. r0 + FD_RC:
// one workgroup per (node, source layer), threads along the layer's sources.
__global__ void __launch_bounds__(256) k_field_spectra(MediumDev m, int R, int Ntot, int Q, double xc,
                                                       const double2* __restrict__ lam, const double2* __restrict__ ky,
                                                       const int* __restrict__ lptr, const int* __restrict__ perm,
                                                       const double* __restrict__ sx, const double* __restrict__ sy,
                                                       const double* __restrict__ sw, const double2* __restrict__ phi,
                                                       int r0, double2* __restrict__ B) {
  const int q = blockIdx.x, ls = blockIdx.y, nl = m.L + 1;
  const zd lm(lam[q].x, lam[q].y), kyl(ky[(int64_t)q * nl + ls].x, ky[(int64_t)q * nl + ls].y);
  const int nr = min(FD_RC, R - r0);
  zd acc[2][2][FD_RC];  // [side][sign][rhs]
  for (int kk = lptr[ls] + threadIdx.x; kk < lptr[ls + 1]; kk += blockDim.x) {
    const int e = perm[kk];
    const zd em = zexp(zd(0.0, -(sx[e] - xc)) * lm);  // e^{-i lam x}
    const zd ep = 1.0 / em;                            // e^{+i lam x}
    zd fs[2];
    for (int s = 0; s < 2; ++s)
      fs[s] = side_exists(m, ls, s) ? zexp(zd(0.0, fmax(side_h(m, ls, s, sy[e]), 0.0)) * kyl) * sw[e] : zd(0.0, 0.0);
#pragma unroll
    for (int r = 0; r < FD_RC; ++r)
      if (r < nr) {
        const double2 v = phi[(int64_t)(r0 + r) * Ntot + e];
        const zd pv(v.x, v.y);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const zd t = fs[s] * pv;
          acc[s][0][r] += t * em;
          acc[s][1][r] += t * ep;
        }
      }
  }
  __shared__ double red[4][FD_RC][2][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int r = 0; r < FD_RC; ++r) {
        double a = acc[s][g][r].re, b = acc[s][g][r].im;
        for (int off = 32; off > 0; off >>= 1) {
          a += __shfl_down(a, off, 64);
          b += __shfl_down(b, off, 64);
        }
        if (lane == 0) {
          red[2 * s + g][r][0][wv] = a;
          red[2 * s + g][r][1][wv] = b;
        }
      }
  __syncthreads();
  if (threadIdx.x < 4 * FD_RC) {
    const int sg = threadIdx.x / FD_RC, r = threadIdx.x % FD_RC;
    const double(*v)[4] = red[sg][r];
    B[(((int64_t)ls * 4 + sg) * Q + q) * FD_RC + r] =
        make_double2(v[0][0] + v[0][1] + v[0][2] + v[0][3], v[1][0] + v[1][1] + v[1][2] + v[1][3]);
  }
}

// out[r][p] += (1/2pi) sum_q wq[q] sum_{ls, t, s} S e^{i ky h_t(p)} (e^{i lam x_p} B+ + e^{-i lam x_p} B-)
// for the receivers of one bin: one workgroup per receiver, threads along the nodes.
__global__ void __launch_bounds__(256) k_field_reaction(MediumDev m, int R, int Q, double xc,
                                                        const double2* __restrict__ lam, const double2* __restrict__ wq,
                                                        const double2* __restrict__ ky, const double2* __restrict__ S,
                                                        const double2* __restrict__ B, const int* __restrict__ pidx,
                                                        const double* __restrict__ px, const double* __restrict__ py,
                                                        const int* __restrict__ pl, int r0, double2* __restrict__ out,
                                                        int n_pts) {
  const int p = pidx[blockIdx.x];
  const int lt = pl[p], nl = m.L + 1;
  const double x = px[p] - xc, y = py[p];
  double ht[2];
  for (int t = 0; t < 2; ++t) ht[t] = side_exists(m, lt, t) ? fmax(side_h(m, lt, t, y), 0.0) : 0.0;
  const int nr = min(FD_RC, R - r0);
  zd acc[FD_RC];
  for (int q = threadIdx.x; q < Q; q += blockDim.x) {
    const zd lm(lam[q].x, lam[q].y), w(wq[q].x, wq[q].y);
    const zd kyt(ky[(int64_t)q * nl + lt].x, ky[(int64_t)q * nl + lt].y);
    const zd ep = zexp(zd(0.0, x) * lm), em = 1.0 / ep;
    zd et[2];
    for (int t = 0; t < 2; ++t) et[t] = side_exists(m, lt, t) ? zexp(zd(0.0, ht[t]) * kyt) * w : zd(0.0, 0.0);
    for (int ls = 0; ls < nl; ++ls) {
      const double2* Sq = S + (((int64_t)q * nl + lt) * nl + ls) * 4;
      for (int s = 0; s < 2; ++s) {
        if (!side_exists(m, ls, s)) continue;
        zd f(0.0, 0.0);
        for (int t = 0; t < 2; ++t) {
          const double2 sv = Sq[t + 2 * s];
          f += zd(sv.x, sv.y) * et[t];
        }
        const double2* Bp = B + (((int64_t)ls * 4 + 2 * s + 0) * Q + q) * FD_RC;
        const double2* Bm = B + (((int64_t)ls * 4 + 2 * s + 1) * Q + q) * FD_RC;
#pragma unroll
        for (int r = 0; r < FD_RC; ++r)
          if (r < nr) acc[r] += f * (ep * zd(Bp[r].x, Bp[r].y) + em * zd(Bm[r].x, Bm[r].y));
      }
    }
  }
  __shared__ double red[2][FD_RC][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < FD_RC; ++r) {
    double a = acc[r].re, b = acc[r].im;
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_down(a, off, 64);
      b += __shfl_down(b, off, 64);
    }
    if (lane == 0) {
      red[0][r][wv] = a;
      red[1][r][wv] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < (unsigned)nr) {
    const int r = threadIdx.x;
    double2& o = out[(int64_t)(r0 + r) * n_pts + p];
    const double s = 1.0 / (2.0 * M_PI);
    o.x += s * (red[0][r][0] + red[0][r][1] + red[0][r][2] + red[0][r][3]);
    o.y += s * (red[1][r][0] + red[1][r][1] + red[1][r][2] + red[1][r][3]);
  }
}

// Quadrature nodes (lam, weight) of one bin: deformed part [0, T] as in the
// direct quadrature with the dip a and panel widths set by the largest
// horizontal offset X, then the real axis from T to T + 36 / h.
void field_nodes(const MediumDev& m, double X, double h, std::vector<double2>& lam, std::vector<double2>& wq) {
  const double T = m.kmax + 1.5;
  const double Xs = std::max(X, 1e-3);
  const double a = std::min(0.5, 3.0 / Xs);
  const double wmax = std::min(std::min(0.3, 0.5 * a), 8.0 / Xs);
  const int np = (int)std::ceil(T / wmax);
  const double hp = T / np;
  for (int q = 0; q < np; ++q) {
    const double c0 = (q + 0.5) * hp;
    for (int j = 0; j < 20; ++j) {
      const double t = c0 + 0.5 * hp * lmq::glx(j), u = t / T;
      const double wgt = 0.5 * hp * lmq::glw(j);
      const double dr = 1.0, di = -a * (4.0 / T) * (1.0 - 2.0 * u);
      lam.push_back(make_double2(t, -a * 4.0 * u * (1.0 - u)));
      wq.push_back(make_double2(dr * wgt, di * wgt));
    }
  }
  const double end = T + 36.0 / h;
  double x0 = T;
  while (x0 < end) {
    const double w = std::min(std::min(8.0 / Xs, 2.5 / h), 0.3 + 0.3 * (x0 - T));
    const double x1 = std::min(end, x0 + w);
    const double hh = 0.5 * (x1 - x0), mid = 0.5 * (x1 + x0);
    for (int j = 0; j < 20; ++j) {
      lam.push_back(make_double2(mid + hh * lmq::glx(j), 0.0));
      wq.push_back(make_double2(hh * lmq::glw(j), 0.0));
    }
    x0 = x1;
  }
}

// Field of sources (device arrays of N, weights sw, densities phi [R][N]) at
// n_pts receivers (host coordinates).
lm_status field_eval(const MediumDev& m, int N, const std::vector<double>& sxh, const std::vector<int>& slh,
                     const double* sx, const double* sy, const double* sw, const double2* phi, int R, int n_pts,
                     const double* pts, double2* out, hipStream_t s) {
  const int nl = m.L + 1;
  constexpr double H_MIN = 1e-4;
  std::vector<double> px(n_pts), py(n_pts), hp(n_pts);
  std::vector<int> pl(n_pts);
  double xmin = 1e300, xmax = -1e300;
  for (int e = 0; e < N; ++e) {
    xmin = std::min(xmin, sxh[e]);
    xmax = std::max(xmax, sxh[e]);
  }
  for (int p = 0; p < n_pts; ++p) {
    px[p] = pts[2 * p];
    py[p] = pts[2 * p + 1];
    LM_CHECK(std::isfinite(px[p]) && std::isfinite(py[p]), LM_EINVAL, "non-finite receiver");
    pl[p] = layer_of(m, py[p]);
    double h = 1e300;
    for (int t = 0; t < 2; ++t)
      if (side_exists(m, pl[p], t)) h = std::min(h, side_h(m, pl[p], t, py[p]));
    LM_CHECK(h >= H_MIN, LM_EINVAL, "receiver %d lies within %g of an interface", p, H_MIN);
    hp[p] = h;
    xmin = std::min(xmin, px[p]);
    xmax = std::max(xmax, px[p]);
  }
  const double xc = 0.5 * (xmin + xmax), X = xmax - xmin;
  // sources sorted by layer
  std::vector<int> lptr(nl + 1, 0), perm(N);
  for (int e = 0; e < N; ++e) ++lptr[slh[e] + 1];
  for (int l = 0; l < nl; ++l) lptr[l + 1] += lptr[l];
  {
    std::vector<int> fill(lptr.begin(), lptr.end() - 1);
    for (int e = 0; e < N; ++e) perm[fill[slh[e]]++] = e;
  }
  DevBuf dpx, dpy, dpl, dlptr, dperm;
  LM_TRY(upload(dpx, px.data(), n_pts * sizeof(double), s));
  LM_TRY(upload(dpy, py.data(), n_pts * sizeof(double), s));
  LM_TRY(upload(dpl, pl.data(), n_pts * sizeof(int), s));
  LM_TRY(upload(dlptr, lptr.data(), lptr.size() * sizeof(int), s));
  LM_TRY(upload(dperm, perm.data(), N * sizeof(int), s));
  for (int r0 = 0; r0 < R; r0 += FD_RC)
    hipLaunchKernelGGL(k_field_free, dim3(n_pts), dim3(256), 0, s, m, R, N, dpx.as<double>(), dpy.as<double>(),
                       dpl.as<int>(), dlptr.as<int>(), dperm.as<int>(), sx, sy, sw, phi, r0, out, n_pts);
  LM_TRY_HIP(hipGetLastError());
  // bins of receivers by the power of two of their distance to the interfaces
  std::map<int, std::vector<int>> bins;
  for (int p = 0; p < n_pts; ++p) bins[(int)std::floor(std::log2(std::min(hp[p], 1e6)))].push_back(p);
  for (auto& kv : bins) {
    std::vector<double2> lam, wq;
    field_nodes(m, X, std::ldexp(1.0, kv.first), lam, wq);
    const int Q = (int)lam.size();
    DevBuf dlam, dwq, dky, dS, dB, didx;
    LM_TRY(upload(dlam, lam.data(), Q * sizeof(double2), s));
    LM_TRY(upload(dwq, wq.data(), Q * sizeof(double2), s));
    LM_TRY(upload(didx, kv.second.data(), kv.second.size() * sizeof(int), s));
    LM_TRY(dky.alloc((size_t)Q * nl * sizeof(double2)));
    LM_TRY(dS.alloc((size_t)Q * nl * nl * 4 * sizeof(double2)));
    LM_TRY(dB.alloc((size_t)nl * 4 * Q * FD_RC * sizeof(double2)));
    LM_TRY_HIP(hipMemsetAsync(dS.p, 0, dS.bytes, s));
    hipLaunchKernelGGL(k_field_tables, dim3(div_up((int64_t)Q * nl * nl, 128)), dim3(128), 0, s, m, Q,
                       dlam.as<double2>(), dky.as<double2>(), dS.as<double2>());
    for (int r0 = 0; r0 < R; r0 += FD_RC) {
      hipLaunchKernelGGL(k_field_spectra, dim3(Q, nl), dim3(256), 0, s, m, R, N, Q, xc, dlam.as<double2>(),
                         dky.as<double2>(), dlptr.as<int>(), dperm.as<int>(), sx, sy, sw, phi, r0,
                         dB.as<double2>());
      hipLaunchKernelGGL(k_field_reaction, dim3(kv.second.size()), dim3(256), 0, s, m, R, Q, xc, dlam.as<double2>(),
                         dwq.as<double2>(), dky.as<double2>(), dS.as<double2>(), dB.as<double2>(), didx.as<int>(),
                         dpx.as<double>(), dpy.as<double>(), dpl.as<int>(), r0, out, n_pts);
    }
    LM_TRY_HIP(hipGetLastError());
    LM_TRY_HIP(hipStreamSynchronize(s));  // the bin's buffers are freed on return
  }
  LM_TRY_HIP(hipStreamSynchronize(s));
  return LM_OK;
}

}  // namespace

extern "C" lm_status lm_field(lm_geom g, int n_rhs, const void* phi_dev, int n_pts, const double* pts_xy,
                              void* out_dev, void* hip_stream) {
  LM_CHECK(g, LM_EINVAL, "geom is NULL");
  LM_CHECK(n_rhs >= 1 && n_pts >= 1 && phi_dev && pts_xy && out_dev, LM_EINVAL, "bad arguments");
  return field_eval(g->m, (int)g->N, g->cx, g->layer, g->d_cx.as<double>(), g->d_cy.as<double>(),
                    g->d_w.as<double>(), (const double2*)phi_dev, n_rhs, n_pts, pts_xy, (double2*)out_dev,
                    (hipStream_t)hip_stream);
}

extern "C" lm_status lm_point_field(lm_layers layers, int n_src, const double* src_xy, int n_pts,
                                    const double* pts_xy, void* out_dev, void* hip_stream) {
  LM_CHECK(layers, LM_EINVAL, "layers is NULL");
  LM_CHECK(n_src >= 1 && n_pts >= 1 && src_xy && pts_xy && out_dev, LM_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)hip_stream;
  const MediumDev& m = layers->m;
  std::vector<double> x(n_src), y(n_src), w(n_src, 1.0);
  std::vector<int> l(n_src);
  std::vector<double2> eye((size_t)n_src * n_src, make_double2(0.0, 0.0));
  for (int r = 0; r < n_src; ++r) {
    x[r] = src_xy[2 * r];
    y[r] = src_xy[2 * r + 1];
    LM_CHECK(std::isfinite(x[r]) && std::isfinite(y[r]), LM_EINVAL, "non-finite source position");
    l[r] = layer_of(m, y[r]);
    eye[(size_t)r * n_src + r] = make_double2(1.0, 0.0);
  }
  DevBuf dx, dy, dw, dphi;
  LM_TRY(upload(dx, x.data(), n_src * sizeof(double), s));
  LM_TRY(upload(dy, y.data(), n_src * sizeof(double), s));
  LM_TRY(upload(dw, w.data(), n_src * sizeof(double), s));
  LM_TRY(upload(dphi, eye.data(), eye.size() * sizeof(double2), s));
  return field_eval(m, n_src, x, l, dx.as<double>(), dy.as<double>(), dw.as<double>(), dphi.as<double2>(), n_src,
                    n_pts, pts_xy, (double2*)out_dev, s);
}
