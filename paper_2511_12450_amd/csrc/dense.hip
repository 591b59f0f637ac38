// Dense plain path: assemble K by direct Sommerfeld quadrature, then y = K x.
// (Dirichlet scatterers below; sound-hard and impedance ones further down;
// then the spectral rule for smooth scatterers.)
//
// Sec. 3.3, eq. matrixelmemts (unscaled rows):
//   K_ie = |Gamma_e| [ delta_{l_i l_e} (i/4) H_0(k |c_i - c_e|) + G^r(c_i | c_e) ]  (e != i)
//   K_ii = |Gamma_i| G^r(c_i | c_i) + I^s_i,
//   I^s = [ i/4 - (gamma + ln(k |Gamma| / 4) - 1) / (2 pi) ] |Gamma|   (eq. ApproximateComputation)
#include "lm_internal.hpp"
#include "sommerfeld.hpp"

static constexpr double kEulerGamma = 0.57721566490153286061;

__device__ __forceinline__ zd self_term(double k, double w) {
  return zd(-(kEulerGamma + log(k * w / 4.0) - 1.0) / (2.0 * M_PI) * w, 0.25 * w);
}

// One thread per matrix entry; row-major K[i][e].
__global__ void __launch_bounds__(256) k_dense_assemble(MediumDev m, int N, const double* __restrict__ cx,
                                                        const double* __restrict__ cy,
                                                        const double* __restrict__ w,
                                                        const int* __restrict__ lay, double2* __restrict__ K) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)N * N) return;
  const int i = (int)(idx / N), e = (int)(idx % N);
  const int li = lay[i], le = lay[e];
  const double dx = cx[i] - cx[e], dy = cy[i] - cy[e];
  zd v = lmq::reaction_direct(m, li, le, fabs(dx), cy[i], cy[e]) * w[e];
  if (i == e) {
    v += self_term(m.k[li], w[i]);
  } else if (li == le) {
    const double kr = m.k[li] * sqrt(dx * dx + dy * dy);
    // (i/4) H_0^(1) = (i/4)(J_0 + i Y_0)
    v += zd(-0.25 * y0(kr), 0.25 * j0(kr)) * w[e];
  }
  K[idx] = make_double2(v.re, v.im);
}

// Sound-hard / impedance scatterers (single-layer representation, exterior
// normal-derivative limit):
//   A_ie = |Gamma_e| n_i . grad G(c_i | c_e) + i beta K_ie  (e != i),
//   A_ii = -1/2 + |Gamma_i| n_i . grad G^r(c_i | c_i) + i beta K_ii;
// grad G^f(c_i | c_e) = -(i/4) k H_1(k r) (c_i - c_e) / r, and the free-space
// part of the self term of K' is zero on a straight element.
__global__ void __launch_bounds__(256) k_dense_assemble_bc(MediumDev m, int N, const double* __restrict__ cx,
                                                           const double* __restrict__ cy,
                                                           const double* __restrict__ w,
                                                           const double* __restrict__ nx,
                                                           const double* __restrict__ ny,
                                                           const int* __restrict__ lay, double beta,
                                                           double2* __restrict__ K) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)N * N) return;
  const int i = (int)(idx / N), e = (int)(idx % N);
  const int li = lay[i], le = lay[e];
  const double dx = cx[i] - cx[e], dy = cy[i] - cy[e];
  zd g, gx, gy;
  lmq::reaction_direct_grad(m, li, le, dx, cy[i], cy[e], g, gx, gy);
  zd dn = gx * nx[i] + gy * ny[i];
  if (i == e) {
    g = g * w[i] + self_term(m.k[li], w[i]);
    dn = dn * w[i] + zd(-0.5, 0.0);
  } else {
    if (li == le) {
      const double r = sqrt(dx * dx + dy * dy), kr = m.k[li] * r;
      g += zd(-0.25 * y0(kr), 0.25 * j0(kr));
      // -(i/4) k H_1(k r) / r, H_1 = J_1 + i Y_1
      const zd d = zd(0.25 * y1(kr), -0.25 * j1(kr)) * (m.k[li] / r);
      dn += d * (dx * nx[i] + dy * ny[i]);
    }
    g = g * w[e];
    dn = dn * w[e];
  }
  const zd v = dn + zd(0.0, beta) * g;
  K[idx] = make_double2(v.re, v.im);
}

// Spectral rule (smooth closed scatterers inside one layer, nodes at equal
// parameter steps): the trapezoidal rule w_e [G^r + delta G^f] for nodes of
// different scatterers, and on a node's own scatterer (same layer)
//   w_e G^r(x_i | x_e) + R_{(i-e) mod M} m1 + (2 pi / M) m2,
//   m1 = -J_0(k r) |x'_e| / (4 pi),
//   m2 = (i/4) H_0(k r) |x'_e| - m1 ln(4 sin^2(pi (i - e) / M))   (e != i),
//   m2 = (i/4 - gamma / (2 pi) - ln(k |x'_i| / 2) / (2 pi)) |x'_i|  (e == i).
__global__ void __launch_bounds__(256) k_dense_assemble_spectral(
    MediumDev m, int N, const double* __restrict__ cx, const double* __restrict__ cy, const double* __restrict__ w,
    const int* __restrict__ lay, const int* __restrict__ sid, const int* __restrict__ loc, const int* __restrict__ cnt,
    const double* __restrict__ speed, const double* __restrict__ logw, const int64_t* __restrict__ roff,
    double2* __restrict__ K) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)N * N) return;
  const int i = (int)(idx / N), e = (int)(idx % N);
  const int li = lay[i], le = lay[e];
  const double dx = cx[i] - cx[e], dy = cy[i] - cy[e];
  zd v = lmq::reaction_direct(m, li, le, fabs(dx), cy[i], cy[e]) * w[e];
  const double k = m.k[li];
  if (sid[i] != sid[e]) {
    if (li == le) {
      const double kr = k * sqrt(dx * dx + dy * dy);
      v += zd(-0.25 * y0(kr), 0.25 * j0(kr)) * w[e];
    }
  } else {
    const int M = cnt[i], d = ((loc[i] - loc[e]) % M + M) % M;
    const double sp = speed[e], kr = k * sqrt(dx * dx + dy * dy);
    const double m1 = -j0(kr) * sp / (4.0 * M_PI);
    zd m2;
    if (d == 0) {
      m2 = zd(-kEulerGamma / (2.0 * M_PI) - log(0.5 * k * sp) / (2.0 * M_PI), 0.25) * sp;
    } else {
      const double sn = sin(M_PI * d / M);
      m2 = zd(-0.25 * y0(kr), 0.25 * j0(kr)) * sp - zd(m1 * log(4.0 * sn * sn), 0.0);
    }
    v += zd(logw[roff[sid[i]] + d] * m1, 0.0) + m2 * (2.0 * M_PI / M);
  }
  K[idx] = make_double2(v.re, v.im);
}

__global__ void k_to_c64(const double2* __restrict__ a, float2* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

lm_status dense_assemble(lm_geom_s* g, hipStream_t s) {
  const int64_t N = g->N, NN = N * N;
  LM_TRY(g->d_K.alloc(NN * sizeof(double2)));
  if (g->quad == LM_QUAD_SPECTRAL)
    hipLaunchKernelGGL(k_dense_assemble_spectral, dim3(div_up(NN, 256)), dim3(256), 0, s, g->m, (int)N,
                       g->d_cx.as<double>(), g->d_cy.as<double>(), g->d_w.as<double>(), g->d_layer.as<int>(),
                       g->d_sid.as<int>(), g->d_loc.as<int>(), g->d_cnt.as<int>(), g->d_speed.as<double>(),
                       g->d_logw.as<double>(), g->d_roff.as<int64_t>(), g->d_K.as<double2>());
  else if (g->bc == LM_BC_DIRICHLET)
    hipLaunchKernelGGL(k_dense_assemble, dim3(div_up(NN, 256)), dim3(256), 0, s, g->m, (int)N, g->d_cx.as<double>(),
                       g->d_cy.as<double>(), g->d_w.as<double>(), g->d_layer.as<int>(), g->d_K.as<double2>());
  else
    hipLaunchKernelGGL(k_dense_assemble_bc, dim3(div_up(NN, 256)), dim3(256), 0, s, g->m, (int)N,
                       g->d_cx.as<double>(), g->d_cy.as<double>(), g->d_w.as<double>(), g->d_nx.as<double>(),
                       g->d_ny.as<double>(), g->d_layer.as<int>(), g->robin_beta, g->d_K.as<double2>());
  LM_TRY_HIP(hipGetLastError());
  LM_TRY(g->d_K32.alloc(NN * sizeof(float2)));
  hipLaunchKernelGGL(k_to_c64, dim3(div_up(NN, 256)), dim3(256), 0, s, g->d_K.as<double2>(), g->d_K32.as<float2>(), NN);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

// y[r] = K x[r]: one 256-thread block per row, all right-hand sides at once.
template <typename T2, typename T, int RMAX>
__global__ void __launch_bounds__(256) k_dense_gemv(int N, int R, const T2* __restrict__ K, const T2* __restrict__ x,
                                                    T2* __restrict__ y) {
  const int i = blockIdx.x;
  const int r0 = blockIdx.y * RMAX;
  const int nr = min(RMAX, R - r0);
  T acc_re[RMAX], acc_im[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) acc_re[r] = acc_im[r] = T(0);
  const T2* row = K + (int64_t)i * N;
  for (int e = threadIdx.x; e < N; e += blockDim.x) {
    const T2 a = row[e];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      if (r < nr) {
        const T2 b = x[(int64_t)(r0 + r) * N + e];
        acc_re[r] += a.x * b.x - a.y * b.y;
        acc_im[r] += a.x * b.y + a.y * b.x;
      }
    }
  }
  __shared__ T red[2][RMAX][256 / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    T a = acc_re[r], b = acc_im[r];
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
  if (threadIdx.x < nr) {
    const int r = threadIdx.x;
    T a = 0, b = 0;
    for (int q = 0; q < 256 / 64; ++q) {
      a += red[0][r][q];
      b += red[1][r][q];
    }
    T2 o;
    o.x = a;
    o.y = b;
    y[(int64_t)(r0 + r) * N + i] = o;
  }
}

lm_status dense_matvec(lm_geom_s* g, int precision, int n_rhs, const void* x, void* y, hipStream_t s) {
  const int N = (int)g->N;
  constexpr int RB = 8;
  dim3 grid(N, div_up(n_rhs, RB));
  if (precision == LM_FP64) {
    hipLaunchKernelGGL((k_dense_gemv<double2, double, RB>), grid, dim3(256), 0, s, N, n_rhs, g->d_K.as<double2>(),
                       (const double2*)x, (double2*)y);
  } else {
    hipLaunchKernelGGL((k_dense_gemv<float2, float, RB>), grid, dim3(256), 0, s, N, n_rhs, g->d_K32.as<float2>(),
                       (const float2*)x, (float2*)y);
  }
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}
