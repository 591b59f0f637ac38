// Expansion arithmetic shared by the FMM kernels (host+device inline).
//
// Notation (complex plane z = x + i h of a tree's coordinates):
//   F_n(z) = J_n(k|z|) e^{i n arg z},   G_n(z) = H^(1)_n(k|z|) e^{i n arg z}.
// Addition theorems (Graf; both follow from the plane-wave generating function
// e^{i k |z| cos(arg z - phi)} = sum_n i^n J_n(k|z|) e^{i n (arg z - phi)}):
//   F_n(a + d) = sum_m F_{n-m}(d) F_m(a)            (all a, d)
//   G_n(a + D) = sum_m G_{n-m}(D) F_m(a)            (|a| < |D|)
// Multipole expansion of a box with centre c (free-space convention):
//   a_n = sum_s q_s J_n(k rho_s) e^{-i n theta_s},  (rho_s, theta_s) = polar(z_s - c)
//   free field: Phi(z) = (i/4) sum_n a_n G_n(z - c)
// Local expansion: Phi(z) = sum_m b_m F_m(z - c).
// Translations:
//   M2M (child c -> parent C):  a^C_n = sum_m F_{m-n}(C - c) a^c_m
//   L2L (parent C -> child c):  b^c_n = sum_m F_{m-n}(c - C) b^C_m
//   free M2L:                   b_m  = (i/4) sum_n G_{n-m}(c_t - c_s) a_n
// Reaction components use the same a_n: their plane-wave source factor
// e^{-i lam (x_s - x_c) + i k'_y (h_s - h_c)} = sum_n w'^n (-1)^n J_n e^{-i n theta_s}
// (Prop. 4.1 of the paper in these coordinates), so the reaction M2L is
//   b_m = sum_n Ttilde_mn a_n,  Ttilde_mn = (-1)^n (1/2pi) int e^{i lam dx + i k_y h_t + i k'_y h_s}
//                                        w(lam,k)^m w(lam,k')^n S(lam) dlam
// with w(lam, k) = (k_y + i lam)/k, dx, h_t, h_s taken between box centres.
#pragma once
#include "zc.hpp"

namespace fm {

// J_n(x), n = 0..N (N <= 96) for 0 <= x <= 10 by downward recurrence started
// from power series at n = N+24 and N+25 (no cancellation there since
// (x/2)^2 < N+25).
LM_HD void bessel_j_seq(double x, int N, double* J) {
  if (x < 1e-300) {
    J[0] = 1.0;
    for (int n = 1; n <= N; ++n) J[n] = 0.0;
    return;
  }
  const int M = N + 24;
  double hx = 0.5 * x, q = -hx * hx;
  // series for J_M and J_{M+1}
  double tM = 1.0;
  for (int i = 1; i <= M; ++i) tM *= hx / i;  // (x/2)^M / M!
  double sM = 0.0, sM1 = 0.0;
  {
    double t = tM;
    for (int k = 0; k < 60; ++k) {
      sM += t;
      t *= q / ((k + 1.0) * (M + k + 1.0));
      if (fabs(t) < 1e-18 * fabs(sM)) break;
    }
    t = tM * hx / (M + 1.0);
    for (int k = 0; k < 60; ++k) {
      sM1 += t;
      t *= q / ((k + 1.0) * (M + k + 2.0));
      if (fabs(t) < 1e-18 * fabs(sM1)) break;
    }
  }
  if (sM == 0.0) {  // underflow: x tiny, use leading terms for every n
    double t = 1.0;
    for (int n = 0; n <= N; ++n) {
      J[n] = t * (1.0 + q / (n + 1.0));
      t *= hx / (n + 1.0);
    }
    return;
  }
  double jp1 = sM1, j = sM;
  for (int n = M; n >= 1; --n) {
    double jm1 = (2.0 * n / x) * j - jp1;
    jp1 = j;
    j = jm1;
    if (n - 1 <= N) J[n - 1] = j;
  }
}

// H^(1)_n(x), n = 0..N by upward recurrence from H_0, H_1 (x > 0).
LM_HD void hankel_seq(double x, int N, zd* H) {
  H[0] = zd(j0(x), y0(x));
  if (N >= 1) H[1] = zd(j1(x), y1(x));
  for (int n = 1; n < N; ++n) H[n + 1] = H[n] * (2.0 * n / x) - H[n - 1];
}

LM_HD zd cis(double t) {
  double s, c;
  sincos(t, &s, &c);
  return zd(c, s);
}

// F_j(d) for j = -J..J into out[j + J].
LM_HD void f_seq(double k, double dx, double dh, int J, zd* out, double* jbuf) {
  const double r = hypot(dx, dh), th = atan2(dh, dx);
  bessel_j_seq(k * r, J, jbuf);
  const zd e = cis(th);
  zd ep(1.0, 0.0);
  out[J] = zd(jbuf[0], 0.0);
  for (int j = 1; j <= J; ++j) {
    ep = ep * e;
    const double sg = (j & 1) ? -1.0 : 1.0;
    out[J + j] = ep * jbuf[j];
    out[J - j] = conj(ep) * (sg * jbuf[j]);  // J_{-j} = (-1)^j J_j, e^{-ij th}
  }
}

// G_j(D) for j = -J..J into out[j + J] (|D| > 0).
LM_HD void g_seq(double k, double dx, double dh, int J, zd* out, zd* hbuf) {
  const double r = hypot(dx, dh), th = atan2(dh, dx);
  hankel_seq(k * r, J, hbuf);
  const zd e = cis(th);
  zd ep(1.0, 0.0);
  out[J] = hbuf[0];
  for (int j = 1; j <= J; ++j) {
    ep = ep * e;
    const double sg = (j & 1) ? -1.0 : 1.0;
    out[J + j] = ep * hbuf[j];
    out[J - j] = conj(ep) * hbuf[j] * sg;
  }
}

}  // namespace fm
