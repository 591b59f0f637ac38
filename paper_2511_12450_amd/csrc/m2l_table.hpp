// Reaction M2L operators by Sommerfeld quadrature (the paper's I_nm integrals,
// eqs. generalintegral and metoleimage, in the side coordinates).
//
// For one component c = (target side, source side) and one pair of box
// centres with horizontal offset dx = x_t - x_s and heights h_t, h_s above
// their interfaces, the operator is
//   Ttilde_mn = (-1)^n (1/2pi) int_{-inf}^{inf} e^{i lam dx + i k_y h_t + i k'_y h_s}
//                w(lam,k)^m w(lam,k')^n S^c(lam) dlam,   |m|, |n| <= p.
// Contour ("class contour", chosen per operator so that the integrand has no
// cancellation): the segment t in [-T, T], lam = t - i a sin(pi t / T)
// (below the positive-axis branch points and guided-mode poles, above the
// negative ones; T = k_max + 1.5, a = min(0.5, 12/|dx|)), then both tails
// along the steepest-descent direction of e^{i lam (dx + i Y)}, Y = h_t + h_s:
//   right tail lam = T + s e_r, left tail lam = -T - s conj(e_r),
//   e_r = e^{i sgn(dx) psi}, psi = atan2(|dx|, Y),
// on which |e^{i lam dx + i k_y Y}| ~ e^{-s sqrt(dx^2 + Y^2)}.  Along these
// rays the integrand of the order-(m+n) operator peaks near
// s ~ (m+n)/dist with the size of the result, so high orders are computed
// without the catastrophic cancellation that a real-axis rule suffers when
// Y << |dx|.  Panels are 20-point Gauss-Legendre.
#pragma once
#include "sommerfeld.hpp"

#define LM_TAIL_PANELS 128

struct ClassNodes {
  double T, a, hm, dx, Y, dist;
  int nm, nt;                   // middle panels, panels per tail
  zd er;                        // right-tail direction
  double se[LM_TAIL_PANELS + 1];  // tail panel edges in s
  LM_HD int total() const { return 20 * (nm + 2 * nt); }
};

LM_HD void class_nodes(ClassNodes& c, double kmax, double dx, double Y, int p) {
  c.T = kmax + 1.5;
  c.dx = dx;
  c.Y = Y;
  const double X = fabs(dx);
  c.dist = hypot(X, Y);
  c.a = fmin(0.5, 12.0 / fmax(X, 1e-300));
  const double wmax = fmin(fmin(0.3, 0.5 * c.a), 8.0 / fmax(X, 1e-300));
  c.nm = (int)ceil(2.0 * c.T / wmax);
  c.hm = 2.0 * c.T / c.nm;
  const double psi = atan2(X, Y);
  c.er = dx >= 0 ? zd(cos(psi), sin(psi)) : zd(cos(psi), -sin(psi));
  const double S = (2.0 * p + 10.0 * sqrt(2.0 * p + 1.0) + 45.0) / c.dist;
  int n = 0;
  double s = 0.0;
  c.se[0] = 0.0;
  while (s < S && n < LM_TAIL_PANELS) {
    s = fmin(S, s + fmin(8.0 / c.dist, 0.5 + 0.5 * s));
    c.se[++n] = s;
  }
  c.nt = n;
}

// Node q: lam and its weight (including dlam and the 1/2pi).
LM_HD void class_node(const ClassNodes& c, int q, zd& lam, zd& wt) {
  const int pan = q / 20, j = q % 20;
  if (pan < c.nm) {
    const double t = -c.T + (pan + 0.5) * c.hm + 0.5 * c.hm * lmq::glx(j);
    const double sn = sin(M_PI * t / c.T), cs = cos(M_PI * t / c.T);
    lam = zd(t, -c.a * sn);
    wt = zd(1.0, -c.a * (M_PI / c.T) * cs) * (0.5 * c.hm * lmq::glw(j) / (2.0 * M_PI));
    return;
  }
  int r = pan - c.nm;
  const bool right = r < c.nt;
  if (!right) r -= c.nt;
  const double s0 = c.se[r], s1 = c.se[r + 1];
  const double s = 0.5 * (s0 + s1) + 0.5 * (s1 - s0) * lmq::glx(j);
  const double w = 0.5 * (s1 - s0) * lmq::glw(j) / (2.0 * M_PI);
  if (right) {
    lam = c.T + c.er * s;
    wt = c.er * w;
  } else {
    lam = -c.T - conj(c.er) * s;
    wt = conj(c.er) * w;
  }
}

// w(lam, k) = (k_y + i lam)/k and its inverse (k_y - i lam)/k.
LM_HD void omega(double k, zd ky, zd lam, zd& w, zd& winv) {
  w = (ky + zd(-lam.im, lam.re)) * (1.0 / k);
  winv = (ky - zd(-lam.im, lam.re)) * (1.0 / k);
}

// Weight of node q for component c between box centres: the factor
// e^{i lam dx + i k_y h_t + i k'_y h_s} S^c(lam) wt, plus the two omegas.
LM_HD void class_factor(const MediumDev& m, int lt, int ls, int comp, const ClassNodes& cn, double ht, double hs,
                        int q, zd& f, zd& wt_, zd& wtinv, zd& ws, zd& wsinv) {
  zd lam, wt;
  class_node(cn, q, lam, wt);
  StackAt st;
  stack_at(m, lam, st);
  zd S[4];
  side_densities(m, st, lt, ls, 1u << comp, S);
  const zd ex = zexp(zd(0.0, 1.0) * (lam * cn.dx + st.ky[lt] * ht + st.ky[ls] * hs));
  f = S[comp] * ex * wt;
  omega(m.k[lt], st.ky[lt], lam, wt_, wtinv);
  omega(m.k[ls], st.ky[ls], lam, ws, wsinv);
}

// Serial evaluation of one operator (row-major T[(m+p)*(2p+1) + (n+p)]).
// Used by the host-side checks; the device kernel parallelises the same sum.
inline void reaction_table_host(const MediumDev& m, int lt, int ls, int comp, double dx, double ht, double hs, int p,
                                zd* T) {
  const int P = 2 * p + 1;
  ClassNodes cn;
  class_nodes(cn, m.kmax, dx, ht + hs, p);
  for (int i = 0; i < P * P; ++i) T[i] = zd(0.0, 0.0);
  const int Q = cn.total();
  zd* wm = new zd[P];
  zd* wn = new zd[P];
  for (int q = 0; q < Q; ++q) {
    zd f, a, ai, b, bi;
    class_factor(m, lt, ls, comp, cn, ht, hs, q, f, a, ai, b, bi);
    // powers a^m (m = -p..p), (-b)^n (n = -p..p)
    wm[p] = zd(1.0, 0.0);
    wn[p] = zd(1.0, 0.0);
    for (int j = 1; j <= p; ++j) {
      wm[p + j] = wm[p + j - 1] * a;
      wm[p - j] = wm[p - j + 1] * ai;
      wn[p + j] = wn[p + j - 1] * (-b);
      wn[p - j] = wn[p - j + 1] * (-bi);
    }
    for (int i = 0; i < P; ++i) {
      const zd fi = f * wm[i];
      for (int j = 0; j < P; ++j) T[i * P + j] += fi * wn[j];
    }
  }
  delete[] wm;
  delete[] wn;
}
