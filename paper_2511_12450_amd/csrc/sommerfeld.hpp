// Direct Sommerfeld quadrature of the reaction part G^r(r | r') for one pair.
//
// The paper evaluates reaction components as Sommerfeld integrals (eq.
// fourreactions) but does not say how.  Here, per pair:
//  * the integrand exp(i lam dx) F(lam) has F even in lam, so the integral
//    folds onto lam >= 0: (1/2pi) int_C [e^{i lam X} + e^{-i lam X}] F dlam,
//    X = |dx|;
//  * C leaves 0 into the fourth quadrant along lam = t - i a q(t),
//    q(t) = 4 (t/T)(1 - t/T), 0 <= t <= T = k_max + 1.5, which passes below
//    the real branch points and guided-mode poles (all at lam <= k_max);
//  * beyond T either the real axis up to T + 36/D (D = smallest decay
//    distance h_t + h_s of the pair's components; used when D >= X/3), or,
//    after T + 1.5, the steepest-descent rays lam = T + 1.5 + s e^{+-i psi},
//    psi = atan2(X, D), on which e^{+-i lam X} F ~ e^{-s sqrt(X^2 + D^2)}.
//    F has no singularities with Re lam > k_max on the sheet Im k_y >= 0, so
//    the rays are a legal deformation.
//  * panels are 20-point Gauss-Legendre.
#pragma once
#include "spectral.hpp"

namespace lmq {

static __device__ __constant__ double GL20_X_D[20] = {-0.99312859918509488, -0.96397192727791381, -0.91223442825132584, -0.83911697182221878, -0.7463319064601508, -0.63605368072651502, -0.51086700195082713, -0.37370608871541955, -0.2277858511416451, -0.076526521133497338, 0.076526521133497338, 0.2277858511416451, 0.37370608871541955, 0.51086700195082713, 0.63605368072651502, 0.7463319064601508, 0.83911697182221878, 0.91223442825132584, 0.96397192727791381, 0.99312859918509488};
static __device__ __constant__ double GL20_W_D[20] = {0.017614007139153273, 0.040601429800386217, 0.062672048334109443, 0.083276741576704671, 0.10193011981724026, 0.11819453196151825, 0.13168863844917653, 0.14209610931838187, 0.14917298647260366, 0.15275338713072578, 0.15275338713072578, 0.14917298647260366, 0.14209610931838187, 0.13168863844917653, 0.11819453196151825, 0.10193011981724026, 0.083276741576704671, 0.062672048334109443, 0.040601429800386217, 0.017614007139153273};
static const double GL20_X_H[20] = {-0.99312859918509488, -0.96397192727791381, -0.91223442825132584, -0.83911697182221878, -0.7463319064601508, -0.63605368072651502, -0.51086700195082713, -0.37370608871541955, -0.2277858511416451, -0.076526521133497338, 0.076526521133497338, 0.2277858511416451, 0.37370608871541955, 0.51086700195082713, 0.63605368072651502, 0.7463319064601508, 0.83911697182221878, 0.91223442825132584, 0.96397192727791381, 0.99312859918509488};
static const double GL20_W_H[20] = {0.017614007139153273, 0.040601429800386217, 0.062672048334109443, 0.083276741576704671, 0.10193011981724026, 0.11819453196151825, 0.13168863844917653, 0.14209610931838187, 0.14917298647260366, 0.15275338713072578, 0.15275338713072578, 0.14917298647260366, 0.14209610931838187, 0.13168863844917653, 0.11819453196151825, 0.10193011981724026, 0.083276741576704671, 0.062672048334109443, 0.040601429800386217, 0.017614007139153273};

LM_HD double glx(int j) {
#ifdef __HIP_DEVICE_COMPILE__
  return GL20_X_D[j];
#else
  return GL20_X_H[j];
#endif
}
LM_HD double glw(int j) {
#ifdef __HIP_DEVICE_COMPILE__
  return GL20_W_D[j];
#else
  return GL20_W_H[j];
#endif
}

struct PairSides {
  unsigned mask;
  double ht[4], hs[4];
  double Dmin;
};

LM_HD PairSides pair_sides(const MediumDev& m, int lt, int ls, double yt, double ys, unsigned want) {
  PairSides p;
  p.mask = 0;
  p.Dmin = 1e300;
  for (int c = 0; c < 4; ++c) {
    int t = c & 1, s = c >> 1;
    p.ht[c] = p.hs[c] = 0.0;
    if (!((want >> c) & 1u)) continue;
    if (!side_exists(m, lt, t) || !side_exists(m, ls, s)) continue;
    p.mask |= 1u << c;
    p.ht[c] = fmax(side_h(m, lt, t, yt), 0.0);
    p.hs[c] = fmax(side_h(m, ls, s, ys), 0.0);
    p.Dmin = fmin(p.Dmin, p.ht[c] + p.hs[c]);
  }
  return p;
}

// F(lam) = sum_c S^c(lam) exp(i k_{lt,y} h_t + i k_{ls,y} h_s)
LM_HD zd integrand(const MediumDev& m, int lt, int ls, const PairSides& p, zd lam) {
  StackAt st;
  stack_at(m, lam, st);
  zd S[4];
  side_densities(m, st, lt, ls, p.mask, S);
  zd f(0.0, 0.0);
  for (int c = 0; c < 4; ++c) {
    if (!((p.mask >> c) & 1u)) continue;
    f += S[c] * zexp(zd(0.0, 1.0) * (st.ky[lt] * p.ht[c] + st.ky[ls] * p.hs[c]));
  }
  return f;
}

// G^r(r | r') for target (layer lt, height yt), source (layer ls, height ys)
// at horizontal distance X = |x - x'|, summed over the components in `want`
// (bit c = target side + 2 * source side; default all).
LM_HD zd reaction_direct(const MediumDev& m, int lt, int ls, double X, double yt, double ys,
                         unsigned want = 0xFu) {
  PairSides p = pair_sides(m, lt, ls, yt, ys, want);
  if (!p.mask) return zd(0.0, 0.0);
  const double T = m.kmax + 1.5;
  const double Xs = fmax(X, 1e-300);
  const double Dm = fmax(p.Dmin, 1e-12);
  zd acc(0.0, 0.0);
  // deformed part
  {
    const double a = fmin(0.5, 3.0 / Xs);
    const double wmax = fmin(fmin(0.3, 0.5 * a), 8.0 / Xs);
    const int np = (int)ceil(T / wmax);
    const double h = T / np;
    for (int q = 0; q < np; ++q) {
      const double c0 = (q + 0.5) * h;
      for (int j = 0; j < 20; ++j) {
        double t = c0 + 0.5 * h * glx(j), u = t / T;
        zd lam(t, -a * 4.0 * u * (1.0 - u));
        zd dl(1.0, -a * (4.0 / T) * (1.0 - 2.0 * u));
        zd e = zexp(zd(0.0, 1.0) * lam * X);
        zd osc = e + 1.0 / e;
        acc += (dl * (0.5 * h * glw(j))) * osc * integrand(m, lt, ls, p, lam);
      }
    }
  }
  if (Dm >= X / 3.0) {
    const double end = T + 36.0 / Dm;
    double x0 = T;
    while (x0 < end) {
      double w = fmin(fmin(8.0 / Xs, 2.5 / Dm), 0.3 + 0.3 * (x0 - T));
      double x1 = fmin(end, x0 + w);
      double hh = 0.5 * (x1 - x0), mid = 0.5 * (x1 + x0);
      for (int j = 0; j < 20; ++j) {
        double lr = mid + hh * glx(j);
        zd lam(lr, 0.0);
        double cs = 2.0 * cos(lr * X);
        acc += integrand(m, lt, ls, p, lam) * (hh * glw(j) * cs);
      }
      x0 = x1;
    }
  } else {
    const double L1 = T + 1.5;
    double x0 = T;
    while (x0 < L1) {
      double x1 = fmin(L1, x0 + fmin(0.3, 8.0 / Xs));
      double hh = 0.5 * (x1 - x0), mid = 0.5 * (x1 + x0);
      for (int j = 0; j < 20; ++j) {
        double lr = mid + hh * glx(j);
        acc += integrand(m, lt, ls, p, zd(lr, 0.0)) * (hh * glw(j) * 2.0 * cos(lr * X));
      }
      x0 = x1;
    }
    const double z = hypot(X, Dm);
    const double psi = atan2(X, Dm);
    zd ep(cos(psi), sin(psi));
    const double S = 50.0 / z;
    double s0 = 0.0;
    while (s0 < S) {
      double s1 = fmin(S, s0 + fmin(2.5 / z, 0.4 + 0.4 * s0));
      double hh = 0.5 * (s1 - s0), mid = 0.5 * (s1 + s0);
      for (int j = 0; j < 20; ++j) {
        double s = mid + hh * glx(j);
        zd lp = L1 + ep * s, lm = L1 + conj(ep) * s;
        zd fp = integrand(m, lt, ls, p, lp) * zexp(zd(0.0, X) * lp);
        zd fm = integrand(m, lt, ls, p, lm) * zexp(zd(0.0, -X) * lm);
        acc += (fp * ep + fm * conj(ep)) * (hh * glw(j));
      }
      s0 = s1;
    }
  }
  return acc * (1.0 / (2.0 * M_PI));
}

// F(lam) as above and its target y-derivative factor: component c gains
// i k_{lt,y} dh_t/dy, dh_t/dy = +1 on the bottom side (h = y + d) and -1 on
// the top side (h = -d - y).
LM_HD void integrand_dy(const MediumDev& m, int lt, int ls, const PairSides& p, zd lam, zd& f, zd& fy) {
  StackAt st;
  stack_at(m, lam, st);
  zd S[4];
  side_densities(m, st, lt, ls, p.mask, S);
  f = zd(0.0, 0.0);
  fy = zd(0.0, 0.0);
  for (int c = 0; c < 4; ++c) {
    if (!((p.mask >> c) & 1u)) continue;
    const zd v = S[c] * zexp(zd(0.0, 1.0) * (st.ky[lt] * p.ht[c] + st.ky[ls] * p.hs[c]));
    f += v;
    const double sy = (c & 1) == SIDE_B ? 1.0 : -1.0;
    fy += v * (zd(0.0, sy) * st.ky[lt]);
  }
}

// G^r(r | r') and its gradient in the target r (signed horizontal offset
// dx = x - x'): the same contour as reaction_direct; d/dx acts on the
// oscillating factor of the folded integral (e^{+i lam X} gains i lam,
// e^{-i lam X} gains -i lam; times the sign of dx), d/dy on the target factor.
LM_HD void reaction_direct_grad(const MediumDev& m, int lt, int ls, double dx, double yt, double ys, zd& g, zd& gx,
                                zd& gy, unsigned want = 0xFu) {
  g = gx = gy = zd(0.0, 0.0);
  PairSides p = pair_sides(m, lt, ls, yt, ys, want);
  if (!p.mask) return;
  const double X = fabs(dx), sx = dx < 0.0 ? -1.0 : 1.0;
  const double T = m.kmax + 1.5;
  const double Xs = fmax(X, 1e-300);
  const double Dm = fmax(p.Dmin, 1e-12);
  zd f, fy;
  {
    const double a = fmin(0.5, 3.0 / Xs);
    const double wmax = fmin(fmin(0.3, 0.5 * a), 8.0 / Xs);
    const int np = (int)ceil(T / wmax);
    const double h = T / np;
    for (int q = 0; q < np; ++q) {
      const double c0 = (q + 0.5) * h;
      for (int j = 0; j < 20; ++j) {
        double t = c0 + 0.5 * h * glx(j), u = t / T;
        zd lam(t, -a * 4.0 * u * (1.0 - u));
        zd dl(1.0, -a * (4.0 / T) * (1.0 - 2.0 * u));
        zd e = zexp(zd(0.0, 1.0) * lam * X), ei = 1.0 / e;
        zd w = dl * (0.5 * h * glw(j));
        integrand_dy(m, lt, ls, p, lam, f, fy);
        g += w * (e + ei) * f;
        gx += w * (zd(0.0, 1.0) * lam * (e - ei)) * f;
        gy += w * (e + ei) * fy;
      }
    }
  }
  if (Dm >= X / 3.0) {
    const double end = T + 36.0 / Dm;
    double x0 = T;
    while (x0 < end) {
      double w = fmin(fmin(8.0 / Xs, 2.5 / Dm), 0.3 + 0.3 * (x0 - T));
      double x1 = fmin(end, x0 + w);
      double hh = 0.5 * (x1 - x0), mid = 0.5 * (x1 + x0);
      for (int j = 0; j < 20; ++j) {
        double lr = mid + hh * glx(j);
        integrand_dy(m, lt, ls, p, zd(lr, 0.0), f, fy);
        double cs = 2.0 * cos(lr * X), sn = -2.0 * lr * sin(lr * X);
        g += f * (hh * glw(j) * cs);
        gx += f * (hh * glw(j) * sn);
        gy += fy * (hh * glw(j) * cs);
      }
      x0 = x1;
    }
  } else {
    const double L1 = T + 1.5;
    double x0 = T;
    while (x0 < L1) {
      double x1 = fmin(L1, x0 + fmin(0.3, 8.0 / Xs));
      double hh = 0.5 * (x1 - x0), mid = 0.5 * (x1 + x0);
      for (int j = 0; j < 20; ++j) {
        double lr = mid + hh * glx(j);
        integrand_dy(m, lt, ls, p, zd(lr, 0.0), f, fy);
        double cs = 2.0 * cos(lr * X), sn = -2.0 * lr * sin(lr * X);
        g += f * (hh * glw(j) * cs);
        gx += f * (hh * glw(j) * sn);
        gy += fy * (hh * glw(j) * cs);
      }
      x0 = x1;
    }
    const double z = hypot(X, Dm);
    const double psi = atan2(X, Dm);
    zd ep(cos(psi), sin(psi));
    const double S = 50.0 / z;
    double s0 = 0.0;
    while (s0 < S) {
      double s1 = fmin(S, s0 + fmin(2.5 / z, 0.4 + 0.4 * s0));
      double hh = 0.5 * (s1 - s0), mid = 0.5 * (s1 + s0);
      for (int j = 0; j < 20; ++j) {
        double s = mid + hh * glx(j);
        zd lp = L1 + ep * s, lm = L1 + conj(ep) * s;
        zd fp, fpy, fm, fmy;
        integrand_dy(m, lt, ls, p, lp, fp, fpy);
        integrand_dy(m, lt, ls, p, lm, fm, fmy);
        const zd xp = zexp(zd(0.0, X) * lp), xm = zexp(zd(0.0, -X) * lm);
        const zd wp = ep * (hh * glw(j)), wm = conj(ep) * (hh * glw(j));
        g += fp * xp * wp + fm * xm * wm;
        gx += (zd(0.0, 1.0) * lp) * fp * xp * wp + (zd(0.0, -1.0) * lm) * fm * xm * wm;
        gy += fpy * xp * wp + fmy * xm * wm;
      }
      s0 = s1;
    }
  }
  const double inv = 1.0 / (2.0 * M_PI);
  g = g * inv;
  gx = gx * (sx * inv);
  gy = gy * inv;
}

}  // namespace lmq
