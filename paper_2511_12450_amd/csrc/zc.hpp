// Minimal complex arithmetic usable in host and device code (double / float).
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

#define LM_HD __host__ __device__ __forceinline__

template <typename T>
struct cx {
  T re, im;
  LM_HD cx() : re(0), im(0) {}
  LM_HD cx(T r, T i = T(0)) : re(r), im(i) {}
  LM_HD cx& operator+=(const cx& o) { re += o.re; im += o.im; return *this; }
  LM_HD cx& operator-=(const cx& o) { re -= o.re; im -= o.im; return *this; }
  LM_HD cx& operator*=(const cx& o) { T r = re * o.re - im * o.im; im = re * o.im + im * o.re; re = r; return *this; }
  LM_HD cx& operator*=(T s) { re *= s; im *= s; return *this; }
};
typedef cx<double> zd;
typedef cx<float> zf;

template <typename T> LM_HD cx<T> operator+(cx<T> a, cx<T> b) { return cx<T>(a.re + b.re, a.im + b.im); }
template <typename T> LM_HD cx<T> operator-(cx<T> a, cx<T> b) { return cx<T>(a.re - b.re, a.im - b.im); }
template <typename T> LM_HD cx<T> operator-(cx<T> a) { return cx<T>(-a.re, -a.im); }
template <typename T> LM_HD cx<T> operator*(cx<T> a, cx<T> b) { return cx<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
template <typename T> LM_HD cx<T> operator*(cx<T> a, T s) { return cx<T>(a.re * s, a.im * s); }
template <typename T> LM_HD cx<T> operator*(T s, cx<T> a) { return cx<T>(a.re * s, a.im * s); }
template <typename T> LM_HD cx<T> operator+(cx<T> a, T s) { return cx<T>(a.re + s, a.im); }
template <typename T> LM_HD cx<T> operator+(T s, cx<T> a) { return cx<T>(a.re + s, a.im); }
template <typename T> LM_HD cx<T> operator-(T s, cx<T> a) { return cx<T>(s - a.re, -a.im); }
template <typename T> LM_HD cx<T> conj(cx<T> a) { return cx<T>(a.re, -a.im); }
template <typename T> LM_HD T abs2(cx<T> a) { return a.re * a.re + a.im * a.im; }

// Division by scaling with the larger component (Smith's method).
template <typename T> LM_HD cx<T> operator/(cx<T> a, cx<T> b) {
  T ar = fabs(b.re), ai = fabs(b.im);
  if (ar >= ai) {
    T r = b.im / b.re, den = b.re + b.im * r;
    return cx<T>((a.re + a.im * r) / den, (a.im - a.re * r) / den);
  }
  T r = b.re / b.im, den = b.re * r + b.im;
  return cx<T>((a.re * r + a.im) / den, (a.im * r - a.re) / den);
}
template <typename T> LM_HD cx<T> operator/(T s, cx<T> b) { return cx<T>(s, T(0)) / b; }

LM_HD zd zexp(zd z) {
  double e = exp(z.re);
  double s, c;
  sincos(z.im, &s, &c);
  return zd(e * c, e * s);
}
LM_HD zf zexpf(zf z) {
  float e = expf(z.re);
  float s, c;
  sincosf(z.im, &s, &c);
  return zf(e * c, e * s);
}

// Principal square root.
LM_HD zd zsqrt(zd z) {
  double r = hypot(z.re, z.im);
  if (r == 0.0) return zd(0.0, 0.0);
  if (z.re >= 0.0) {
    double t = sqrt(0.5 * (r + z.re));
    return zd(t, 0.5 * z.im / t);
  }
  double t = sqrt(0.5 * (r - z.re));
  return zd(0.5 * fabs(z.im) / t, copysign(t, z.im));
}

// Vertical wavenumber sqrt(k^2 - lam^2) on the sheet Im >= 0.
LM_HD zd zky(double k, zd lam) {
  zd v = zsqrt(zd(k * k, 0.0) - lam * lam);
  if (v.im < 0.0 || (v.im == 0.0 && v.re < 0.0)) v = -v;
  return v;
}
