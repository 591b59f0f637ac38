// Spectral densities of the layered Green's function in "side" form.
//
// Sec. 3.1 of the paper gives G^r_{l l'} as four Sommerfeld integrals
// (eq. fourreactions) with densities sigma from the generalized reflection /
// transmission recursions (eqs. Rellrecursionup, Rellrecursiondown,
// generaltransmission; Cases I-III: densityinsourcelayer, disity1, disity2).
//
// This library rewrites every non-zero component in one form.  A layer l has
// a bottom side B (interface y = -d_l, exists for l < L) and a top side T
// (interface y = -d_{l-1}, exists for l > 0); h_B(y) = y + d_l and
// h_T(y) = -d_{l-1} - y are the distances from a point of layer l to them.
// The wave that arrives at the target travelling up came last from its B
// side, one travelling down from its T side; the wave leaving the source
// downward goes to its B side, upward to its T side.  With
// c = (target side t, source side s):
//
//   G^c(r, r') = (1/2pi) int exp(i lam (x - x')) exp(i k_{l,y} h_t(y)
//                 + i k_{l',y} h_s(y')) S^c(lam) dlam,
//   S^c = sigma^c_{l l'} * i/(2 k_{l',y}) * exp(i (k_{l,y} a_t + k_{l',y} a_s)),
//
// where a_t, a_s = +-(depth of the side's interface) make up the difference
// between the paper's exponent and the h-form (the paper references
// amplitudes to y = 0).  The factor i/(2 k_{l',y}) is the paper's printed
// 1/(2 k_{l',y}) read with the factor i that the Sommerfeld identity needs.
// The round-trip factor printed exp(-2 k_{l,y} h_l) is read exp(2 i k_{l,y} h_l).
// Every (target side, source side) pair is a non-zero component: 2L x 2L = 4L^2
// (the Remark of Sec. 3.1).  Component index c = t + 2 s with t, s in {B=0, T=1}.
#pragma once
#include "zc.hpp"

#define LM_MAXL 8  // max layers

struct MediumDev {
  int L;                    // number of interfaces; layers 0..L
  double d[LM_MAXL];        // interface depths (y = -d[l])
  double k[LM_MAXL];        // wavenumbers per layer
  double eta[LM_MAXL];      // transmission weights per layer
  double kmax;
};

enum { SIDE_B = 0, SIDE_T = 1 };

LM_HD bool side_exists(const MediumDev& m, int l, int side) {
  return side == SIDE_B ? (l < m.L) : (l > 0);
}

// Distance of height y (in layer l) from the interface of the given side.
LM_HD double side_h(const MediumDev& m, int l, int side, double y) {
  return side == SIDE_B ? (y + m.d[l]) : (-m.d[l - 1] - y);
}

LM_HD double layer_thickness(const MediumDev& m, int l) {
  return (l >= 1 && l <= m.L - 1) ? (m.d[l] - m.d[l - 1]) : 0.0;
}

// All spectral quantities of the stack at one lam.
struct StackAt {
  zd ky[LM_MAXL];
  zd Rloc[LM_MAXL];   // R_{l,l+1}
  zd Tdn[LM_MAXL];    // T_{l,l+1}
  zd Tup[LM_MAXL];    // T_{l+1,l}
  zd Rup[LM_MAXL];    // R~_{l,l-1}, Rup[0] = 0
  zd Rdn[LM_MAXL];    // R~_{l,l+1}, Rdn[L] = 0
  zd ph[LM_MAXL];     // exp(2 i k_{l,y} h_l)
};

LM_HD void stack_at(const MediumDev& m, zd lam, StackAt& s) {
  const int L = m.L;
  for (int l = 0; l <= L; ++l) {
    s.ky[l] = zky(m.k[l], lam);
    s.ph[l] = zexp(zd(0.0, 2.0 * layer_thickness(m, l)) * s.ky[l]);
  }
  for (int l = 0; l < L; ++l) {
    zd a = s.ky[l] * m.eta[l], b = s.ky[l + 1] * m.eta[l + 1];
    zd inv = 1.0 / (a + b);
    s.Rloc[l] = (a - b) * inv;
    s.Tdn[l] = (a * 2.0) * inv;
    s.Tup[l] = (b * 2.0) * inv;
  }
  s.Rup[0] = zd(0.0, 0.0);
  for (int l = 0; l < L; ++l) {
    zd r = -s.Rloc[l];               // R_{l+1,l}
    zd t = s.Rup[l] * s.ph[l];
    s.Rup[l + 1] = (r + t) / (1.0 + r * t);
  }
  s.Rdn[L] = zd(0.0, 0.0);
  for (int l = L - 1; l >= 0; --l) {
    zd t = s.Rdn[l + 1] * s.ph[l + 1];
    s.Rdn[l] = (s.Rloc[l] + t) / (1.0 + s.Rloc[l] * t);
  }
}

// Generalized transmission T~_{lp -> l}.
LM_HD zd gen_transmission(const MediumDev& m, const StackAt& s, int lp, int l) {
  zd v(1.0, 0.0);
  if (l < lp) {
    for (int j = lp - 1; j >= l; --j) {
      zd num = s.Tup[j] * zexp(zd(0.0, m.d[j]) * (s.ky[j] - s.ky[j + 1]));
      zd den = 1.0 - s.Rloc[j] * s.Rup[j] * s.ph[j];   // 1 + R_{j+1,j} R~_{j,j-1} e^{2ikh}
      v = num * v / den;
    }
  } else if (l > lp) {
    for (int j = lp + 1; j <= l; ++j) {
      zd num = s.Tdn[j - 1] * zexp(zd(0.0, m.d[j - 1]) * (s.ky[j - 1] - s.ky[j]));
      zd den = 1.0 + s.Rloc[j - 1] * s.Rdn[j] * s.ph[j];
      v = num * v / den;
    }
  }
  return v;
}

// S^c(lam) for the components of (target layer lt, source layer ls) selected
// by mask (bit c).  Components whose sides do not exist are left untouched.
LM_HD void side_densities(const MediumDev& m, const StackAt& s, int lt, int ls, unsigned mask, zd* S) {
  // Case I quantities of the source layer
  zd D = 1.0 - s.Rdn[ls] * s.Rup[ls] * s.ph[ls];
  zd invD = 1.0 / D;
  zd sig[4];  // index c = t + 2 s: 0 = (up,down) 1 = (down,down) 2 = (up,up) 3 = (down,up)
  if (lt == ls) {
    zd ud = s.Rdn[ls] * invD, du = s.Rup[ls] * invD, uu = s.Rup[ls] * ud;
    sig[0] = ud; sig[1] = uu; sig[2] = uu; sig[3] = du;
  } else if (lt < ls) {
    zd T = gen_transmission(m, s, ls, lt);
    zd ud = T * (s.Rdn[ls] * invD);
    zd uu = T * (1.0 + s.Rup[ls] * s.Rdn[ls] * invD * s.ph[ls]);
    sig[0] = ud; sig[2] = uu; sig[1] = s.Rup[lt] * ud; sig[3] = s.Rup[lt] * uu;
  } else {
    zd T = gen_transmission(m, s, ls, lt);
    zd du = T * (s.Rup[ls] * invD);
    zd dd = T * (1.0 + s.Rup[ls] * s.Rdn[ls] * invD * s.ph[ls]);
    sig[3] = du; sig[1] = dd; sig[2] = s.Rdn[lt] * du; sig[0] = s.Rdn[lt] * dd;
  }
  zd pref = zd(0.0, 0.5) / s.ky[ls];  // i / (2 k_{l',y})
  for (int c = 0; c < 4; ++c) {
    if (!((mask >> c) & 1u)) continue;
    int ts = c & 1, ss = c >> 1;
    if (!side_exists(m, lt, ts) || !side_exists(m, ls, ss)) continue;
    double at, as;
    if (ts == SIDE_B) {
      bool direct = (ss == SIDE_B) ? (lt <= ls) : (lt < ls);
      at = direct ? -m.d[lt] : m.d[lt];
    } else {
      bool direct = (ss == SIDE_B) ? (lt > ls) : (lt >= ls);
      at = direct ? m.d[lt - 1] : -m.d[lt - 1];
    }
    if (ss == SIDE_B) as = (lt <= ls) ? m.d[ls] : -m.d[ls];
    else as = (lt < ls) ? m.d[ls - 1] : -m.d[ls - 1];
    zd e = zexp(zd(0.0, 1.0) * (s.ky[lt] * at + s.ky[ls] * as));
    S[c] = sig[c] * pref * e;
  }
}
