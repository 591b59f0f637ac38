"""The oracle's quadrature for Sommerfeld integrals.

Oracle (test infrastructure): see the package docstring.

The paper gives the reaction components as Sommerfeld integrals
(eq. fourreactions, uniform form eq. planewavekernel) but is silent on how
they are evaluated (reading: any convergent quadrature is admissible).  Every reaction component has
the form

    I = (1/2pi) int_{-inf}^{inf} exp(i lam dx) F(lam) dlam,

with F even in lam (it depends on lam only through the k_{l,y}) and
|F(lam)| ~ exp(-D |lam|) for large |lam| where D >= 0 is the vertical decay
distance.  Evenness folds the integral onto [0, inf):

    I = (1/2pi) int_C [exp(i lam X) + exp(-i lam X)] F(lam) dlam,  X = |dx|,

where C leaves 0 into the fourth quadrant to pass below the real branch points
and guided-mode poles (lam = t - i a sin(pi t / Tc), 0 <= t <= Tc, Tc = k_max+2)
and then follows the real axis.  Two tails:

* "real" (D >= X/4): the real axis up to Tc + 40/D, where exp(-lam D) is 4e-18;
* "ray"  (D <  X/4): after Tc + 1 each exponential leaves along its own
  steepest-descent ray lam = Lam1 + s exp(+-i psi), psi = atan2(X, D), on which
  exp(+-i lam X) F decays like exp(-s sqrt(X^2 + D^2)).  The deformation is
  legal because F has no singularities with Re lam > k_max on the sheet
  Im k_{l,y} >= 0.

Pairs are binned by (X, D) in powers of two so that node sets (and the
expensive densities evaluated on them) are shared by all pairs of a bin.
All panels are 16-point Gauss-Legendre.
"""

import functools

import numpy as np

_NGL = 16
_XGL, _WGL = np.polynomial.legendre.leggauss(_NGL)

BIN_MIN = -30  # 2**-30 ~ 1e-9


def _panels(edges):
    """Gauss-Legendre nodes/weights on consecutive intervals given by edges."""
    a = np.asarray(edges[:-1], dtype=float)
    b = np.asarray(edges[1:], dtype=float)
    half = 0.5 * (b - a)
    mid = 0.5 * (b + a)
    t = (mid[:, None] + half[:, None] * _XGL[None, :]).ravel()
    w = (half[:, None] * _WGL[None, :]).ravel()
    return t, w


def _grow(a, b, width_fn):
    """Edges from a to b with panel width width_fn(left_edge)."""
    edges = [a]
    x = a
    while x < b:
        x = min(b, x + width_fn(x))
        edges.append(x)
    return np.asarray(edges)


def bin_index(v):
    """Power-of-two bin of a non-negative distance (v < 2**BIN_MIN -> BIN_MIN)."""
    v = np.asarray(v, dtype=float)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.maximum(v, 2.0 ** (BIN_MIN - 1))))
    return np.maximum(e, BIN_MIN).astype(int)


@functools.lru_cache(maxsize=4096)
def node_set(kmax, ix, idd):
    """Nodes for the bin X in [2^ix, 2^(ix+1)), D in [2^idd, 2^(idd+1)).

    Returns (lam_c, w_c, lam_p, w_p, lam_m, w_m): lam_c/w_c carry the
    symmetric part [exp(i lam X) + exp(-i lam X)], lam_p/w_p the exp(+i lam X)
    ray and lam_m/w_m the exp(-i lam X) ray (empty in the real regime).
    Weights include dlam/dt.
    """
    X_lo = 0.0 if ix <= BIN_MIN else 2.0 ** ix
    X_hi = 2.0 ** (ix + 1)
    D_lo = 0.0 if idd <= BIN_MIN else 2.0 ** idd
    D_hi = 2.0 ** (idd + 1)
    Tc = kmax + 2.0
    a = min(0.4, 4.0 / X_hi)
    # deformed part: width limited by the pole clearance a and the oscillation
    wc = min(0.25, a / 2.0, 6.0 / X_hi)
    t, w = _panels(_grow(0.0, Tc, lambda x: wc))
    lam0 = t - 1j * a * np.sin(np.pi * t / Tc)
    dl0 = 1.0 - 1j * a * (np.pi / Tc) * np.cos(np.pi * t / Tc)
    w0 = w * dl0
    real_regime = D_lo >= X_hi / 4.0
    empty = np.zeros(0, dtype=complex)
    if real_regime:
        Dd = max(D_lo, 2.0 ** BIN_MIN)
        lam_end = Tc + 40.0 / Dd
        width = lambda x: min(6.0 / X_hi, 2.0 / Dd, 0.25 + 0.25 * (x - Tc))
        t1, w1 = _panels(_grow(Tc, lam_end, width))
        lam_c = np.concatenate([lam0, t1.astype(complex)])
        w_c = np.concatenate([w0, w1.astype(complex)])
        return lam_c, w_c, empty, empty, empty, empty
    Lam1 = Tc + 1.0
    t1, w1 = _panels(_grow(Tc, Lam1, lambda x: min(0.25, 6.0 / X_hi)))
    lam_c = np.concatenate([lam0, t1.astype(complex)])
    w_c = np.concatenate([w0, w1.astype(complex)])
    Xc = np.sqrt(X_lo * X_hi) if X_lo > 0 else X_hi / 2
    Dc = np.sqrt(D_lo * D_hi) if D_lo > 0 else 0.0
    psi = np.arctan2(Xc, Dc)
    z_lo = max(np.hypot(X_lo, D_lo), 2.0 ** BIN_MIN)
    z_hi = np.hypot(X_hi, D_hi)
    S = 60.0 / z_lo
    ts, ws = _panels(_grow(0.0, S, lambda s: min(2.0 / z_hi, 0.5 + 0.5 * s)))
    ep = np.exp(1j * psi)
    lam_p = Lam1 + ts * ep
    w_p = ws * ep
    lam_m = Lam1 + ts * np.conj(ep)
    w_m = ws * np.conj(ep)
    return lam_c, w_c, lam_p, w_p, lam_m, w_m


def sommerfeld(X, fac_c, fac_p, fac_m, nodes):
    """Evaluate (1/2pi) int exp(i lam dx) F dlam for pairs sharing one node set.

    X: (n,) |dx| per pair.  fac_*: (n, q_*) values of F on the three node
    groups (pair-dependent).  nodes: output of node_set.
    """
    lam_c, w_c, lam_p, w_p, lam_m, w_m = nodes
    X = np.asarray(X, dtype=float)[:, None]
    out = ((2.0 * np.cos(lam_c[None, :] * X)) * fac_c) @ w_c
    if lam_p.size:
        out = out + (np.exp(1j * lam_p[None, :] * X) * fac_p) @ w_p
        out = out + (np.exp(-1j * lam_m[None, :] * X) * fac_m) @ w_m
    return out / (2.0 * np.pi)


def sommerfeld_dx(X, fac_c, fac_p, fac_m, nodes):
    """d/dX of ``sommerfeld``: the lam-integrand gains i lam on the e^{+i lam X}
    branch and -i lam on the e^{-i lam X} branch (so 2 cos(lam X) becomes
    -2 lam sin(lam X) on the shared nodes)."""
    lam_c, w_c, lam_p, w_p, lam_m, w_m = nodes
    X = np.asarray(X, dtype=float)[:, None]
    out = ((-2.0 * lam_c[None, :] * np.sin(lam_c[None, :] * X)) * fac_c) @ w_c
    if lam_p.size:
        out = out + (1j * lam_p[None, :] * np.exp(1j * lam_p[None, :] * X) * fac_p) @ w_p
        out = out + (-1j * lam_m[None, :] * np.exp(-1j * lam_m[None, :] * X) * fac_m) @ w_m
    return out / (2.0 * np.pi)
