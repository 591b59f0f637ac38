"""Scattered field from the density: receivers and far-field patterns.

Oracle (test infrastructure): see the package docstring.

Paper, eq. integralrep: u^s at r is the single-layer potential of the density
over all Gamma_l.  In the unscaled form (see ``nystrom``) that is
u^s(r) = sum_e |Gamma_e| phi_e G_{l(r) l_e}(r | c_e).

The paper defines no far field for layered media (reading "Z22").  This oracle
uses the stationary-phase limit of the spectral representation: for r in the
top layer at angle theta in (0, pi),

    u^s(R, theta) ~ exp(i k_0 R) / sqrt(R) * u_top(theta),
    u_top(theta)  = e^{-i pi/4} sqrt(k_0 / 2pi) sin(theta) S_0(k_0 cos theta),
    S_0(lam)      = sum_e |Gamma_e| phi_e e^{-i lam x_e} a_e(lam),

where a_e collects the free-space term (source in layer 0) and every reaction
component G^{up,star}_{0 l_e} of eq. fourreactions with its target factor
exp(i k_{0,y} y) removed.  The bottom pattern is the mirror image in layer L
with the down components and theta in (pi, 2pi).  In a homogeneous medium this
reduces to the usual e^{i pi/4}/sqrt(8 pi k) sum |Gamma| phi e^{-i k xhat.c}.
"""

import numpy as np

from .green import LayeredGreen
from .medium import nonzero_components


def scattered_field(med, el, phi, x, y, green=None):
    """u^s at observation points (x, y) off the boundary (eq. integralrep)."""
    G = LayeredGreen(med) if green is None else green
    x = np.atleast_1d(np.asarray(x, dtype=float))
    y = np.atleast_1d(np.asarray(y, dtype=float))
    q = el.w * np.asarray(phi)
    out = np.zeros(x.shape, dtype=complex)
    for r in range(x.size):
        for lp in range(med.L + 1):
            idx = np.nonzero(el.layer == lp)[0]
            if idx.size == 0:
                continue
            g = G.green(x[r], y[r], el.cx[idx], el.cy[idx], lp=lp)
            out[r] += g @ q[idx]
    return out


def _spectral_source_factor(med, el, lam, target_layer, arrival):
    """a_e(lam) for every element: the lam-integrand of G_{target, l_e}(r|c_e)
    with exp(i lam x) exp(+-i k_{target,y} y) removed."""
    C = med.coefficients(np.array([lam], dtype=complex))
    ky = np.array([C["ky"][l][0] for l in range(med.L + 1)])
    lt = target_layer
    a = np.zeros(el.n, dtype=complex)
    for lp in range(med.L + 1):
        idx = np.nonzero(el.layer == lp)[0]
        if idx.size == 0:
            continue
        ys = el.cy[idx]
        acc = np.zeros(idx.size, dtype=complex)
        if lp == lt:
            # free space (1/2pi) int e^{i lam (x-x')} e^{i k_y |y-y'|} i/(2 k_y)
            sgn = 1.0 if arrival == "u" else -1.0
            acc += 1j / (2.0 * ky[lt]) * np.exp(-1j * sgn * ky[lt] * ys)
        sig = med.densities(np.array([lam], dtype=complex), lt, lp, C)
        for c in nonzero_components(lt, lp, med.L):
            if c[0] != arrival:
                continue
            # Theta = k_{lt,y} A + k_{lp,y} B and A = +-y + const; keep only the
            # source part and the constant
            A0, B = med.theta_coeffs(c, lt, lp, 0.0, ys)
            acc += sig[c][0] * 1j / (2.0 * ky[lp]) * np.exp(1j * (ky[lt] * A0 + ky[lp] * B))
        a[idx] = acc * np.exp(-1j * lam * el.cx[idx])
    return a


def far_field(med, el, phi, theta):
    """Top (0 < theta < pi) or bottom (pi < theta < 2 pi) far-field pattern."""
    theta = np.atleast_1d(np.asarray(theta, dtype=float))
    q = el.w * np.asarray(phi)
    out = np.zeros(theta.shape, dtype=complex)
    for j, th in enumerate(theta):
        s = np.sin(th)
        if s > 0:
            lt, arr, kk = 0, "u", med.k[0]
        elif s < 0:
            lt, arr, kk = med.L, "d", med.k[med.L]
        else:
            raise ValueError("far field is defined off the horizontal directions")
        lam = kk * np.cos(th)
        a = _spectral_source_factor(med, el, lam, lt, arr)
        out[j] = np.exp(-0.25j * np.pi) * np.sqrt(kk / (2.0 * np.pi)) * abs(s) * (a @ q)
    return out
