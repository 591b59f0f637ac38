"""Layered Green's function G_{l l'}(r, r'): field at r (layer l) due to a point
source at r' (layer l').

Oracle (test infrastructure): see the package docstring.

Paper, Sec. 3.1: G = delta_{l l'} G^f_l + G^r_{l l'} (eq. layeredGreensfun),
G^f_l = (i/4) H_0^(1)(k_l |r - r'|) (eq. freegreensfun), and G^r the sum of
the four components of eq. fourreactions with tau_m(a) = -2 d_m - a
(eq. reflections) and the densities of Cases I-III.

Reading: the spectral prefactor printed as 1/(2 k_{l',y}) is read as
i/(2 k_{l',y}); only that form reproduces (i/4) H_0 through the Sommerfeld
identity, which the tests pin.
"""

import numpy as np
from scipy.special import hankel1

from .medium import nonzero_components
from .quadrature import bin_index, node_set, sommerfeld, sommerfeld_dx


def free_space(k, x, y, xs, ys, dy=False):
    """(i/4) H_0^(1)(k |r - r'|) and optionally its y-derivative."""
    rx = np.asarray(x) - np.asarray(xs)
    ry = np.asarray(y) - np.asarray(ys)
    rho = np.hypot(rx, ry)
    g = 0.25j * hankel1(0, k * rho)
    if not dy:
        return g
    dg = -0.25j * k * hankel1(1, k * rho) * ry / rho
    return g, dg


def free_space_grad(k, x, y, xs, ys):
    """(i/4) H_0^(1)(k |r - r'|) and its gradient in the target r:
    -(i/4) k H_1^(1)(k rho) (r - r') / rho."""
    rx = np.asarray(x) - np.asarray(xs)
    ry = np.asarray(y) - np.asarray(ys)
    rho = np.hypot(rx, ry)
    g = 0.25j * hankel1(0, k * rho)
    d = -0.25j * k * hankel1(1, k * rho) / rho
    return g, d * rx, d * ry


class _SigmaCache:
    """Densities and k_y on a bin's node set, keyed by (l, l', comp, bin)."""

    def __init__(self, med):
        self.med = med
        self.kmax = float(np.max(med.k))
        self.store = {}

    def get(self, l, lp, ix, idd):
        key = (l, lp, ix, idd)
        hit = self.store.get(key)
        if hit is not None:
            return hit
        nodes = node_set(self.kmax, ix, idd)
        groups = []
        for lam in (nodes[0], nodes[2], nodes[4]):
            if lam.size == 0:
                groups.append(None)
                continue
            C = self.med.coefficients(lam)
            sig = self.med.densities(lam, l, lp, C)
            ky = C["ky"]
            pref = 1j / (2.0 * ky[lp])  # reading: i/(2 k_{l',y})
            groups.append((ky[l], ky[lp], {c: sig[c] * pref for c in sig}))
        hit = (nodes, groups)
        self.store[key] = hit
        return hit


class LayeredGreen:
    """Evaluator of G and its pieces for one medium."""

    def __init__(self, med):
        self.med = med
        self.cache = _SigmaCache(med)

    def reaction_component(self, comp, l, lp, x, y, xs, ys, dy=False):
        """One reaction component G^{comp}_{l l'}(r, r') for one target r and
        arrays of sources r' (all in layer l').  If dy, also d/dy."""
        med = self.med
        xs = np.atleast_1d(np.asarray(xs, dtype=float))
        ys = np.atleast_1d(np.asarray(ys, dtype=float))
        A, B = med.theta_coeffs(comp, l, lp, y, ys)
        A = np.broadcast_to(np.asarray(A, dtype=float), ys.shape)
        B = np.broadcast_to(np.asarray(B, dtype=float), ys.shape)
        # dA/dy is +1 or -1 depending on the case
        dAdy = med.theta_coeffs(comp, l, lp, y + 1.0, ys)[0] - A
        D = np.maximum(A + B, 0.0)
        X = np.abs(x - xs)
        out = np.zeros(xs.shape, dtype=complex)
        dout = np.zeros(xs.shape, dtype=complex)
        ib_x, ib_d = bin_index(X), bin_index(D)
        keys = ib_x.astype(np.int64) * 1000 + (ib_d.astype(np.int64) + 500)
        for key in np.unique(keys):
            sel = np.nonzero(keys == key)[0]
            ix, idd = int(ib_x[sel[0]]), int(ib_d[sel[0]])
            nodes, groups = self.cache.get(l, lp, ix, idd)
            if all(g is None or not np.any(g[2][comp]) for g in groups):
                continue  # density is exactly zero on every node: the sum is zero
            facs, dfacs = [], []
            for g in groups:
                if g is None:
                    facs.append(None)
                    dfacs.append(None)
                    continue
                kyl, kylp, sig = g
                ph = np.exp(1j * (kyl[None, :] * A[sel, None] + kylp[None, :] * B[sel, None]))
                f = ph * sig[comp][None, :]
                facs.append(f)
                if dy:
                    dfacs.append(f * (1j * kyl[None, :]) * dAdy[sel, None])
            out[sel] = sommerfeld(X[sel], facs[0], facs[1], facs[2], nodes)
            if dy:
                dout[sel] = sommerfeld(X[sel], dfacs[0], dfacs[1], dfacs[2], nodes)
        if dy:
            return out, dout
        return out

    def reaction_component_grad(self, comp, l, lp, x, y, xs, ys):
        """One reaction component and its gradient in the target (x, y).
        d/dx acts on e^{i lam (x - x')} through the sign of x - x' and the
        X-derivative of the folded integral; d/dy on e^{i Theta} through
        dTheta/dy = k_{l,y} dA/dy (dA/dy = +-1)."""
        med = self.med
        xs = np.atleast_1d(np.asarray(xs, dtype=float))
        ys = np.atleast_1d(np.asarray(ys, dtype=float))
        A, B = med.theta_coeffs(comp, l, lp, y, ys)
        A = np.broadcast_to(np.asarray(A, dtype=float), ys.shape)
        B = np.broadcast_to(np.asarray(B, dtype=float), ys.shape)
        dAdy = med.theta_coeffs(comp, l, lp, y + 1.0, ys)[0] - A
        D = np.maximum(A + B, 0.0)
        X = np.abs(x - xs)
        sgn = np.sign(x - xs)
        g = np.zeros(xs.shape, dtype=complex)
        gx = np.zeros(xs.shape, dtype=complex)
        gy = np.zeros(xs.shape, dtype=complex)
        ib_x, ib_d = bin_index(X), bin_index(D)
        keys = ib_x.astype(np.int64) * 1000 + (ib_d.astype(np.int64) + 500)
        for key in np.unique(keys):
            sel = np.nonzero(keys == key)[0]
            ix, idd = int(ib_x[sel[0]]), int(ib_d[sel[0]])
            nodes, groups = self.cache.get(l, lp, ix, idd)
            if all(gg is None or not np.any(gg[2][comp]) for gg in groups):
                continue
            facs, dfacs = [], []
            for gg in groups:
                if gg is None:
                    facs.append(None)
                    dfacs.append(None)
                    continue
                kyl, kylp, sig = gg
                ph = np.exp(1j * (kyl[None, :] * A[sel, None] + kylp[None, :] * B[sel, None]))
                f = ph * sig[comp][None, :]
                facs.append(f)
                dfacs.append(f * (1j * kyl[None, :]) * dAdy[sel, None])
            g[sel] = sommerfeld(X[sel], facs[0], facs[1], facs[2], nodes)
            gx[sel] = sgn[sel] * sommerfeld_dx(X[sel], facs[0], facs[1], facs[2], nodes)
            gy[sel] = sommerfeld(X[sel], dfacs[0], dfacs[1], dfacs[2], nodes)
        return g, gx, gy

    def green_grad(self, x, y, xs, ys, l, lp):
        """G_{l l'}(r | r') and its gradient in the target r, for one target
        and an array of sources in layer l'."""
        med = self.med
        xs = np.atleast_1d(np.asarray(xs, dtype=float))
        ys = np.atleast_1d(np.asarray(ys, dtype=float))
        g = np.zeros(xs.shape, dtype=complex)
        gx = np.zeros(xs.shape, dtype=complex)
        gy = np.zeros(xs.shape, dtype=complex)
        for c in nonzero_components(l, lp, med.L):
            a, b, cc = self.reaction_component_grad(c, l, lp, x, y, xs, ys)
            g += a
            gx += b
            gy += cc
        if l == lp:
            a, b, cc = free_space_grad(med.k[l], x, y, xs, ys)
            g += a
            gx += b
            gy += cc
        return g, gx, gy

    def reaction(self, l, lp, x, y, xs, ys, dy=False):
        """G^r_{l l'}: sum of the non-zero components (Remark: 4L^2 of them)."""
        xs = np.atleast_1d(np.asarray(xs, dtype=float))
        tot = np.zeros(xs.shape, dtype=complex)
        dtot = np.zeros(xs.shape, dtype=complex)
        for c in nonzero_components(l, lp, self.med.L):
            r = self.reaction_component(c, l, lp, x, y, xs, ys, dy=dy)
            if dy:
                tot += r[0]
                dtot += r[1]
            else:
                tot += r
        return (tot, dtot) if dy else tot

    def green(self, x, y, xs, ys, l=None, lp=None, dy=False):
        """Full G_{l l'}(r, r') for one target and an array of sources in a
        single layer l' (layers are inferred from the coordinates unless
        given)."""
        med = self.med
        xs = np.atleast_1d(np.asarray(xs, dtype=float))
        ys = np.atleast_1d(np.asarray(ys, dtype=float))
        if l is None:
            l = int(med.layer_of(y))
        if lp is None:
            lps = med.layer_of(ys)
            assert np.all(lps == lps[0]), "sources must lie in one layer"
            lp = int(lps[0])
        r = self.reaction(l, lp, x, y, xs, ys, dy=dy)
        if l == lp:
            f = free_space(med.k[l], x, y, xs, ys, dy=dy)
            if dy:
                return r[0] + f[0], r[1] + f[1]
            return r + f
        return r
