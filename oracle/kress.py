"""Spectrally accurate Nystrom discretisation of smooth closed scatterers.

Oracle (test infrastructure): see the package docstring.

Beyond the paper's discretisation: Sec. 3.3 and Sec. 5 use the lowest-order
rule (chords, midpoint collocation, eqs. ApproximateComputation and
matrixelmemts), first order in the element size.  For scatterers that are
smooth closed curves lying inside one layer, the product quadrature for
logarithmic kernels of Martensen and Kussmaul (as presented by Kress, Linear
Integral Equations, Sec. 12.3) reaches spectral order:

* a scatterer is x(t), t in [0, 2 pi), sampled at its M = 2n input nodes
  t_j = 2 pi j / M (the nodes are read as samples at equal parameter steps);
  x'(t_j) is the derivative of the trigonometric interpolant of the samples;
* the unknown is the density at the nodes; node j carries the weight
  w_j = (2 pi / M) |x'(t_j)|, so every sum over smooth integrands (other
  scatterers, the reaction part G^r, far fields, fields off the boundary) is
  the trapezoidal rule;
* within a scatterer the free-space kernel
  m(t, s) = (i/4) H_0(k |x(t) - x(s)|) |x'(s)| splits as
  m = m1(t, s) ln(4 sin^2((t - s)/2)) + m2(t, s) with
  m1 = -J_0(k |x(t) - x(s)|) |x'(s)| / (4 pi) and m2 smooth,
  m2(t, t) = (i/4 - gamma/(2 pi) - ln(k |x'(t)| / 2)/(2 pi)) |x'(t)|
  (from the logarithmic term of Y_0); the logarithm is integrated exactly
  against the trigonometric interpolant,
  int ln(4 sin^2((t - s)/2)) f(s) ds ~ sum_j R_j(t) f(t_j),
  R_j(t) = -(2 pi / n) sum_{m=1}^{n-1} cos(m (t - t_j)) / m
           - (pi / n^2) cos(n (t - t_j)),
  and m2 by the trapezoidal rule.

Readings (the paper does not treat this rule): every scatterer has an even
number of nodes (>= 6) and lies inside one layer without touching an
interface, so the reaction part is smooth on it; the outward unit normal is
x'(t) turned by -90 degrees for counter-clockwise nodes (+90 for clockwise).
"""

import numpy as np
from scipy.special import hankel1, j0

from .green import LayeredGreen, free_space

EULER_GAMMA = 0.57721566490153286061


def spectral_derivative(f):
    """d/dt of the trigonometric interpolant of the samples f(2 pi j / M),
    j = 0..M-1, at the same points (the unpaired mode of an even M dropped)."""
    f = np.asarray(f, dtype=float)
    M = f.size
    m = np.fft.fftfreq(M, d=1.0 / M)
    if M % 2 == 0:
        m[M // 2] = 0.0
    return np.real(np.fft.ifft(1j * m * np.fft.fft(f)))


def log_weights(M):
    """R_j(t_i) as a function of k = (i - j) mod M, for M = 2n nodes."""
    if M % 2 or M < 6:
        raise ValueError("the logarithmic weights need an even number of nodes >= 6")
    n = M // 2
    d = 2.0 * np.pi * np.arange(M) / M
    m = np.arange(1, n)
    return -(2.0 * np.pi / n) * (np.cos(np.outer(d, m)) / m).sum(axis=1) - (np.pi / n ** 2) * np.cos(n * d)


class Nodes:
    """Quadrature nodes of smooth closed scatterers (one node list per
    scatterer, equal parameter steps).  Attributes as ``nystrom.Elements``
    (cx, cy, w, layer, scatterer, nx, ny, n) plus the speed |x'(t_j)|, the
    local index j and the node count M of each node's scatterer."""

    def __init__(self, med, polygons):
        cols = {k: [] for k in ("cx", "cy", "w", "speed", "sid", "loc", "M", "nx", "ny", "layer")}
        for s, P in enumerate(polygons):
            P = np.asarray(P, dtype=float)
            M = P.shape[0]
            if P.ndim != 2 or P.shape[1] != 2 or M < 6 or M % 2:
                raise ValueError("each scatterer needs an even number (>= 6) of nodes")
            lay = med.layer_of(P[:, 1])
            if np.any(lay != lay[0]):
                raise ValueError(f"scatterer {s} crosses an interface")
            dx, dy = spectral_derivative(P[:, 0]), spectral_derivative(P[:, 1])
            sp = np.hypot(dx, dy)
            Q = np.roll(P, -1, axis=0)
            o = 1.0 if np.sum(P[:, 0] * Q[:, 1] - Q[:, 0] * P[:, 1]) > 0 else -1.0
            cols["cx"].append(P[:, 0])
            cols["cy"].append(P[:, 1])
            cols["speed"].append(sp)
            cols["w"].append(2.0 * np.pi / M * sp)
            cols["sid"].append(np.full(M, s))
            cols["loc"].append(np.arange(M))
            cols["M"].append(np.full(M, M))
            cols["nx"].append(o * dy / sp)
            cols["ny"].append(-o * dx / sp)
            cols["layer"].append(lay)
        self.cx = np.concatenate(cols["cx"])
        self.cy = np.concatenate(cols["cy"])
        self.w = np.concatenate(cols["w"])
        self.speed = np.concatenate(cols["speed"])
        self.scatterer = np.concatenate(cols["sid"])
        self.local = np.concatenate(cols["loc"])
        self.count = np.concatenate(cols["M"])
        self.nx = np.concatenate(cols["nx"])
        self.ny = np.concatenate(cols["ny"])
        self.layer = np.concatenate(cols["layer"])
        self.med = med
        self.n = self.cx.size


def matrix(med, nd, green=None):
    """Dense matrix of the single-layer operator on the nodes: row i is the
    target node, column j the source node (field at x_i of the density at
    x_j), in the unscaled form of ``nystrom``."""
    G = LayeredGreen(med) if green is None else green
    A = np.zeros((nd.n, nd.n), dtype=complex)
    layers = range(med.L + 1)
    src = {lp: np.nonzero(nd.layer == lp)[0] for lp in layers}
    for i in range(nd.n):
        l, s = int(nd.layer[i]), int(nd.scatterer[i])
        x, y = nd.cx[i], nd.cy[i]
        # trapezoidal rule: the reaction part everywhere, the free-space part
        # on the other scatterers of the same layer
        for lp in layers:
            idx = src[lp]
            if idx.size == 0:
                continue
            vals = G.reaction(l, lp, x, y, nd.cx[idx], nd.cy[idx])
            if lp == l:
                other = nd.scatterer[idx] != s
                vals[other] += free_space(med.k[l], x, y, nd.cx[idx[other]], nd.cy[idx[other]])
            A[i, idx] = vals * nd.w[idx]
        # the free-space part on the node's own scatterer: logarithmic split
        J = np.nonzero(nd.scatterer == s)[0]
        M, k = int(nd.count[i]), med.k[l]
        kk = (nd.local[i] - nd.local[J]) % M
        R = log_weights(M)[kk]
        r = np.hypot(nd.cx[J] - x, nd.cy[J] - y)
        sp = nd.speed[J]
        m1 = -j0(k * r) * sp / (4.0 * np.pi)
        m2 = np.empty(J.size, dtype=complex)
        off = kk != 0
        logf = np.log(4.0 * np.sin(np.pi * kk[off] / M) ** 2)
        m2[off] = 0.25j * hankel1(0, k * r[off]) * sp[off] - m1[off] * logf
        m2[~off] = (0.25j - EULER_GAMMA / (2.0 * np.pi) - np.log(k * sp[~off] / 2.0) / (2.0 * np.pi)) * sp[~off]
        A[i, J] += R * m1 + (2.0 * np.pi / M) * m2
    return A
