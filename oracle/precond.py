"""Overlapping domain-decomposition preconditioner, built densely.

Oracle (test infrastructure): see the package docstring.

Paper, Sec. 4.2.  The reaction part of the diagonal blocks K_ll is dropped,
which leaves per layer l the matrix of the free-space interaction plus the
singular self terms.  Its inverse is approximated with the tree of the
free-space FMM: for every box B of layer l's tree, J = the elements of B and
of its neighbour boxes (B included), and the local matrix (eq. localmatix) is

    P_B[a][b] = |Gamma_{j_b}| G^f_l(c_{j_a}, c_{j_b})   (a != b),
    P_B[a][a] = I^s_{j_a}.

The local solve keeps the entries of B (Q_B) and the local solutions are
added (S_B):  P^{-1} = sum_B S_B Q_B P_B^{-1} R_B, block-diagonal over the
layers.  The paper writes the local system for eta_l g; within one layer eta
is a constant factor, so the same operator serves the unscaled system the
oracle uses (P^{-1}(eta g) = eta P^{-1} g and the unknowns are eta phi).

Readings (the paper names "leaf boxes" of "the FMM tree" but does not fix the
tree):
* the tree of layer l is a uniform quadtree in (x, h) with h the height of
  the point above the layer's bottom interface (below the top interface for
  the bottom layer; clamped at 0), level widths w_lev = w_top / 2^lev with
  w_top = 8 / max_l k_l, and one x-origin shared by every layer,
  x0 = min x - 1e-7 (1 + |min x|) - (median element length) / 2;
* the leaf level is the first level whose non-empty boxes hold on average at
  most ``leaf_size`` elements (over the trees of all layers), at most 12;
* the subdomains may be the boxes of a coarser level than the leaves
  (ancestors of the leaf boxes): ``level_for(..., precond=c)`` gives the
  leaf level for c = 1, c - 1 levels above it for c >= 2, and for c < 0
  the coarsest level whose neighbourhoods hold at most 8192 elements;
* neighbours are the (up to 8) boxes of the same layer and level whose
  column and row differ by at most one.
"""

import numpy as np
from scipy.special import hankel1

from .nystrom import self_term

TOP_KW = 8.0     # top-level box width times the largest wavenumber
MAX_LEVEL = 12
QMAX_AUTO = 8192  # largest neighbourhood of the automatic subdomain level


def box_height(med, layer, y):
    """Height of points y of a layer above its bottom interface (below the
    top interface for the bottom layer), clamped at 0."""
    layer = np.asarray(layer)
    y = np.asarray(y, dtype=float)
    h = np.empty(y.shape)
    for l in range(med.L + 1):
        sel = layer == l
        h[sel] = (y[sel] + med.d[l]) if l < med.L else (-med.d[l - 1] - y[sel])
    return np.maximum(h, 0.0)


class BoxGrid:
    """Cell indices of every element in the uniform trees of its layer."""

    def __init__(self, med, el):
        self.med, self.el = med, el
        xmin = float(np.min(el.cx))
        hmed = float(np.sort(el.w)[el.n // 2])
        self.w_top = TOP_KW / float(np.max(med.k))
        self.x0 = xmin - 1e-7 * (1.0 + abs(xmin)) - 0.5 * hmed
        self.h = box_height(med, el.layer, el.cy)

    def width(self, lev):
        return self.w_top / float(1 << lev)

    def cells(self, lev):
        """(column, row) of every element at level lev."""
        w = self.width(lev)
        i = np.floor((self.el.cx - self.x0) / w).astype(np.int64)
        j = np.floor(self.h / w).astype(np.int64)
        return i, j

    def leaf_level(self, leaf_size):
        for lev in range(MAX_LEVEL):
            i, j = self.cells(lev)
            nbox = len(set(zip(self.el.layer.tolist(), i.tolist(), j.tolist())))
            if self.el.n / nbox <= leaf_size:
                return lev
        return MAX_LEVEL

    def boxes(self, lev, leaf_level):
        """{(layer, column, row): element indices} at level lev <= leaf_level:
        the level-lev ancestors of the leaf boxes."""
        i, j = self.cells(leaf_level)
        sh = leaf_level - lev
        i, j = i >> sh, j >> sh
        out = {}
        for e in range(self.el.n):
            out.setdefault((int(self.el.layer[e]), int(i[e]), int(j[e])), []).append(e)
        return out


def subdomains(med, el, lev, leaf_level):
    """[(own elements, neighbourhood elements)] for the boxes of level lev;
    the neighbourhood lists the box's own elements first."""
    bx = BoxGrid(med, el).boxes(lev, leaf_level)
    out = []
    for (l, i, j), own in sorted(bx.items()):
        J = list(own)
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                if di == 0 and dj == 0:
                    continue
                J += bx.get((l, i + di, j + dj), [])
        out.append((np.array(own, dtype=np.int64), np.array(J, dtype=np.int64)))
    return out


def level_for(med, el, precond, leaf_size=48):
    """(subdomain level, leaf level) of the option ``precond`` (see the
    module docstring)."""
    grid = BoxGrid(med, el)
    lf = grid.leaf_level(leaf_size)
    if precond >= 1:
        return max(0, lf - (precond - 1)), lf
    for lev in range(lf + 1):
        q = max(len(J) for _, J in subdomains(med, el, lev, lf))
        if q <= QMAX_AUTO:
            return lev, lf
    return lf, lf


def local_matrix(med, el, J):
    """P_B over the neighbourhood J (eq. localmatix)."""
    l = int(el.layer[J[0]])
    assert np.all(el.layer[J] == l)
    k = med.k[l]
    dx = el.cx[J][:, None] - el.cx[J][None, :]
    dy = el.cy[J][:, None] - el.cy[J][None, :]
    r = np.hypot(dx, dy)
    q = len(J)
    P = np.zeros((q, q), dtype=complex)
    off = ~np.eye(q, dtype=bool)
    P[off] = (0.25j * hankel1(0, k * r[off])) * np.broadcast_to(el.w[J][None, :], (q, q))[off]
    P[np.diag_indices(q)] = self_term(k, el.w[J])
    return P


def dense(med, el, lev, leaf_level):
    """P^{-1} = sum_B S_B Q_B P_B^{-1} R_B as a dense N x N matrix."""
    M = np.zeros((el.n, el.n), dtype=complex)
    for own, J in subdomains(med, el, lev, leaf_level):
        Pinv = np.linalg.inv(local_matrix(med, el, J))
        nb = len(own)
        # rows of B (the first nb entries of J), columns of J
        M[np.ix_(J[:nb], J)] += Pinv[:nb, :]
    return M


def apply(med, el, lev, leaf_level, x):
    """y = P^{-1} x for x of shape (N,) or (R, N), one local solve per box."""
    x = np.atleast_2d(np.asarray(x, dtype=complex))
    y = np.zeros_like(x)
    for own, J in subdomains(med, el, lev, leaf_level):
        P = local_matrix(med, el, J)
        t = np.linalg.solve(P, x[:, J].T).T
        y[:, J[: len(own)]] += t[:, : len(own)]
    return y
