"""Lowest-order Nystrom discretisation and the dense matrix.

Oracle (test infrastructure): see the package docstring.

Paper, Sec. 3.3:
* boundaries are split into straight segments, the density is constant on
  each, the collocation point is the element centre (eq. linearSystem);
* the singular self term I^s = [i/4 - (gamma + ln(k |Gamma|/4) - 1)/(2 pi)] |Gamma|
  (eq. ApproximateComputation); the regular remainder is dropped;
* off the diagonal the rectangle rule K = G(c_i | c_e) |Gamma_e|, on the
  diagonal G^r(c_i, c_i) |Gamma_i| + I^s_i (eq. matrixelmemts).

Reading: elements are chords between consecutive polygon nodes (node j to
node j+1, closing the polygon); |Gamma_e| is the chord length; the element
belongs to the layer of its midpoint (ties to the upper layer).

Row i is the collocation point c_i, column e the source element e.  The
paper writes the system source-first with eta scaling (eqs. linearSystem,
matrixandvec: K_{ei}^{l l'} = int_{Gamma_{le}} G_{l l'}(r, c_{l'i}) ds,
unknowns eta_l phi, right side eta_{l'} g).  By the eta-weighted reciprocity
eta_l G_{l l'}(r, r') = eta_{l'} G_{l' l}(r', r), row i of that system is
eta_{l_i} times row i of the unscaled system K phi = g with
K_{ie} = |Gamma_e| G_{l_i l_e}(c_i | c_e) (field at c_i due to c_e).  The
oracle uses the unscaled form; ``paper_form_matrix`` builds the paper's form
so a test can check both give the same phi.
"""

import numpy as np

from .green import LayeredGreen, free_space
from .medium import nonzero_components

EULER_GAMMA = 0.57721566490153286061


class Elements:
    """Chord elements of closed polygons (one polygon per scatterer), with the
    unit normal of every chord pointing out of its polygon (the sign of the
    polygon's signed area decides the orientation)."""

    def __init__(self, med, polygons):
        cx, cy, w, sid, nx, ny = [], [], [], [], [], []
        for j, P in enumerate(polygons):
            P = np.asarray(P, dtype=float)
            if P.ndim != 2 or P.shape[1] != 2 or P.shape[0] < 3:
                raise ValueError("each polygon needs >= 3 nodes of (x, y)")
            Q = np.roll(P, -1, axis=0)
            cx.append(0.5 * (P[:, 0] + Q[:, 0]))
            cy.append(0.5 * (P[:, 1] + Q[:, 1]))
            ln = np.hypot(Q[:, 0] - P[:, 0], Q[:, 1] - P[:, 1])
            w.append(ln)
            sid.append(np.full(P.shape[0], j))
            area2 = np.sum(P[:, 0] * Q[:, 1] - Q[:, 0] * P[:, 1])  # twice the signed area
            o = 1.0 if area2 > 0 else -1.0  # counter-clockwise: the right-hand normal points out
            nx.append(o * (Q[:, 1] - P[:, 1]) / ln)
            ny.append(-o * (Q[:, 0] - P[:, 0]) / ln)
        self.nx = np.concatenate(nx)
        self.ny = np.concatenate(ny)
        self.cx = np.concatenate(cx)
        self.cy = np.concatenate(cy)
        self.w = np.concatenate(w)
        self.scatterer = np.concatenate(sid)
        self.layer = med.layer_of(self.cy)
        self.med = med
        self.n = self.cx.size


def self_term(k, w):
    """I^s (eq. ApproximateComputation)."""
    return (0.25j - (EULER_GAMMA + np.log(k * w / 4.0) - 1.0) / (2.0 * np.pi)) * w


def matrix_rows(med, el, rows, green=None, chunk=None):
    """Rows of the unscaled dense matrix K (complex128, shape (len(rows), N)).

    chunk: evaluate the sources of a layer in blocks of at most this many
    (bounds the memory of the vectorised quadrature at large N; every entry
    is computed the same way)."""
    G = LayeredGreen(med) if green is None else green
    out = np.zeros((len(rows), el.n), dtype=complex)
    layers = range(med.L + 1)
    src_idx = {lp: np.nonzero(el.layer == lp)[0] for lp in layers}
    for r, i in enumerate(rows):
        l = int(el.layer[i])
        x, y = el.cx[i], el.cy[i]
        for lp in layers:
            idx_all = src_idx[lp]
            step = idx_all.size if chunk is None else int(chunk)
            for c0 in range(0, idx_all.size, max(step, 1)):
                idx = idx_all[c0:c0 + step]
                vals = G.reaction(l, lp, x, y, el.cx[idx], el.cy[idx])
                if lp == l:
                    off = idx != i
                    vals[off] += free_space(med.k[l], x, y, el.cx[idx[off]], el.cy[idx[off]])
                out[r, idx] = vals * el.w[idx]
        out[r, i] += self_term(med.k[l], el.w[i])
    return out


def matrix_bc(med, el, beta=None, green=None):
    """Matrix of a sound-hard (beta None) or impedance scatterer.

    Reading (the paper names Neumann and Robin conditions in Sec. 2.1 and
    treats only the Dirichlet one): the same single-layer representation
    u^s = S phi, with the exterior limit of its normal derivative
    d_n S phi = (-1/2 + K') phi (n pointing out of the scatterer) and the
    condition (d_n + i beta) u = 0 on the boundary; collocated at the chord
    midpoints with the rectangle rule:

        A_ie = |Gamma_e| n_i . grad_r G(c_i | c_e) [+ i beta K_ie],   e != i,
        A_ii = -1/2 + |Gamma_i| n_i . grad_r G^r(c_i | c_i) [+ i beta K_ii];

    the free-space part of the self term of K' vanishes on a straight element
    ((c - r') . n = 0 along it)."""
    G = LayeredGreen(med) if green is None else green
    A = np.zeros((el.n, el.n), dtype=complex)
    for i in range(el.n):
        l = int(el.layer[i])
        for lp in range(med.L + 1):
            idx = np.nonzero(el.layer == lp)[0]
            if idx.size == 0:
                continue
            g, gx, gy = G.green_grad(el.cx[i], el.cy[i], el.cx[idx], el.cy[idx], l, lp)
            if lp == l:
                # the self pair keeps only its reaction part
                j = np.nonzero(idx == i)[0]
                rg = [G.reaction_component_grad(c, l, l, el.cx[i], el.cy[i], el.cx[i:i + 1], el.cy[i:i + 1])
                      for c in nonzero_components(l, l, med.L)]
                g[j] = sum(r[0] for r in rg) if rg else 0.0
                gx[j] = sum(r[1] for r in rg) if rg else 0.0
                gy[j] = sum(r[2] for r in rg) if rg else 0.0
            A[i, idx] = (el.nx[i] * gx + el.ny[i] * gy) * el.w[idx]
            if beta is not None:
                A[i, idx] += 1j * beta * g * el.w[idx]
        A[i, i] -= 0.5
        if beta is not None:
            A[i, i] += 1j * beta * self_term(med.k[l], el.w[i])
    return A


def matrix(med, el, green=None):
    return matrix_rows(med, el, range(el.n), green)


def paper_form_matrix(med, el, green=None):
    """The paper's source-first, eta-scaled matrix (eqs. linearSystem,
    matrixelementsexpression, matrixelmemts): entry (i, e) multiplies
    Phi_e = eta_{l_e} phi_e and equals |Gamma_e| G_{l_e l_i}(c_e, c_i) off the
    diagonal, with right side eta_{l_i} g_i."""
    G = LayeredGreen(med) if green is None else green
    Kp = np.zeros((el.n, el.n), dtype=complex)
    for e in range(el.n):
        le = int(el.layer[e])
        for li in range(med.L + 1):
            idx = np.nonzero(el.layer == li)[0]
            if idx.size == 0:
                continue
            # G_{l_e l_i}(c_e, c_i): field at c_e (layer l_e) due to a source at c_i
            vals = G.reaction(le, li, el.cx[e], el.cy[e], el.cx[idx], el.cy[idx])
            if li == le:
                off = idx != e
                vals[off] += free_space(med.k[le], el.cx[e], el.cy[e], el.cx[idx[off]], el.cy[idx[off]])
            Kp[idx, e] = vals * el.w[e]
        Kp[e, e] += self_term(med.k[le], el.w[e])
    # the diagonal carries eta of its own layer through Phi_e = eta phi_e; the
    # self term in eq. matrixelmemts multiplies Phi, so it is unscaled here
    return Kp


def matvec(K, x):
    return K @ x
