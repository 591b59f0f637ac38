"""Scattered field at receivers off the boundary (lm_field, lm_point_field;
eq. integralrep) against the oracle, through the C-ABI.

A three-layer eta != 1 medium with scatterers crossing both interfaces;
receivers on a ring around them, inside every layer, between scatterers and
at 0.01 and 0.001 from each interface (the spectral reaction sum extends its
nodes with the inverse of that distance).  Bar: 1e-9 relative to the largest
value per right-hand side, entry by entry (both sides FP64; the oracle's
quadrature is converged to about 1e-13 per Green's function value).

Far field (lm_far_field) of given densities on a geometry large enough that
the launch splits its elements over several workgroup chunks and adds their
partial sums: entry by entry against the oracle's closed form (eq.
integralrep at large distance), top and bottom directions.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.farfield import far_field, scattered_field
from oracle.green import LayeredGreen
from oracle.medium import Medium
from oracle.nystrom import Elements
from paper_2511_12450_amd import lmfmm
from paper_2511_12450_amd import workloads as wl
from tests.parity import check

pytestmark = pytest.mark.gpu


def _case():
    polys = [wl.ellipse((0.2, -0.6), 0.9, 0.45, 1.2, 72), wl.circle((1.9, 0.7), 0.35, 40),
             wl.star((-1.6, -2.1), 0.3, 48, 0.4)]
    return wl.Workload("straddle3", np.array([0.0, 1.1]), np.array([2.0, 3.5, 2.5]), np.array([1.0, 2.0, 1.5]),
                       polys, np.array([40.0]))


def _receivers(med):
    t = np.linspace(0.0, 2.0 * np.pi, 20, endpoint=False)
    ring = np.stack([0.1 + 3.6 * np.cos(t), -0.7 + 3.6 * np.sin(t)], axis=1)
    ring = ring[np.min(np.abs(ring[:, 1:2] + med.d[None, :]), axis=1) > 0.05]
    extra = [(-0.5, 1.3), (0.9, 0.01), (0.9, -0.01), (-2.7, 0.001), (-2.7, -0.001), (1.2, -1.1 + 0.01),
             (1.2, -1.1 - 0.01), (-0.3, -1.1 + 0.001), (3.0, -1.1 - 0.001), (0.8, -2.9)]
    return np.concatenate([ring, np.array(extra)], axis=0)


def test_field_at_receivers_vs_oracle():
    w = _case()
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    pts = _receivers(med)
    print(f"case: straddle3 field, N={el.n}, {len(pts)} receivers", flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=0)
    phi = wl.random_vector(el.n, seed=8, n_rhs=2)
    u = geo.field(torch.from_numpy(phi).cuda(), pts).cpu().numpy()
    ref = np.array([scattered_field(med, el, phi[r], pts[:, 0], pts[:, 1]) for r in range(2)])
    check(u, ref, 1e-9, "field at receivers vs oracle")


def test_point_field_vs_oracle():
    w = _case()
    med = Medium(w.d, w.k, w.eta)
    pts = _receivers(med)
    srcs = np.array([[0.3, 0.6], [-1.0, -0.5], [2.2, -2.4], [0.5, -1.1 + 0.02]])  # every layer, one by an interface
    lay = lmfmm.Layers(w.d, w.k, w.eta)
    u = lmfmm.point_field(lay, srcs, pts).cpu().numpy()
    G = LayeredGreen(med)
    ref = np.zeros_like(u)
    for r, s in enumerate(srcs):
        ls = int(med.layer_of(np.array([s[1]]))[0])
        for p, q in enumerate(pts):
            ref[r, p] = G.green(q[0], q[1], [s[0]], [s[1]], lp=ls)[0]
    check(u, ref, 1e-9, "point-source field at receivers vs oracle")


def test_far_field_chunked_vs_oracle():
    w = wl.three_layer_mini(seed=6, n_scat=80)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    assert el.n >= 3 * 4096  # three or more element chunks in the launch below
    obs = np.concatenate([np.radians(np.linspace(5.0, 175.0, 24)), np.radians(np.linspace(185.0, 355.0, 16))])
    print(f"case: chunked far field, N={el.n}, {obs.size} angles", flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=0)
    phi = wl.random_vector(el.n, seed=9, n_rhs=3)
    ff = geo.far_field(torch.from_numpy(phi).cuda(), obs).cpu().numpy()
    ref = np.array([far_field(med, el, phi[r], obs) for r in range(3)])
    check(ff, ref, 1e-11, "chunked far field vs oracle")
