"""Parity of the dense plain path (direct Sommerfeld quadrature + device GMRES)
with the FP64 oracle, called through the C-ABI.

Tolerances: FP64 form 1e-10 on the matvec (the quadratures agree to ~1e-13
per entry), FP32 storage of K 1e-5; solution far field 1e-6 at GMRES tol
1e-10 (the first-kind system amplifies the residual into phi, the far field
is stable)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.farfield import far_field
from oracle.incident import boundary_data
from oracle.medium import Medium
from oracle.nystrom import Elements, matrix
from oracle.solve import lu_solve
from paper_2511_12450_amd import lmfmm
from paper_2511_12450_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def plain_small():
    print("case: plain_small N=256 (dense)", flush=True)
    w = wl.plain_small()
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_DENSE)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    K = matrix(med, el)
    return w, geo, med, el, K


def _straddle_case():
    """Three layers with eta != 1 and a scatterer crossing both interfaces."""
    polys = [wl.ellipse((0.2, -0.6), 0.9, 0.45, 1.2, 72), wl.circle((1.9, 0.7), 0.35, 40),
             wl.star((-1.6, -2.1), 0.3, 48, 0.4)]
    return wl.Workload("straddle3", np.array([0.0, 1.1]), np.array([2.0, 3.5, 2.5]), np.array([1.0, 2.0, 1.5]),
                       polys, np.array([40.0, 95.0]))


def test_elements_match(plain_small):
    w, geo, med, el, K = plain_small
    cx, cy, ww, lay = geo.elements()
    assert np.array_equal(cx, el.cx) and np.array_equal(cy, el.cy)
    assert np.allclose(ww, el.w, rtol=1e-15, atol=0)
    assert np.array_equal(lay, el.layer)


def test_dense_matvec_fp64_and_fp32(plain_small):
    w, geo, med, el, K = plain_small
    x = wl.random_vector(el.n, seed=11, n_rhs=3)
    ref = (K @ x.T).T
    xt = torch.from_numpy(x).cuda()
    y = geo.matvec(xt).cpu().numpy()
    assert _rel(y, ref) < 1e-10
    y32 = geo.matvec(xt.to(torch.complex64), precision=lmfmm.LM_MIXED).cpu().numpy()
    assert _rel(y32, ref) < 1e-5


def test_rhs(plain_small):
    w, geo, med, el, K = plain_small
    th = np.radians([30.0, 77.0, 150.0])
    g = geo.rhs(th).cpu().numpy()
    for r, t in enumerate(th):
        assert _rel(g[r], boundary_data(med, t, el.cx, el.cy)) < 1e-13


def test_gmres_solution_and_far_field(plain_small):
    w, geo, med, el, K = plain_small
    th = np.radians(w.angles_deg)
    phi, rep, st = geo.solve(th, tol=1e-10, max_iter=300, restart=300)
    assert st == lmfmm.LM_OK and rep[0][1] < 1e-10
    g = boundary_data(med, th[0], el.cx, el.cy)
    ref = lu_solve(K, g)
    ph = phi.cpu().numpy()[0]
    assert _rel(ph, ref) < 1e-7
    obs = lmfmm.far_field_angles()[::17]
    ff = geo.far_field(phi, obs).cpu().numpy()[0]
    ff_ref = far_field(med, el, ref, obs)
    assert _rel(ff, ff_ref) < 1e-6


def test_far_field_of_given_density(plain_small):
    w, geo, med, el, K = plain_small
    x = wl.random_vector(el.n, seed=5, n_rhs=2)
    obs = lmfmm.far_field_angles()[::23]
    ff = geo.far_field(torch.from_numpy(x).cuda(), obs).cpu().numpy()
    for r in range(2):
        assert _rel(ff[r], far_field(med, el, x[r], obs)) < 1e-12


def test_gmres_restart_and_multi_rhs(plain_small):
    w, geo, med, el, K = plain_small
    th = np.radians([30.0, 60.0, 120.0])
    phi, rep, st = geo.solve(th, tol=1e-8, max_iter=400, restart=15)
    assert st == lmfmm.LM_OK
    ph = phi.cpu().numpy()
    for r, t in enumerate(th):
        ref = lu_solve(K, boundary_data(med, t, el.cx, el.cy))
        assert rep[r][1] <= 1e-8
        assert _rel(ph[r], ref) < 1e-4


def test_dense_three_layers_straddling():
    w = _straddle_case()
    print("case: straddle3 dense", flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_DENSE)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    K = matrix(med, el)
    x = wl.random_vector(el.n, seed=2, n_rhs=1)
    y = geo.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert _rel(y[0], K @ x[0]) < 1e-10
    g = geo.rhs(np.radians(w.angles_deg)).cpu().numpy()
    for r, t in enumerate(np.radians(w.angles_deg)):
        assert _rel(g[r], boundary_data(med, t, el.cx, el.cy)) < 1e-13


def test_tiny_and_invalid_inputs():
    lay = lmfmm.Layers([0.0], [2.0, 3.0])
    tri = np.array([[0.0, 1.0], [1.0, 1.0], [0.5, 2.0]])
    geo = lmfmm.Geometry(lay, np.array([0, 3]), tri, method=lmfmm.LM_DENSE)
    assert geo.n == 3
    x = torch.ones((1, 3), dtype=torch.complex128, device="cuda")
    y = geo.matvec(x)
    assert torch.isfinite(y).all()
    with pytest.raises(lmfmm.LmError):
        geo.rhs(np.array([-0.3]))  # wave must come from above
    with pytest.raises(lmfmm.LmError):
        geo.far_field(x, np.array([0.0]))  # horizontal direction
