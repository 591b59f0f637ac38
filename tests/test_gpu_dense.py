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
from tests.parity import check

pytestmark = pytest.mark.gpu


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
    check(y, ref, 1e-10, "dense matvec FP64")
    y32 = geo.matvec(xt.to(torch.complex64), precision=lmfmm.LM_MIXED).cpu().numpy()
    check(y32, ref, 1e-5, "dense matvec FP32 storage")


def test_rhs(plain_small):
    w, geo, med, el, K = plain_small
    th = np.radians([30.0, 77.0, 150.0])
    g = geo.rhs(th).cpu().numpy()
    check(g, np.array([boundary_data(med, t, el.cx, el.cy) for t in th]), 1e-13, "rhs two layers")


def test_gmres_solution_and_far_field(plain_small):
    w, geo, med, el, K = plain_small
    th = np.radians(w.angles_deg)
    phi, rep, st = geo.solve(th, tol=1e-10, max_iter=300, restart=300)
    assert st == lmfmm.LM_OK and rep[0][1] < 1e-10
    g = boundary_data(med, th[0], el.cx, el.cy)
    ref = lu_solve(K, g)
    ph = phi.cpu().numpy()[0]
    check(ph, ref, 1e-7, "dense solve phi")
    obs = lmfmm.far_field_angles()[::17]
    ff = geo.far_field(phi, obs).cpu().numpy()[0]
    ff_ref = far_field(med, el, ref, obs)
    check(ff, ff_ref, 1e-6, "dense solve far field")


def test_far_field_of_given_density(plain_small):
    w, geo, med, el, K = plain_small
    x = wl.random_vector(el.n, seed=5, n_rhs=2)
    obs = lmfmm.far_field_angles()[::23]
    ff = geo.far_field(torch.from_numpy(x).cuda(), obs).cpu().numpy()
    check(ff, np.array([far_field(med, el, x[r], obs) for r in range(2)]), 1e-12, "far field of given density")


def test_gmres_restart_and_multi_rhs(plain_small):
    w, geo, med, el, K = plain_small
    th = np.radians([30.0, 60.0, 120.0])
    phi, rep, st = geo.solve(th, tol=1e-8, max_iter=400, restart=15)
    assert st == lmfmm.LM_OK
    ph = phi.cpu().numpy()
    refs = []
    for r, t in enumerate(th):
        refs.append(lu_solve(K, boundary_data(med, t, el.cx, el.cy)))
        assert rep[r][1] <= 1e-8
    check(ph, np.array(refs), 1e-4, "restarted multi-rhs phi")


def test_dense_three_layers_straddling():
    w = _straddle_case()
    print("case: straddle3 dense", flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_DENSE)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    K = matrix(med, el)
    x = wl.random_vector(el.n, seed=2, n_rhs=1)
    y = geo.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    check(y, (K @ x.T).T, 1e-10, "dense straddle3 matvec")
    g = geo.rhs(np.radians(w.angles_deg)).cpu().numpy()
    check(g, np.array([boundary_data(med, t, el.cx, el.cy) for t in np.radians(w.angles_deg)]), 1e-13,
          "rhs straddle3 (eta != 1, every layer)")


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


def _tie_polygon():
    """A zigzag across the interface y = -1 closed below it: consecutive
    nodes at -1 + 0.25 + t_j and -1 - 0.25 + t_{j+1}, so chord midpoints sit
    at -1 + (t_j + t_{j+1}) / 2: exactly on the interface (t = 0), within
    1e-13 above and below (inside the 1e-12 tie band: upper layer), and 2e-12
    below / above (outside it)."""
    offs = [0.0, 0.0, 2e-13, 0.0, -2e-13, 0.0, 4e-12, 0.0, -4e-12, 0.0, 0.0, 0.0]
    top = []
    for j, t in enumerate(offs):
        top.append((0.2 * j, -1.0 + (0.25 if j % 2 == 0 else -0.25) + t))
    x_end = 0.2 * (len(offs) - 1)
    bottom = [(x_end, -1.8), (0.5 * x_end, -2.0), (0.0, -1.8)]
    P = np.array(top[::-1] + bottom[::-1])  # closed, non-self-intersecting
    return P


@pytest.mark.parametrize("method", [lmfmm.LM_DENSE, lmfmm.LM_FMM])
def test_midpoints_on_and_next_to_an_interface(method):
    """Element layers where the midpoint lies exactly on the interface or
    within 1e-13 / 2e-12 of it: bit-exact with the oracle's rule (ties to the
    upper layer); the matvec there against the oracle entry by entry."""
    P = _tie_polygon()
    polys = [P, wl.circle((0.7, 0.6), 0.3, 24)]
    w = wl.Workload("tie", np.array([1.0]), np.array([2.0, 3.0]), np.ones(2), polys, np.array([60.0]))
    print(f"case: interface ties method={method}", flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=method, precond=0)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    cx, cy, ww, lay = geo.elements()
    assert np.array_equal(cx, el.cx) and np.array_equal(cy, el.cy)
    assert np.array_equal(lay, el.layer)
    dy = cy + 1.0
    on = np.abs(dy) <= 1e-12
    assert on.sum() >= 6 and np.any(dy == 0.0) and np.any((dy > 0) & on) and np.any((dy < 0) & on)
    assert np.all(lay[on] == 0)
    assert np.any((dy < -1e-12) & (dy > -1e-11) & (lay == 1)) and np.any((dy > 1e-12) & (dy < 1e-11) & (lay == 0))
    K = matrix(med, el)
    x = wl.random_vector(el.n, seed=17, n_rhs=2)
    y = geo.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    check(y, (K @ x.T).T, 1e-10 if method == lmfmm.LM_DENSE else 1e-6, f"interface ties matvec method={method}")
