"""End-to-end parity of the fast path (FMM + preconditioned GMRES + far field)
with the FP64 oracle, and properties of the domain-decomposition
preconditioner, through the C-ABI.

Bars: far field of the solution 1e-6 (FP64 form, tol 1e-10); the
preconditioner is exact when one leaf holds every element of a homogeneous
medium (GMRES converges in one iteration); on N = 4000 it reduces the
iteration count and does not change the solution beyond the tolerance."""

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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _straddle():
    polys = [wl.ellipse((0.2, -0.6), 0.9, 0.45, 1.2, 96), wl.circle((1.9, 0.7), 0.35, 60),
             wl.star((-1.6, -2.1), 0.3, 64, 0.4)]
    return wl.Workload("straddle3", np.array([0.0, 1.1]), np.array([2.0, 3.5, 2.5]), np.array([1.0, 2.0, 1.5]),
                       polys, np.array([40.0, 120.0]))


@pytest.mark.parametrize("name", ["plain_small", "straddle3"])
def test_fmm_solve_far_field_matches_oracle(name):
    w = wl.plain_small() if name == "plain_small" else _straddle()
    print("case:", name, flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=1)
    th = np.radians(w.angles_deg)
    phi, rep, st = geo.solve(th, tol=1e-10, max_iter=600, restart=600, precond=1)
    assert st == lmfmm.LM_OK
    obs = lmfmm.far_field_angles()[::13]
    ff = geo.far_field(phi, obs).cpu().numpy()
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    K = matrix(med, el)
    print(name, "iterations", [r[0] for r in rep], flush=True)
    ref = np.array([far_field(med, el, lu_solve(K, boundary_data(med, t, el.cx, el.cy)), obs) for t in th])
    check(ff, ref, 1e-6, f"{name} FP64 solve far field")


def test_preconditioner_exact_on_one_leaf():
    lay = lmfmm.Layers([0.0], [2.5, 2.5])
    P = wl.circle((0.1, 0.6), 0.4, 40)
    geo = lmfmm.Geometry(lay, np.array([0, 40]), P, method=lmfmm.LM_FMM, leaf_size=1000, precond=1)
    assert geo.fmm_stats()["free_leaf_level"] == 0
    phi, rep, st = geo.solve(np.radians([60.0]), tol=1e-10, max_iter=50, restart=50, precond=1)
    assert st == lmfmm.LM_OK
    assert rep[0][0] == 1, rep
    assert rep[0][1] < 1e-10


def test_preconditioner_reduces_iterations_same_solution():
    w = wl.three_layer_mini(seed=3)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=1)
    th = np.radians([30.0])
    p1, r1, s1 = geo.solve(th, tol=1e-8, max_iter=800, restart=800, precond=1)
    p0, r0, s0 = geo.solve(th, tol=1e-8, max_iter=800, restart=800, precond=0)
    print("iterations with / without preconditioner:", r1[0][0], r0[0][0], flush=True)
    assert s1 == lmfmm.LM_OK and s0 == lmfmm.LM_OK
    assert r1[0][0] < 0.8 * r0[0][0]
    obs = lmfmm.far_field_angles()[::7]
    f1 = geo.far_field(p1, obs).cpu().numpy()[0]
    f0 = geo.far_field(p0, obs).cpu().numpy()[0]
    check(f1, f0, 1e-6, "far field with / without preconditioner")


def test_restarted_gmres_same_solution():
    w = wl.three_layer_mini(seed=3)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=1)
    th = np.radians([75.0])
    pa, ra, sa = geo.solve(th, tol=1e-8, max_iter=800, restart=800)
    pb, rb, sb = geo.solve(th, tol=1e-8, max_iter=800, restart=20)
    assert sa == lmfmm.LM_OK and sb == lmfmm.LM_OK
    obs = lmfmm.far_field_angles()[::11]
    check(geo.far_field(pb, obs).cpu().numpy(), geo.far_field(pa, obs).cpu().numpy(), 1e-6, "restart 20 vs 800")


def test_not_converged_status():
    w = wl.three_layer_mini(seed=3)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=1)
    phi, rep, st = geo.solve(np.radians([30.0]), tol=1e-12, max_iter=3, restart=3)
    assert st == lmfmm.LM_NOT_CONVERGED
    assert rep[0][0] == 3 and rep[0][1] > 1e-12
    assert torch.isfinite(phi).all()


def test_coarser_subdomains_fewer_iterations_same_solution():
    w = wl.three_layer_mini(seed=3)
    g1 = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=1)
    g2 = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=2)
    th = np.radians([45.0])
    p1, r1, s1 = g1.solve(th, tol=1e-8, max_iter=800, restart=800)
    p2, r2, s2 = g2.solve(th, tol=1e-8, max_iter=800, restart=800)
    print("iterations with leaf / coarser subdomains:", r1[0][0], r2[0][0], flush=True)
    assert s1 == lmfmm.LM_OK and s2 == lmfmm.LM_OK
    assert r2[0][0] < r1[0][0]
    obs = lmfmm.far_field_angles()[::7]
    check(g2.far_field(p2, obs).cpu().numpy(), g1.far_field(p1, obs).cpu().numpy(), 1e-6, "coarser subdomains")
    # the default picks the coarsest level that fits: no more iterations
    g3 = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM)
    p3, r3, s3 = g3.solve(th, tol=1e-8, max_iter=800, restart=800)
    print("iterations with the default subdomains:", r3[0][0], flush=True)
    assert s3 == lmfmm.LM_OK and r3[0][0] <= r2[0][0]
    check(g3.far_field(p3, obs).cpu().numpy(), g1.far_field(p1, obs).cpu().numpy(), 1e-6, "default subdomains")


def test_fp32_preconditioner_is_one_fixed_complex_linear_operator():
    """The FP32 form applies the preconditioner rows in binary16 on matrix
    cores; GMRES with right preconditioning needs the same complex-linear
    operator at every application, which is what this checks (it need only
    be close to the FP64 operator)."""
    w = wl.three_layer_mini(seed=3)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM)
    x = torch.from_numpy(wl.random_vector(geo.n, seed=11, n_rhs=3)).cuda()
    y64 = geo.precond_apply(x, precision=lmfmm.LM_FP64).cpu().numpy()
    y32 = geo.precond_apply(x, precision=lmfmm.LM_MIXED).cpu().numpy()
    for r in range(3):
        d = _rel(y32[r], y64[r])
        print(f"rhs {r}: binary16 vs FP64 operator rel diff {d:.2e}", flush=True)
        assert d < 2e-3
        one = geo.precond_apply(x[r:r + 1].contiguous(), precision=lmfmm.LM_MIXED).cpu().numpy()[0]
        assert np.array_equal(one, y32[r])  # alone = in a batch, bit for bit
    a, b = 0.3 - 1.7j, -2.1 + 0.4j
    z = (a * x[0] + b * x[1])[None].contiguous()
    yz = geo.precond_apply(z, precision=lmfmm.LM_MIXED).cpu().numpy()[0]
    lin = _rel(yz, a * y32[0] + b * y32[1])
    print(f"complex linearity rel diff {lin:.2e}", flush=True)
    assert lin < 1e-5
