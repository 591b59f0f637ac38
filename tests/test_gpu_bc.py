"""Sound-hard (Neumann) and impedance (Robin) scatterers on the dense path
(Sec. 2.1 names both conditions; the single-layer second-kind system
(-1/2 + K' + i beta S) phi = -(d_n + i beta)(u^inc + u^b)) against the
oracle, through the C-ABI:

* outward element normals bit-exact;
* the matrix (through lm_matvec) entry-wise within 1e-10 on a three-layer
  eta != 1 medium with scatterers crossing both interfaces (the reaction
  gradients by direct Sommerfeld quadrature on both sides);
* the right-hand side within 1e-13; the far field of the GMRES solution
  within 1e-6 (FP64 form) and 1e-4 (FP32 form) of the oracle's LU solution;
* the same on the FMM path: matvec within 1e-8 (FP64) / 2e-5 (FP32, one and
  eight right-hand sides), far fields of GMRES solutions against the
  oracle's LU solution;
* a sound-hard disk in a homogeneous medium: the scattered field at
  receivers (lm_field) against the Bessel series, at the oracle's own
  discretisation error.
"""

import numpy as np
import pytest
from scipy.special import h1vp, hankel1, jvp

torch = pytest.importorskip("torch")

from oracle.farfield import far_field, scattered_field
from oracle.incident import boundary_data_bc
from oracle.medium import Medium
from oracle.nystrom import Elements, matrix_bc
from oracle.solve import lu_solve
from paper_2511_12450_amd import lmfmm
from paper_2511_12450_amd import workloads as wl
from tests.parity import check

pytestmark = pytest.mark.gpu


def _case():
    polys = [wl.ellipse((0.2, -0.6), 0.9, 0.45, 1.2, 64), wl.circle((1.9, 0.7), 0.35, 40)[::-1],
             wl.star((-1.6, -2.1), 0.3, 48, 0.4)]  # the circle clockwise
    return wl.Workload("straddle3", np.array([0.0, 1.1]), np.array([2.0, 3.5, 2.5]), np.array([1.0, 2.0, 1.5]),
                       polys, np.array([40.0, 125.0]))


@pytest.mark.parametrize("bc,beta", [(lmfmm.LM_BC_NEUMANN, None), (lmfmm.LM_BC_ROBIN, 1.7)])
def test_neumann_robin_dense_vs_oracle(bc, beta):
    w = _case()
    print(f"case: straddle3 dense bc={bc} beta={beta}", flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_DENSE, bc=bc, robin_beta=beta or 0.0)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    nx, ny = geo.normals()
    assert np.array_equal(nx, el.nx) and np.array_equal(ny, el.ny)
    A = matrix_bc(med, el, beta)
    x = wl.random_vector(el.n, seed=12, n_rhs=2)
    y = geo.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    check(y, (A @ x.T).T, 1e-10, f"bc={bc} matrix")
    th = np.radians(w.angles_deg)
    g = geo.rhs(th).cpu().numpy()
    gref = np.array([boundary_data_bc(med, t, el.cx, el.cy, el.nx, el.ny, beta) for t in th])
    check(g, gref, 1e-13, f"bc={bc} right-hand side")
    obs = lmfmm.far_field_angles()[::11]
    fref = np.array([far_field(med, el, lu_solve(A, gref[r]), obs) for r in range(len(th))])
    for prec, tol, bar in ((lmfmm.LM_FP64, 1e-11, 1e-6), (lmfmm.LM_MIXED, 1e-6, 1e-4)):
        phi, rep, st = geo.solve(th, tol=tol, max_iter=400, restart=400, precond=0, precision=prec)
        assert st == lmfmm.LM_OK, rep
        print(f"bc={bc} precision={prec} iterations {[r[0] for r in rep]}", flush=True)
        check(geo.far_field(phi, obs).cpu().numpy(), fref, bar, f"bc={bc} precision={prec} far field vs oracle LU")


@pytest.mark.parametrize("bc,beta", [(lmfmm.LM_BC_NEUMANN, None), (lmfmm.LM_BC_ROBIN, 1.7)])
def test_neumann_robin_fmm_vs_oracle(bc, beta):
    """The same operators on the FMM (targets evaluate n . grad + i beta of
    the local expansions and of the near-field kernel; reaction near pairs
    by direct quadrature of the gradient), leaf boxes of 8 elements so that
    the expansions carry most pairs."""
    w = _case()
    print(f"case: straddle3 FMM bc={bc} beta={beta}", flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, bc=bc, robin_beta=beta or 0.0, leaf_size=8,
                                       precond=0)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    A = matrix_bc(med, el, beta)
    x1 = wl.random_vector(el.n, seed=31, n_rhs=1)
    y = geo.matvec(torch.from_numpy(x1).cuda()).cpu().numpy()
    check(y, (A @ x1.T).T, 1e-8, f"bc={bc} FMM FP64 matvec (R = 1)")
    y = geo.matvec(torch.from_numpy(x1).to(torch.complex64).cuda(), precision=lmfmm.LM_MIXED).cpu().numpy()
    check(y, (A @ x1.T).T, 2e-5, f"bc={bc} FMM FP32 matvec (R = 1)")
    x8 = wl.random_vector(el.n, seed=32, n_rhs=8)
    y = geo.matvec(torch.from_numpy(x8).to(torch.complex64).cuda(), precision=lmfmm.LM_MIXED).cpu().numpy()
    check(y, (A @ x8.T).T, 2e-5, f"bc={bc} FMM FP32 matvec (R = 8, matrix cores)")
    th = np.radians(w.angles_deg)
    gref = np.array([boundary_data_bc(med, t, el.cx, el.cy, el.nx, el.ny, beta) for t in th])
    obs = lmfmm.far_field_angles()[::11]
    fref = np.array([far_field(med, el, lu_solve(A, gref[r]), obs) for r in range(len(th))])
    for prec, tol, bar in ((lmfmm.LM_FP64, 1e-11, 1e-6), (lmfmm.LM_MIXED, 1e-6, 1e-4)):
        phi, rep, st = geo.solve(th, tol=tol, max_iter=400, restart=400, precond=0, precision=prec)
        assert st == lmfmm.LM_OK, rep
        print(f"FMM bc={bc} precision={prec} iterations {[r[0] for r in rep]}", flush=True)
        check(geo.far_field(phi, obs).cpu().numpy(), fref, bar, f"FMM bc={bc} precision={prec} far field vs oracle LU")


def test_fmm_rejects_preconditioner_for_neumann():
    w = _case()
    with pytest.raises(lmfmm.LmError) as e:
        lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, bc=lmfmm.LM_BC_NEUMANN, precond=1)
    assert e.value.status == -1


def test_sound_hard_disk_field_vs_bessel_series():
    k, a, cy = 2.0, 1.0, 2.0
    w = wl.Workload("disk", np.array([0.0]), np.array([k, k]), np.ones(2), [wl.circle((0.0, cy), a, 256)],
                    np.array([30.0]))
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_DENSE, bc=lmfmm.LM_BC_NEUMANN)
    phi, rep, st = geo.solve(np.radians([30.0]), tol=1e-12, max_iter=400, restart=400, precond=0)
    assert st == lmfmm.LM_OK
    t = np.linspace(0, 2 * np.pi, 16, endpoint=False)
    pts = np.stack([2.5 * np.cos(t), cy + 2.5 * np.sin(t)], axis=1)
    pts = pts[np.abs(pts[:, 1]) > 0.05]
    u = geo.field(phi, pts).cpu().numpy()[0]
    n = np.arange(-60, 61)
    c = -(1j ** n) * jvp(n, k * a) / h1vp(n, k * a)
    r = np.hypot(pts[:, 0], pts[:, 1] - cy)
    ph = np.arctan2(pts[:, 1] - cy, pts[:, 0])
    alpha = -np.radians(30.0)
    exact = np.sum(c[:, None] * hankel1(n[:, None], k * r[None, :]) * np.exp(1j * n[:, None] * (ph[None, :] - alpha)),
                   axis=0) * np.exp(-1j * k * np.sin(np.radians(30.0)) * cy)
    err = np.abs(u - exact).max() / np.abs(exact).max()
    # the oracle's own discretisation error at N = 256 is 4.1e-3 (first order)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    po = lu_solve(matrix_bc(med, el), boundary_data_bc(med, np.radians(30.0), el.cx, el.cy, el.nx, el.ny))
    uo = scattered_field(med, el, po, pts[:, 0], pts[:, 1])
    print(f"sound-hard disk N=256: library error vs Bessel series {err:.3e}", flush=True)
    check(u, uo, 1e-8, "sound-hard disk field vs oracle")
    assert err < 6e-3
