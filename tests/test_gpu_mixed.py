"""The mixed-precision (FP32 translation and near-field arithmetic) form and
multi-right-hand-side launches of the layered FMM matvec, through the C-ABI.

Bars: FP32 form within 1e-4 (relative 2-norm) of the FP64 oracle for the
matvec and for the far field of a solve; a launch with R right-hand sides
equal to R single launches (FP64: 1e-12, i.e. identical arithmetic up to
summation order), including R above the per-launch chunk of 64.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.farfield import far_field
from oracle.incident import boundary_data
from oracle.medium import Medium
from oracle.nystrom import Elements, matrix, matrix_rows
from oracle.solve import lu_solve
from paper_2511_12450_amd import lmfmm
from paper_2511_12450_amd import workloads as wl
from tests.parity import check

pytestmark = pytest.mark.gpu


def _straddle():
    polys = [wl.ellipse((0.2, -0.6), 0.9, 0.45, 1.2, 96), wl.circle((1.9, 0.7), 0.35, 60),
             wl.star((-1.6, -2.1), 0.3, 64, 0.4), wl.circle((-0.8, 1.2), 0.3, 48)]
    return wl.Workload("straddle3", np.array([0.0, 1.1]), np.array([2.0, 3.5, 2.5]), np.array([1.0, 2.0, 1.5]),
                       polys, np.array([40.0, 120.0]))


@pytest.fixture(scope="module")
def straddle():
    w = _straddle()
    print("case: straddle3", flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=1)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    return w, geo, med, el, matrix(med, el)


@pytest.fixture(scope="module")
def mini():
    w = wl.three_layer_mini(seed=3)
    print("case: three_layer_mini N=", w.n_elements, flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=0)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    return w, geo, med, el


def test_fp32_matvec_vs_oracle(straddle):
    w, geo, med, el, K = straddle
    x = wl.random_vector(el.n, seed=4, n_rhs=3)
    y = geo.matvec(torch.from_numpy(x).to(torch.complex64).cuda(), precision=lmfmm.LM_MIXED).cpu().numpy()
    ref = (K @ x.astype(np.complex64).astype(np.complex128).T).T
    check(y.astype(np.complex128), ref, 1e-4, "straddle3 FP32 matvec")


def test_fp32_matvec_sampled_rows(mini):
    w, geo, med, el = mini
    x = wl.random_vector(el.n, seed=9, n_rhs=1)[0].astype(np.complex64)
    y = geo.matvec(torch.from_numpy(x[None]).cuda(), precision=lmfmm.LM_MIXED).cpu().numpy()[0]
    rng = np.random.default_rng(1)
    near = np.nonzero(np.min(np.abs(el.cy[:, None] + med.d[None, :]), axis=1) < 0.05)[0]
    rows = np.unique(np.concatenate([rng.choice(near, 10, replace=False), rng.choice(el.n, 10, replace=False)]))
    ref = matrix_rows(med, el, rows) @ x.astype(np.complex128)
    check(y[rows].astype(np.complex128), ref, 1e-4, "mini FP32 sampled rows", idx=rows)


@pytest.mark.parametrize("n_rhs", [5, 70])
def test_multi_rhs_equals_single(mini, n_rhs):
    w, geo, med, el = mini
    x = torch.from_numpy(wl.random_vector(el.n, seed=20 + n_rhs, n_rhs=n_rhs)).cuda()
    yb = geo.matvec(x).cpu().numpy()
    picks = [0, n_rhs // 2, n_rhs - 1]
    ys = np.array([geo.matvec(x[r:r + 1].contiguous()).cpu().numpy()[0] for r in picks])
    check(yb[picks], ys, 1e-12, f"R={n_rhs}: batched vs single")
    x32 = x.to(torch.complex64)
    y32 = geo.matvec(x32, precision=lmfmm.LM_MIXED).cpu().numpy()
    check(y32[picks].astype(np.complex128), yb[picks], 1e-4, f"R={n_rhs}: FP32 vs FP64")


@pytest.mark.parametrize("n_rhs", [2, 7, 16])
def test_fp32_few_rhs_matches_many(mini, n_rhs):
    """FP32 launches of few right-hand sides (up to 8: operator-major M2L;
    16: target-major) against the same vectors inside a 64-wide launch and
    against FP64."""
    w, geo, med, el = mini
    x = torch.from_numpy(wl.random_vector(el.n, seed=40, n_rhs=64)).cuda()
    y64 = geo.matvec(x).cpu().numpy()
    x32 = x.to(torch.complex64)
    wide = geo.matvec(x32, precision=lmfmm.LM_MIXED).cpu().numpy()
    few = geo.matvec(x32[:n_rhs].contiguous(), precision=lmfmm.LM_MIXED).cpu().numpy()
    check(few.astype(np.complex128), wide[:n_rhs].astype(np.complex128), 1e-5, f"R={n_rhs}: FP32 few vs wide launch")
    check(few.astype(np.complex128), y64[:n_rhs], 1e-4, f"R={n_rhs}: FP32 few vs FP64")


def test_fp32_solve_far_field_vs_oracle(straddle):
    w, geo, med, el, K = straddle
    th = np.radians(w.angles_deg)
    phi, rep, st = geo.solve(th, tol=1e-6, max_iter=600, restart=600, precond=1, precision=lmfmm.LM_MIXED)
    print("mixed solve reports", rep, "status", st, flush=True)
    assert st == lmfmm.LM_OK
    obs = lmfmm.far_field_angles()[::13]
    ff = geo.far_field(phi, obs).cpu().numpy()
    ref = np.array([far_field(med, el, lu_solve(K, boundary_data(med, t, el.cx, el.cy)), obs) for t in th])
    check(ff, ref, 1e-4, "straddle3 mixed solve far field")


def test_fp32_dense_solve_far_field_vs_oracle():
    w = wl.plain_small()
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_DENSE)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    th = np.radians(w.angles_deg)
    phi, rep, st = geo.solve(th, tol=1e-6, max_iter=300, restart=300, precond=0, precision=lmfmm.LM_MIXED)
    assert st == lmfmm.LM_OK
    obs = lmfmm.far_field_angles()[::7]
    ff = geo.far_field(phi, obs).cpu().numpy()[0]
    ref = lu_solve(matrix(med, el), boundary_data(med, th[0], el.cx, el.cy))
    check(ff, far_field(med, el, ref, obs), 1e-4, "plain_small mixed dense solve far field")
