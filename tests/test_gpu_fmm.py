"""Parity of the layered FMM matvec with the FP64 oracle (through the C-ABI).

Bar: relative 2-norm error <= 1e-6 for the FP64 form (the stated parity for
matvec and far field), on
* a 3-layer eta != 1 medium with scatterers crossing both interfaces (full
  oracle matrix),
* the three-layer medium of the 64k-element workload at 25 scatterers
  (N = 4000; oracle rows sampled, plus the GPU dense path on the full vector),
* a homogeneous medium (reaction part identically zero) and a tiny input.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.medium import Medium
from oracle.nystrom import Elements, matrix, matrix_rows
from paper_2511_12450_amd import lmfmm
from paper_2511_12450_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _straddle():
    polys = [wl.ellipse((0.2, -0.6), 0.9, 0.45, 1.2, 96), wl.circle((1.9, 0.7), 0.35, 60),
             wl.star((-1.6, -2.1), 0.3, 64, 0.4), wl.circle((-0.8, 1.2), 0.3, 48)]
    return wl.Workload("straddle3", np.array([0.0, 1.1]), np.array([2.0, 3.5, 2.5]), np.array([1.0, 2.0, 1.5]),
                       polys, np.array([40.0]))


def test_fmm_matvec_straddling_eta():
    w = _straddle()
    print("case: straddle3 fmm", flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=0)
    st = geo.fmm_stats()
    print(st, flush=True)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    K = matrix(med, el)
    x = wl.random_vector(el.n, seed=4, n_rhs=2)
    y = geo.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    for r in range(2):
        err = _rel(y[r], K @ x[r])
        print("straddle3 rel err", err, flush=True)
        assert err < 1e-6


@pytest.fixture(scope="module")
def mini():
    w = wl.three_layer_mini(seed=3)
    print("case: three_layer_mini fmm N=", w.n_elements, flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=0)
    print(geo.fmm_stats(), flush=True)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    return w, geo, med, el


def test_fmm_matvec_sampled_rows(mini):
    w, geo, med, el = mini
    x = wl.random_vector(el.n, seed=9, n_rhs=1)[0]
    y = geo.matvec(torch.from_numpy(x[None]).cuda()).cpu().numpy()[0]
    rng = np.random.default_rng(0)
    # half the rows among elements near an interface, half anywhere
    near = np.nonzero(np.min(np.abs(el.cy[:, None] + med.d[None, :]), axis=1) < 0.05)[0]
    rows = np.unique(np.concatenate([rng.choice(near, 12, replace=False), rng.choice(el.n, 12, replace=False)]))
    ref = matrix_rows(med, el, rows) @ x
    err = _rel(y[rows], ref)
    print("mini sampled-row rel err", err, flush=True)
    assert err < 1e-6


def test_fmm_vs_dense_full_vector(mini):
    w, geo, med, el = mini
    dense = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_DENSE)
    x = torch.from_numpy(wl.random_vector(el.n, seed=10, n_rhs=1)).cuda()
    yf = geo.matvec(x).cpu().numpy()[0]
    yd = dense.matvec(x).cpu().numpy()[0]
    err = _rel(yf, yd)
    print("mini fmm vs dense rel err", err, flush=True)
    assert err < 1e-6


def test_fmm_homogeneous_medium():
    w = _straddle()
    w = wl.Workload("homog", w.d, np.array([3.0, 3.0, 3.0]), np.ones(3), w.polygons, w.angles_deg)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=0)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    K = matrix(med, el)
    x = wl.random_vector(el.n, seed=6, n_rhs=1)[0]
    y = geo.matvec(torch.from_numpy(x[None]).cuda()).cpu().numpy()[0]
    assert _rel(y, K @ x) < 1e-6


def test_fmm_tiny():
    lay = lmfmm.Layers([0.0], [2.0, 3.0])
    tri = np.array([[0.0, 0.01], [0.3, -0.02], [0.1, 0.2], [-0.2, 0.1]])
    geo = lmfmm.Geometry(lay, np.array([0, 4]), tri, method=lmfmm.LM_FMM, precond=0)
    med = Medium([0.0], [2.0, 3.0])
    el = Elements(med, [tri])
    K = matrix(med, el)
    x = wl.random_vector(4, seed=1)[0]
    y = geo.matvec(torch.from_numpy(x[None]).cuda()).cpu().numpy()[0]
    assert _rel(y, K @ x) < 1e-6
