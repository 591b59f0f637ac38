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
from tests.parity import check

pytestmark = pytest.mark.gpu


def _straddle():
    polys = [wl.ellipse((0.2, -0.6), 0.9, 0.45, 1.2, 96), wl.circle((1.9, 0.7), 0.35, 60),
             wl.star((-1.6, -2.1), 0.3, 64, 0.4), wl.circle((-0.8, 1.2), 0.3, 48)]
    return wl.Workload("straddle3", np.array([0.0, 1.1]), np.array([2.0, 3.5, 2.5]), np.array([1.0, 2.0, 1.5]),
                       polys, np.array([40.0]))


@pytest.mark.parametrize("top_fft", [-1, 1])
def test_fmm_matvec_straddling_eta(top_fft):
    w = _straddle()
    print(f"case: straddle3 fmm top_fft={top_fft}", flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=0, top_fft=top_fft)
    st = geo.fmm_stats()
    print(st, flush=True)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    K = matrix(med, el)
    x = wl.random_vector(el.n, seed=4, n_rhs=2)
    y = geo.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    check(y, (K @ x.T).T, 1e-6, f"straddle3 fmm top_fft={top_fft}")


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
    check(y[rows], ref, 1e-6, "mini sampled rows", idx=rows)


def test_fmm_vs_dense_full_vector(mini):
    w, geo, med, el = mini
    dense = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_DENSE)
    x = torch.from_numpy(wl.random_vector(el.n, seed=10, n_rhs=1)).cuda()
    yf = geo.matvec(x).cpu().numpy()[0]
    yd = dense.matvec(x).cpu().numpy()[0]
    check(yf, yd, 1e-6, "mini fmm vs dense full vector")


@pytest.mark.parametrize("top_fft", [-1, 1])
def test_fmm_homogeneous_medium(top_fft):
    w = _straddle()
    w = wl.Workload("homog", w.d, np.array([3.0, 3.0, 3.0]), np.ones(3), w.polygons, w.angles_deg)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=0, top_fft=top_fft)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    K = matrix(med, el)
    x = wl.random_vector(el.n, seed=6, n_rhs=1)[0]
    y = geo.matvec(torch.from_numpy(x[None]).cuda()).cpu().numpy()[0]
    check(y, K @ x, 1e-6, f"homogeneous fmm top_fft={top_fft}")


@pytest.mark.parametrize("top_fft", [-1, 1])
def test_fmm_tiny(top_fft):
    lay = lmfmm.Layers([0.0], [2.0, 3.0])
    tri = np.array([[0.0, 0.01], [0.3, -0.02], [0.1, 0.2], [-0.2, 0.1]])
    geo = lmfmm.Geometry(lay, np.array([0, 4]), tri, method=lmfmm.LM_FMM, precond=0, top_fft=top_fft)
    med = Medium([0.0], [2.0, 3.0])
    el = Elements(med, [tri])
    K = matrix(med, el)
    x = wl.random_vector(4, seed=1)[0]
    y = geo.matvec(torch.from_numpy(x[None]).cuda()).cpu().numpy()[0]
    check(y, K @ x, 1e-6, f"tiny fmm top_fft={top_fft}")


@pytest.mark.parametrize("precision", [lmfmm.LM_FP64, lmfmm.LM_MIXED])
def test_level0_convolution_equals_direct_lists(mini, precision):
    """The coarsest level by FFT along x (top_fft=1) against the same
    interactions as explicit M2L list entries (top_fft=-1): same operator up
    to rounding, for one and several right-hand sides, and against the
    oracle's sampled rows."""
    w, _, med, el = mini
    on = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=0, top_fft=1)
    off = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=0, top_fft=-1)
    s_on, s_off = on.fmm_stats(), off.fmm_stats()
    print("lists with / without the level-0 convolution", s_on, s_off, flush=True)
    assert s_on["m2l_free_entries"] + s_on["m2l_reaction_entries"] < \
        s_off["m2l_free_entries"] + s_off["m2l_reaction_entries"]
    dt = torch.complex128 if precision == lmfmm.LM_FP64 else torch.complex64
    bar = 1e-11 if precision == lmfmm.LM_FP64 else 1e-5
    for R in (1, 5):
        x = torch.from_numpy(wl.random_vector(el.n, seed=20 + R, n_rhs=R)).to(dt).cuda()
        a = on.matvec(x, precision=precision).cpu().numpy()
        b = off.matvec(x, precision=precision).cpu().numpy()
        check(a, b, bar, f"precision {precision} R={R}: level-0 convolution vs lists")
    y = torch.empty_like(x)
    st_on = on.stage_times(x, y, reps=2, precision=precision)
    st_off = off.stage_times(x, y, reps=2, precision=precision)
    print("stage ms on", np.round(st_on, 3).tolist(), "off", np.round(st_off, 3).tolist(), flush=True)
    assert st_on[8] > 0  # (off: the events bracket no kernel)
    xr = wl.random_vector(el.n, seed=9, n_rhs=1)[0]
    yr = on.matvec(torch.from_numpy(xr[None]).to(dt).cuda(), precision=precision).cpu().numpy()[0]
    rng = np.random.default_rng(0)
    near = np.nonzero(np.min(np.abs(el.cy[:, None] + med.d[None, :]), axis=1) < 0.05)[0]
    rows = np.unique(np.concatenate([rng.choice(near, 12, replace=False), rng.choice(el.n, 12, replace=False)]))
    xo = xr.astype(np.complex64).astype(np.complex128) if precision == lmfmm.LM_MIXED else xr
    check(yr[rows].astype(np.complex128), matrix_rows(med, el, rows) @ xo,
          1e-6 if precision == lmfmm.LM_FP64 else 1e-4, f"precision {precision}: level-0 convolution sampled rows",
          idx=rows)
    on.close()
    off.close()


def test_level0_convolution_wide_sparse_rows():
    """A wide medium with few scatterers: level-0 rows with empty columns,
    rows holding one box, a scatterer across an eta != 1 interface.  The
    convolution against the lists and both against the full oracle matrix."""
    polys = [wl.circle((-5.6, 0.9), 0.18, 40), wl.star((-3.1, -0.6), 0.2, 48, 0.3), wl.circle((-0.4, -1.25), 0.22, 48),
             wl.ellipse((1.7, 0.05), 0.3, 0.15, 0.4, 48), wl.circle((4.9, -2.3), 0.15, 32), wl.star((5.8, 1.6), 0.16, 40, 1.1)]
    w = wl.Workload("wide6", np.array([0.0, 1.2]), np.array([6.0, 8.0, 5.0]), np.array([1.0, 1.5, 1.0]), polys,
                    np.array([60.0]))
    print("case: wide6 level-0 convolution", flush=True)
    on = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=0, top_fft=1)
    off = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=0, top_fft=-1)
    s_on, s_off = on.fmm_stats(), off.fmm_stats()
    print(s_on, s_off, flush=True)
    assert s_on["m2l_reaction_entries"] < s_off["m2l_reaction_entries"]
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    K = matrix(med, el)
    x = wl.random_vector(el.n, seed=13, n_rhs=3)
    xt = torch.from_numpy(x).cuda()
    y_on = on.matvec(xt).cpu().numpy()
    y_off = off.matvec(xt).cpu().numpy()
    y32 = on.matvec(xt.to(torch.complex64), precision=lmfmm.LM_MIXED).cpu().numpy()
    ref = (K @ x.T).T
    check(y_on, y_off, 1e-11, "wide6 convolution vs lists")
    check(y_on, ref, 1e-6, "wide6 convolution vs oracle")
    check(y_off, ref, 1e-6, "wide6 lists vs oracle")
    x32 = x.astype(np.complex64).astype(np.complex128)
    check(y32.astype(np.complex128), (K @ x32.T).T, 1e-4, "wide6 FP32 form vs oracle")
    on.close()
    off.close()


def test_level0_convolution_over_launch_chunks(mini):
    """More right-hand sides than one launch holds (70 = 64 + 6): the level-0
    convolution's frequency buffers are reused by the second chunk."""
    w, _, med, el = mini
    on = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=0, top_fft=1)
    off = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=0, top_fft=-1)
    x = torch.from_numpy(wl.random_vector(el.n, seed=71, n_rhs=70)).cuda()
    for precision, dt, bar in ((lmfmm.LM_FP64, torch.complex128, 1e-11), (lmfmm.LM_MIXED, torch.complex64, 1e-5)):
        xx = x.to(dt)
        a = on.matvec(xx, precision=precision).cpu().numpy().astype(np.complex128)
        b = off.matvec(xx, precision=precision).cpu().numpy().astype(np.complex128)
        check(a, b, bar, f"precision {precision}, R=70: convolution vs lists")
    on.close()
    off.close()
