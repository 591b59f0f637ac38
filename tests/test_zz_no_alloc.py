"""lm_matvec_noalloc (workspace in the library's static device array, no
device allocation) against lm_matvec, through the C-ABI.

Two calls in a row on each case, the second with a smaller input (fewer
right-hand sides, then a smaller geometry after a larger one), so a result
that depended on what the previous call left in the shared array would show.
Both entry points run the same kernels on the same chunks here, so they
agree to the rounding of the form (checked at 1e-12 relative for FP64 and
1e-6 for the FP32 form; the bars of the parity against the oracle are 1e-6
and 1e-4).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2511_12450_amd import lmfmm
from paper_2511_12450_amd import workloads as wl
from tests.parity import check

pytestmark = pytest.mark.gpu


def _small():
    polys = [wl.ellipse((0.2, -0.6), 0.9, 0.45, 1.2, 96), wl.circle((1.9, 0.7), 0.35, 60),
             wl.star((-1.6, -2.1), 0.3, 64, 0.4)]
    return wl.Workload("small3", np.array([0.0, 1.1]), np.array([2.0, 3.5, 2.5]), np.array([1.0, 2.0, 1.5]),
                       polys, np.array([50.0]))


def _run(geo, prec, R, seed):
    dt = torch.complex128 if prec == lmfmm.LM_FP64 else torch.complex64
    x = torch.from_numpy(wl.random_vector(geo.n, seed=seed, n_rhs=R)).to(dt).cuda()
    ref = geo.matvec(x, precision=prec)
    y = torch.full_like(x, float("nan"))
    geo.matvec_noalloc(x, y, precision=prec)
    torch.cuda.synchronize()
    same = bool(torch.equal(y, ref))
    print(f"noalloc prec={prec} N={geo.n} R={R}: bit-identical to lm_matvec: {same}", flush=True)
    bar = 1e-12 if prec == lmfmm.LM_FP64 else 1e-6
    check(y.cpu().numpy(), ref.cpu().numpy(), bar, f"noalloc vs lm_matvec prec={prec} R={R}")


def test_noalloc_matvec_matches_matvec():
    big = wl.three_layer_mini(seed=3)
    print(f"case: noalloc three_layer_mini N={big.n_elements}", flush=True)
    g1 = lmfmm.Geometry.from_workload(big, method=lmfmm.LM_FMM, precond=0)
    g2 = lmfmm.Geometry.from_workload(_small(), method=lmfmm.LM_FMM, precond=0)
    for prec, Rs in ((lmfmm.LM_FP64, (3, 1)), (lmfmm.LM_MIXED, (16, 2))):
        for i, R in enumerate(Rs):
            _run(g1, prec, R, seed=30 + i)
        _run(g2, prec, 1, seed=40)  # smaller geometry after the larger one


def test_noalloc_dense_geometry():
    w = wl.plain_small()
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_DENSE)
    for R in (4, 1):
        _run(geo, lmfmm.LM_FP64, R, seed=50 + R)
