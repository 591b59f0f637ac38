"""Full-size parity of the layered FMM matvec with the oracle, on sampled rows.

The oracle's rows of the Nystrom matrix (Sec. 3.3) times seeded vectors are
stored under tests/golden/ (written by make_fullsize_rows.py, oracle only).
Here the library computes the whole product at full size, in the launch
shapes a solve uses, and the sampled rows are compared:

* three-layer medium, 400 scatterers, N = 64,000, p = 20: 64 right-hand
  sides in one launch (the fused multi-angle launch of the served solve) in
  the FP32 form, and in the FP64 form;
* five-layer medium, 4,000 scatterers, N = 1,000,000, p = 24: 8
  right-hand sides (its 8 incident angles) in both forms, on eight rows,
  four of them within 0.05 of an interface (one oracle row takes 20-30
  minutes there).

Bars, per right-hand side over the sampled rows, entry by entry (relative to
the largest entry) and in the 2-norm: 1e-6 (FP64 form) and 1e-4 (FP32
form).
"""

import os
import re

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2511_12450_amd import lmfmm
from paper_2511_12450_amd import workloads as wl
from tests.parity import check

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    path = os.path.join(GOLDEN, f"fullsize_rows_{name}.txt")
    with open(path) as f:
        head = f.read(1024)
    m = re.search(r"random_vector\(N, seed=(\d+), n_rhs=(\d+)\)", head)
    seed, nrhs = int(m.group(1)), int(m.group(2))
    a = np.loadtxt(path)
    rows = np.unique(a[:, 0].astype(np.int64))
    Y = np.zeros((rows.size, nrhs), dtype=complex)
    ri = np.searchsorted(rows, a[:, 0].astype(np.int64))
    Y[ri, a[:, 1].astype(np.int64)] = a[:, 2] + 1j * a[:, 3]
    return seed, nrhs, rows, Y


def _check(name, w):
    seed, nrhs, rows, ref = _golden(name)
    print(f"case: {w.name} full-size sampled rows, R={nrhs}", flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, p=w.p, precond=0)
    try:
        assert geo.n == w.n_elements
        X = torch.from_numpy(wl.random_vector(geo.n, seed=seed, n_rhs=nrhs)).cuda()
        idx = torch.from_numpy(rows).cuda()
        y64 = geo.matvec(X)[:, idx].T.cpu().numpy()
        y32 = geo.matvec(X.to(torch.complex64), precision=lmfmm.LM_MIXED)[:, idx].T.cpu().numpy()
        del X
        # per right-hand side over the sampled rows, entry by entry
        check(y64.T, ref.T, 1e-6, f"{w.name} FP64 form, R={nrhs}, {rows.size} sampled rows", idx=rows)
        check(y32.T.astype(np.complex128), ref.T, 1e-4, f"{w.name} FP32 form, R={nrhs}, {rows.size} sampled rows",
              idx=rows)
    finally:
        geo.close()
        torch.cuda.empty_cache()


def test_three_layer_64k_sampled_rows():
    _check("three_layer", wl.three_layer())


@pytest.mark.timeout(900)
def test_five_layer_1m_sampled_rows():
    _check("five_layer", wl.five_layer())
