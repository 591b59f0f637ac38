"""The multi-angle precision form on the mini workload against the oracle,
angle by angle: the three-layer generator at 25 scatterers (N = 4,000, the
density of the 64,000-element workload), 64 incidence angles in [10, 170]
deg.  The expected far fields are the oracle's LU solutions (dense FP64
matrix by direct Sommerfeld quadrature), stored under tests/golden/ by
make_mini_far_fields.py, which calls only the oracle.

* served FP32 form: the serving loop in LM_MIXED, 16 requests of 4 angles
  submitted at once, GMRES tol 1e-6: every angle within 1e-4;
* FP64 form: one 64-right-hand-side lm_gmres_solve at tol 1e-9: every angle
  within 1e-6.
"""

import importlib.util
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2511_12450_amd import lmfmm
from paper_2511_12450_amd import workloads as wl
from tests.parity import check

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden():
    spec = importlib.util.spec_from_file_location("make_mini_far_fields", os.path.join(GOLDEN, "make_mini_far_fields.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    a = np.loadtxt(os.path.join(GOLDEN, "mini_far_fields.txt"))
    obs = mod.obs_angles()
    ff = np.zeros((64, obs.size), dtype=complex)
    ff[a[:, 0].astype(int), a[:, 1].astype(int)] = a[:, 2] + 1j * a[:, 3]
    return obs, ff


@pytest.fixture(scope="module")
def mini():
    w = wl.three_layer_mini(seed=3)
    print(f"case: three_layer_mini, N={w.n_elements}, 64 angles", flush=True)
    return w, lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM)


def test_served_fp32_every_angle_vs_oracle(mini):
    w, geo = mini
    obs, ref = _golden()
    th = np.radians(w.angles_deg)
    srv = lmfmm.Server(precision=lmfmm.LM_MIXED)
    try:
        ids = [srv.submit(geo, th[i:i + 4], tol=1e-6, max_iter=2000, restart=500, obs_rad=obs) for i in range(0, 64, 4)]
        ff = np.zeros_like(ref)
        its = []
        for q, rid in enumerate(ids):
            st, status, lat, rep, phi, f = srv.wait(rid)
            assert st == lmfmm.LM_DONE and status == lmfmm.LM_OK, (q, st, status)
            ff[4 * q:4 * q + 4] = f
            its += [r[0] for r in rep]
    finally:
        srv.close()
    print(f"served iterations {min(its)}..{max(its)}", flush=True)
    per = [float(np.linalg.norm(ff[r] - ref[r]) / np.linalg.norm(ref[r])) for r in range(64)]
    print("served FP32 per-angle far-field error vs oracle:", [f"{e:.1e}" for e in per], flush=True)
    check(ff, ref, 1e-4, "served FP32 64 angles vs oracle LU")


def test_fp64_every_angle_vs_oracle(mini):
    w, geo = mini
    obs, ref = _golden()
    th = np.radians(w.angles_deg)
    phi, rep, st = geo.solve(th, tol=1e-9, max_iter=2000, restart=500, precision=lmfmm.LM_FP64)
    assert st == lmfmm.LM_OK
    ff = geo.far_field(phi, obs).cpu().numpy()
    check(ff, ref, 1e-6, "FP64 64 angles vs oracle LU")
