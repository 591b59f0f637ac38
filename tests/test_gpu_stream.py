"""A serving stream over several geometries, through lm_submit / lm_poll.

The request mix of the serving workload: Poisson arrivals of solves drawn
from layered media of 2-4 layers (k per layer U[1, 10], scatterers crossing
interfaces), 1-16 incident angles per request, admitted by HBM footprint
(the budget holds only part of the stream, so requests queue), Krylov state
on the device, served in the FP32 form.  Four pool geometries of the
generator, the smallest ones (N = 4,640 .. 15,040), keep the test short.

Bars: every request completes; the far field of every angle within 1e-4 of
an FP64 direct solve (tol 1e-8) of the same geometry and angle; a request
solved again alone returns the same density as in the mix (columns are
computed independently inside the fused launches).  p50 / p99 latency are
printed.
"""

import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2511_12450_amd import lmfmm
from paper_2511_12450_amd import workloads as wl
from tests.parity import check

pytestmark = pytest.mark.gpu

OBS = lmfmm.far_field_angles()[::11]


def test_stream_of_mixed_geometries():
    gs = [9, 12, 7, 1]
    ws = [wl.stream_geometry(g) for g in gs]
    print("case: stream over", [(w.name, len(w.k)) for w in ws], flush=True)
    geos = [lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, p=w.p) for w in ws]
    rng = np.random.default_rng(17)
    n_req = 12
    which = rng.integers(0, len(geos), size=n_req)
    n_ang = rng.integers(1, 17, size=n_req)
    angles = [np.radians(rng.uniform(10.0, 170.0, size=n)) for n in n_ang]
    t_arr = np.cumsum(rng.exponential(0.03, size=n_req))
    opts = dict(tol=1e-6, max_iter=1000, restart=300)
    fp = max(lmfmm.request_footprint(geos[i], int(n), tol=1e-6, max_iter=1000, restart=300)
             for i, n in zip(which, n_ang))
    srv = lmfmm.Server(precision=lmfmm.LM_MIXED, hbm_budget_bytes=int(2.5 * fp))
    try:
        ids, done = [], {}
        t0 = time.time()
        k = 0
        while len(done) < n_req:
            now = time.time() - t0
            while k < n_req and t_arr[k] <= now:
                ids.append(srv.submit(geos[which[k]], angles[k], obs_rad=OBS, **opts))
                k += 1
            for q, rid in enumerate(ids):
                if q in done:
                    continue
                out = srv.poll(rid, results=True)
                if out[0] in (lmfmm.LM_DONE, lmfmm.LM_FAILED, lmfmm.LM_CANCELLED):
                    done[q] = out
            assert time.time() - t0 < 240, "stream did not finish"
            time.sleep(0.002)
        lat = np.array([done[q][2] for q in range(n_req)])
        print(f"stream: {n_req} requests, {int(n_ang.sum())} solves in {time.time() - t0:.2f} s, "
              f"latency p50 {np.percentile(lat, 50):.3f} s, p99 {np.percentile(lat, 99):.3f} s", flush=True)
        for q in range(n_req):
            st, status, _, rep, phi, ff = done[q]
            assert st == lmfmm.LM_DONE and status == lmfmm.LM_OK, (q, st, status, rep)
            g = geos[which[q]]
            ref_phi, _, rst = g.solve(angles[q], tol=1e-8, max_iter=2000, restart=500, precision=lmfmm.LM_FP64)
            assert rst == lmfmm.LM_OK
            ref = g.far_field(ref_phi, OBS).cpu().numpy()
            check(ff, ref, 1e-4, f"stream request {q} ({n_ang[q]} angles) far field vs FP64 direct solves")
        # the request with most angles, alone on a fresh server
        q = int(np.argmax(n_ang))
        srv1 = lmfmm.Server(precision=lmfmm.LM_MIXED)
        try:
            rid = srv1.submit(geos[which[q]], angles[q], obs_rad=OBS, **opts)
            st, status, _, rep, phi1, _ = srv1.wait(rid)
            assert st == lmfmm.LM_DONE and status == lmfmm.LM_OK
        finally:
            srv1.close()
        check(phi1, done[q][4], 1e-6, f"stream: request {q} ({n_ang[q]} angles) phi alone vs in the mix")
    finally:
        srv.close()
        for g in geos:
            g.close()
