"""Request-serving loop (lm_server_*, continuous batching) through the C-ABI.

Each result must be the same alone and in a mix of concurrent requests on
several geometries (within the form's tolerance: 1e-4 relative far-field
difference for the FP32 form), and the same as the direct solver
(lm_gmres_solve) and the FP64 oracle; requests on one geometry must be fused
into shared multi-right-hand-side launches; cancellation, invalid input,
admission by right-hand-side slots and HBM budget, and non-convergence are
reported as documented.
"""

import time

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
def geoms():
    mini = wl.three_layer_mini(seed=3)
    small = wl.plain_small()
    print("case: server geometries mini N=", mini.n_elements, "plain_small N=", small.n_elements, flush=True)
    g_mini = lmfmm.Geometry.from_workload(mini, method=lmfmm.LM_FMM, precond=1)
    g_small = lmfmm.Geometry.from_workload(small, method=lmfmm.LM_DENSE)
    return mini, g_mini, small, g_small


OBS = lmfmm.far_field_angles()[::17]


def test_server_fp64_matches_direct_solve_and_oracle(geoms):
    mini, g_mini, small, g_small = geoms
    srv = lmfmm.Server(precision=lmfmm.LM_FP64)
    try:
        th = np.radians([35.0, 110.0])
        rid = srv.submit(g_small, th, tol=1e-10, max_iter=300, restart=300, precond=0, obs_rad=OBS)
        st, status, lat, rep, phi, ff = srv.wait(rid)
        assert st == lmfmm.LM_DONE and status == lmfmm.LM_OK, (st, status)
        print("plain_small server reports", rep, "latency", lat, flush=True)
        med = Medium(small.d, small.k, small.eta)
        el = Elements(med, small.polygons)
        K = matrix(med, el)
        ref = np.array([far_field(med, el, lu_solve(K, boundary_data(med, t, el.cx, el.cy)), OBS) for t in th])
        check(ff, ref, 1e-6, "server FP64 far field vs oracle")
        # same as the direct solver on the FMM geometry
        th2 = np.radians([60.0])
        rid2 = srv.submit(g_mini, th2, tol=1e-8, max_iter=800, restart=400, precond=1, obs_rad=OBS)
        st, status, lat, rep, phi_s, ff_s = srv.wait(rid2)
        assert st == lmfmm.LM_DONE and status == lmfmm.LM_OK
        phi_d, rep_d, sd = g_mini.solve(th2, tol=1e-8, max_iter=800, restart=400, precond=1)
        ff_d = g_mini.far_field(phi_d, OBS).cpu().numpy()
        print("server its", rep, "direct its", rep_d, flush=True)
        assert abs(rep[0][0] - rep_d[0][0]) <= 2
        check(ff_s, ff_d, 1e-6, "server vs direct solve far field")
        srv.release(rid)
        srv.release(rid2)
    finally:
        srv.close()


def test_alone_equals_in_mix_and_fusion(geoms):
    mini, g_mini, small, g_small = geoms
    srv = lmfmm.Server(precision=lmfmm.LM_MIXED)
    try:
        thA = np.radians([30.0, 75.0])
        ridA = srv.submit(g_mini, thA, tol=1e-6, max_iter=800, restart=400, obs_rad=OBS)
        stA, sA, latA, repA, _, ffA = srv.wait(ridA)
        assert stA == lmfmm.LM_DONE and sA == lmfmm.LM_OK
        alone_stats = srv.stats()
        # the mix: A again between requests on both geometries; the last one
        # arrives while the others are on the GPU
        ids = [srv.submit(g_mini, np.radians([50.0, 140.0, 100.0]), tol=1e-6, max_iter=800, restart=400, obs_rad=OBS),
               srv.submit(g_small, np.radians([20.0, 160.0]), tol=1e-6, max_iter=300, restart=300, precond=0,
                          obs_rad=OBS)]
        ridA2 = srv.submit(g_mini, thA, tol=1e-6, max_iter=800, restart=400, obs_rad=OBS)
        time.sleep(0.02)
        ids.append(srv.submit(g_mini, np.radians([120.0]), tol=1e-6, max_iter=800, restart=400, obs_rad=OBS))
        st2, s2, lat2, rep2, _, ffA2 = srv.wait(ridA2)
        assert st2 == lmfmm.LM_DONE and s2 == lmfmm.LM_OK
        its = sum(r[0] for r in rep2)
        for rid in ids:
            st, s, lat, rep, _, ff = srv.wait(rid)
            assert st == lmfmm.LM_DONE and s == lmfmm.LM_OK, (rid, st, s)
            assert np.all(np.isfinite(ff))
            its += sum(r[0] for r in rep)
        print(f"alone its {[r[0] for r in repA]}, in mix its {[r[0] for r in rep2]}", flush=True)
        check(ffA2, ffA, 1e-4, "far field alone vs in the mix")
        stt = srv.stats()
        mix_rounds = stt["rounds"] - alone_stats["rounds"]
        mix_launches = stt["launches"] - alone_stats["launches"]
        mix_rhs = stt["fused_rhs"] - alone_stats["fused_rhs"]
        print("stats alone", alone_stats, "after mix", stt, "iterations in the mix", its, flush=True)
        assert mix_rhs / mix_launches > 1.5  # requests on one geometry shared launches
        assert mix_rounds < 0.6 * its  # solves advanced together, not one after another
    finally:
        srv.close()


def test_cancel_and_release(geoms):
    mini, g_mini, small, g_small = geoms
    srv = lmfmm.Server(precision=lmfmm.LM_MIXED, max_active_rhs=2)
    try:
        # restarted every 5 steps and checked against the true FP32 residual: cannot reach 1e-13
        long_id = srv.submit(g_mini, np.radians([40.0, 80.0]), tol=1e-13, max_iter=20000, restart=5)
        queued_id = srv.submit(g_mini, np.radians([60.0]), tol=1e-6)
        time.sleep(0.2)
        assert srv.poll(queued_id)[0] == lmfmm.LM_QUEUED  # no right-hand-side slot free
        srv.cancel(queued_id)
        assert srv.poll(queued_id)[0] == lmfmm.LM_CANCELLED
        assert srv.poll(long_id)[0] == lmfmm.LM_RUNNING
        with pytest.raises(lmfmm.LmError):
            srv.release(long_id)  # still running
        srv.cancel(long_id)
        st = srv.wait(long_id, results=False)[0]
        assert st == lmfmm.LM_CANCELLED
        assert srv.stats()["active_rhs"] == 0
        srv.release(long_id)
        srv.release(queued_id)
        # the server keeps working after cancellations
        rid = srv.submit(g_small, np.radians([30.0]), tol=1e-6, precond=0)
        assert srv.wait(rid)[0] == lmfmm.LM_DONE
    finally:
        srv.close()


def test_invalid_and_never_admissible(geoms):
    mini, g_mini, small, g_small = geoms
    srv = lmfmm.Server(precision=lmfmm.LM_MIXED, max_active_rhs=4, hbm_budget_bytes=8 << 20)
    try:
        with pytest.raises(lmfmm.LmError) as e:
            srv.submit(g_small, np.array([np.nan]))
        assert e.value.status == -1
        with pytest.raises(lmfmm.LmError) as e:
            srv.submit(g_small, np.radians([30.0]), tol=float("nan"))
        assert e.value.status == -1
        with pytest.raises(lmfmm.LmError) as e:
            srv.submit(g_small, np.radians(np.linspace(10, 170, 5)))  # more than max_active_rhs
        assert e.value.status == lmfmm.LM_ENOMEM
        with pytest.raises(lmfmm.LmError) as e:
            srv.submit(g_mini, np.radians([30.0]), restart=400, max_iter=800)  # basis alone ~ 26 MB > 8 MB
        assert e.value.status == lmfmm.LM_ENOMEM
        rid = srv.submit(g_small, np.radians([30.0]), tol=1e-6, restart=50, max_iter=100, precond=0)
        assert srv.wait(rid)[0] == lmfmm.LM_DONE
    finally:
        srv.close()


def test_admission_by_hbm_budget(geoms):
    mini, g_mini, small, g_small = geoms
    # restarted every 5 steps against the true FP32 residual: cannot reach 1e-13
    long_opts = dict(tol=1e-13, restart=5, max_iter=20000)
    one = lmfmm.request_footprint(g_mini, 1, **long_opts)
    print("footprint of one request:", one, flush=True)
    assert one > 5 * 4000 * 16
    srv = lmfmm.Server(precision=lmfmm.LM_MIXED, hbm_budget_bytes=int(one * 1.5))
    try:
        a = srv.submit(g_mini, np.radians([30.0]), **long_opts)
        b = srv.submit(g_mini, np.radians([70.0]), tol=1e-6, restart=5, max_iter=800)
        time.sleep(0.1)
        sa, sb = srv.poll(a)[0], srv.poll(b)[0]
        print("states while the first runs:", sa, sb, srv.stats(), flush=True)
        assert sa == lmfmm.LM_RUNNING and sb == lmfmm.LM_QUEUED  # the budget holds one request
        srv.cancel(a)
        assert srv.wait(a, results=False)[0] == lmfmm.LM_CANCELLED
        assert srv.wait(b)[0] == lmfmm.LM_DONE  # admitted once the memory was free
    finally:
        srv.close()


def test_memory_stays_within_budget():
    """A stream over three geometries of different sizes under a budget that
    holds about two requests: the device memory the server holds (bases and
    work vectors of admitted and spare solves, fused-launch buffers, round
    buffers) never exceeds the budget, spare solves of other shapes are freed
    when an admission needs the room, and the fused-launch buffers of an idle
    geometry are released."""
    ws = [wl.three_layer_mini(seed=s, n_scat=n) for s, n in ((3, 25), (4, 18), (5, 12))]
    print("case: memory budget, N =", [w.n_elements for w in ws], flush=True)
    gs = [lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=1) for w in ws]
    opts = dict(tol=1e-6, max_iter=600, restart=40)
    rng = np.random.default_rng(5)
    reqs = [(int(rng.integers(0, 3)), np.radians(rng.uniform(10, 170, size=int(rng.integers(1, 4)))))
            for _ in range(10)]
    big = max(lmfmm.request_footprint(gs[g], th.size, **opts) for g, th in reqs)
    budget = int(2.2 * big)
    srv = lmfmm.Server(precision=lmfmm.LM_MIXED, hbm_budget_bytes=budget)
    try:
        ids = []
        peak = 0
        for g, th in reqs:
            ids.append((srv.submit(gs[g], th, obs_rad=OBS, **opts), g, th))
            time.sleep(0.01)
            peak = max(peak, srv.memory()["held"])
        pending = list(ids)
        t0 = time.time()
        while pending:
            m = srv.memory()
            peak = max(peak, m["held"])
            assert m["held"] <= budget, (m, budget)
            for item in list(pending):
                st = srv.poll(item[0])[0]
                if st in (lmfmm.LM_DONE, lmfmm.LM_FAILED, lmfmm.LM_CANCELLED):
                    pending.remove(item)
            assert time.time() - t0 < 120, "requests did not finish"
            time.sleep(0.002)
        for rid, g, th in ids:
            st, status, lat, rep, phi, ff = srv.wait(rid)
            assert st == lmfmm.LM_DONE and status == lmfmm.LM_OK, (st, status)
            assert np.all(np.isfinite(ff))
        time.sleep(0.05)
        m = srv.memory()
        print(f"budget {budget}, peak held {peak}, at rest {m}", flush=True)
        assert peak <= budget
        assert m["admitted"] == 0 and m["held"] == m["spare"] <= budget
        # the last request's results against its geometry's direct solve
        rid, g, th = ids[-1]
        st, status, lat, rep, phi, ff = srv.wait(rid)
        pd, rd, sd = gs[g].solve(th, tol=1e-9, max_iter=800, restart=400, precond=1)
        check(ff, gs[g].far_field(pd, OBS).cpu().numpy(), 1e-4, "budgeted stream vs direct solve")
    finally:
        srv.close()
        for g in gs:
            g.close()


def test_not_converged_reported(geoms):
    mini, g_mini, small, g_small = geoms
    srv = lmfmm.Server(precision=lmfmm.LM_FP64)
    try:
        rid = srv.submit(g_mini, np.radians([30.0]), tol=1e-12, max_iter=4, restart=4, obs_rad=OBS)
        st, status, lat, rep, phi, ff = srv.wait(rid)
        assert st == lmfmm.LM_DONE and status == lmfmm.LM_NOT_CONVERGED
        assert rep[0][0] == 4 and rep[0][1] > 1e-12
        assert np.all(np.isfinite(phi))
    finally:
        srv.close()


def test_batched_finish_matches_direct_solves(geoms):
    """Columns finishing in the same round share one preconditioner launch;
    requests with the same observation angles share one far-field launch."""
    mini, g_mini, small, g_small = geoms
    obs2 = lmfmm.far_field_angles()[5::23]
    thA, thB, thC = np.radians([35.0, 65.0]), np.radians([95.0, 125.0]), np.radians([150.0])
    ref = {}
    for th in np.concatenate([thA, thB, thC]):
        phi, rep, st = g_mini.solve(np.array([th]), tol=1e-10, max_iter=800, restart=400, precond=1)
        assert st == lmfmm.LM_OK
        ref[float(th)] = phi
    for prec, tol, bar in ((lmfmm.LM_FP64, 1e-9, 1e-6), (lmfmm.LM_MIXED, 1e-6, 1e-4)):
        srv = lmfmm.Server(precision=prec)
        try:
            ids = [srv.submit(g_mini, thA, tol=tol, max_iter=800, restart=400, obs_rad=OBS),
                   srv.submit(g_mini, thB, tol=tol, max_iter=800, restart=400, obs_rad=OBS),
                   srv.submit(g_mini, thC, tol=tol, max_iter=800, restart=400, obs_rad=obs2)]
            for rid, th, ob in zip(ids, (thA, thB, thC), (OBS, OBS, obs2)):
                st, status, lat, rep, phi, ff = srv.wait(rid)
                assert st == lmfmm.LM_DONE and status == lmfmm.LM_OK, (prec, st, status)
                want = np.array([g_mini.far_field(ref[float(t)], ob).cpu().numpy()[0] for t in th])
                print(f"precision {prec}: its {[r[0] for r in rep]}", flush=True)
                check(ff, want, bar, f"precision {prec}: batched finish far field vs direct")
            print("rounds", srv.stats()["rounds"], flush=True)
        finally:
            srv.close()


def test_odd_n_basis_padding():
    """N odd: the last element pair of every basis vector ends in padding."""
    w0 = wl.plain_small()
    polys = [wl.circle((float(p[:, 0].mean()), float(p[:, 1].mean())), 0.3, n)
             for p, n in zip(w0.polygons, (63, 64, 64, 64))]
    w = wl.Workload("odd_N255", w0.d, w0.k, w0.eta, polys, np.array([40.0]))
    assert w.n_elements % 2 == 1
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_DENSE)
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    th = np.radians([40.0, 140.0])
    K = matrix(med, el)
    for prec, tol, bar in ((lmfmm.LM_FP64, 1e-10, 1e-6), (lmfmm.LM_MIXED, 1e-6, 1e-4)):
        srv = lmfmm.Server(precision=prec)
        try:
            rid = srv.submit(geo, th, tol=tol, max_iter=300, restart=300, precond=0, obs_rad=OBS)
            st, status, lat, rep, phi, ff = srv.wait(rid)
            assert st == lmfmm.LM_DONE and status == lmfmm.LM_OK
            want = np.array([far_field(med, el, lu_solve(K, boundary_data(med, t, el.cx, el.cy)), OBS) for t in th])
            check(ff, want, bar, f"N={el.n} precision {prec}: far field vs oracle")
        finally:
            srv.close()


def test_same_results_with_kept_and_released_buffers(geoms):
    """A request submitted at once after another (fused-launch, round and
    finishing buffers kept), and again after the server has been idle long
    enough to give them back, returns the same phi and far field bit for bit
    (each column is computed independently of what the buffers held)."""
    mini, g_mini, small, g_small = geoms
    srv = lmfmm.Server(precision=lmfmm.LM_MIXED)
    try:
        th = np.radians([35.0, 80.0, 125.0])
        outs = []
        for pause in (0.0, 0.0, 0.2):
            time.sleep(pause)
            rid = srv.submit(g_mini, th, tol=1e-6, max_iter=800, restart=400, obs_rad=OBS)
            st, s, lat, rep, phi, ff = srv.wait(rid)
            assert st == lmfmm.LM_DONE and s == lmfmm.LM_OK
            outs.append((phi, ff, [r[0] for r in rep]))
            srv.release(rid)
            if pause > 0.0:
                assert srv.memory()["held"] > 0
        time.sleep(0.1)
        m = srv.memory()
        print("iterations", [o[2] for o in outs], "memory at rest", m, flush=True)
        assert m["held"] == m["spare"]  # the idle release ran
        for phi, ff, its in outs[1:]:
            assert its == outs[0][2]
            assert np.array_equal(phi, outs[0][0]) and np.array_equal(ff, outs[0][1])
    finally:
        srv.close()
