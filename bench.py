"""Benchmark: GMRES solves/sec (+ p50/p99 latency) of the layered-medium
Nystrom solver on one MI355X, served FP32 form vs plain FP64 form.

Workload (default): three layers (interfaces y = 0, -2; k = 5, 7, 4), 400
scatterers (circles and 5-petal stars), N = 64,000 elements, FMM order
p = 20, GMRES tol 1e-6 with the domain-decomposition preconditioner; the
geometry's operator data (trees, Sommerfeld M2L tables, near-field matrix,
preconditioner) are built once and stay resident in HBM.

* plain FP64 form: one lm_gmres_solve per incidence angle (every step FP64),
  then the far field on 682 angles; solves run one after another.
* served FP32 form (the value): the request-serving loop in LM_MIXED
  precision; a step is one batch of 64 incidence angles in [10, 170] deg
  submitted at once as 16 requests of 4 angles (each request also asks for
  the 682-angle far field); the server fuses them into multi-right-hand-side
  launches.  solves/s = angles / wall time of the batch; latency = per
  request, submission to completion.  The same batch is also served with the
  preconditioner applied from its FP64 rows instead of the binary16 copy.
* latency under load: an open-loop Poisson stream on the same geometry, and
  a stream over a pool of seeded geometries of 2-4 layers (different media
  and sizes, 1-16 angles per request, admission by HBM footprint).

Every solve of every form is checked against a tight FP64 reference (all 64
angles solved together at tol 1e-9, outside the timed region): the far-field
relative error per angle is reported (bar 1e-4).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP64_VALU_TFLOPS = 78.6
STAGES = ("P2M", "M2M", "M2L", "L2L", "L2P", "near", "M2L_sums", "total", "level0_conv")


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1, help="served batches of --angles incidence angles")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--angles", type=int, default=64)
    ap.add_argument("--requests", type=int, default=16)
    ap.add_argument("--plain-solves", type=int, default=16)
    ap.add_argument("--restart", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stream-requests", type=int, default=550,
                    help="requests of the open-loop Poisson stream (0: skip); the first 50 are warm-up")
    ap.add_argument("--stream-rho", type=float, default=0.5, help="arrival rate as a fraction of the served capacity")
    ap.add_argument("--stream-max-angles", type=int, default=4)
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--pool-geometries", type=int, default=6,
                    help="serve open-loop streams over this many pool geometries (2-4 layers, N in "
                         "[4,000, 250,000], 1-16 angles per request); 0: skip")
    ap.add_argument("--pool-requests", type=int, default=20, help="requests per pool stream")
    ap.add_argument("--pool-rho", type=str, default="0.5,0.9",
                    help="arrival rates of the pool streams as fractions of the pool's served capacity")
    ap.add_argument("--replica", type=str, default="",
                    help="run a paper replica instead of the benchmark: 'example1', 'example2' or 'example3' "
                         "(Sec. 5, Tables 5.1-5.3), or 'spectral' (the spectral rule against the lowest-order "
                         "one; --replica-n gives the nodes per scatterer, e.g. 16,32,64,128,256)")
    ap.add_argument("--replica-n", type=str, default="960,1920,3840,7680,15360",
                    help="example1: nodes per unit length of the L-shape (N = 12.5 x this)")
    ap.add_argument("--pool-budget-gb", type=float, default=0.0,
                    help="also run the first pool stream under this HBM budget (restart 100); 0: skip")
    return ap.parse_args()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _traffic():
    """HBM bytes per launch from the committed rocprofv3 counter record, or
    None when the kernel sources changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic_three_layer_N64000.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    for f, h in rec["source_sha256"].items():
        if hashlib.sha256(open(os.path.join(ROOT, f), "rb").read()).hexdigest() != h:
            return None
    return rec


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _oracle_rows(args):
    """Worker: rows of the dense oracle matrix until budget_s has passed."""
    name, rows, budget_s = args
    from threadpoolctl import threadpool_limits

    from oracle.nystrom import matrix_rows

    med, el = _ORACLE[name]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        done = 0
        K = None
        while done < len(rows) and (done == 0 or time.perf_counter() - t0 < budget_s):
            K = matrix_rows(med, el, [int(rows[done])])
            done += 1
        row_s = (time.perf_counter() - t0) / done
        x = np.ones(el.n, dtype=complex)
        t1 = time.perf_counter()
        for _ in range(10):
            K @ x
        gemv_row_s = (time.perf_counter() - t1) / 10
    return done, row_s, gemv_row_s


_ORACLE = {}


def cpu_baseline_time(w, budget_s):
    """The oracle as it stands, timed on the host cores before the GPU is
    touched: one worker process per core (one BLAS thread each, at most 16,
    the host share of one GPU) computes rows of the dense Nystrom matrix by
    direct Sommerfeld quadrature for budget_s seconds."""
    import multiprocessing as mp

    from oracle.medium import Medium
    from oracle.nystrom import Elements

    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    _ORACLE[w.name] = (med, el)
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    rows = np.random.default_rng(0).permutation(el.n)
    chunks = [(w.name, rows[i::cores][:1000], budget_s) for i in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_rows, chunks)
    wall = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    return {"n": el.n, "cores": cores, "rows": done, "wall_s": wall, "rows_per_s": done / wall,
            "gemv_row_s": float(np.median([r[2] for r in res])), "row_s_per_core": float(np.median([r[1] for r in res]))}


def cpu_baseline(w, t, iterations):
    """One solve projected from the timed sample: N rows of assembly at the
    measured rate of all workers plus (iterations + 1) dense matvecs spread
    over the same cores."""
    n = t["n"]
    projected = n / t["rows_per_s"] + (iterations + 1) * n * t["gemv_row_s"] / t["cores"]
    return {"value": 1.0 / projected, "unit": "solves/s", "cores": t["cores"], "kind": "oracle",
            "sample": (f"{t['rows']} rows of the dense FP64 matrix of {w.name} by direct Sommerfeld quadrature in "
                       f"{t['wall_s']:.1f} s on {t['cores']} worker processes ({t['row_s_per_core']:.2f} s/row per "
                       f"core); one solve projected as {n} rows + {iterations + 1} dense matvecs = "
                       f"{projected:.3g} s (projected, not run)")}


def _pool_stream(lmfmm, srv, pgeos, gi, th_q, t_arr, obs, gm_of, fref_of=None):
    """Open-loop stream: request i arrives at t_arr[i]; returns per-request
    latency, iterations, far-field errors (when references are given) and
    the span."""
    pend, lat, its, errs = {}, {}, [], []
    i, t0 = 0, time.perf_counter()
    nq = len(t_arr)
    while i < nq or pend:
        now = time.perf_counter() - t0
        while i < nq and t_arr[i] <= now:
            pend[srv.submit(pgeos[gi[i]], th_q[i], obs_rad=obs, **gm_of(gi[i]))] = i
            i += 1
        for rid in list(pend):
            out_q = srv.poll(rid, results=True)
            if out_q[0] in (lmfmm.LM_DONE, lmfmm.LM_FAILED, lmfmm.LM_CANCELLED):
                assert out_q[0] == lmfmm.LM_DONE, out_q[:2]
                k = pend.pop(rid)
                lat[k] = out_q[2]
                its += [r_[0] for r_ in out_q[3]]
                if fref_of is not None:
                    errs += fref_of(k, out_q[5])
                srv.release(rid)
                if len(lat) % 20 == 0:
                    _log(f"  {len(lat)} of {nq} requests done")
        time.sleep(0.0005)
    return lat, its, errs, time.perf_counter() - t0


# Table 5.1 of the paper (Example 1; CPU time, hardware not reported): N,
# GMRES iterations without / with the preconditioner, time in s without /
# with it, L-infinity error of the preconditioned solve.
PAPER_TABLE_5_1 = [(12000, 140, 60, 739.71, 573.37, 2.282e-2), (24000, 163, 68, 918.03, 650.14, 1.151e-2),
                   (48000, 190, 77, 1142.87, 783.46, 5.782e-3), (96000, 278, 86, 2110.27, 1014.66, 2.897e-3),
                   (192000, 331, 99, 3535.53, 1501.94, 1.450e-3)]


def replica_example1(a):
    """Example 1 of Sec. 5: the L-shaped scatterer across four of five
    layers (eta = 1..5, k = 3.2, 2.5, 5.1, 8.6, 6.9), manufactured solution
    G(. | s) of a unit point source at s = (0, 0.375) inside it; FP64 GMRES
    at tol 1e-8 with and without the preconditioner; error of the far-field
    pattern (682 angles) against the exact one, per N."""
    import torch

    from paper_2511_12450_amd import lmfmm
    from paper_2511_12450_amd import workloads as wl

    torch.cuda.set_device(0)
    obs = lmfmm.far_field_angles()
    src = np.array([[0.0, 0.375]])
    # receivers: 256 points on a circle of 1.5 times the geometry's radius
    # about its centre, those within 0.05 of an interface left out
    w0 = wl.paper_example1(n_per_side_unit=8)
    P = np.concatenate(w0.polygons)
    ctr = 0.5 * (P.min(axis=0) + P.max(axis=0))
    rad = 1.5 * np.max(np.hypot(P[:, 0] - ctr[0], P[:, 1] - ctr[1]))
    t = 2.0 * np.pi * np.arange(256) / 256
    rec = np.stack([ctr[0] + rad * np.cos(t), ctr[1] + rad * np.sin(t)], axis=1)
    rec = rec[np.min(np.abs(rec[:, 1:2] + w0.d[None, :]), axis=1) > 0.05]
    lay0 = lmfmm.Layers(w0.d, w0.k, w0.eta)
    u_exact = lmfmm.point_field(lay0, src, rec).cpu().numpy()[0]
    rows = []
    for n in [int(v) for v in a.replica_n.split(",") if v]:
        w = wl.paper_example1(n_per_side_unit=n)
        t0 = time.perf_counter()
        geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        g = geo.point_source_rhs(src)
        exact = lmfmm.point_far_field(geo.layers, src, obs).cpu().numpy()[0]
        row = {"N": int(geo.n), "setup_s": setup}
        for pc, key in ((1, "preconditioned"), (0, "plain")):
            t1 = time.perf_counter()
            phi, rep, st = geo.solve_rhs(g, tol=1e-8, max_iter=5000, restart=1000, precond=pc)
            torch.cuda.synchronize()
            ts = time.perf_counter() - t1
            ff = geo.far_field(phi, obs).cpu().numpy()[0]
            row[key] = {"iterations": int(rep[0][0]), "solve_s": ts, "status": int(st),
                        "far_field_err_l2": _rel(ff, exact),
                        "far_field_err_linf": float(np.abs(ff - exact).max() / np.abs(exact).max())}
            if pc == 1:
                u = geo.field(phi, rec).cpu().numpy()[0]
                row[key]["receiver_err_l2"] = _rel(u, u_exact)
                row[key]["receiver_err_linf"] = float(np.abs(u - u_exact).max() / np.abs(u_exact).max())
        _log(f"example1 N={geo.n}: its {row['preconditioned']['iterations']} / {row['plain']['iterations']}, "
             f"far-field err {row['preconditioned']['far_field_err_linf']:.3e}, receiver err "
             f"{row['preconditioned']['receiver_err_linf']:.3e}, setup {setup:.1f} s")
        rows.append(row)
        geo.close()
        torch.cuda.empty_cache()
    for i in range(1, len(rows)):
        p0, p1 = rows[i - 1]["preconditioned"], rows[i]["preconditioned"]
        rows[i]["ratio_linf"] = p0["far_field_err_linf"] / p1["far_field_err_linf"]
        rows[i]["ratio_l2"] = p0["far_field_err_l2"] / p1["far_field_err_l2"]
        rows[i]["receiver_ratio_linf"] = p0["receiver_err_linf"] / p1["receiver_err_linf"]
    print(json.dumps({"replica": "example1", "workload": "L-shape across 4 of 5 layers, eta 1..5, point source "
                      "(0, 0.375), FP64, GMRES tol 1e-8", "receivers": int(len(rec)),
                      "receiver_circle": {"centre": ctr.tolist(), "radius": float(rad)}, "rows": rows,
                      "paper_table_5_1": [dict(zip(("N", "its", "its_preconditioned", "time_s",
                                                    "time_s_preconditioned", "linf_error"), r))
                                          for r in PAPER_TABLE_5_1],
                      "paper_hardware": "not reported (CPU time)"}))


# Tables 5.2 and 5.3 of the paper (Examples 2 and 3; CPU time, hardware not
# reported): N, iterations without / with the preconditioner, time in s
# without / with it.
PAPER_TABLE_5_2 = [(12000, 93, 59, 1628.33, 1362.33), (24000, 104, 66, 1822.82, 1520.70),
                   (48000, 115, 72, 2429.23, 1685.44), (96000, 132, 81, 3042.68, 2058.86),
                   (192000, 162, 93, 3807.98, 2827.82)]
PAPER_TABLE_5_3 = [(12000, 125, 71, 1638.88, 1553.62), (24000, 138, 79, 1742.52, 1639.49),
                   (48000, 156, 88, 2031.50, 1831.76), (96000, 173, 101, 2708.44, 2649.50),
                   (192000, 192, 112, 3782.74, 3056.38)]


def replica_plane_wave(a, which):
    """Examples 2 and 3 of Sec. 5 (plane-wave incidence, no closed-form
    solution): FP64 GMRES at tol 1e-8 with and without the preconditioner
    per N, and the self-convergence of the far-field pattern (682 angles):
    the difference to the next finer N, whose ratio per doubling is about 2
    at first order."""
    import torch

    from paper_2511_12450_amd import lmfmm
    from paper_2511_12450_amd import workloads as wl

    torch.cuda.set_device(0)
    gen, table = (wl.paper_example2, PAPER_TABLE_5_2) if which == "example2" else (wl.paper_example3, PAPER_TABLE_5_3)
    obs = lmfmm.far_field_angles()
    rows, ffs = [], []
    for n_el in [int(12.5 * int(v)) for v in a.replica_n.split(",") if v]:
        w = gen(n_el)
        t0 = time.perf_counter()
        geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM)
        torch.cuda.synchronize()
        row = {"N": int(geo.n), "setup_s": time.perf_counter() - t0}
        th = np.radians(w.angles_deg)
        for pc, key in ((1, "preconditioned"), (0, "plain")):
            t1 = time.perf_counter()
            phi, rep, st = geo.solve(th, tol=1e-8, max_iter=5000, restart=1000, precond=pc)
            torch.cuda.synchronize()
            row[key] = {"iterations": int(rep[0][0]), "solve_s": time.perf_counter() - t1, "status": int(st)}
            if pc == 1:
                ffs.append(geo.far_field(phi, obs).cpu().numpy()[0])
        _log(f"{which} N={geo.n}: its {row['preconditioned']['iterations']} / {row['plain']['iterations']}")
        rows.append(row)
        geo.close()
        torch.cuda.empty_cache()
    for i in range(len(rows) - 1):
        rows[i]["far_field_diff_to_next"] = _rel(ffs[i], ffs[i + 1])
    for i in range(1, len(rows) - 1):
        rows[i]["diff_ratio"] = rows[i - 1]["far_field_diff_to_next"] / rows[i]["far_field_diff_to_next"]
    print(json.dumps({"replica": which, "workload": gen.__doc__.split(":")[0].strip(), "rows": rows,
                      "paper_table": [dict(zip(("N", "its", "its_preconditioned", "time_s", "time_s_preconditioned"),
                                               r)) for r in table],
                      "paper_hardware": "not reported (CPU time)"}))


def replica_spectral(a):
    """The spectral Nystrom rule against the paper's lowest-order rule on
    smooth scatterers: 100 circles, ellipses and stars inside the three
    layers of the headline workload (none touching an interface), Dirichlet
    data of a unit point source at the centre of scatterer 0 (manufactured
    solution); per node count, both rules on the FMM with the
    preconditioner, FP64 (tol 1e-10) and the FP32 form (tol 1e-6): the far
    field's error against the source's, iterations and solve time."""
    import torch

    from paper_2511_12450_amd import lmfmm
    from paper_2511_12450_amd import workloads as wl

    torch.cuda.set_device(0)
    obs = lmfmm.far_field_angles()
    rows = []
    for n in [int(v) for v in a.replica_n.split(",") if v]:
        w = wl.three_layer_smooth(n_nodes=n)
        src = w.extra["source"]
        for quad, name in ((lmfmm.LM_QUAD_LOWEST, "lowest"), (lmfmm.LM_QUAD_SPECTRAL, "spectral")):
            t0 = time.perf_counter()
            geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, quad=quad)
            torch.cuda.synchronize()
            row = {"nodes_per_scatterer": n, "N": int(geo.n), "rule": name, "setup_s": time.perf_counter() - t0}
            exact = lmfmm.point_far_field(geo.layers, src, obs).cpu().numpy()[0]
            g = geo.point_source_rhs(src)
            for prec, tol, key in ((lmfmm.LM_FP64, 1e-10, "fp64"), (lmfmm.LM_MIXED, 1e-6, "fp32")):
                geo.solve_rhs(g, tol=tol, max_iter=3000, restart=500, precision=prec)  # warm-up
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                phi, rep, st = geo.solve_rhs(g, tol=tol, max_iter=3000, restart=500, precision=prec)
                torch.cuda.synchronize()
                ff = geo.far_field(phi, obs).cpu().numpy()[0]
                row[key] = {"iterations": int(rep[0][0]), "solve_s": time.perf_counter() - t1, "status": int(st),
                            "far_field_err_l2": _rel(ff, exact),
                            "far_field_err_linf": float(np.abs(ff - exact).max() / np.abs(exact).max())}
            _log(f"spectral replica n={n} {name}: N={geo.n}, err fp64 {row['fp64']['far_field_err_linf']:.2e} "
                 f"fp32 {row['fp32']['far_field_err_linf']:.2e}, its {row['fp64']['iterations']}, "
                 f"solve {row['fp64']['solve_s']:.3f} / {row['fp32']['solve_s']:.3f} s")
            rows.append(row)
            geo.close()
            torch.cuda.empty_cache()
    print(json.dumps({"replica": "spectral", "workload": wl.three_layer_smooth.__doc__.replace("\n", " "),
                      "rows": rows}))


def main():
    a = _args()
    if a.replica:
        if a.replica == "example1":
            replica_example1(a)
        elif a.replica in ("example2", "example3"):
            replica_plane_wave(a, a.replica)
        elif a.replica == "spectral":
            replica_spectral(a)
        else:
            sys.exit(f"unknown replica {a.replica}")
        return
    if a.gpus != 1:
        print(json.dumps({"error": "lmfmm runs on one GPU; sharding across GPUs is not implemented",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    from paper_2511_12450_amd import workloads as wl

    w = wl.three_layer()
    # the oracle's sample runs on the host cores before the GPU is touched
    cpu_t = None if a.no_cpu_baseline else cpu_baseline_time(w, a.cpu_seconds)
    if cpu_t:
        _log(f"oracle: {cpu_t['rows']} rows in {cpu_t['wall_s']:.1f} s on {cpu_t['cores']} cores")

    import torch

    from paper_2511_12450_amd import lmfmm

    torch.cuda.set_device(0)
    obs = lmfmm.far_field_angles()
    t0 = time.perf_counter()
    # default preconditioner: the coarsest subdomain level that fits
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, p=w.p)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    _log(f"geometry ready in {setup_s:.1f} s")
    N = geo.n
    th_all = np.radians(np.linspace(10.0, 170.0, a.angles))
    gm = dict(tol=w.tol, max_iter=3000, restart=a.restart)

    # tight FP64 reference of every angle, solved together (untimed)
    tr0 = time.perf_counter()
    fref = np.zeros((a.angles, obs.size), dtype=complex)
    for c0 in range(0, a.angles, 64):
        pr, rr, _ = geo.solve(th_all[c0:c0 + 64], tol=1e-9, max_iter=3000, restart=a.restart)
        fref[c0:c0 + 64] = geo.far_field(pr, obs).cpu().numpy()
        del pr
    _log(f"FP64 reference of {a.angles} angles (tol 1e-9) in {time.perf_counter() - tr0:.1f} s")

    # ---- plain FP64 form: single solves, one after another -----------------------
    def plain(th):
        phi, rep, st = geo.solve(np.array([th]), precision=lmfmm.LM_FP64, precond=1, **gm)
        ff = geo.far_field(phi, obs)
        torch.cuda.synchronize()
        return rep[0], st, ff.cpu().numpy()[0]

    plain_idx = [int(v) for v in np.linspace(0, a.angles - 1, a.plain_solves).round()]
    for _ in range(a.warmup):
        plain(th_all[plain_idx[0]])
    lat_p, its_p, err_p = [], [], []
    tp = time.perf_counter()
    for k in plain_idx:
        t1 = time.perf_counter()
        rep, st, ff = plain(th_all[k])
        lat_p.append(time.perf_counter() - t1)
        its_p.append(rep[0])
        err_p.append(_rel(ff, fref[k]))
    plain_s = time.perf_counter() - tp
    _log(f"plain FP64: {a.plain_solves} solves in {plain_s:.2f} s")

    # ---- served FP32 form: batches through the serving loop ----------------------
    per = max(1, a.angles // a.requests)

    def served(srv, steps, warmup):
        for _ in range(warmup):  # warm-up batches have the timed batch's shape
            for rid in [srv.submit(geo, th_all[i:i + per], obs_rad=obs, **gm) for i in range(0, a.angles, per)]:
                srv.wait(rid, results=False)
                srv.release(rid)
        ph0, st0 = srv.phase_times(), srv.stats()
        lat, its, err = [], [], np.zeros(a.angles)
        t_0 = time.perf_counter()
        for _ in range(steps):
            ids = [(srv.submit(geo, th_all[i:i + per], obs_rad=obs, **gm), i) for i in range(0, a.angles, per)]
            for rid, i0 in ids:
                st, status, lt, rep, phi, ff = srv.wait(rid)
                assert st == lmfmm.LM_DONE, (st, status)
                lat.append(lt)
                its += [r[0] for r in rep]
                for r in range(len(rep)):
                    err[i0 + r] = max(err[i0 + r], _rel(ff[r], fref[i0 + r]))
                srv.release(rid)
        span = time.perf_counter() - t_0
        ph1, st1 = srv.phase_times(), srv.stats()
        return span, lat, its, err, {k: ph1[k] - ph0[k] for k in ph1}, st0, st1

    srv = lmfmm.Server(precision=lmfmm.LM_MIXED, max_active_rhs=max(64, a.angles))
    served_s, lat_s, its_s, err_s, ph, st0, st1 = served(srv, a.steps, a.warmup)
    srv.close()
    n_served = a.steps * a.angles
    _log(f"served FP32: {n_served} solves in {served_s:.2f} s")
    # the same batch with the preconditioner applied from its FP64 rows
    srv = lmfmm.Server(precision=lmfmm.LM_MIXED, max_active_rhs=max(64, a.angles), precond_fp64=True)
    served64_s, _, its_s64, err_s64, ph64, _, _ = served(srv, 1, 0)
    srv.close()
    _log(f"served FP32 with the FP64 preconditioner: {a.angles} solves in {served64_s:.2f} s")

    # ---- served FP32 form under an open-loop stream: Poisson arrivals at
    # rho x the capacity just measured, 1..max angles per request drawn from the
    # batch's angle grid; latency per request from submit to done
    stream = None
    if a.stream_requests > 0:
        rng = np.random.default_rng(7)
        cap = n_served / served_s
        n_ang = rng.integers(1, a.stream_max_angles + 1, size=a.stream_requests)
        rate = a.stream_rho * cap / float(np.mean(n_ang))  # requests per second
        t_arr = np.cumsum(rng.exponential(1.0 / rate, size=a.stream_requests))
        picks = [np.sort(rng.choice(a.angles, size=int(k), replace=False)) for k in n_ang]
        srv2 = lmfmm.Server(precision=lmfmm.LM_MIXED, max_active_rhs=max(64, a.angles))

        def ref_err(k, ff):
            return [_rel(ff[r_], fref[ai]) for r_, ai in enumerate(picks[k])]

        lat_q, its_q, err_q, span = _pool_stream(lmfmm, srv2, [geo], np.zeros(a.stream_requests, dtype=int),
                                                 [th_all[p_] for p_ in picks], t_arr, obs, lambda g_: gm, ref_err)
        srv2.close()
        keep = [lat_q[k] for k in range(50, a.stream_requests)] if a.stream_requests > 100 else list(lat_q.values())
        stream = {"requests": a.stream_requests, "warmup_requests_excluded": 50 if a.stream_requests > 100 else 0,
                  "rho": a.stream_rho, "arrival_rate_solves_s": float(rate * np.mean(n_ang)),
                  "angles_per_request": [1, a.stream_max_angles], "solves": int(np.sum(n_ang)),
                  "solves_per_s": float(np.sum(n_ang) / span),
                  "p50_s": float(np.percentile(keep, 50)), "p99_s": float(np.percentile(keep, 99)),
                  "iterations_min_max": [int(min(its_q)), int(max(its_q))],
                  "rel_err_far_field_max": float(max(err_q)), "checked_solves": len(err_q)}
        _log(f"stream: {a.stream_requests} requests in {span:.1f} s, p50 {stream['p50_s']:.3f} s, "
             f"p99 {stream['p99_s']:.3f} s")

    # ---- streams over a pool of geometries (different media and sizes, 1-16
    # angles per request, admission by HBM footprint): the pool's served
    # capacity from a closed batch, then Poisson streams at fractions of it
    pool = None
    if a.pool_geometries > 0:
        ws = [wl.stream_geometry(g) for g in range(a.pool_geometries)]
        t0p = time.perf_counter()
        pgeos = [lmfmm.Geometry.from_workload(w_, method=lmfmm.LM_FMM, p=w_.p) for w_ in ws]
        pool_setup = time.perf_counter() - t0p
        _log(f"pool: {len(ws)} geometries (N {min(w_.n_elements for w_ in ws)}..{max(w_.n_elements for w_ in ws)}) "
             f"ready in {pool_setup:.1f} s")
        budget = int(0.8 * torch.cuda.mem_get_info()[0])
        rng = np.random.default_rng(11)
        gmp = lambda g_: gm  # noqa: E731
        # closed batch: one request of 8 angles per geometry, all at once
        srvc = lmfmm.Server(precision=lmfmm.LM_MIXED, hbm_budget_bytes=budget)
        thc = [np.radians(np.linspace(20.0, 160.0, 8)) for _ in pgeos]
        latc, itsc, _, spanc = _pool_stream(lmfmm, srvc, pgeos, list(range(len(pgeos))), thc,
                                            np.zeros(len(pgeos)), obs, gmp)
        srvc.close()
        cap_pool = 8 * len(pgeos) / spanc
        _log(f"pool: closed batch of {8 * len(pgeos)} solves in {spanc:.1f} s ({cap_pool:.1f} solves/s)")
        runs = []
        rhos = [float(v) for v in a.pool_rho.split(",") if v]
        plan = [(r_, budget, a.restart) for r_ in rhos]
        if a.pool_budget_gb > 0:
            plan.append((rhos[0], int(a.pool_budget_gb * 2 ** 30), 100))
        for rho, bud, rst in plan:
            nq = a.pool_requests
            gi = rng.integers(0, len(pgeos), size=nq)
            na = rng.integers(1, 17, size=nq)
            th_q = [np.radians(rng.uniform(10.0, 170.0, size=int(k))) for k in na]
            rate = rho * cap_pool / float(np.mean(na))
            t_arr = np.cumsum(rng.exponential(1.0 / rate, size=nq))
            gmr = dict(gm, restart=rst)
            srv3 = lmfmm.Server(precision=lmfmm.LM_MIXED, hbm_budget_bytes=bud)
            lat_g, its_g, _, span = _pool_stream(lmfmm, srv3, pgeos, gi, th_q, t_arr, obs, lambda g_: gmr)
            mem = srv3.memory()
            srv3.close()
            keep = [lat_g[k] for k in range(nq // 10, nq)]
            runs.append({"rho": rho, "hbm_budget_bytes": bud, "gmres_restart": rst, "requests": nq,
                         "warmup_requests_excluded": nq // 10, "arrival_rate_solves_s": float(rate * np.mean(na)),
                         "solves": int(np.sum(na)), "solves_per_s": float(np.sum(na) / span), "span_s": span,
                         "p50_s": float(np.percentile(keep, 50)), "p99_s": float(np.percentile(keep, 99)),
                         "iterations_min_max": [int(min(its_g)), int(max(its_g))],
                         "server_bytes_at_end": mem["held"]})
            _log(f"pool rho {rho}: {nq} requests, {int(np.sum(na))} solves in {span:.1f} s, "
                 f"p50 {runs[-1]['p50_s']:.3f} s, p99 {runs[-1]['p99_s']:.3f} s")
        for g_ in pgeos:
            g_.close()
        pool = {"geometries": [w_.name for w_ in ws], "layers": [int(len(w_.k)) for w_ in ws],
                "N": [int(w_.n_elements) for w_ in ws], "setup_s": pool_setup, "angles_per_request": [1, 16],
                "capacity_solves_s": cap_pool, "capacity_batch": f"{len(pgeos)} requests of 8 angles, one per geometry",
                "runs": runs}

    # ---- kernel rooflines (HIP events on the launch stream, inside the timed batch)
    stats = geo.fmm_stats()
    rounds = st1["rounds"] - st0["rounds"]
    m2l_avg_s = ph["m2l_ms"] * 1e-3 / max(ph["m2l_launches"], 1)
    m2l_flops = ph["m2l_flops"] / max(ph["m2l_launches"], 1)
    m2l_roof = {"bound": "mfma", "achieved": m2l_flops / m2l_avg_s / 1e12, "peak": PEAK_FP32_MFMA_TFLOPS,
                "unit": "TFLOP/s", "traffic": None, "kernel": "k_m2l_mfma<4, 1, 0, true> (M2L lists)",
                "kernel_avg_us": m2l_avg_s * 1e6, "launches": int(ph["m2l_launches"]),
                "algorithmic_flops_per_launch": m2l_flops,
                "entries": stats["m2l_free_entries"] + stats["m2l_reaction_entries"]}
    m2l_roof["frac"] = m2l_roof["achieved"] / PEAK_FP32_MFMA_TFLOPS
    gs_avg_s = ph["gs_ms"] * 1e-3 / max(rounds, 1)
    gs_bytes = ph["gs_bytes"] / max(rounds, 1)
    gs_roof = {"bound": "hbm", "achieved": gs_bytes / gs_avg_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
               "traffic": None, "kernel": "k_s_dots2 + k_s_update2 (delayed CGS2; + k_s_dots2_final, k_s_resid, k_s_norm_final, k_s_norm_to)",
               "kernel_avg_us": gs_avg_s * 1e6, "launches": int(rounds), "algorithmic_bytes_per_launch": gs_bytes}
    gs_roof["frac"] = gs_roof["achieved"] / PEAK_HBM_GBS
    tr = _traffic()
    if tr is not None:
        m2l_roof["traffic"] = tr["k_m2l_mfma_list"]["hbm_bytes_per_launch"]
        gs_roof["traffic"] = tr["cgs2_phase"]["hbm_bytes_per_round"]
    # the dominant single kernel of the served step is the M2L; the CGS2 phase
    # (several kernels) is reported beside it
    roof, other = m2l_roof, gs_roof
    x1 = torch.from_numpy(wl.random_vector(N, seed=1, n_rhs=1)).cuda()
    y1 = torch.empty_like(x1)
    t_fp64 = geo.stage_times(x1, y1, reps=10, precision=lmfmm.LM_FP64)
    R = min(64, a.angles)
    x = torch.from_numpy(wl.random_vector(N, seed=1, n_rhs=R)).to(torch.complex64).cuda()
    y = torch.empty_like(x)
    t_mix = geo.stage_times(x, y, reps=5, precision=lmfmm.LM_MIXED)
    # near field (the P2P step): leaf blocks on matrix cores at R = 64 (FP32),
    # the FP64 CSR at R = 1; stage 5, HIP events on the near-field stream
    pairs = stats["free_near_pairs"] + stats["reaction_near_pairs"]
    p2p = [{"bound": "mfma", "kernel": "k_block_mfma (free-space near field + self terms, leaf blocks) + "
                                       "k_near_csr (reaction near pairs), FP32, R = 64",
            "near_pairs": pairs, "algorithmic_flops_per_launch": 8.0 * R * pairs, "kernel_avg_us": 1e3 * t_mix[5],
            "achieved": 8.0 * R * pairs / (1e-3 * t_mix[5]) / 1e12, "peak": PEAK_FP32_MFMA_TFLOPS,
            "unit": "TFLOP/s"},
           {"bound": "hbm", "kernel": "k_near_csr<double, 4> (near field + self terms, CSR), FP64, R = 1",
            "near_pairs": pairs, "algorithmic_bytes_per_launch": 20.0 * pairs + 32.0 * N,
            "kernel_avg_us": 1e3 * t_fp64[5],
            "achieved": (20.0 * pairs + 32.0 * N) / (1e-3 * t_fp64[5]) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}]
    for e in p2p:
        e["frac"] = e["achieved"] / e["peak"]

    cfg = {"workload": w.name, "N": int(N), "layers": int(len(w.k)), "k": [float(v) for v in w.k], "p": int(w.p),
           "gmres_tol": w.tol, "gmres_restart": a.restart, "preconditioner": "overlapping DD (Sec. 4.2), default subdomain level (coarsest that fits)",
           "served": {"angles_per_step": a.angles, "requests_per_step": len(range(0, a.angles, per)),
                      "angles_per_request": per, "far_field_angles": int(obs.size),
                      "iterations_min_max": [int(min(its_s)), int(max(its_s))], "rounds": int(rounds),
                      "fused_rhs_per_launch": (st1["fused_rhs"] - st0["fused_rhs"]) /
                                              max(1, st1["launches"] - st0["launches"]),
                      "km_phase_ms": ph["km_ms"], "gs_phase_ms": ph["gs_ms"], "m2l_ms": ph["m2l_ms"],
                      "round_host_ms": ph["round_ms"], "finish_host_ms": ph["finish_ms"],
                      "round_queue_ms": ph["launch_ms"], "round_wait_ms": ph["wait_ms"],
                      "round_step_ms": ph["step_ms"]},
           "setup_s": setup_s, "device_bytes": int(geo.device_bytes), "fmm": stats,
           "matvec_fp32_R64_ms": float(t_mix[7]),
           "matvec_fp32_R64_stage_ms": {s_: float(t) for s_, t in zip(STAGES, t_mix) if s_ != "total"},
           "matvec_fp64_R1_ms": float(t_fp64[7]),
           "matvec_fp64_R1_stage_ms": {s_: float(t) for s_, t in zip(STAGES, t_fp64) if s_ != "total"}}
    errs_all = list(err_s) + (([stream["rel_err_far_field_max"]]) if stream else [])
    out = {
        "metric": "GMRES solves/sec + p50/p99 latency, served FP32 vs plain FP64, at rel err 1e-4",
        "value": n_served / served_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * served_s / a.steps,
        # per-request latency over the open-loop stream (requests 50.. of 550),
        # else over the timed batch
        "p50_s": stream["p50_s"] if stream else float(np.percentile(lat_s, 50)),
        "p99_s": stream["p99_s"] if stream else float(np.percentile(lat_s, 99)),
        "batch_p50_s": float(np.percentile(lat_s, 50)),
        "batch_p99_s": float(np.percentile(lat_s, 99)),
        "rel_err_far_field_max": float(max(errs_all)),
        "rel_err_far_field_per_angle": [float(f"{v:.3g}") for v in err_s],
        "stream": stream,
        "pool_stream": pool,
        "served_fp64_preconditioner": {"value": a.angles / served64_s, "unit": "solves/s", "solves": a.angles,
                                       "iterations_min_max": [int(min(its_s64)), int(max(its_s64))],
                                       "rel_err_far_field_max": float(max(err_s64)),
                                       "km_phase_ms": ph64["km_ms"]},
        "plain_fp64": {"value": a.plain_solves / plain_s, "unit": "solves/s", "solves": a.plain_solves,
                       "p50_s": float(np.percentile(lat_p, 50)), "p99_s": float(np.percentile(lat_p, 99)),
                       "iterations": [int(v) for v in its_p], "rel_err_far_field_max": float(max(err_p))},
        "speedup_served_vs_plain": (n_served / served_s) / (a.plain_solves / plain_s),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "precision_split": ("f32 translations and near field (matrix cores, f32 accumulation); binary16 preconditioner "
                            "products on a split input (fixed operator, f32 accumulation; served_fp64_preconditioner "
                            "is the same form with the FP64 preconditioner rows); complex64 Krylov basis storage; f64 "
                            "Arnoldi and Givens arithmetic, spectral tables and self terms"),
        "data": "synthetic",
        "config": cfg,
        "roofline": roof,
        "roofline_other": other,
        "roofline_p2p": p2p,
    }
    if cpu_t:
        out["cpu_baseline"] = cpu_baseline(w, cpu_t, int(np.median(its_p)))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
