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
  request, submission to completion.

Both forms are checked against a tight FP64 reference (tol 1e-9, computed
outside the timed region) on four of the angles: the far-field relative
error of each form is reported (bar 1e-4).

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
    ap.add_argument("--plain-solves", type=int, default=4)
    ap.add_argument("--restart", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stream-requests", type=int, default=550,
                    help="requests of the open-loop Poisson stream (0: skip); the first 50 are warm-up")
    ap.add_argument("--stream-rho", type=float, default=0.5, help="arrival rate as a fraction of the served capacity")
    ap.add_argument("--stream-max-angles", type=int, default=4)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--pool-geometries", type=int, default=0,
                    help="also serve an open-loop stream over this many pool geometries (2-4 layers, "
                         "N in [4,000, 250,000], 1-16 angles per request); 0: skip")
    ap.add_argument("--pool-requests", type=int, default=60)
    ap.add_argument("--pool-rate", type=float, default=0.35, help="requests per second of the pool stream")
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


def cpu_baseline(w, iterations, budget_s):
    """The oracle as it stands on one host core: rows of the dense Nystrom
    matrix by direct Sommerfeld quadrature, timed until budget_s has passed;
    the full solve is projected as N rows of assembly plus (iterations + 1)
    dense matvecs."""
    from threadpoolctl import threadpool_limits

    from oracle.medium import Medium
    from oracle.nystrom import Elements, matrix_rows

    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    rng = np.random.default_rng(0)
    rows = rng.permutation(el.n)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        done = 0
        K = None
        while done == 0 or time.perf_counter() - t0 < budget_s:
            K = matrix_rows(med, el, [int(rows[done])])
            done += 1
            if done >= el.n:
                break
        row_s = (time.perf_counter() - t0) / done
        x = np.ones(el.n, dtype=complex)
        t1 = time.perf_counter()
        for _ in range(20):
            K @ x
        gemv_row_s = (time.perf_counter() - t1) / 20
    n = el.n
    projected = n * row_s + (iterations + 1) * n * gemv_row_s
    return {"value": 1.0 / projected, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"{done} rows of the dense FP64 matrix of {w.name} by direct Sommerfeld quadrature "
                       f"({row_s:.2f} s/row on one core); one solve projected as {n} rows + "
                       f"{iterations + 1} dense matvecs = {projected:.3g} s (projected, not run)")}


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "lmfmm runs on one GPU; sharding across GPUs is not implemented",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    from paper_2511_12450_amd import lmfmm
    from paper_2511_12450_amd import workloads as wl

    torch.cuda.set_device(0)
    w = wl.three_layer()
    obs = lmfmm.far_field_angles()
    t0 = time.perf_counter()
    # default preconditioner: the coarsest subdomain level that fits
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, p=w.p)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    _log(f"geometry ready in {setup_s:.1f} s")
    N, P = geo.n, 2 * w.p + 1
    th_all = np.radians(np.linspace(10.0, 170.0, a.angles))
    ref_idx = list(range(0, a.angles, max(1, a.angles // 4)))[:4]
    gm = dict(tol=w.tol, max_iter=3000, restart=a.restart)

    # tight FP64 reference (untimed)
    pr, rr, _ = geo.solve(th_all[ref_idx], tol=1e-9, max_iter=3000, restart=a.restart)
    fref = geo.far_field(pr, obs).cpu().numpy()
    del pr

    # ---- plain FP64 form: single solves, one after another -----------------------
    def plain(th):
        phi, rep, st = geo.solve(np.array([th]), precision=lmfmm.LM_FP64, precond=1, **gm)
        ff = geo.far_field(phi, obs)
        torch.cuda.synchronize()
        return rep[0], st, ff.cpu().numpy()[0]

    for _ in range(a.warmup):
        plain(th_all[ref_idx[0]])
    lat_p, its_p, err_p = [], [], []
    tp = time.perf_counter()
    for i in range(a.plain_solves):
        k = ref_idx[i % len(ref_idx)]
        t1 = time.perf_counter()
        rep, st, ff = plain(th_all[k])
        lat_p.append(time.perf_counter() - t1)
        its_p.append(rep[0])
        err_p.append(_rel(ff, fref[ref_idx.index(k)]))
    plain_s = time.perf_counter() - tp
    _log(f"plain FP64: {a.plain_solves} solves in {plain_s:.2f} s")

    # ---- served FP32 form: batches through the serving loop ----------------------
    srv = lmfmm.Server(precision=lmfmm.LM_MIXED, max_active_rhs=max(64, a.angles))
    per = max(1, a.angles // a.requests)
    for _ in range(a.warmup):  # warm-up batches have the timed batch's shape
        for rid in [srv.submit(geo, th_all[i:i + per], obs_rad=obs, **gm) for i in range(0, a.angles, per)]:
            srv.wait(rid, results=False)
            srv.release(rid)
    ph0 = srv.phase_times()
    st0 = srv.stats()
    lat_s, its_s, err_s = [], [], []
    tsrv = time.perf_counter()
    for _ in range(a.steps):
        ids = [(srv.submit(geo, th_all[i:i + per], obs_rad=obs, **gm), i) for i in range(0, a.angles, per)]
        for rid, i0 in ids:
            st, status, lat, rep, phi, ff = srv.wait(rid)
            assert st == lmfmm.LM_DONE, (st, status)
            lat_s.append(lat)
            its_s += [r[0] for r in rep]
            for r in range(len(rep)):
                if i0 + r in ref_idx:
                    err_s.append(_rel(ff[r], fref[ref_idx.index(i0 + r)]))
            srv.release(rid)
    served_s = time.perf_counter() - tsrv
    ph1 = srv.phase_times()
    ph = {k: ph1[k] - ph0[k] for k in ph1}
    st1 = srv.stats()
    srv.close()
    n_served = a.steps * a.angles
    _log(f"served FP32: {n_served} solves in {served_s:.2f} s")

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
        pend, lat_q, err_q, its_q = {}, {}, [], []
        i, t0s = 0, time.perf_counter()
        while i < len(t_arr) or pend:
            now = time.perf_counter() - t0s
            while i < len(t_arr) and t_arr[i] <= now:
                pend[srv2.submit(geo, th_all[picks[i]], obs_rad=obs, **gm)] = i
                i += 1
            for rid in list(pend):
                out_q = srv2.poll(rid, results=True)
                if out_q[0] in (lmfmm.LM_DONE, lmfmm.LM_FAILED, lmfmm.LM_CANCELLED):
                    assert out_q[0] == lmfmm.LM_DONE, out_q[:2]
                    k = pend.pop(rid)
                    lat_q[k] = out_q[2]
                    its_q += [r_[0] for r_ in out_q[3]]
                    for r_, ai in enumerate(picks[k]):
                        if ai in ref_idx:
                            err_q.append(_rel(out_q[5][r_], fref[ref_idx.index(ai)]))
                    srv2.release(rid)
            time.sleep(0.0005)
        span = time.perf_counter() - t0s
        srv2.close()
        keep = [lat_q[k] for k in range(50, a.stream_requests)] if a.stream_requests > 100 else list(lat_q.values())
        stream = {"requests": a.stream_requests, "warmup_requests_excluded": 50 if a.stream_requests > 100 else 0,
                  "rho": a.stream_rho, "arrival_rate_solves_s": float(rate * np.mean(n_ang)),
                  "angles_per_request": [1, a.stream_max_angles], "solves": int(np.sum(n_ang)),
                  "solves_per_s": float(np.sum(n_ang) / span),
                  "p50_s": float(np.percentile(keep, 50)), "p99_s": float(np.percentile(keep, 99)),
                  "iterations_min_max": [int(min(its_q)), int(max(its_q))],
                  "rel_err_far_field_max": float(max(err_q)) if err_q else None,
                  "checked_solves": len(err_q)}
        _log(f"stream: {a.stream_requests} requests in {span:.1f} s, p50 {stream['p50_s']:.3f} s, "
             f"p99 {stream['p99_s']:.3f} s")

    # ---- optional: a stream over several pool geometries (different media and
    # sizes, 1-16 angles per request, admission by HBM footprint)
    pool = None
    if a.pool_geometries > 0:
        ws = [wl.stream_geometry(g) for g in range(a.pool_geometries)]
        t0p = time.perf_counter()
        pgeos = [lmfmm.Geometry.from_workload(w_, method=lmfmm.LM_FMM, p=w_.p) for w_ in ws]
        _log(f"pool: {len(ws)} geometries (N {min(w_.n_elements for w_ in ws)}..{max(w_.n_elements for w_ in ws)}) "
             f"ready in {time.perf_counter() - t0p:.1f} s")
        rng = np.random.default_rng(11)
        nq = a.pool_requests
        gi = rng.integers(0, len(pgeos), size=nq)
        na = rng.integers(1, 17, size=nq)
        th_q = [np.radians(rng.uniform(10.0, 170.0, size=int(k))) for k in na]
        t_arr = np.cumsum(rng.exponential(1.0 / a.pool_rate, size=nq))
        srv3 = lmfmm.Server(precision=lmfmm.LM_MIXED, hbm_budget_bytes=int(160e9))
        pend, lat_g, its_g = {}, {}, []
        i, t0s = 0, time.perf_counter()
        while i < nq or pend:
            now = time.perf_counter() - t0s
            while i < nq and t_arr[i] <= now:
                pend[srv3.submit(pgeos[gi[i]], th_q[i], obs_rad=obs, **gm)] = i
                i += 1
            for rid in list(pend):
                out_q = srv3.poll(rid, results=True)
                if out_q[0] in (lmfmm.LM_DONE, lmfmm.LM_FAILED, lmfmm.LM_CANCELLED):
                    assert out_q[0] == lmfmm.LM_DONE, out_q[:2]
                    k = pend.pop(rid)
                    lat_g[k] = out_q[2]
                    its_g += [r_[0] for r_ in out_q[3]]
                    srv3.release(rid)
                    if len(lat_g) % 25 == 0:
                        _log(f"pool: {len(lat_g)} of {nq} requests done")
            time.sleep(0.0005)
        span = time.perf_counter() - t0s
        srv3.close()
        for g_ in pgeos:
            g_.close()
        keep = [lat_g[k] for k in range(nq // 10, nq)]
        pool = {"geometries": [w_.name for w_ in ws], "layers": [int(len(w_.k)) for w_ in ws],
                "requests": nq, "warmup_requests_excluded": nq // 10, "arrival_rate_requests_s": a.pool_rate,
                "angles_per_request": [1, 16], "solves": int(np.sum(na)),
                "solves_per_s": float(np.sum(na) / span), "span_s": span,
                "p50_s": float(np.percentile(keep, 50)), "p99_s": float(np.percentile(keep, 99)),
                "iterations_min_max": [int(min(its_g)), int(max(its_g))]}
        _log(f"pool: {nq} requests, {int(np.sum(na))} solves in {span:.1f} s, p50 {pool['p50_s']:.3f} s, "
             f"p99 {pool['p99_s']:.3f} s")

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

    cfg = {"workload": w.name, "N": int(N), "layers": int(len(w.k)), "k": [float(v) for v in w.k], "p": int(w.p),
           "gmres_tol": w.tol, "gmres_restart": a.restart, "preconditioner": "overlapping DD (Sec. 4.2), default subdomain level (coarsest that fits)",
           "served": {"angles_per_step": a.angles, "requests_per_step": len(range(0, a.angles, per)),
                      "angles_per_request": per, "far_field_angles": int(obs.size),
                      "iterations_min_max": [int(min(its_s)), int(max(its_s))], "rounds": int(rounds),
                      "fused_rhs_per_launch": (st1["fused_rhs"] - st0["fused_rhs"]) /
                                              max(1, st1["launches"] - st0["launches"]),
                      "km_phase_ms": ph["km_ms"], "gs_phase_ms": ph["gs_ms"], "m2l_ms": ph["m2l_ms"]},
           "setup_s": setup_s, "device_bytes": int(geo.device_bytes), "fmm": stats,
           "matvec_fp32_R64_ms": float(t_mix[7]),
           "matvec_fp32_R64_stage_ms": {s_: float(t) for s_, t in zip(STAGES, t_mix) if s_ != "total"},
           "matvec_fp64_R1_ms": float(t_fp64[7]),
           "matvec_fp64_R1_stage_ms": {s_: float(t) for s_, t in zip(STAGES, t_fp64) if s_ != "total"}}
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
        "rel_err_far_field_max": float(max(err_s + (stream["rel_err_far_field_max"] and [stream["rel_err_far_field_max"]] or []))) if stream else float(max(err_s)),
        "stream": stream,
        "pool_stream": pool,
        "plain_fp64": {"value": a.plain_solves / plain_s, "unit": "solves/s", "solves": a.plain_solves,
                       "p50_s": float(np.percentile(lat_p, 50)), "p99_s": float(np.percentile(lat_p, 99)),
                       "iterations": [int(v) for v in its_p], "rel_err_far_field_max": float(max(err_p))},
        "speedup_served_vs_plain": (n_served / served_s) / (a.plain_solves / plain_s),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "precision_split": ("f32 translations and near field (matrix cores, f32 accumulation); binary16 preconditioner "
                            "products on a split input (fixed operator, f32 accumulation); complex64 Krylov basis "
                            "storage; f64 Arnoldi and Givens arithmetic, spectral tables and self terms"),
        "data": "synthetic",
        "config": cfg,
        "roofline": roof,
        "roofline_other": other,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, int(np.median(its_p)), a.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
