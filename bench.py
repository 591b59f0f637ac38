"""Benchmark: GMRES solves/sec (+ p50/p99 latency) of the layered-medium
Nystrom solver on one MI355X.

A step is one complete solve of the hot path for one incidence angle on a
geometry whose operator data (trees, Sommerfeld M2L tables, near-field
entries, preconditioner) are already resident in HBM: right-hand side ->
preconditioned GMRES (layered FMM matvec inside) -> far-field pattern on 682
angles.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Workloads: three_layer (default: 3 layers, k = (5,7,4), 400 scatterers,
N = 64,000, p = 20, GMRES tol 1e-6 with the domain-decomposition
preconditioner) and plain_small (2 layers, N = 256, dense matrix).
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
PEAK_FP64_VALU_TFLOPS = 78.6
STAGES = ("P2M", "M2M", "M2L", "L2L", "L2P", "near", "unused")
KERNEL_OF_STAGE = {"P2M": "k_p2m", "M2M": "k_m2m", "M2L": "k_m2l_apply+k_m2l_reduce", "L2L": "k_l2l",
                   "L2P": "k_l2p", "near": "k_near_csr"}


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="three_layer")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def _workload(name):
    from paper_2511_12450_amd import workloads as wl

    if name == "three_layer":
        return wl.three_layer(), "fmm"
    if name == "plain_small":
        return wl.plain_small(), "dense"
    raise SystemExit(f"unknown workload {name}")


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
            "sample": (f"{done} rows of the dense matrix of {w.name} ({row_s:.2f} s/row on one core); "
                       f"solve projected as {n} rows + {iterations + 1} dense matvecs = {projected:.3g} s "
                       "(projected, not run)")}


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is a design only (DESIGN.md)",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    from paper_2511_12450_amd import lmfmm

    torch.cuda.set_device(0)
    w, kind = _workload(a.workload)
    th = np.radians(w.angles_deg[:1])
    obs = lmfmm.far_field_angles()
    t0 = time.perf_counter()
    method = lmfmm.LM_DENSE if kind == "dense" else lmfmm.LM_FMM
    geo = lmfmm.Geometry.from_workload(w, method=method, p=w.p, precond=1 if kind == "fmm" else 0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    opts = dict(tol=w.tol, max_iter=2000, restart=500, precond=1 if kind == "fmm" else 0)

    def step():
        phi, rep, st = geo.solve(th, **opts)
        ff = geo.far_field(phi, obs)
        return phi, rep, st, ff

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    for _ in range(a.steps):
        t1 = time.perf_counter()
        phi, rep, st, ff = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t1)
    elapsed = time.perf_counter() - t_start
    iters = int(rep[0][0])

    x = torch.from_numpy(np.exp(1j * np.linspace(0, 50, geo.n))[None, :].copy()).cuda()
    y = torch.empty_like(x)
    N = geo.n
    P = 2 * w.p + 1
    cfg = {"workload": w.name, "N": int(N), "layers": int(len(w.k)), "k": [float(v) for v in w.k],
           "method": kind, "p": int(w.p), "angle_deg": float(w.angles_deg[0]), "gmres_tol": w.tol,
           "gmres_iterations": iters, "converged": st == 0, "rel_residual": float(rep[0][1]),
           "setup_s": setup_s, "device_bytes": int(geo.device_bytes)}
    if kind == "fmm":
        stats = geo.fmm_stats()
        cfg["fmm"] = stats
        times = geo.stage_times(x, y, reps=10)
        cfg["matvec_ms"] = float(times[7])
        cfg["stage_ms"] = {s_: float(t) for s_, t in zip(STAGES, times[:7])}
        dom = STAGES[int(np.argmax(times[:7]))]
        t_dom = float(times[STAGES.index(dom)]) * 1e-3
        if dom == "M2L":
            # each list entry: one (2p+1)^2 operator applied to one expansion
            n_e = stats["m2l_free_entries"] + stats["m2l_reaction_entries"]
            flops = 8.0 * P * P * n_e
            bytes_ = (16.0 * P * P * stats["reaction_tables"] + 16.0 * (4 * w.p + 1) * stats["free_classes"]
                      + 16.0 * P * n_e + 16.0 * P * stats["boxes"])
        elif dom == "near":
            nnz = stats["free_near_pairs"] - N + stats["reaction_near_pairs"] + N
            flops = 8.0 * nnz
            bytes_ = 20.0 * nnz + 16.0 * 3 * N + 4.0 * N  # value + column index, x gather, y read/write, row ptr
        else:
            flops, bytes_ = float("nan"), float("nan")
        intensity = flops / bytes_
        ridge = PEAK_FP64_VALU_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
        if intensity < ridge:
            roof = {"bound": "hbm", "achieved": bytes_ / t_dom / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
        else:
            roof = {"bound": "alu", "achieved": flops / t_dom / 1e12, "peak": PEAK_FP64_VALU_TFLOPS,
                    "unit": "TFLOP/s"}
        roof["frac"] = roof["achieved"] / roof["peak"]
        roof["traffic"] = None
        roof.update({"stage": dom, "kernel": KERNEL_OF_STAGE[dom], "kernel_avg_us": t_dom * 1e6,
                     "algorithmic_bytes_per_launch": bytes_, "algorithmic_flops_per_launch": flops})
    else:
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(5):
            geo.matvec(x, y)
        ev0.record()
        for _ in range(200):
            geo.matvec(x, y)
        ev1.record()
        torch.cuda.synchronize()
        t_dom = ev0.elapsed_time(ev1) / 1e3 / 200
        bytes_ = 16.0 * N * N + 32.0 * N
        roof = {"bound": "hbm", "achieved": bytes_ / t_dom / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": bytes_ / t_dom / 1e9 / PEAK_HBM_GBS, "traffic": None, "kernel": "k_dense_gemv",
                "kernel_avg_us": t_dom * 1e6, "algorithmic_bytes_per_launch": bytes_}

    out = {
        "metric": "GMRES solves/sec (plain FP64 single-solve form)",
        "value": a.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": cfg,
        "roofline": roof,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, iters, a.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
