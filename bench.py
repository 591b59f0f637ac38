"""Benchmark: GMRES solves/sec (+ p50/p99 latency) of the layered-medium
Nystrom solver on one MI355X.

A step is one complete solve of the hot path for one incidence angle:
right-hand side -> GMRES (matvec inside) -> far-field pattern, on a geometry
whose operator data are already resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plain_small")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def _workload(name):
    from paper_2511_12450_amd import workloads as wl

    if name == "plain_small":
        return wl.plain_small(), "dense"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(w, theta):
    """The oracle as it stands on the host: dense assembly + LU + far field
    for one angle of the same workload, on one thread."""
    from threadpoolctl import threadpool_limits

    from oracle.farfield import far_field
    from oracle.incident import boundary_data
    from oracle.medium import Medium
    from oracle.nystrom import Elements, matrix
    from oracle.solve import lu_solve
    from paper_2511_12450_amd import lmfmm

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        med = Medium(w.d, w.k, w.eta)
        el = Elements(med, w.polygons)
        K = matrix(med, el)
        phi = lu_solve(K, boundary_data(med, theta, el.cx, el.cy))
        ff = far_field(med, el, phi, lmfmm.far_field_angles())
        dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"one full solve of {w.name} (assembly + LU + 682 far-field angles), {dt:.2f} s"}, ff


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is a design only (see DESIGN.md)"}))
        sys.exit(2)
    import torch

    from paper_2511_12450_amd import lmfmm

    torch.cuda.set_device(0)
    w, kind = _workload(a.workload)
    th = np.radians(w.angles_deg[:1])
    obs = lmfmm.far_field_angles()
    t0 = time.perf_counter()
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_DENSE if kind == "dense" else lmfmm.LM_FMM)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    opts = dict(tol=w.tol, max_iter=1000, restart=300, precond=1)

    def step():
        phi, rep, st = geo.solve(th, **opts)
        ff = geo.far_field(phi, obs)
        return phi, rep, ff

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    for _ in range(a.steps):
        t1 = time.perf_counter()
        phi, rep, ff = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    iters = rep[0][0]

    # dominant kernel: the operator apply (dense: one GEMV launch per matvec),
    # timed with events on the stream it runs on
    x = torch.randn((1, geo.n), dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        geo.matvec(x, y)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 200
    ev0.record()
    for _ in range(reps):
        geo.matvec(x, y)
    ev1.record()
    torch.cuda.synchronize()
    mv_s = ev0.elapsed_time(ev1) / 1e3 / reps
    N = geo.n
    alg_bytes = 16.0 * N * N + 2 * 16.0 * N
    achieved = alg_bytes / mv_s / 1e9

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
        "config": {"workload": w.name, "N": int(N), "layers": int(len(w.k)), "method": kind,
                   "angle_deg": float(w.angles_deg[0]), "gmres_tol": w.tol, "gmres_iterations": int(iters),
                   "setup_s": setup_s},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None, "kernel": "k_dense_gemv",
                     "kernel_avg_us": mv_s * 1e6, "algorithmic_bytes_per_launch": alg_bytes},
    }
    if not a.no_cpu_baseline:
        cb, ff_ref = cpu_baseline(w, th[0])
        out["cpu_baseline"] = cb
        ffg = ff.cpu().numpy()[0]
        out["far_field_rel_err_vs_oracle"] = float(np.linalg.norm(ffg - ff_ref) / np.linalg.norm(ff_ref))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
