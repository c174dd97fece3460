"""Benchmark: spin-updates/s of the whole replica-batched PA solve on one MI355X.

One benchmark step = one complete solve of the workload through the C ABI: App. A
canonicalisation + validation, initial state, all PA steps of App. B, exact FP64/int64
energies of every replica's final spins and the best-of-replica reduction.  Inputs are
uploaded to HBM before the timed region; value = n * replicas * PA-steps * K / seconds.

Default workload: dense SK n=4096, 1024 replicas, 2000 PA steps, couplings in BF16 on
the matrix cores (FP32 accumulation).  The same solve with FP32 couplings on the FP32
path is timed once beside it, and both best energies are compared in FP64 ("BF16 vs FP32
form at matched best energy").

    python bench.py [--steps K] [--warmup W] [--workload sk4096|chimera16|dense20|planted3r]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-updates/s (n×replicas×steps/s), BF16 vs FP32 form at matched best energy"
PEAK_BF16_TFLOPS = 2500.0     # MI355X dense BF16 matrix peak
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sk4096")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-form", action="store_true")
    return ap.parse_args()


def cpu_baseline(inst, wl, prec):
    """The CPU oracle (untuned) on a bounded replica x step sample of the same workload,
    replicas split over host threads (the oracle releases the GIL)."""
    import oracle as orc
    cores = max(1, min(16, os.cpu_count() or 1))
    n = inst.n
    if inst.dense is not None and not np.issubdtype(inst.dense.dtype, np.integer):
        J = inst.dense
        if prec == "bf16":
            J = orc.bf16_quantise(J, orc.bf16_scale_exponent(J))
        reps, steps = 2 * cores, 40
        lam = orc.lambda_linear(wl.steps, wl.lambda0)

        def work(r0, cnt):
            x, m = orc.pa_init(n, cnt, wl.seed, np.float32(wl.sigma0), r0=r0)
            orc.pa_steps_dense_float(J, inst.lin, x, m, 0, steps, lam, wl.eta, wl.alpha)
    elif inst.dense is not None:
        J, b, _ = orc.qubo_to_ising_int(inst.dense, inst.lin)
        reps, steps = wl.replicas, wl.steps
        lam = orc.lambda_linear(wl.steps, wl.lambda0)

        def work(r0, cnt):
            x, m = orc.pa_init(n, cnt, wl.seed, np.float32(wl.sigma0), r0=r0)
            orc.pa_steps_dense_int(J, b, x, m, 0, steps, lam, wl.eta, wl.alpha)
    else:
        c = inst.csr
        rp = c.rp.astype(np.int64)
        reps = min(wl.replicas, 4 * cores)
        steps = max(1, min(wl.steps, int(2.0e9 / max(1, c.nnz * reps))))
        lam = orc.lambda_linear(wl.steps, wl.lambda0)

        def work(r0, cnt):
            x, m = orc.pa_init(n, cnt, wl.seed, np.float32(wl.sigma0), r0=r0)
            orc.pa_steps_csr_int(rp, c.col, c.w, inst.lin, x, m, 0, steps, lam, wl.eta, wl.alpha)
    per = [reps // cores + (1 if k < reps % cores else 0) for k in range(cores)]
    starts = np.concatenate([[0], np.cumsum(per)[:-1]])
    threads = [threading.Thread(target=work, args=(int(s), int(c))) for s, c in zip(starts, per) if c]
    t0 = time.perf_counter()
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    dt = time.perf_counter() - t0
    return {"value": n * reps * steps / dt, "unit": "spin-updates/s", "cores": len(threads),
            "kind": "oracle",
            "sample": "%d replicas x %d PA steps of the same instance (%s couplings), %.1f s wall"
                      % (reps, steps, "bf16-rounded" if prec == "bf16" else "exact", dt)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build runs the whole solve on a single "
              "MI355X (replica/variable sharding across GPUs is a design note, not code). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2501_19221_amd import qpa
    from paper_2501_19221_amd.configs import WORKLOADS

    wl = WORKLOADS[a.workload]
    log("generating workload %s" % wl.name)
    inst = wl.make()
    prec = wl.precision
    eng = qpa.Engine(0)
    prob = qpa.Problem.from_instance(inst)
    pcode = qpa.QPA_PREC_BF16 if prec == "bf16" else qpa.QPA_PREC_FP32
    params = qpa.make_params(wl.replicas, wl.steps, wl.eta, wl.alpha, wl.lambda0, wl.sigma0,
                             wl.seed, pcode)
    torch.cuda.synchronize()
    for w in range(a.warmup):
        out = eng.solve(prob, params)
        torch.cuda.synchronize()
        log("warmup %d done" % w)
    qpa.qpa_profile_read(eng.ctx, reset=True)
    qpa.qpa_profile_enable(eng.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        out = eng.solve(prob, params)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    qpa.qpa_profile_enable(eng.ctx, False)
    step_ms, launches = qpa.qpa_profile_read(eng.ctx, reset=True)
    log("timed %d solves in %.3f s" % (a.steps, dt))
    n, R, T = inst.n, wl.replicas, wl.steps
    su = n * R * T * a.steps / dt
    energy = out["energy"].cpu().numpy()
    best = int(out["best"].cpu()[0])
    avg_launch_s = step_ms / 1e3 / max(1, launches)

    if inst.dense is not None:
        flops = 2.0 * R * n * n           # one field product per launch
        achieved = flops / avg_launch_s / 1e12
        roof = {"bound": "mfma" if prec == "bf16" else "alu", "achieved": achieved,
                "peak": PEAK_BF16_TFLOPS if prec == "bf16" else 78.6, "unit": "TFLOP/s"}
        roof["frac"] = achieved / roof["peak"]
        roof["kernel"] = "k_mfma_step" if prec == "bf16" else "k_dense_*"
        roof["per_launch"] = "2*R*n^2 = %.4g flop (one PA step of every replica)" % flops
    else:
        c = inst.csr
        idx = c.col.dtype.itemsize
        wbytes = c.w.dtype.itemsize
        byts = (4 * (n + 1) + c.nnz * (idx + wbytes) + 16 * n * R) * 1.0
        achieved = byts / avg_launch_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "kernel": "k_csr_step",
                "per_launch": "row_ptr + nnz*(index+weight) + 16 B of x,m read+write per "
                              "(variable, replica) = %.4g B" % byts}
    roof["traffic"] = None
    roof["avg_launch_us"] = avg_launch_s * 1e6
    roof["launches"] = launches

    res = {"metric": METRIC, "value": su, "unit": "spin-updates/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt / a.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": prec, "data": "synthetic",
           "config": {"workload": wl.name, "description": wl.note, "n": n, "replicas": R,
                      "pa_steps": T, "precision": prec, "eta": wl.eta, "alpha": wl.alpha,
                      "lambda0": wl.lambda0, "parallelism": "single GPU"},
           "best_energy": float(energy[best]), "best_replica": best,
           "roofline": roof}

    if prec == "bf16" and not a.no_fp32_form:
        p32 = qpa.make_params(R, T, wl.eta, wl.alpha, wl.lambda0, wl.sigma0, wl.seed,
                              qpa.QPA_PREC_FP32)
        log("FP32 form")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        o32 = eng.solve(prob, p32)
        torch.cuda.synchronize()
        d32 = time.perf_counter() - t1
        e32 = o32["energy"].cpu().numpy()
        eb, ef = float(energy.min()), float(e32.min())
        res["fp32_form"] = {"value": n * R * T / d32, "unit": "spin-updates/s",
                            "best_energy": ef, "bf16_best_energy": eb,
                            "matched": bool(eb <= ef + 1e-6 * abs(ef)),
                            "bf16_speedup": (n * R * T * a.steps / dt) / (n * R * T / d32)}
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(inst, wl, prec)
    eng.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
