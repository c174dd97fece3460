"""Benchmark: spin-updates/s of the whole replica-batched PA solve on one MI355X.

One benchmark step = one complete solve of the workload through the C ABI: App. A
canonicalisation + validation, initial state, all PA steps of App. B, exact FP64/int64
energies of every replica's final spins and the best-of-replica reduction.  Inputs are
uploaded to HBM before the timed region; value = n * replicas * PA-steps * K / seconds.

Default workload: dense SK n=4096, 1024 replicas, 2000 PA steps, couplings in BF16 on
the matrix cores (FP32 accumulation).  The same solve with FP32 couplings on the FP32
path is timed once beside it, and both best energies are compared in FP64 ("BF16 vs FP32
form at matched best energy").

    python bench.py [--steps K] [--warmup W]
                    [--workload sk4096|chimera16|dense20|er512|planted3r|sbm_sk4096|sbm_chimera16
                                |er512_grad]

The sbm_* workloads time whole Simulated Bifurcation Machine solves (App. B) instead;
er512_grad times the relaxed-energy gradient of the whole er512 batch.
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
    ap.add_argument("--precision", choices=["bf16", "fp32"], default=None,
                    help="dense field arithmetic instead of the workload's own (e.g. the "
                         "FP32 form of sk4096 alone)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-form", action="store_true")
    ap.add_argument("--no-measured-peaks", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device to device 4 times (the reference kernel for "
                         "scaling the HBM byte counters) and exit")
    return ap.parse_args()


def measured_traffic(workload, kernel):
    """HBM bytes per launch of the dominant kernel, from the committed rocprofv3 counter
    table (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when the table has no
    entry for it or the kernel's sources changed since the counters were taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(root, "profiles", "hbm_traffic.json")) as f:
            entry = json.load(f)["kernels"][workload]
    except (OSError, KeyError, ValueError):
        return None
    if entry.get("kernel") != kernel:
        return None
    h = hashlib.sha256()
    for rel in entry["source"]:
        with open(os.path.join(root, "paper_2501_19221_amd", rel), "rb") as f:
            h.update(f.read())
    return entry["hbm_bytes_per_dispatch"] if h.hexdigest() == entry["source_sha256"] else None


def calibrate_copy(torch):
    """A plain device-to-device copy of 1 GiB, four times: under rocprofv3 --pmc its
    FETCH_SIZE and WRITE_SIZE per dispatch, against the 1 GiB moved, give the factors that
    turn those counters into HBM bytes."""
    a = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": a.numel() * 4, "copies": 4}), flush=True)


def measured_peaks(torch):
    """Achievable rates on this GPU, as references for the roofline fractions: a 2 GiB
    device-to-device copy (HBM read + write) and a 8192^3 BF16 GEMM from the vendor BLAS."""
    out = {}
    a = torch.empty(2 ** 29, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    it = 10
    e0.record()
    for _ in range(it):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    out["hbm_copy_GBps"] = 2.0 * a.numel() * 4 * it / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    n = 8192
    x = torch.randn(n, n, device="cuda").to(torch.bfloat16)
    y = torch.randn(n, n, device="cuda").to(torch.bfloat16)
    for _ in range(3):
        z = x @ y
    torch.cuda.synchronize()
    it = 20
    e0.record()
    for _ in range(it):
        z = x @ y
    e1.record()
    torch.cuda.synchronize()
    out["bf16_gemm_TFLOPs"] = 2.0 * n ** 3 * it / (e0.elapsed_time(e1) / 1e3) / 1e12
    del x, y, z
    torch.cuda.empty_cache()
    return out


# Host threads the CPU baseline may use: the CPUs this process may run on, at most 16 (the
# host share of one GPU on the measurement machines, whatever the machine's count is).
HOST_THREADS_MAX = 16


def host_cpus():
    """What the host offers: logical CPUs of the machine, CPUs this process may run on, the
    threads the baseline uses, and the CPU model name."""
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count() or 1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"machine_cpus": os.cpu_count(), "allowed_cpus": allowed,
            "threads": max(1, min(HOST_THREADS_MAX, allowed)), "model": model}


def _both_rates(rate_fn, target_s):
    """The oracle on one thread, then on every thread the baseline may use."""
    hc = host_cpus()
    one = rate_fn(1, target_s / 2)
    r = rate_fn(hc["threads"], target_s / 2) if hc["threads"] > 1 else dict(one)
    r["value_1core"] = one["value"]
    r["sample_1core"] = "%d replicas x %d steps, %.1f s wall on 1 thread" % (
        one["reps"], one["steps"], one["seconds"])
    r["host"] = hc
    return r


def cpu_baseline(inst, wl, prec, target_s=20.0):
    """The CPU oracle (untuned) on a bounded sample of the same workload: a set of replicas
    split over host threads (the oracle releases the GIL), initialised outside the timing,
    run for a number of PA steps chosen from a short probe so that the timed part takes
    about target_s / 2 (steps beyond the schedule's T continue from the state, restarting
    the schedule); once on one thread and once on every thread the baseline may use."""
    import oracle as orc
    n = inst.n
    lam = orc.lambda_linear(wl.steps, wl.lambda0)
    if inst.dense is not None and not np.issubdtype(inst.dense.dtype, np.integer):
        J = inst.dense
        if prec == "bf16":
            J = orc.bf16_quantise(J, orc.bf16_scale_exponent(J))
        kind = "bf16-rounded" if prec == "bf16" else "exact"

        def steps_fn(x, m, t0, t1):
            orc.pa_steps_dense_float(J, inst.lin, x, m, t0, t1, lam, wl.eta, wl.alpha)
    elif inst.dense is not None:
        J, b, _ = orc.qubo_to_ising_int(inst.dense, inst.lin)
        kind = "exact"

        def steps_fn(x, m, t0, t1):
            orc.pa_steps_dense_int(J, b, x, m, t0, t1, lam, wl.eta, wl.alpha)
    else:
        c = inst.csr
        if inst.kind == "qubo":
            rp, col, w, b, _ = orc.qubo_to_ising_csr_int(c.rp, c.col, c.w, inst.lin)
        else:
            rp, col, w, b = c.rp.astype(np.int64), c.col, c.w, inst.lin
        kind = "exact"

        def steps_fn(x, m, t0, t1):
            orc.pa_steps_csr_int(rp, col, w, b, x, m, t0, t1, lam, wl.eta, wl.alpha)
    r = _both_rates(lambda cores, ts: _oracle_rate(n, wl.replicas, wl.steps, wl.seed, wl.sigma0,
                                                   steps_fn, cores, ts), target_s)
    r["sample"] = "%d replicas x %d PA steps of the same instance (%s couplings), " \
                  "%.1f s wall on %d threads" % (r.pop("reps"), r.pop("steps"), kind,
                                                 r.pop("seconds"), r["cores"])
    return r


def _oracle_rate(n, R, T, seed, sigma0, steps_fn, cores, target_s):
    """Time steps_fn(x, m, t0, t1) (an oracle stepper, which releases the GIL) on a set of
    replicas split over host threads, initialised outside the timing; the number of steps
    comes from a short probe so that the timed part takes about target_s (steps beyond the
    schedule's T continue from the state, restarting the schedule)."""
    import oracle as orc
    reps = min(R, 4 * cores)
    per = [reps // cores + (1 if k < reps % cores else 0) for k in range(cores)]
    starts = np.concatenate([[0], np.cumsum(per)[:-1]])
    chunks = [(int(s0), int(cnt)) for s0, cnt in zip(starts, per) if cnt]
    states = [orc.pa_init(n, cnt, seed, np.float32(sigma0), r0=s0) for s0, cnt in chunks]

    def timed(steps):
        def work(k):
            x, m = states[k]
            done = 0
            while done < steps:                   # whole schedules, then the remainder
                t1 = min(T, steps - done)
                steps_fn(x, m, 0, t1)
                done += t1
        threads = [threading.Thread(target=work, args=(k,)) for k in range(len(chunks))]
        t0 = time.perf_counter()
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        return time.perf_counter() - t0

    probe_steps, probe = 1, timed(1)
    while probe < 0.25:                       # grow the probe until it measures work
        probe_steps *= 4
        probe = timed(probe_steps)
    steps = max(1, int(probe_steps * target_s / probe))
    dt = timed(steps)
    return {"value": n * reps * steps / dt, "unit": "spin-updates/s", "cores": len(chunks),
            "kind": "oracle", "reps": reps, "steps": steps, "seconds": dt}


def cpu_baseline_sbm(inst, swl, target_s=20.0):
    """The CPU oracle's SBM steps on a bounded sample of the same workload (see
    _oracle_rate), on one thread and on every thread the baseline may use; c0 = 1 / rho
    from the oracle's own power method when the workload asks for it."""
    import oracle as orc
    n = inst.n
    if inst.dense is not None:
        J = np.asarray(inst.dense, np.float32)
        b = np.asarray(inst.lin, np.float32)
        D = J.astype(np.float64)
    else:
        c = inst.csr
        rp, col, w = c.rp.astype(np.int64), c.col, c.w.astype(np.float32)
        b = np.zeros(n, np.float32) if inst.lin is None else np.asarray(inst.lin, np.float32)
        D = c.to_dense(np.float64)
    c0 = swl.c0 if swl.c0 > 0 else float(np.float32(
        1.0 / orc.spectral_radius_power(D, swl.power_iters, swl.seed)))
    if inst.dense is not None:
        def steps_fn(q, p, t0, t1):
            orc.sbm_steps_dense(J, b, q, p, t0, t1, swl.steps, swl.a0, c0, swl.dt)
    else:
        def steps_fn(q, p, t0, t1):
            orc.sbm_steps_csr(rp, col, w, b, q, p, t0, t1, swl.steps, swl.a0, c0, swl.dt)
    r = _both_rates(lambda cores, ts: _oracle_rate(n, swl.replicas, swl.steps, swl.seed,
                                                   swl.sigma0, steps_fn, cores, ts), target_s)
    r["sample"] = "%d replicas x %d SBM steps of the same instance, %.1f s wall on %d " \
                  "threads" % (r.pop("reps"), r.pop("steps"), r.pop("seconds"), r["cores"])
    return r


PEAK_ALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # 32-bit VALU lane-ops/s, no packed math
PEAK_FP32_TFLOPS = 78.6                          # FP32 FMA without packed math


def run_solves(eng, qpa, torch, inst, prob, params, steps, warmup, batch):
    """Time `steps` whole solves; returns (seconds, last output, step-kernel ms, launches)."""
    solve = (lambda: eng.solve_batch(prob, params)) if batch else (lambda: eng.solve(prob, params))
    torch.cuda.synchronize()
    for w in range(warmup):
        solve()
        torch.cuda.synchronize()
        log("warmup %d done" % w)
    qpa.qpa_profile_read(eng.ctx, reset=True)
    qpa.qpa_profile_enable(eng.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = solve()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    qpa.qpa_profile_enable(eng.ctx, False)
    per_path = {}
    for code in (qpa.QPA_PATH_DENSE_RESIDENT, qpa.QPA_PATH_DENSE_TILED, qpa.QPA_PATH_DENSE_MFMA,
                 qpa.QPA_PATH_CSR, qpa.QPA_PATH_BATCH_SPARSE, qpa.QPA_PATH_BATCH_DENSE,
                 qpa.QPA_PATH_CSR_RESIDENT, qpa.QPA_PATH_CSR_BINNED):
        pm, pl = qpa.qpa_profile_read_path(eng.ctx, code)
        if pl:
            per_path[code] = (pm, pl)
    ms, launches = qpa.qpa_profile_read(eng.ctx, reset=True)
    return dt, out, ms, launches, per_path


def bench_sbm(a, torch, qpa, swl):
    """One benchmark step = one whole SBM solve (canonicalisation, initial state, power
    method for c0, all steps, exact energies, best replica)."""
    log("generating SBM workload %s" % swl.name)
    inst = swl.make()
    eng = qpa.Engine(0)
    prob = qpa.Problem.from_instance(inst)
    R, T, n = swl.replicas, swl.steps, inst.n
    sp = qpa.make_sbm_params(R, T, swl.dt, swl.a0, swl.c0, swl.sigma0, swl.seed,
                             swl.power_iters)
    torch.cuda.synchronize()
    for w in range(a.warmup):
        eng.sbm_solve(prob, sp)
        torch.cuda.synchronize()
        log("warmup %d done" % w)
    qpa.qpa_profile_read(eng.ctx, reset=True)
    qpa.qpa_profile_enable(eng.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        out = eng.sbm_solve(prob, sp)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    qpa.qpa_profile_enable(eng.ctx, False)
    dense = inst.dense is not None
    code = qpa.QPA_PATH_SBM_DENSE if dense else qpa.QPA_PATH_SBM_CSR
    step_ms, launches = qpa.qpa_profile_read_path(eng.ctx, code)
    resident = False
    if not dense and launches == 0:
        code = qpa.QPA_PATH_SBM_CSR_RESIDENT
        step_ms, launches = qpa.qpa_profile_read_path(eng.ctx, code)
        resident = True
    qpa.qpa_profile_read(eng.ctx, reset=True)
    avg_s = step_ms / 1e3 / max(1, launches)
    if resident:
        c = inst.csr
        flops = 2.0 * c.nnz * R * T
        roof = {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "kernel": "k_sbm_csr_resident",
                "per_launch": "2*nnz*R*T = %.4g flop (one FMA per stored entry, replica and "
                              "step; all steps in one launch, state on chip)" % flops}
    elif dense:
        flops = 2.0 * R * n * n
        roof = {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "kernel": "k_fp32_tiled_step",
                "per_launch": "2*R*n^2 = %.4g flop (one FMA per coupling, replica; one SBM "
                              "step of every replica)" % flops}
    else:
        c = inst.csr
        byts = (4.0 * (n + 1) + c.nnz * (c.col.dtype.itemsize + c.w.dtype.itemsize)
                + 16.0 * n * R)
        roof = {"bound": "hbm", "achieved": byts / avg_s / 1e9, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "kernel": "k_sbm_csr_step",
                "per_launch": "4(n+1) + nnz*(index+weight) + 16*n*R (q read and written, p "
                              "read and written) = %.4g B (one SBM step of every replica)"
                              % byts}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(swl.name, roof["kernel"])
    roof["avg_launch_us"] = avg_s * 1e6
    roof["launches"] = launches
    e = out["energy"].cpu().numpy()
    res = {"metric": METRIC, "value": n * R * T * a.steps / dt, "unit": "spin-updates/s",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": swl.name, "description": swl.note, "n": n, "replicas": R,
                      "sbm_steps": T, "dt": swl.dt, "a0": swl.a0,
                      "c0": "1/rho (power method)" if swl.c0 == 0 else swl.c0,
                      "parallelism": "single GPU"},
           "roofline": roof, "best_energy": float(e.min()),
           "best_replica": int(out["best"].cpu()[0])}
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline_sbm(inst, swl)
    eng.close()
    print(json.dumps(res), flush=True)


def bench_relaxed(a, torch, qpa, wl, ckpt=50):
    """One benchmark step = the mean relaxed final energy of the whole batch and its
    gradient with respect to (eta, alpha, lambda_t): forward pass with a checkpoint every
    `ckpt` steps, recomputation of each segment and the reverse pass (App. B dynamics with
    analog spins in the target part)."""
    log("generating workload %s" % wl.name)
    insts = wl.make()
    eng = qpa.Engine(0)
    probs = [qpa.Problem.from_instance(i) for i in insts]
    R, T = wl.replicas, wl.steps
    params = qpa.make_params(R, T, wl.eta, wl.alpha, wl.lambda0, wl.sigma0, wl.seed)
    torch.cuda.synchronize()
    for w in range(a.warmup):
        eng.relaxed_grad(probs, params, ckpt)
        torch.cuda.synchronize()
        log("warmup %d done" % w)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        L, de, da, dl = eng.relaxed_grad(probs, params, ckpt)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_total = sum(i.n for i in insts)
    nnz = sum(i.csr.nnz for i in insts)
    res = {"metric": "relaxed-gradient spin-steps/s (n x replicas x steps / s; forward, "
                     "recomputation and reverse pass)",
           "value": n_total * R * T * a.steps / dt, "unit": "spin-steps/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt / a.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "er512_grad", "description": wl.note, "n": n_total,
                      "nnz": nnz, "instances": len(insts), "replicas": R, "pa_steps": T,
                      "checkpoint_every": ckpt, "parallelism": "single GPU"},
           "loss": float(L.cpu()[0]), "d_eta": float(de.cpu()[0]),
           "d_alpha": float(da.cpu()[0])}
    eng.close()
    print(json.dumps(res), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library runs the whole solve on a single "
              "MI355X (replica/variable sharding across GPUs is a design note, not code). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    if a.calibrate_copy:
        calibrate_copy(torch)
        return
    from paper_2501_19221_amd import qpa
    from paper_2501_19221_amd.configs import SBM_WORKLOADS, WORKLOADS

    if a.workload in SBM_WORKLOADS:
        bench_sbm(a, torch, qpa, SBM_WORKLOADS[a.workload])
        return
    if a.workload == "er512_grad":
        bench_relaxed(a, torch, qpa, WORKLOADS["er512"])
        return
    wl = WORKLOADS[a.workload]
    log("generating workload %s" % wl.name)
    made = wl.make()
    batch = isinstance(made, list)
    insts = made if batch else [made]
    prec = a.precision or wl.precision
    eng = qpa.Engine(0)
    probs = [qpa.Problem.from_instance(i) for i in insts]
    prob = probs if batch else probs[0]
    pcode = qpa.QPA_PREC_BF16 if prec == "bf16" else qpa.QPA_PREC_FP32
    R, T = wl.replicas, wl.steps
    params = qpa.make_params(R, T, wl.eta, wl.alpha, wl.lambda0, wl.sigma0, wl.seed, pcode)
    tuned = None
    if batch:
        # batch path rates measured by the library's batch autotuner (set-up, not timed)
        dense_bps, sparse_adds = eng.autotune_batch(prob, params, 20)
        tuned = {"dense_Bps": dense_bps, "sparse_adds_per_s": sparse_adds, "probe_steps": 20}
        log("autotune_batch: dense %.3g B/s, sparse %.3g adds/s" % (dense_bps, sparse_adds))
    if not batch and insts[0].csr is not None and insts[0].n <= 8192:
        # sparse kernel configuration by the library's autotuner (set-up, not timed)
        choice, ms = eng.autotune(prob, params, 100)
        tuned = {"choice": "streamed" if choice == 0 else "resident G=%d" % choice,
                 "probe_ms": dict(zip(["streamed", "G1", "G2", "G4", "G8"], ms)),
                 "probe_steps": 100}
        log("autotune: %s" % tuned["choice"])
    dt, out, step_ms, launches, per_path = run_solves(eng, qpa, torch, insts, prob, params,
                                                      a.steps, a.warmup, batch)
    log("timed %d solves in %.3f s" % (a.steps, dt))
    n_total = sum(i.n for i in insts)
    su = n_total * R * T * a.steps / dt
    avg_launch_s = step_ms / 1e3 / max(1, launches)
    per_solve_launches = launches / max(1, a.steps)

    inst0 = insts[0]
    if batch:
        paths = qpa.qpa_batch_paths(eng.ctx, len(insts))
        grouped = (qpa.QPA_PATH_BATCH_DENSE, qpa.QPA_PATH_BATCH_DENSE_I8,
                   qpa.QPA_PATH_BATCH_SPARSE_I8)
        dense = np.isin(paths, grouped)
        roofs = {}
        if qpa.QPA_PATH_BATCH_DENSE in per_path:
            pm, pl = per_path[qpa.QPA_PATH_BATCH_DENSE]
            # one step: the couplings read once (BF16: 2 bytes per element, int8 rows: 1 byte
            # per element, int8 entry lists: 4 bytes per nonzero), x and m read and written
            jb, kinds = 0.0, set()
            for i, pth in zip(insts, paths):
                if pth not in grouped:
                    continue
                kinds.add(int(pth))
                if pth == qpa.QPA_PATH_BATCH_SPARSE_I8:
                    jb += 4.0 * np.count_nonzero(i.csr.w)
                else:
                    jb += (1.0 if pth == qpa.QPA_PATH_BATCH_DENSE_I8 else 2.0) * i.n * i.n
            nd = np.array([i.n for i, d in zip(insts, dense) if d], np.float64)
            byts = float(jb + np.sum(16.0 * R * nd))
            pl = pl / max(1, len(kinds))          # launches per step: one per tile kind present
            roofs["dense"] = {
                "bound": "hbm", "achieved": byts / (pm / 1e3 / pl) / 1e9, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "kernel": "k_mfma_grouped", "ms": pm, "launches": pl,
                "instances": int(dense.sum()),
                "per_launch": "sum over the grouped instances of their couplings (2n^2 BF16, "
                              "n^2 int8 rows, 4 bytes per nonzero as int8 entry lists) + 16nR "
                              "(x, m read and written) = %.4g B (one PA step of every replica "
                              "of every grouped instance; 'launch' = the grouped launches of "
                              "one step)" % byts,
                "int8_instances": int(np.sum(paths == qpa.QPA_PATH_BATCH_DENSE_I8)),
                "int8_entry_list_instances": int(np.sum(paths == qpa.QPA_PATH_BATCH_SPARSE_I8))}
        if qpa.QPA_PATH_BATCH_SPARSE in per_path:
            pm, pl = per_path[qpa.QPA_PATH_BATCH_SPARSE]
            nnz = sum(i.csr.nnz for i, d in zip(insts, dense) if not d)
            ops = float(nnz) * R * T          # one signed coupling add per entry, replica, step
            roofs["sparse"] = {
                "bound": "alu", "achieved": ops / (pm / 1e3 / pl) / 1e12, "peak": PEAK_ALU_TOPS,
                "unit": "Tops/s", "kernel": "k_csr_batch", "ms": pm, "launches": pl,
                "instances": int((~dense).sum()),
                "per_launch": "sum(nnz)*R*T = %.4g signed coupling adds (sparse instances, "
                              "all steps, one launch)" % ops}
        if "dense" in roofs:
            # the same step counted as the streamed CSR form would move it: int16 index and
            # weight per stored entry, row pointers, x and m read and written, byte spins
            # written and read -- the bytes the batch workload's scope states
            csr_b = float(sum(4.0 * i.csr.nnz + 4.0 * (i.n + 1) + 18.0 * R * i.n
                              for i in insts))
            rd = roofs["dense"]
            rd["csr_form_bytes_per_step"] = csr_b
            rd["frac_on_csr_form_bytes"] = csr_b / (rd["ms"] / 1e3 / rd["launches"]) / 1e9 / \
                PEAK_HBM_GBS
        main_path = max(roofs, key=lambda k: roofs[k]["ms"])
        roof = dict(roofs[main_path])
        avg_launch_s = roof.pop("ms") / 1e3 / roof["launches"]
        launches = roof.pop("launches")
        if len(roofs) > 1:
            other = [k for k in roofs if k != main_path][0]
            o = dict(roofs[other])
            o["frac"] = o["achieved"] / o["peak"]
            roof["other_path"] = o
        best = [int(o["best"].cpu()[0]) for o in out]
        bestE = [float(o["energy"].cpu().numpy()[b]) for o, b in zip(out, best)]
        extra = {"mean_best_energy": float(np.mean(bestE))}
    elif inst0.dense is not None:
        n = inst0.n
        if per_solve_launches <= 1.0:      # resident kernels: all steps in one launch
            flops = 2.0 * R * n * n * T
            what = "2*R*n^2*T = %.4g flop (all steps of all replicas, one launch)" % flops
        else:
            flops = 2.0 * R * n * n
            what = "2*R*n^2 = %.4g flop (one PA step of every replica)" % flops
        achieved = flops / avg_launch_s / 1e12
        if prec == "bf16":
            roof = {"bound": "mfma", "peak": PEAK_BF16_TFLOPS, "kernel": "k_mfma_step"}
        else:
            roof = {"bound": "alu", "peak": PEAK_FP32_TFLOPS,
                    "kernel": ("k_dense_wave" if n <= 64 else "k_dense_resident")
                    if per_solve_launches <= 1.0 else "k_fp32_tiled_step"}
        roof.update({"achieved": achieved, "unit": "TFLOP/s", "per_launch": what})
        e = out["energy"].cpu().numpy()
        extra = {"best_energy": float(e.min()), "best_replica": int(out["best"].cpu()[0])}
    elif qpa.QPA_PATH_CSR_RESIDENT in per_path:
        c = inst0.csr
        ops = float(c.nnz) * R * T            # one signed coupling add per entry, replica, step
        roof = {"bound": "alu", "achieved": ops / avg_launch_s / 1e12, "peak": PEAK_ALU_TOPS,
                "unit": "Tops/s", "kernel": "k_csr_resident",
                "per_launch": "nnz*R*T = %.4g signed coupling adds (all steps of all replicas, "
                              "one launch; state on chip)" % ops}
        e = out["energy"].cpu().numpy()
        extra = {"best_energy": float(e.min()), "best_replica": int(out["best"].cpu()[0])}
    else:
        c = inst0.csr
        n = inst0.n
        byts = (4.0 * (n + 1) + c.nnz * (c.col.dtype.itemsize + c.w.dtype.itemsize)
                + 16.0 * n * R)
        binned = qpa.QPA_PATH_CSR_BINNED in per_path
        # the binned step is two launches (gather, then fields + update): one 'launch'
        # below is the pair, so the bytes of a step are set against the time of a step
        step_s = avg_launch_s * (2.0 if binned else 1.0)
        achieved = byts / step_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "kernel": "k_bin_gather+k_bin_update" if binned else "k_csr_step",
                "per_launch": "4(n+1) + nnz*(index+weight) + 16*n*R (x, m read and written) "
                              "= %.4g B (one PA step of every replica%s)"
                              % (byts, "; the two launches of a binned step together"
                                 if binned else "")}
        if binned:
            avg_launch_s = step_s
            launches //= 2
        e = out["energy"].cpu().numpy()
        extra = {"best_energy": float(e.min()), "best_replica": int(out["best"].cpu()[0])}
    if not batch and "planted_state" in inst0.meta and inst0.csr is not None:
        # planted optimum E* = -sum over edges of |w| (every coupling satisfied by s*)
        c = inst0.csr
        e_star = -float(np.abs(c.w.astype(np.int64)).sum()) / 2.0
        extra["planted_energy"] = e_star
        extra["optimality_gap"] = (extra["best_energy"] - e_star) / abs(e_star)
    roof["frac"] = roof["achieved"] / roof["peak"]
    if not a.no_measured_peaks:
        log("measured peaks")
        mp = measured_peaks(torch)
        res_peaks = mp
        ref = {"GB/s": mp["hbm_copy_GBps"], "TFLOP/s": mp["bf16_gemm_TFLOPs"]}.get(roof["unit"])
        if ref is not None and roof["bound"] in ("hbm", "mfma"):
            roof["frac_of_measured"] = roof["achieved"] / ref
    else:
        res_peaks = None
    roof["traffic"] = measured_traffic(wl.name, roof["kernel"])
    roof["avg_launch_us"] = avg_launch_s * 1e6
    roof["launches"] = launches

    res = {"metric": METRIC, "value": su, "unit": "spin-updates/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt / a.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": prec, "data": "synthetic",
           "config": {"workload": wl.name, "description": wl.note, "n": n_total,
                      "instances": len(insts), "replicas": R, "pa_steps": T,
                      "precision": prec, "eta": wl.eta, "alpha": wl.alpha,
                      "lambda0": wl.lambda0, "parallelism": "single GPU"},
           "roofline": roof}
    if res_peaks is not None:
        res["measured_peak"] = res_peaks
    if tuned is not None:
        res["autotune"] = tuned
    res.update(extra)

    if prec == "bf16" and not a.no_fp32_form:
        # the same solve with FP32 couplings; when BF16's best energy is worse, BF16 is
        # rerun with twice the replicas (and its cost counted) until it matches
        # (each form: one warm-up solve, then FORM_SOLVES timed solves)
        FORM_SOLVES = 3
        p32 = qpa.make_params(R, T, wl.eta, wl.alpha, wl.lambda0, wl.sigma0, wl.seed,
                              qpa.QPA_PREC_FP32)
        log("FP32 form")
        d32, o32, _, _, _ = run_solves(eng, qpa, torch, insts, prob, p32, FORM_SOLVES, 1, False)
        d32 /= FORM_SOLVES
        ef = float(o32["energy"].cpu().numpy().min())
        eb = float(out["energy"].cpu().numpy().min())
        t_bf = dt / a.steps
        reps = R
        while eb > ef + 1e-6 * abs(ef) and reps < 8 * R:
            reps *= 2
            log("BF16 with %d replicas" % reps)
            pb = qpa.make_params(reps, T, wl.eta, wl.alpha, wl.lambda0, wl.sigma0, wl.seed,
                                 qpa.QPA_PREC_BF16)
            tb, ob, _, _, _ = run_solves(eng, qpa, torch, insts, prob, pb, FORM_SOLVES, 1, False)
            t_bf = tb / FORM_SOLVES
            eb = float(ob["energy"].cpu().numpy().min())
        matched = bool(eb <= ef + 1e-6 * abs(ef))
        res["fp32_form"] = {"value": n_total * R * T / d32, "unit": "spin-updates/s",
                            "seconds_per_solve": d32, "solves_timed": FORM_SOLVES,
                            "best_energy": ef, "bf16_best_energy": eb,
                            "bf16_replicas_to_match": reps, "matched": matched,
                            "bf16_seconds_per_solve_at_match": t_bf,
                            "bf16_value_at_matched_energy": n_total * reps * T / t_bf,
                            "bf16_speedup_at_matched_energy": d32 / t_bf,
                            "bf16_speedup_at_config_replicas": d32 / (dt / a.steps)}
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(inst0, wl, prec)
        if batch:
            res["cpu_baseline"]["sample"] += " (first instance of the batch)"
    eng.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
