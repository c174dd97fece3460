"""Optimality gaps of PA and SBM on the planted families of Sec. VIII.

    python -m paper_2501_19221_amd.gaps [--families 3r3x,tp_easy,tp_hard,wp_easy,wp_hard]
                                        [--replicas 256] [--steps 2000] [--seeds 1]

Every instance has a known ground-state energy E0 (the planted state's energy, scored by
the engine itself).  Both solvers run through the C ABI on one GPU; the gap of a run is
(E_best - E0) / |E0|.  PA runs on the scale-free parameters eta = 0.5 / rho,
lambda0 = 2 rho, alpha = 0.8 (rho: the spectral radius of J from the engine's power
method; the PA dynamics are invariant under J -> cJ with eta -> eta/c, lambda -> c
lambda), SBM on a0 = 1, c0 = 1/rho, dt = 0.5.  One JSON line per instance on stdout.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import instances as gen

FAMILIES = {
    "3r3x": (lambda size, seed: gen.xorsat_3r3x(size, seed=seed), (128, 1024, 8192, 65536)),
    "tp_easy": (lambda size, seed: gen.tile_planted(size, (0, 0.2, 0, 0.8), seed=seed),
                (16, 64, 128, 300)),
    "tp_hard": (lambda size, seed: gen.tile_planted(size, (0, 0.8, 0, 0.2), seed=seed),
                (16, 64, 128, 300)),
    "wp_easy": (lambda size, seed: gen.wishart_planted(size, 1.0, seed=seed), (128, 512, 2048)),
    "wp_hard": (lambda size, seed: gen.wishart_planted(size, 0.2, seed=seed), (128, 512, 2048)),
}


def run_instance(eng, qpa, torch, inst, R, T, seed=1):
    prob = qpa.Problem.from_instance(inst)
    rho = float(eng.spectral_radius(prob, qpa.make_sbm_params(1, 0, 0.5, seed=seed,
                                                             power_iters=200)).cpu()[0])
    dev = "cuda:%d" % eng.device
    s_star = torch.from_numpy(inst.meta["planted_state"][None, :].astype(np.int8)).to(dev)
    pe = qpa.make_params(1, 0, 0.1, 0.8, 1.0)
    E0 = float(eng.energy(prob, pe, s_star)[0].cpu()[0])
    p = qpa.make_params(R, T, 0.5 / rho, 0.8, 2.0 * rho, 0.1, seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = eng.solve(prob, p)
    torch.cuda.synchronize()
    t_pa = time.perf_counter() - t0
    e_pa = float(out["energy"].min().cpu())
    sp = qpa.make_sbm_params(R, T, 0.5, a0=1.0, c0=0.0, sigma0=0.1, seed=seed,
                             power_iters=200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = eng.sbm_solve(prob, sp)
    torch.cuda.synchronize()
    t_sbm = time.perf_counter() - t0
    e_sbm = float(out["energy"].min().cpu())
    return {"n": inst.n, "rho": rho, "E0": E0,
            "pa_best": e_pa, "pa_gap": (e_pa - E0) / abs(E0), "pa_seconds": t_pa,
            "sbm_best": e_sbm, "sbm_gap": (e_sbm - E0) / abs(E0), "sbm_seconds": t_sbm}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--families", default=",".join(FAMILIES))
    ap.add_argument("--replicas", type=int, default=256)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--seeds", type=int, default=1)
    ap.add_argument("--max-size", type=int, default=0, help="skip sizes above this")
    a = ap.parse_args(argv)
    import torch
    from . import qpa
    eng = qpa.Engine(0)
    for fam in a.families.split(","):
        make, sizes = FAMILIES[fam]
        for size in sizes:
            if a.max_size and size > a.max_size:
                continue
            for seed in range(1, a.seeds + 1):
                inst = make(size, seed)
                r = run_instance(eng, qpa, torch, inst, a.replicas, a.steps)
                r.update({"family": fam, "size": size, "seed": seed, "replicas": a.replicas,
                          "steps": a.steps})
                print(json.dumps(r), flush=True)
    eng.close()


if __name__ == "__main__":
    sys.exit(main())
