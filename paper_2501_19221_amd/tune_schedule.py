"""Tuning the PA step size, momentum and schedule with the hand-written adjoint.

    python -m paper_2501_19221_amd.tune_schedule [--n 400] [--iters 30] [--replicas 64]
                                                 [--steps 500] [--ckpt 50]

The relaxed final energy L(eta, alpha, lambda) (App. B with the analog spins in the
target part, mean over replicas) is differentiable; its gradient comes from the
library's adjoint (qpa_relaxed_grad, checkpointed every `ckpt` steps) through
RelaxedEnergy.  Adam on (log eta, logit alpha, log lambda0, log gamma) of the schedule
lambda_t = lambda0 (1 - t/T)^gamma lowers L (the lowest-loss parameters seen are kept);
the tool then runs the ordinary binarised PA solve with the initial and the tuned
parameters and reports both best and mean energies.  One JSON line per iteration, then a
summary line.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import instances as gen


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=400)
    ap.add_argument("--density", type=float, default=0.1)
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--replicas", type=int, default=64)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--ckpt", type=int, default=50)
    ap.add_argument("--lr", type=float, default=0.02)
    ap.add_argument("--seed", type=int, default=4)
    a = ap.parse_args(argv)
    import torch
    from . import qpa
    eng = qpa.Engine(0)
    rng = np.random.default_rng(a.seed)
    inst = gen.er_qubo(a.n, a.density, 100, rng, idx_dtype=np.int16)
    prob = qpa.Problem.from_instance(inst)
    T, R = a.steps, a.replicas
    # start from the er512 workload's hand-picked parameters
    log_eta = torch.tensor(np.log(2e-4), dtype=torch.float64, requires_grad=True)
    logit_alpha = torch.tensor(np.log(0.8 / 0.2), dtype=torch.float64, requires_grad=True)
    log_lam0 = torch.tensor(np.log(200.0), dtype=torch.float64, requires_grad=True)
    log_gamma = torch.tensor(0.0, dtype=torch.float64, requires_grad=True)
    frac = 1.0 - torch.arange(T, dtype=torch.float64) / T
    opt = torch.optim.Adam([log_eta, logit_alpha, log_lam0, log_gamma], lr=a.lr)

    def params_now():
        eta = torch.exp(log_eta)
        alpha = torch.sigmoid(logit_alpha)
        lam = torch.exp(log_lam0) * frac ** torch.exp(log_gamma)
        return eta, alpha, lam

    def solve_energies(eta, alpha, lam):
        p = qpa.make_params(R, T, float(eta), float(alpha), 0.0, 0.1, a.seed,
                            lambda_table=lam.detach().numpy().astype(np.float32))
        e = eng.solve(prob, p)["energy"].cpu().numpy()
        return float(e.min()), float(e.mean())

    with torch.no_grad():
        start = solve_energies(*params_now())
    first, best = None, None
    for it in range(a.iters):
        eta, alpha, lam = params_now()
        L = qpa.RelaxedEnergy.apply(eta, alpha, lam, eng, prob, R, 0.1, a.seed, a.ckpt)
        if best is None or float(L) < best[0]:
            best = (float(L), eta.detach().clone(), alpha.detach().clone(),
                    lam.detach().clone())
        opt.zero_grad()
        L.backward()
        opt.step()
        first = float(L) if first is None else first
        print(json.dumps({"iter": it, "relaxed_loss": float(L), "eta": float(eta),
                          "alpha": float(alpha), "lambda0": float(lam[0]),
                          "gamma": float(torch.exp(log_gamma))}), flush=True)
    with torch.no_grad():
        Lend, eta, alpha, lam = best
        end = solve_energies(eta, alpha, lam)
    print(json.dumps({"summary": True, "n": a.n, "replicas": R, "steps": T,
                      "relaxed_loss_start": first, "relaxed_loss_end": Lend,
                      "pa_best_start": start[0], "pa_mean_start": start[1],
                      "pa_best_tuned": end[0], "pa_mean_tuned": end[1],
                      "eta": float(eta), "alpha": float(alpha)}), flush=True)
    eng.close()


if __name__ == "__main__":
    sys.exit(main())
