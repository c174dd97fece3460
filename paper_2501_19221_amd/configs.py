"""The five synthetic workloads the engine is measured and checked on, with their pinned
PA hyperparameters.

The paper prints no PA hyperparameters (App. B asks only for a lambda(t) that falls from
a sufficiently large value to zero); each workload's (lambda0, eta, alpha, sigma0) was
chosen once by a small sweep on the CPU oracle and is frozen here.
"""
from __future__ import annotations

from dataclasses import dataclass

from . import instances as gen


@dataclass(frozen=True)
class Workload:
    name: str
    replicas: int
    steps: int
    eta: float
    alpha: float
    lambda0: float
    sigma0: float
    seed: int
    precision: str          # "fp32" | "bf16" (dense field arithmetic)
    make: object            # () -> Instance | list[Instance]
    note: str


WORKLOADS = {
    "dense20": Workload(
        "dense20", 256, 2000, 0.002, 0.9, 30.0, 0.1, 1, "fp32",
        lambda: gen.dense_int_qubo(20, -10, 10, seed=1),
        "dense QUBO n=20, int32 Q and c uniform in [-10,10], 256 replicas, 2000 steps"),
    "chimera16": Workload(
        "chimera16", 1024, 5000, 0.2, 0.8, 10.0, 0.1, 1, "fp32",
        lambda: gen.chimera_ising(16, seed=2),
        "Chimera C16 (16x16 K4,4 cells, 2048 vars, 6016 edges), +-1 couplings, CSR int8, "
        "1024 replicas, 5000 steps"),
    "sk4096": Workload(
        "sk4096", 1024, 2000, 0.2, 0.8, 4.0, 0.1, 1, "bf16",
        lambda: gen.sk_ising(4096, 0.1, seed=3),
        "dense SK n=4096, J ~ N(0,1/n), b ~ N(0,0.1), 1024 replicas, 2000 steps"),
    "er512": Workload(
        "er512", 64, 500, 0.0002, 0.8, 200.0, 0.1, 1, "fp32",
        lambda: gen.er_qubo_batch(512, 100, 2000, 0.1, 100, seed=4),
        "512 Erdos-Renyi QUBOs, n uniform in [100,2000], p=0.1, int16 weights in [-100,100], "
        "64 replicas each, 500 steps"),
    "planted3r": Workload(
        "planted3r", 4, 1000, 0.1, 0.8, 10.0, 0.1, 1, "fp32",
        lambda: gen.planted_3regular(100_000_000, 1, 7, seed=5),
        "planted random 3-regular Ising graph, n=1e8, |w| in [1,7], CSR int32 indices + int8 "
        "weights, 4 replicas, 1000 steps"),
}


@dataclass(frozen=True)
class SbmWorkload:
    """A Simulated Bifurcation Machine run (App. B).  c0 = 0 takes c0 = 1 / rho from
    `power_iters` power-method iterations, the prescription App. B gives; a0 = 1 as it
    suggests.  dt was chosen once by a small sweep on the CPU oracle (dt = 1 diverges
    on SK couplings, dt = 0.25 and 0.5 reach similar energies)."""
    name: str
    replicas: int
    steps: int
    dt: float
    a0: float
    c0: float
    sigma0: float
    seed: int
    power_iters: int
    make: object
    note: str


SBM_WORKLOADS = {
    "sbm_sk4096": SbmWorkload(
        "sbm_sk4096", 1024, 1000, 0.5, 1.0, 0.0, 0.1, 1, 100,
        lambda: gen.sk_ising(4096, 0.1, seed=3),
        "SBM on dense SK n=4096 (the sk4096 instance), FP32 couplings, 1024 replicas, "
        "1000 symplectic-Euler steps, dt=0.5, a0=1, c0=1/rho"),
    "sbm_chimera16": SbmWorkload(
        "sbm_chimera16", 1024, 2000, 0.5, 1.0, 0.0, 0.1, 1, 100,
        lambda: gen.chimera_ising(16, seed=2),
        "SBM on Chimera C16 (the chimera16 instance), CSR int8, 1024 replicas, 2000 steps, "
        "dt=0.5, a0=1, c0=1/rho"),
}
