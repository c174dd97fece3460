"""PA and SBM on the planted families (Sec. VIII) on the GPU: no replica ever scores
below the planted ground-state energy (exactly, for the integer families), every
returned energy is the oracle's energy of the returned spins, and the easy instances are
solved to small gaps where the paper reports the solver strong (Sec. VIII).""" 
import sys

import numpy as np
import pytest

import oracle as orc
from paper_2501_19221_amd import instances as gen

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-planted] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def q():
    from paper_2501_19221_amd import qpa
    return qpa


@pytest.fixture(scope="module")
def eng(q):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    e = q.Engine(0)
    yield e
    e.close()


CASES = {
    "3r3x": lambda: gen.xorsat_3r3x(200, seed=3),
    "tp_easy": lambda: gen.tile_planted(24, (0, 0.2, 0, 0.8), seed=4),
    "tp_hard": lambda: gen.tile_planted(24, (0, 0.8, 0, 0.2), seed=5),
    "wp_easy": lambda: gen.wishart_planted(200, 1.0, seed=6),
}


def _oracle_energies(inst, s):
    if inst.dense is not None:
        J = inst.dense.astype(np.float64)
        return np.array([orc.ising_energy_float(J, np.zeros(inst.n), s[r])
                         for r in range(len(s))])
    c = inst.csr
    return np.array([orc.ising_energy_csr_int(c.rp, c.col, c.w, inst.lin.astype(np.int64),
                                              s[r]) for r in range(len(s))])


@pytest.mark.parametrize("family", list(CASES))
@pytest.mark.parametrize("solver", ["pa", "sbm"])
def test_planted_energy_is_a_floor(q, eng, family, solver):
    inst = CASES[family]()
    prob = q.Problem.from_instance(inst)
    J = inst.dense.astype(np.float64) if inst.dense is not None else \
        inst.csr.to_dense(np.float64)
    rho = orc.spectral_radius_power(J, 200, 1)
    R, T = 64, 1500
    say("%s %s n=%d" % (solver, family, inst.n))
    if solver == "pa":
        out = eng.solve(prob, q.make_params(R, T, 0.5 / rho, 0.8, 2.0 * rho, 0.1, 1))
    else:
        out = eng.sbm_solve(prob, q.make_sbm_params(R, T, 0.5, c0=float(1.0 / rho), seed=1))
    s = out["spins"].cpu().numpy()
    e = out["energy"].cpu().numpy()
    ref = _oracle_energies(inst, s)
    E0 = _oracle_energies(inst, inst.meta["planted_state"][None, :])[0]
    if inst.dense is not None:
        np.testing.assert_allclose(e, ref, rtol=1e-12, atol=1e-9)
        assert e.min() >= E0 - 1e-6 * abs(E0)
    else:
        assert np.array_equal(out["energy_i64"].cpu().numpy(), ref)
        assert E0 == inst.meta["planted_energy"]
        assert ref.min() >= E0
    gap = (e.min() - E0) / abs(E0)
    say("gap %.4g" % gap)
    # quality on the regimes where the section reports each solver strong: both on easy
    # tile planting, SBM on easy Wishart, PA on 3R3X
    if (family == "tp_easy" or (family == "wp_easy" and solver == "sbm")
            or (family == "3r3x" and solver == "pa")):
        assert gap <= 0.05
