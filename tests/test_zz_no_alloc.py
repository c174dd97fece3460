"""The allocation-free solve (qpa_solve_noalloc, static device workspace) against
qpa_solve with a caller workspace: identical outputs bit for bit, on two calls in a row
with the second on a smaller input (the static workspace then still holds the first
call's contents), for a dense and a sparse instance; limits rejected with clear errors."""
import sys

import numpy as np
import pytest

from paper_2501_19221_amd import instances as gen

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-noalloc] " + msg, flush=True)
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


def _same(a, b):
    for k in ("spins", "energy", "energy_i64", "best", "x", "m"):
        assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()), k


PAIRS = [
    # two instances of one kind, the second smaller:
    # (label, instance factory, replicas, steps, eta, alpha, lambda0, precision)
    [("dense qubo n=400 bf16", lambda: gen.dense_int_qubo(400, seed=3), 256, 150, 0.002, 0.9,
      30.0, 1),
     ("dense qubo n=90 fp32", lambda: gen.dense_int_qubo(90, seed=4), 64, 120, 0.002, 0.9,
      30.0, 0)],
    [("chimera C8 csr", lambda: gen.chimera_ising(8, seed=5), 512, 200, 0.2, 0.8, 10.0, 0),
     ("chimera C2 csr", lambda: gen.chimera_ising(2, seed=6), 40, 90, 0.2, 0.8, 10.0, 0)],
]


@pytest.mark.parametrize("pair", [0, 1])
def test_noalloc_equals_solve_two_calls_in_a_row(q, eng, pair):
    import torch
    runs = []
    for label, make, R, T, eta, alpha, lam0, prec in PAIRS[pair]:
        prob = q.Problem.from_instance(make())
        p = q.make_params(R, T, eta, alpha, lam0, 0.1, 11, prec)
        need = q.qpa_workspace_size(eng.ctx, prob.struct(), p)
        assert need <= q.QPA_NOALLOC_WORKSPACE_BYTES, (label, need)
        runs.append((label, prob, p))
    # the two allocation-free calls back to back, the second on the smaller input
    got = []
    for label, prob, p in runs:
        say("noalloc %s: R=%d T=%d" % (label, p.replicas, p.steps))
        got.append(eng.solve(prob, p, want_state=True, noalloc=True))
    torch.cuda.synchronize()
    for (label, prob, p), a in zip(runs, got):
        say("qpa_solve %s" % label)
        b = eng.solve(prob, p, want_state=True)
        torch.cuda.synchronize()
        _same(a, b)


def test_noalloc_rejects_what_it_cannot_hold(q, eng):
    big = gen.dense_int_qubo(3000, seed=7)          # FP32 couplings alone: 36 MB
    prob = q.Problem.from_instance(big)
    p = q.make_params(1024, 10, 0.002, 0.9, 30.0)
    assert q.qpa_workspace_size(eng.ctx, prob.struct(), p) > q.QPA_NOALLOC_WORKSPACE_BYTES
    with pytest.raises(q.QpaError, match="static workspace holds"):
        eng.solve(prob, p, noalloc=True)
    small = q.Problem.from_instance(gen.dense_int_qubo(20, seed=8))
    with pytest.raises(q.QpaError, match="QPA_NOALLOC_MAX_STEPS"):
        eng.solve(small, q.make_params(8, q.QPA_NOALLOC_MAX_STEPS + 1, 0.002, 0.9, 30.0),
                  noalloc=True)
    with pytest.raises(q.QpaError, match="QPA_SOLVE_GRAPH"):
        eng.solve(small, q.make_params(8, 10, 0.002, 0.9, 30.0, flags=q.QPA_SOLVE_GRAPH),
                  noalloc=True)
    # the context still solves after the rejections
    out = eng.solve(small, q.make_params(8, 10, 0.002, 0.9, 30.0), noalloc=True)
    assert out["energy"].shape[0] == 8
