"""Parity of the GPU low-energy spectrum (Sec. V.A) with the oracle: the distinct
states, their energies, multiplicities and first replicas must match exactly."""
import sys

import numpy as np
import pytest

import oracle as orc
from paper_2501_19221_amd import instances as gen

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-spectrum] " + msg, flush=True)
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


def _samples(R, n, distinct, seed):
    """R samples drawn from `distinct` random states, with integer energies of a random
    coupling matrix (so equal-energy distinct states occur)."""
    rng = np.random.default_rng(seed)
    pool = (2 * rng.integers(0, 2, (distinct, n)) - 1).astype(np.int8)
    s = pool[rng.integers(0, distinct, R)]
    J = rng.integers(-2, 3, (n, n))
    J = np.triu(J, 1)
    J = (J + J.T).astype(np.int32)
    e = np.array([orc.ising_energy_int(J, np.zeros(n, np.int64), s[r]) for r in range(R)],
                 np.float64)
    return s, e


def _check(eng, s, e, k, flags=0):
    import torch
    out = eng.spectrum(torch.from_numpy(s).cuda(), torch.from_numpy(e).cuda(), k, flags)
    st, E, cnt, first, distinct = orc.spectrum(s, e, k)
    assert out["distinct"] == distinct
    assert np.array_equal(out["spins"].cpu().numpy(), st)
    assert np.array_equal(out["energy"].cpu().numpy(), E)
    assert np.array_equal(out["count"].cpu().numpy(), cnt)
    assert np.array_equal(out["first"].cpu().numpy(), first)


@pytest.mark.parametrize("R,n,distinct,k", [(1000, 9, 300, 50), (1024, 130, 40, 1024),
                                            (4096, 64, 4096, 10), (1, 5, 1, 3),
                                            (3000, 200, 7, 7), (777, 1, 2, 5)])
@pytest.mark.parametrize("flags", [0, 1])
def test_spectrum_matches_oracle(q, eng, R, n, distinct, k, flags):
    say("spectrum R=%d n=%d distinct<=%d k=%d flags=%d" % (R, n, distinct, k, flags))
    s, e = _samples(R, n, distinct, seed=R + n)
    _check(eng, s, e, k, flags)


def test_spectrum_of_pa_samples(q, eng):
    """2^10 PA samples of a Chimera instance (the oracle's own run supplies them)."""
    inst = gen.chimera_ising(3, seed=2)
    c = inst.csr
    lam = orc.lambda_linear(300, 10.0)
    ref = orc.solve_csr_int(c.rp, c.col, c.w, np.zeros(inst.n, np.int64), 1024, 300, lam, 0.2,
                            0.8, 1, np.float32(0.1))
    say("spectrum of 1024 PA samples")
    _check(eng, ref.spins, ref.energy.astype(np.float64), 64)


def test_spectrum_signed_zero_and_limits(q, eng):
    import torch
    s = np.array([[1, 1], [-1, -1], [1, -1]], np.int8)
    e = np.array([0.0, -0.0, -1.0])
    _check(eng, s, e, 5)
    big = torch.ones((q.QPA_SPECTRUM_MAX_R + 1, 4), dtype=torch.int8, device="cuda")
    with pytest.raises(q.QpaError) as ei:
        eng.spectrum(big, torch.zeros(big.shape[0], dtype=torch.float64, device="cuda"), 4)
    assert ei.value.status == q.QPA_E_UNSUPPORTED
