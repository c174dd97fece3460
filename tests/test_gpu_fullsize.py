"""Parity of the dense step kernels at the benchmarked size (n = 4096, R = 1024) and at
reduction depths where every LDS stage of the matrix-core loop is refilled and read.

* BF16 matrix cores, float couplings (the sk4096 workload, its own launch shape):
  teacher-forced steps at t = 0, 1, 999 and 1999 -- the GPU runs to step t, its state
  is copied, one more GPU step returns the fields, and the oracle takes the same step
  from the copied state on sampled replicas with the BF16-rounded couplings.  Fields
  must agree within 1e-5 of each row's magnitude (sum_j |J_ij| + |b_i|); given the GPU's
  fields, the oracle's update must reproduce the GPU's x and m bit for bit.
* BF16 matrix cores, integer couplings (exact in BF16) over 8 reduction chunks: whole
  solve bit-exact.
* FP32 tiled product at n = 4096, R = 1024: 20 steps bit-exact on sampled replicas.
"""
import sys

import numpy as np
import pytest

import oracle as orc
from paper_2501_19221_amd import instances as gen
from paper_2501_19221_amd.configs import WORKLOADS

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-fullsize] " + msg, flush=True)
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


@pytest.fixture(scope="module")
def sk4096():
    return WORKLOADS["sk4096"].make()


def host(t):
    return t.detach().cpu().numpy()


def _paths(q, eng, fn):
    q.qpa_profile_read(eng.ctx, reset=True)
    q.qpa_profile_enable(eng.ctx, True)
    try:
        res = fn()
    finally:
        q.qpa_profile_enable(eng.ctx, False)
    used = {}
    for code in range(0, 12):
        _, k = q.qpa_profile_read_path(eng.ctx, code)
        if k:
            used[code] = k
    q.qpa_profile_read(eng.ctx, reset=True)
    return res, used


SAMPLE = [0, 127, 128, 511, 1023]          # first/last of a 128-replica tile, both ends


def test_sk4096_bf16_teacher_forced_full_depth(q, eng, sk4096):
    import torch
    wl = WORKLOADS["sk4096"]
    inst = sk4096
    n, R, T = inst.n, wl.replicas, wl.steps
    e = orc.bf16_scale_exponent(inst.dense)
    Jq = orc.bf16_quantise(inst.dense, e)
    rowmag = np.abs(Jq.astype(np.float64)).sum(1) + np.abs(inst.lin.astype(np.float64))
    lam = orc.lambda_linear(T, wl.lambda0)
    prob = q.Problem.from_instance(inst)
    p = q.make_params(R, T, wl.eta, wl.alpha, wl.lambda0, wl.sigma0, wl.seed, q.QPA_PREC_BF16)
    x0, m0 = orc.pa_init(n, R, wl.seed, np.float32(wl.sigma0))
    xd, md = torch.from_numpy(x0).cuda(), torch.from_numpy(m0).cuda()
    t_done = 0
    for t in [0, 1, 999, 1999]:
        if t > t_done:
            eng.steps(prob, p, t_done, t, xd, md)
        t_done = t
        xs, ms = host(xd), host(md)
        say("sk4096 bf16: step %d from the GPU state" % t)
        h, used = _paths(q, eng, lambda: eng.steps(prob, p, t, t + 1, xd, md, want_h=True))
        assert list(used) == [q.QPA_PATH_DENSE_MFMA], used
        t_done = t + 1
        hg, xg, mg = host(h), host(xd), host(md)
        xr, mr = xs[SAMPLE].copy(), ms[SAMPLE].copy()
        h_ref = orc.pa_steps_dense_float(Jq, inst.lin, xr, mr, t, t + 1, lam, wl.eta, wl.alpha,
                                         want_h=True)
        dh = np.abs(hg[SAMPLE] - h_ref)
        assert np.all(dh <= 1e-5 * rowmag[None, :]), (t, float((dh / rowmag).max()))
        # the field against its exact value (FP64 sum of the BF16 couplings, +-1 spins)
        s = np.where(xs[SAMPLE] >= 0, 1.0, -1.0)
        exact = s @ Jq.astype(np.float64).T + inst.lin.astype(np.float64)
        assert np.all(np.abs(hg[SAMPLE] - exact) <= 1e-5 * rowmag[None, :])
        # given the GPU's fields, the update is the oracle's, bit for bit, on every replica
        xu, mu = xs.copy(), ms.copy()
        orc.pa_update(hg, xu, mu, lam[t], wl.eta, wl.alpha)
        assert np.array_equal(xu, xg) and np.array_equal(mu, mg), t
        # spins near zero are where the two sums may disagree on a sign; count them
        flips = int((np.sign(xg[SAMPLE]) != np.sign(xr)).sum())
        say("sk4096 bf16 step %d: max |dh|/rowmag %.2e, sign disagreements %d"
            % (t, float((dh / rowmag).max()), flips))


def test_bf16_integer_bit_exact_eight_chunks(q, eng):
    """Integer couplings (|J| <= 50, exact in BF16) at n = 1000: 8 reduction chunks, so
    stages refilled in the loop are read; 130 replicas = a full and a ragged tile."""
    inst = gen.dense_int_ising(1000, -50, 50, seed=31)
    R, T, eta, alpha, lam0 = 130, 25, 0.001, 0.7, 50.0
    prob = q.Problem.from_instance(inst)
    p = q.make_params(R, T, eta, alpha, lam0, 0.1, 5, q.QPA_PREC_BF16)
    say("bf16 integer n=1000 R=130 T=25")
    out, used = _paths(q, eng, lambda: eng.solve(prob, p, want_state=True))
    assert list(used) == [q.QPA_PATH_DENSE_MFMA], used
    ref = orc.solve_dense_int(inst.dense, inst.lin, "ising", R, T, orc.lambda_linear(T, lam0),
                              eta, alpha, 5, 0.1)
    assert np.array_equal(host(out["x"]), ref.x)
    assert np.array_equal(host(out["m"]), ref.m)
    assert np.array_equal(host(out["spins"]), ref.spins)
    assert np.array_equal(host(out["energy_i64"]), ref.energy)
    assert int(host(out["best"])[0]) == ref.best


def test_sk4096_fp32_tiled_sampled_bit_exact(q, eng, sk4096):
    """The FP32 form (the metric's comparator) at the benchmarked size: 20 steps of all
    1024 replicas, sampled replicas bit-exact against the oracle's sequential FP32 sums."""
    import torch
    wl = WORKLOADS["sk4096"]
    inst = sk4096
    n, R, T = inst.n, wl.replicas, 20
    prob = q.Problem.from_instance(inst)
    p = q.make_params(R, T, wl.eta, wl.alpha, wl.lambda0, wl.sigma0, wl.seed, q.QPA_PREC_FP32)
    x0, m0 = orc.pa_init(n, R, wl.seed, np.float32(wl.sigma0))
    xd, md = torch.from_numpy(x0).cuda(), torch.from_numpy(m0).cuda()
    say("sk4096 fp32 tiled, 20 steps")
    h, used = _paths(q, eng, lambda: eng.steps(prob, p, 0, T, xd, md, want_h=True))
    assert list(used) == [q.QPA_PATH_DENSE_TILED], used
    lam = orc.lambda_linear(T, wl.lambda0)
    xr, mr = x0[SAMPLE].copy(), m0[SAMPLE].copy()
    h_ref = orc.pa_steps_dense_float(inst.dense, inst.lin, xr, mr, 0, T, lam, wl.eta, wl.alpha,
                                     want_h=True)
    assert np.array_equal(host(xd)[SAMPLE], xr)
    assert np.array_equal(host(md)[SAMPLE], mr)
    assert np.array_equal(host(h)[SAMPLE], h_ref)
