"""Parity of the HIP path (called through the C ABI) with the CPU oracle.

Integer couplings, and float couplings on the FP32 paths (which sum every field in
ascending column order, as the oracle does), must match bit for bit: final analog
states, momenta, spins, exact energies and the best replica.  The BF16 matrix-core path
sums in another order, so float couplings there are checked one step at a time from the
oracle's state (teacher forcing) within 1e-5 relative to each row's magnitude; integer
couplings small enough to be exact in BF16 must again match bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle as orc
from paper_2501_19221_amd import instances as gen
from paper_2501_19221_amd.configs import WORKLOADS

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-parity] " + msg, flush=True)
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


def host(t):
    return t.detach().cpu().numpy()


def _params(q, R, T, eta, alpha, lam0, sigma0=0.1, seed=1, prec="fp32", flags=0):
    return q.make_params(R, T, eta, alpha, lam0, sigma0, seed,
                         q.QPA_PREC_BF16 if prec == "bf16" else q.QPA_PREC_FP32, flags=flags)


def _check_solve_dense_int(q, eng, inst, R, T, eta, alpha, lam0, prec="fp32", seed=1):
    prob = q.Problem.from_instance(inst)
    p = _params(q, R, T, eta, alpha, lam0, seed=seed, prec=prec)
    say("dense int %s n=%d R=%d T=%d prec=%s" % (inst.kind, inst.n, R, T, prec))
    out = eng.solve(prob, p, want_state=True)
    lam = orc.lambda_linear(T, lam0)
    ref = orc.solve_dense_int(inst.dense, inst.lin, inst.kind, R, T, lam, eta, alpha, seed, 0.1)
    assert np.array_equal(host(out["x"]), ref.x)
    assert np.array_equal(host(out["m"]), ref.m)
    assert np.array_equal(host(out["spins"]), ref.spins)
    assert np.array_equal(host(out["energy_i64"]), ref.energy)
    assert np.array_equal(host(out["energy"]), ref.energy.astype(np.float64))
    assert int(host(out["best"])[0]) == ref.best
    return out, ref


# ------------------------------------------------------------------ dense, integer
def test_dense20_full_workload_bit_exact(q, eng):
    wl = WORKLOADS["dense20"]
    inst = wl.make()
    out, ref = _check_solve_dense_int(q, eng, inst, wl.replicas, wl.steps, wl.eta, wl.alpha,
                                      wl.lambda0)
    J, b, K = orc.qubo_to_ising_int(inst.dense, inst.lin)
    Hmin, _ = orc.bruteforce_ising_int(J, b)
    assert ref.energy.min() == (Hmin + K) // 2          # best-of-replica reaches the optimum


def test_dense20_bf16_path_is_exact_for_small_integers(q, eng):
    wl = WORKLOADS["dense20"]
    _check_solve_dense_int(q, eng, wl.make(), wl.replicas, wl.steps, wl.eta, wl.alpha,
                           wl.lambda0, prec="bf16")


@pytest.mark.parametrize("n,R,T", [(300, 70, 50), (129, 3, 30), (1, 1, 5), (2, 1, 0)])
def test_dense_int_ising_ragged(q, eng, n, R, T):
    inst = gen.dense_int_ising(n, -9, 9, seed=n)
    _check_solve_dense_int(q, eng, inst, R, T, 0.01, 0.7, 5.0)


@pytest.mark.parametrize("n", [17, 33, 63, 64, 65, 100, 128])
def test_dense_resident_sizes(q, eng, n):
    """Small dense instances run all steps in one launch: one wave per replica for n <= 64
    (row of J in registers, spins as a ballot), a workgroup of replicas above; both equal
    the oracle bit for bit, fields of the last step included."""
    import torch
    inst = gen.dense_int_ising(n, -9, 9, seed=100 + n)
    _check_solve_dense_int(q, eng, inst, 7, 40, 0.01, 0.7, 5.0)
    prob = q.Problem.from_instance(inst)
    R, T = 5, 23
    p = _params(q, R, T, 0.02, 0.8, 6.0)
    x0, _ = orc.pa_init(n, R, 1, np.float32(0.1))
    xd = torch.from_numpy(x0.copy()).cuda()
    md = torch.zeros_like(xd)
    h = eng.steps(prob, p, 0, T, xd, md, want_h=True)
    x, m = x0.copy(), np.zeros_like(x0)
    hr = orc.pa_steps_dense_int(inst.dense, inst.lin, x, m, 0, T, orc.lambda_linear(T, 6.0),
                                0.02, 0.8, want_h=True)
    assert np.array_equal(host(xd), x) and np.array_equal(host(md), m)
    assert np.array_equal(host(h), hr)


def test_dense_int_bf16_ragged_tiles(q, eng):
    inst = gen.dense_int_ising(200, -50, 50, seed=8)
    _check_solve_dense_int(q, eng, inst, 130, 40, 0.001, 0.7, 50.0, prec="bf16")


# ------------------------------------------------------------------ dense, float
def _oracle_dense_float(J, b, R, T, lam, eta, alpha, seed=1):
    x, m = orc.pa_init(J.shape[0], R, seed, np.float32(0.1))
    orc.pa_steps_dense_float(J, b, x, m, 0, T, lam, eta, alpha)
    return x, m


@pytest.mark.parametrize("n,R,T", [(300, 70, 40), (64, 5, 100), (20, 9, 50), (45, 3, 60), (100, 4, 30)])
def test_dense_float_fp32_bit_exact(q, eng, n, R, T):
    inst = gen.sk_ising(n, 0.1, seed=n)
    prob = q.Problem.from_instance(inst)
    p = _params(q, R, T, 0.2, 0.8, 4.0)
    say("dense float fp32 n=%d R=%d T=%d" % (n, R, T))
    out = eng.solve(prob, p, want_state=True)
    x, m = _oracle_dense_float(inst.dense, inst.lin, R, T, orc.lambda_linear(T, 4.0), 0.2, 0.8)
    assert np.array_equal(host(out["x"]), x)
    assert np.array_equal(host(out["m"]), m)
    s = np.where(x >= 0, 1, -1).astype(np.int8)
    e = np.array([orc.ising_energy_float(inst.dense.astype(np.float64),
                                         inst.lin.astype(np.float64), s[r]) for r in range(R)])
    np.testing.assert_allclose(host(out["energy"]), e, rtol=1e-12, atol=1e-9)
    assert int(host(out["best"])[0]) == int(np.argmin(e))


def test_mfma_float_teacher_forced(q, eng):
    n, R, T = 300, 70, 60
    inst = gen.sk_ising(n, 0.1, seed=5)
    e = orc.bf16_scale_exponent(inst.dense)
    Jq = orc.bf16_quantise(inst.dense, e)
    lam = orc.lambda_linear(T, 4.0)
    prob = q.Problem.from_instance(inst)
    p = _params(q, R, T, 0.2, 0.8, 4.0, prec="bf16")
    x, m = orc.pa_init(n, R, 1, np.float32(0.1))
    rowmag = np.abs(Jq.astype(np.float64)).sum(1) + np.abs(inst.lin)
    eta, alpha = 0.2, 0.8
    import torch
    for t in range(T):
        x0, m0 = x.copy(), m.copy()
        h_ref = orc.pa_steps_dense_float(Jq, inst.lin, x0, m0, t, t + 1, lam, eta, alpha,
                                         want_h=True)
        if t % 15 == 0 or t == T - 1:
            say("mfma teacher-forced step %d" % t)
            xd = torch.from_numpy(x).cuda()
            md = torch.from_numpy(m).cuda()
            h = eng.steps(prob, p, t, t + 1, xd, md, want_h=True)
            # field: 1e-5 relative to the row's magnitude sum_j |J_ij| + |b_i|
            tol_h = 1e-5 * rowmag[None, :]
            dh = np.abs(host(h) - h_ref)
            assert np.all(dh <= tol_h), dh.max()
            # states: m' = alpha m - eta (lambda x + h) and x' = clip(x + m') move by eta
            # times the field difference, plus 1e-5 of the magnitude of the update's terms
            terms = (np.abs(x) + alpha * np.abs(m)
                     + eta * (np.abs(lam[t] * x) + np.abs(h_ref)))
            tol_s = eta * tol_h + 1e-5 * terms
            assert np.all(np.abs(host(md) - m0) <= tol_s)
            assert np.all(np.abs(host(xd) - x0) <= tol_s)
        x, m = x0, m0


# ------------------------------------------------------------------ CSR
def _oracle_csr(inst, R, T, lam, eta, alpha, r0=0, seed=1):
    c = inst.csr
    if inst.kind == "qubo":
        rp, col, w, b, K = orc.qubo_to_ising_csr_int(c.rp, c.col, c.w, inst.lin)
    else:
        rp, col, w, b, K = c.rp, c.col, c.w, inst.lin, 0
    x, m = orc.pa_init(inst.n, R, seed, np.float32(0.1), r0=r0)
    if np.issubdtype(np.asarray(w).dtype, np.floating):
        orc.pa_steps_csr_float(rp, col, w, b, x, m, 0, T, lam, eta, alpha)
    else:
        orc.pa_steps_csr_int(rp, col, w, b, x, m, 0, T, lam, eta, alpha)
    return x, m, (rp, col, w, b, K)


def _energies_csr_int(canon, kind, s):
    rp, col, w, b, K = canon
    H = np.array([orc.ising_energy_csr_int(rp, col, w, b, s[r]) for r in range(len(s))])
    return (H + K) // 2 if kind == "qubo" else H


def _launches_by_path(q, eng, fn):
    """Runs fn() with kernel profiling on; returns {path code: step-kernel launches}."""
    q.qpa_profile_read(eng.ctx, reset=True)
    q.qpa_profile_enable(eng.ctx, True)
    try:
        res = fn()
    finally:
        q.qpa_profile_enable(eng.ctx, False)
    paths = {}
    for code in range(0, 7):
        _, n = q.qpa_profile_read_path(eng.ctx, code)
        if n:
            paths[code] = n
    q.qpa_profile_read(eng.ctx, reset=True)
    return res, paths


@pytest.mark.parametrize("streamed", [False, True])
@pytest.mark.parametrize("m_,R,T", [(4, 70, 200), (2, 1, 30), (3, 64, 50)])
def test_csr_chimera_bit_exact(q, eng, m_, R, T, streamed):
    inst = gen.chimera_ising(m_, seed=m_)
    prob = q.Problem.from_instance(inst)
    p = _params(q, R, T, 0.2, 0.8, 10.0, flags=q.QPA_SOLVE_STREAMED if streamed else 0)
    say("csr chimera m=%d R=%d T=%d streamed=%s" % (m_, R, T, streamed))
    out, paths = _launches_by_path(q, eng, lambda: eng.solve(prob, p, want_state=True))
    want = q.QPA_PATH_CSR if streamed else q.QPA_PATH_CSR_RESIDENT
    assert list(paths) == [want], paths
    x, m, canon = _oracle_csr(inst, R, T, orc.lambda_linear(T, 10.0), 0.2, 0.8)
    assert np.array_equal(host(out["x"]), x)
    assert np.array_equal(host(out["m"]), m)
    s = np.where(x >= 0, 1, -1).astype(np.int8)
    assert np.array_equal(host(out["spins"]), s)
    e = _energies_csr_int(canon, "ising", s)
    assert np.array_equal(host(out["energy_i64"]), e)
    assert int(host(out["best"])[0]) == int(np.flatnonzero(e == e.min())[0])


@pytest.mark.parametrize("scale,G", [(10900, 4), (10900, 8), (11000, 2), (20000, 4)])
def test_csr_resident_weight_bound(q, eng, scale, G):
    """Resident kernel on either side of its packed-sum bound: rows with a sum of |w|
    below 2^16 (6 x 10900 = 65400 plus a field) take two replicas per 32-bit word,
    6 x 11000 and 6 x 20000 the general int32 sums; both equal the oracle bit for bit."""
    base = gen.chimera_ising(4, seed=9)
    rng = np.random.default_rng(scale)
    c = base.csr
    w = c.w.astype(np.int32) * scale
    # symmetric magnitudes in [scale - 100, scale]: perturb the upper triangle, mirror it
    rows = np.repeat(np.arange(base.n), np.diff(c.rp)).astype(np.int64)
    cols = c.col.astype(np.int64)
    pair = np.minimum(rows, cols) * base.n + np.maximum(rows, cols)
    uniq, inv = np.unique(pair, return_inverse=True)
    d = rng.integers(0, 101, size=len(uniq))[inv]
    w = (np.sign(w) * (np.abs(w) - d)).astype(np.int16)
    lin = rng.integers(-50, 51, size=base.n).astype(np.int16)
    inst = gen.Instance("ising", base.n, csr=gen.CSR(base.n, c.rp, c.col, w), lin=lin, meta={})
    prob = q.Problem.from_instance(inst)
    R, T = 4 * G, 25
    eng.tune_set(prob, _params(q, R, T, 0.0002, 0.8, 20000.0), G)
    p = _params(q, R, T, 0.0002, 0.8, 20000.0)
    say("resident weight bound scale=%d G=%d" % (scale, G))
    out, paths = _launches_by_path(q, eng, lambda: eng.solve(prob, p, want_state=True))
    assert paths == {q.QPA_PATH_CSR_RESIDENT: 1}, paths
    x, m, canon = _oracle_csr(inst, R, T, orc.lambda_linear(T, 20000.0), 0.0002, 0.8)
    assert np.array_equal(host(out["x"]), x) and np.array_equal(host(out["m"]), m)
    s = np.where(x >= 0, 1, -1).astype(np.int8)
    assert np.array_equal(host(out["energy_i64"]), _energies_csr_int(canon, "ising", s))


# replica groups G = 8, 4, 2, 1 and 2, 2, 4, 8, 1 variables per thread of the resident
# kernel, with replica counts that leave a partial group (the n = 6000 graph has degree 3,
# so that its CSR fits in LDS)
@pytest.mark.parametrize("graph,R,T", [("chimera14", 2050, 12), ("chimera14", 1100, 15),
                                       ("chimera19", 515, 10), ("planted6000", 300, 6),
                                       ("chimera1", 7, 40)])
def test_csr_resident_groups_bit_exact(q, eng, graph, R, T):
    if graph.startswith("chimera"):
        m_ = int(graph[len("chimera"):])
        inst = gen.chimera_ising(m_, seed=m_ + 1)
    else:
        inst = gen.planted_3regular(6000, 1, 7, seed=3)
    prob = q.Problem.from_instance(inst)
    p = _params(q, R, T, 0.2, 0.8, 10.0)
    say("csr resident chimera n=%d R=%d T=%d" % (inst.n, R, T))
    out, paths = _launches_by_path(q, eng, lambda: eng.solve(prob, p, want_state=True))
    assert list(paths) == [q.QPA_PATH_CSR_RESIDENT], paths
    x, m, canon = _oracle_csr(inst, R, T, orc.lambda_linear(T, 10.0), 0.2, 0.8)
    assert np.array_equal(host(out["x"]), x)
    assert np.array_equal(host(out["m"]), m)
    s = np.where(x >= 0, 1, -1).astype(np.int8)
    e = _energies_csr_int(canon, "ising", s)
    assert np.array_equal(host(out["energy_i64"]), e)


def test_chimera16_full_workload_replica_subset(q, eng):
    wl = WORKLOADS["chimera16"]
    inst = wl.make()
    prob = q.Problem.from_instance(inst)
    p = _params(q, wl.replicas, wl.steps, wl.eta, wl.alpha, wl.lambda0)
    say("chimera16 full workload R=%d T=%d" % (wl.replicas, wl.steps))
    out = eng.solve(prob, p, want_state=True)
    gx, gm, gs = host(out["x"]), host(out["m"]), host(out["spins"])
    lam = orc.lambda_linear(wl.steps, wl.lambda0)
    for r0 in [0, 1, 511, 1023]:
        x, m, canon = _oracle_csr(inst, 1, wl.steps, lam, wl.eta, wl.alpha, r0=r0)
        assert np.array_equal(gx[r0], x[0]) and np.array_equal(gm[r0], m[0])
    e = _energies_csr_int((inst.csr.rp, inst.csr.col, inst.csr.w, inst.lin, 0), "ising", gs)
    assert np.array_equal(host(out["energy_i64"]), e)
    assert int(host(out["best"])[0]) == int(np.flatnonzero(e == e.min())[0])


@pytest.mark.parametrize("streamed", [False, True])
def test_csr_er_qubo_int16(q, eng, streamed):
    rng = np.random.default_rng(3)
    inst = gen.er_qubo(300, 0.1, 100, rng)
    # add diagonal terms to exercise the QUBO fold
    c = inst.csr
    n = inst.n
    d = c.to_dense(np.int32)
    d[np.arange(n), np.arange(n)] = rng.integers(-20, 21, n)
    rows, cols = np.nonzero(d)
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    inst.csr = gen.CSR(n, rp.astype(np.int32), cols.astype(np.int16), d[rows, cols].astype(np.int16))
    R, T = 5, 100
    prob = q.Problem.from_instance(inst)
    p = _params(q, R, T, 0.0002, 0.8, 200.0, flags=q.QPA_SOLVE_STREAMED if streamed else 0)
    say("csr ER qubo int16 n=%d R=%d T=%d streamed=%s" % (n, R, T, streamed))
    out = eng.solve(prob, p, want_state=True)
    x, m, canon = _oracle_csr(inst, R, T, orc.lambda_linear(T, 200.0), 0.0002, 0.8)
    assert np.array_equal(host(out["x"]), x) and np.array_equal(host(out["m"]), m)
    s = np.where(x >= 0, 1, -1).astype(np.int8)
    e = _energies_csr_int(canon, "qubo", s)
    assert np.array_equal(host(out["energy_i64"]), e)
    # independent check of the QUBO objective on x = (1+s)/2
    for r in range(R):
        xb = ((s[r] + 1) // 2).astype(np.int8)
        assert e[r] == orc.qubo_energy_int(d, inst.lin, xb)


@pytest.mark.parametrize("streamed", [False, True])
def test_csr_float_weights_bit_exact(q, eng, streamed):
    inst = gen.chimera_ising(3, seed=4)
    rng = np.random.default_rng(0)
    c = inst.csr
    D = c.to_dense(np.int32).astype(np.float32)
    W = np.triu(rng.standard_normal(D.shape).astype(np.float32) * (D != 0), 1)
    W = W + W.T
    rows, cols = np.nonzero(D)
    inst.csr = gen.CSR(inst.n, c.rp, c.col, W[rows, cols].astype(np.float32))
    inst.lin = rng.standard_normal(inst.n).astype(np.float32) * 0.3
    R, T = 3, 80
    prob = q.Problem.from_instance(inst)
    p = _params(q, R, T, 0.1, 0.8, 2.0, flags=q.QPA_SOLVE_STREAMED if streamed else 0)
    say("csr float weights n=%d streamed=%s" % (inst.n, streamed))
    out = eng.solve(prob, p, want_state=True)
    x, m, _ = _oracle_csr(inst, R, T, orc.lambda_linear(T, 2.0), 0.1, 0.8)
    assert np.array_equal(host(out["x"]), x) and np.array_equal(host(out["m"]), m)


# ------------------------------------------------------------------ best state over the trajectory
@pytest.mark.parametrize("case", ["csr_ising", "csr_qubo", "dense_bf16"])
def test_solve_track_matches_oracle(q, eng, case):
    """qpa_solve_track: each replica's best sampled state (after every `every` steps and
    after the last) is the oracle's -- exact integer energies, the step, the spins -- and
    the final outputs are qpa_solve's."""
    if case == "csr_ising":
        inst, R, T, every, prec = gen.chimera_ising(3, seed=12), 20, 120, 10, "fp32"
    elif case == "csr_qubo":
        inst, R, T, every, prec = gen.er_qubo(150, 0.1, 100, np.random.default_rng(13)), 70, 90, 7, "fp32"
    else:
        inst, R, T, every, prec = gen.dense_int_ising(300, -20, 20, seed=14), 130, 60, 8, "bf16"
    eta, alpha, lam0, seed = 0.05, 0.8, 3.0, 6
    prob = q.Problem.from_instance(inst)
    p = _params(q, R, T, eta, alpha, lam0, seed=seed, prec=prec)
    say("solve_track %s n=%d R=%d T=%d every=%d" % (case, inst.n, R, T, every))
    out = eng.solve_track(prob, p, every, want_state=True)
    ref = eng.solve(prob, p, want_state=True)
    for key in ("x", "m", "spins", "energy_i64", "best"):
        assert np.array_equal(host(out[key]), host(ref[key])), key
    lam = orc.lambda_linear(T, lam0)
    x, m = orc.pa_init(inst.n, R, seed, np.float32(0.1))
    if inst.dense is not None:
        J, b = inst.dense, inst.lin
        step = lambda x_, m_, t0, t1: orc.pa_steps_dense_int(J, b, x_, m_, t0, t1, lam, eta, alpha)
        energy = lambda s_: np.array([orc.ising_energy_int(J, b, s_[r]) for r in range(R)])
    else:
        c = inst.csr
        canon = (orc.qubo_to_ising_csr_int(c.rp, c.col, c.w, inst.lin) if inst.kind == "qubo"
                 else (c.rp, c.col, c.w, inst.lin, 0))
        step = lambda x_, m_, t0, t1: orc.pa_steps_csr_int(canon[0], canon[1], canon[2],
                                                           canon[3], x_, m_, t0, t1, lam, eta,
                                                           alpha)
        energy = lambda s_: _energies_csr_int(canon, inst.kind, s_)
    be, bt, bs = orc.track_best(x, m, T, every, step, energy)
    assert np.array_equal(host(out["best_energy"]), be.astype(np.float64))
    assert np.array_equal(host(out["best_step"]), bt)
    assert np.array_equal(host(out["best_spins"]), bs)
    assert (bt < T).any()                    # some replica's best is not its final state


def test_solve_track_argument_errors(q, eng):
    """every < 1 and missing track outputs are rejected before any work."""
    import ctypes
    inst = gen.chimera_ising(2, seed=1)
    prob = q.Problem.from_instance(inst)
    p = _params(q, 4, 10, 0.1, 0.8, 2.0)
    say("solve_track argument errors")
    for every in (0, -3):
        with pytest.raises(q.QpaError) as ei:
            eng.solve_track(prob, p, every)
        assert ei.value.status == q.QPA_E_ARG, str(ei.value)
    ps = prob.struct()
    ws, nbytes = eng.workspace(ps, p)
    out = eng.solve(prob, p)
    o = q.qpa_outputs()
    o.energy = out["energy"].data_ptr()
    o.best = out["best"].data_ptr()
    tr = q.qpa_track_outputs()                      # all three outputs missing
    with pytest.raises(q.QpaError) as ei:
        q.qpa_solve_track(eng.ctx, ps, p, 5, ctypes.c_void_p(ws.data_ptr()), nbytes,
                          eng._stream(), o, tr)
    assert ei.value.status == q.QPA_E_ARG, str(ei.value)


# ------------------------------------------------------------------ energies, resume, errors
def test_energy_entry_point(q, eng):
    import torch
    rng = np.random.default_rng(11)
    # R = 1100: the dense energies' replicas span three blocks of 512 (the last ragged)
    for inst, R in [(gen.dense_int_qubo(50, seed=3), 33), (gen.sk_ising(70, seed=2), 33),
                    (gen.chimera_ising(3, seed=1), 33), (gen.dense_int_qubo(40, seed=5), 1100),
                    (gen.sk_ising(30, seed=6), 1100)]:
        s = (2 * rng.integers(0, 2, (R, inst.n)) - 1).astype(np.int8)
        prob = q.Problem.from_instance(inst)
        say("energy entry point %s n=%d" % (inst.kind, inst.n))
        e, ei, best = eng.energy(prob, _params(q, R, 1, 0.1, 0.5, 1.0), torch.from_numpy(s).cuda())
        if inst.dense is not None and inst.kind == "qubo":
            ref = np.array([orc.qubo_energy_int(inst.dense, inst.lin, ((s[r] + 1) // 2).astype(np.int8))
                            for r in range(R)])
            assert np.array_equal(host(ei), ref)
        elif inst.dense is not None:
            ref = np.array([orc.ising_energy_float(inst.dense.astype(np.float64),
                                                   inst.lin.astype(np.float64), s[r]) for r in range(R)])
            np.testing.assert_allclose(host(e), ref, rtol=1e-12, atol=1e-9)
        else:
            ref = _energies_csr_int((inst.csr.rp, inst.csr.col, inst.csr.w, inst.lin, 0), "ising", s)
            assert np.array_equal(host(ei), ref)
        assert int(host(best)[0]) == int(np.flatnonzero(ref == ref.min())[0])


@pytest.mark.parametrize("which", ["dense-tiled", "csr", "csr-streamed", "mfma"])
def test_resume_split_equals_uninterrupted(q, eng, which):
    import torch
    flags = 0
    if which.startswith("csr"):
        inst, prec = gen.chimera_ising(4, seed=9), "fp32"
        flags = q.QPA_SOLVE_STREAMED if which == "csr-streamed" else 0
    elif which == "mfma":
        inst, prec = gen.dense_int_ising(150, seed=4), "bf16"
    else:
        inst, prec = gen.dense_int_ising(150, seed=4), "fp32"
    R, T = 9, 120
    prob = q.Problem.from_instance(inst)
    p = _params(q, R, T, 0.01, 0.8, 5.0, prec=prec, flags=flags)
    say("resume split %s" % which)
    full = eng.solve(prob, p, want_state=True)
    x, m = orc.pa_init(inst.n, R, 1, np.float32(0.1))
    xd, md = torch.from_numpy(x).cuda(), torch.from_numpy(m).cuda()
    eng.steps(prob, p, 0, 37, xd, md)
    eng.steps(prob, p, 37, 37, xd, md)
    eng.steps(prob, p, 37, T, xd, md)
    assert torch.equal(xd, full["x"]) and torch.equal(md, full["m"])


def _expect_status(q, eng, inst, status, prec="fp32"):
    prob = q.Problem.from_instance(inst)
    with pytest.raises(q.QpaError) as ei:
        eng.solve(prob, _params(q, 4, 3, 0.1, 0.5, 1.0, prec=prec))
    assert ei.value.status == status, str(ei.value)


def test_invalid_inputs_are_rejected(q, eng):
    say("error paths")
    a = gen.dense_int_qubo(10, seed=1)
    a.dense = a.dense.copy()
    a.dense[2, 3] += 1
    _expect_status(q, eng, a, q.QPA_E_ASYM)
    b = gen.dense_int_ising(10, seed=1)
    b.dense = b.dense.copy()
    b.dense[4, 4] = 1
    _expect_status(q, eng, b, q.QPA_E_ASYM)
    c = gen.dense_int_ising(10, seed=1)
    c.dense = np.full((10, 10), 2**22, np.int32)
    np.fill_diagonal(c.dense, 0)
    _expect_status(q, eng, c, q.QPA_E_RANGE)
    d = gen.chimera_ising(2, seed=1)
    col = d.csr.col.copy()
    col[[0, 1]] = col[[1, 0]]
    d.csr = gen.CSR(d.n, d.csr.rp, col, d.csr.w)
    _expect_status(q, eng, d, q.QPA_E_SHAPE)
    e = gen.chimera_ising(2, seed=1)
    w = e.csr.w.copy()
    w[0] = -w[0]
    e.csr = gen.CSR(e.n, e.csr.rp, e.csr.col, w)
    _expect_status(q, eng, e, q.QPA_E_ASYM)


def test_workspace_too_small(q, eng):
    import ctypes
    import torch
    inst = gen.dense_int_qubo(20, seed=1)
    prob = q.Problem.from_instance(inst)
    p = _params(q, 4, 3, 0.1, 0.5, 1.0)
    ps = prob.struct()
    need = q.qpa_workspace_size(eng.ctx, ps, p)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    out = {k: torch.empty(4, dtype=dt, device="cuda") for k, dt in
           [("e", torch.float64), ("b", torch.int32)]}
    o = q.qpa_outputs()
    o.energy = out["e"].data_ptr()
    o.best = out["b"].data_ptr()
    st = q._lib.qpa_solve(eng.ctx, ctypes.byref(ps), ctypes.byref(p),
                          ctypes.c_void_p(ws.data_ptr()), need - 1, None, ctypes.byref(o))
    assert st == q.QPA_E_WORKSPACE


def test_zero_steps_scores_initial_state(q, eng):
    inst = gen.chimera_ising(2, seed=3)
    prob = q.Problem.from_instance(inst)
    say("zero steps")
    out = eng.solve(prob, _params(q, 6, 0, 0.1, 0.5, 1.0), want_state=True)
    x, m = orc.pa_init(inst.n, 6, 1, np.float32(0.1))
    assert np.array_equal(host(out["x"]), x)
    s = np.where(x >= 0, 1, -1).astype(np.int8)
    e = _energies_csr_int((inst.csr.rp, inst.csr.col, inst.csr.w, inst.lin, 0), "ising", s)
    assert np.array_equal(host(out["energy_i64"]), e)


def test_empty_csr(q, eng):
    inst = gen.Instance("ising", 5, csr=gen.CSR(5, np.zeros(6, np.int32), np.zeros(0, np.int32),
                                                np.zeros(0, np.int8)),
                        lin=np.array([1, -2, 0, 3, -1], np.int8))
    prob = q.Problem.from_instance(inst)
    say("empty csr")
    out = eng.solve(prob, _params(q, 2, 400, 0.05, 0.5, 1.0))
    # with no couplings each spin settles opposite to its field
    assert int(host(out["energy_i64"]).min()) == -7


# ------------------------------------------------------------------ batched instances
def _oracle_instance(inst, R, T, lam, eta, alpha, seed, r0=0):
    x, m, canon = _oracle_csr(inst, R, T, lam, eta, alpha, r0=r0, seed=seed)
    return x, m, canon


@pytest.mark.parametrize("R", [70, 40])
@pytest.mark.parametrize("path", ["auto", "sparse", "dense"])
def test_batch_uneven_instances_bit_exact(q, eng, path, R):
    # Both batch paths give the oracle's bits on integer instances.  The last instance has
    # couplings up to 300 (not exact in BF16), so it stays sparse even when dense is forced.
    # R = 70: a full and a partial group of 64 (sparse kernel), live replicas in both halves
    # of the matrix-core tile; R = 40: only the first half of the tile is live.
    rng = np.random.default_rng(7)
    insts = [gen.er_qubo(int(n), 0.1, 100, rng) for n in rng.integers(30, 400, size=9)]
    insts.append(gen.er_qubo(200, 0.5, 100, rng))       # too dense for int8 entry lists
    insts.append(gen.chimera_ising(3, seed=5))          # an Ising instance in the same batch
    insts.append(gen.er_qubo(400, 0.005, 100, rng))     # sparse enough for the sparse kernel
    insts.append(gen.er_qubo(250, 0.1, 200, rng))       # |w| up to 200: BF16 tiles, not int8
    insts.append(gen.er_qubo(300, 0.2, 300, rng))
    T, eta, alpha, lam0 = 60, 0.0002, 0.8, 200.0
    probs = [q.Problem.from_instance(i) for i in insts]
    flags = {"auto": 0, "sparse": q.QPA_BATCH_SPARSE, "dense": q.QPA_BATCH_DENSE}[path]
    p = _params(q, R, T, eta, alpha, lam0, seed=11, flags=flags)
    say("batch of %d uneven instances, R=%d T=%d path=%s" % (len(insts), R, T, path))
    outs = eng.solve_batch(probs, p, want_state=True)
    paths = q.qpa_batch_paths(eng.ctx, len(insts))
    assert paths[-1] == q.QPA_PATH_BATCH_SPARSE           # |w| up to 300: never densified
    if path == "sparse":
        assert (paths == q.QPA_PATH_BATCH_SPARSE).all()
    elif path == "dense":
        # |w| <= 127: int8 tiles, as entry lists where every 16 x 128 block is sparse enough
        assert (paths[:9] == q.QPA_PATH_BATCH_SPARSE_I8).all()
        assert paths[9] == q.QPA_PATH_BATCH_DENSE_I8             # half of all pairs
        assert (paths[10:12] == q.QPA_PATH_BATCH_SPARSE_I8).all()
        assert paths[-2] == q.QPA_PATH_BATCH_DENSE               # |w| <= 200: BF16 tiles
    else:                                                  # the cost model mixes both
        assert paths[0] == q.QPA_PATH_BATCH_SPARSE_I8       # n=379, 10% of pairs
        assert paths[9] == q.QPA_PATH_BATCH_DENSE_I8        # n=200, 50% of pairs
        assert paths[-3] == q.QPA_PATH_BATCH_SPARSE         # n=400, 0.5% of pairs
    lam = orc.lambda_linear(T, lam0)
    for k, (inst, out) in enumerate(zip(insts, outs)):
        x, m, canon = _oracle_instance(inst, R, T, lam, eta, alpha, seed=11 + k)
        assert np.array_equal(host(out["x"]), x), k
        assert np.array_equal(host(out["m"]), m), k
        s = np.where(x >= 0, 1, -1).astype(np.int8)
        assert np.array_equal(host(out["spins"]), s), k
        e = _energies_csr_int(canon, inst.kind, s)
        assert np.array_equal(host(out["energy_i64"]), e), k
        assert int(host(out["best"])[0]) == int(np.flatnonzero(e == e.min())[0]), k


def _float_chimera(m, seed):
    """A Chimera Ising instance with Gaussian float couplings and fields on its graph."""
    inst = gen.chimera_ising(m, seed=seed)
    rng = np.random.default_rng(seed)
    c = inst.csr
    D = c.to_dense(np.int32).astype(np.float32)
    W = np.triu(rng.standard_normal(D.shape).astype(np.float32) * (D != 0), 1)
    W = W + W.T
    rows, cols = np.nonzero(D)
    inst.csr = gen.CSR(inst.n, c.rp, c.col, W[rows, cols].astype(np.float32))
    inst.lin = rng.standard_normal(inst.n).astype(np.float32) * 0.3
    return inst


def test_batch_float_couplings_on_the_sparse_kernel(q, eng):
    """Float couplings are not exact in BF16, so a batch sends them to the sparse task
    kernel (FP32 sums of +-w in row order): the oracle's bits, next to an integer instance,
    with a full and a partial group of 64 replicas."""
    insts = [_float_chimera(3, 41), gen.chimera_ising(2, seed=42), _float_chimera(2, 43)]
    R, T, eta, alpha, lam0 = 70, 60, 0.1, 0.8, 2.0
    probs = [q.Problem.from_instance(i) for i in insts]
    p = _params(q, R, T, eta, alpha, lam0, seed=21)
    say("batch with float couplings, R=%d T=%d" % (R, T))
    outs = eng.solve_batch(probs, p, want_state=True)
    paths = q.qpa_batch_paths(eng.ctx, len(insts))
    assert paths[0] == q.QPA_PATH_BATCH_SPARSE and paths[2] == q.QPA_PATH_BATCH_SPARSE
    lam = orc.lambda_linear(T, lam0)
    for k, (inst, out) in enumerate(zip(insts, outs)):
        x, m, _ = _oracle_instance(inst, R, T, lam, eta, alpha, seed=21 + k)
        assert np.array_equal(host(out["x"]), x), k
        assert np.array_equal(host(out["m"]), m), k


def _with_diagonal(inst, rng, lo=-20, hi=20):
    """The CSR QUBO with Q_ii drawn in [lo, hi] stored as entries (App. A folds them into b)."""
    c, n = inst.csr, inst.n
    d = c.to_dense(np.int32)
    d[np.arange(n), np.arange(n)] = rng.integers(lo, hi + 1, n)
    rows, cols = np.nonzero(d)
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    inst.csr = gen.CSR(n, rp.astype(np.int32), cols.astype(c.col.dtype),
                       d[rows, cols].astype(c.w.dtype))
    return inst


def test_batch_sparse_kernel_with_stored_diagonals(q, eng):
    """QUBOs with stored diagonal entries on the sparse task kernel (the diagonal adds
    nothing to the field there: it is folded into b), a full and a partial replica group:
    the oracle's bits."""
    rng = np.random.default_rng(61)
    insts = [_with_diagonal(gen.er_qubo(int(n), 0.1, 100, rng), rng) for n in (90, 333)]
    insts.append(_with_diagonal(gen.er_qubo(150, 0.05, 100, rng, idx_dtype=np.int32), rng))
    R, T, eta, alpha, lam0 = 70, 50, 0.0002, 0.8, 200.0
    probs = [q.Problem.from_instance(i) for i in insts]
    p = _params(q, R, T, eta, alpha, lam0, seed=31, flags=q.QPA_BATCH_SPARSE)
    say("batch with stored diagonals on the sparse kernel, R=%d T=%d" % (R, T))
    outs = eng.solve_batch(probs, p, want_state=True)
    assert (q.qpa_batch_paths(eng.ctx, len(insts)) == q.QPA_PATH_BATCH_SPARSE).all()
    lam = orc.lambda_linear(T, lam0)
    for k, (inst, out) in enumerate(zip(insts, outs)):
        x, m, canon = _oracle_instance(inst, R, T, lam, eta, alpha, seed=31 + k)
        assert np.array_equal(host(out["x"]), x), k
        assert np.array_equal(host(out["m"]), m), k
        s = np.where(x >= 0, 1, -1).astype(np.int8)
        assert np.array_equal(host(out["energy_i64"]), _energies_csr_int(canon, "qubo", s)), k


def test_batch_autotune_measures_rates_and_chooses_by_them(q, eng):
    """qpa_autotune_batch measures both paths on the device; afterwards every instance
    takes the path the cost model gives with the measured rates (dense when BF16-exact and
    (J bytes + 16 R np) / dense rate < nnz R / sparse rate, J bytes 4 nnz for integer
    couplings with nnz <= np^2 / 10, else 2 np^2), and the results are the oracle's
    bits."""
    rng = np.random.default_rng(17)
    insts = [gen.er_qubo(int(n), 0.1, 100, rng) for n in (60, 200, 350)]
    insts += [gen.chimera_ising(4, seed=3), gen.er_qubo(600, 0.004, 100, rng),
              gen.er_qubo(200, 0.1, 300, rng)]
    R, T, eta, alpha, lam0 = 64, 40, 0.0002, 0.8, 200.0
    probs = [q.Problem.from_instance(i) for i in insts]
    p = _params(q, R, T, eta, alpha, lam0, seed=9)
    say("batch autotune")
    dense_bps, sparse_adds = eng.autotune_batch(probs, p, probe_steps=20)
    say("measured rates: dense %.3g B/s, sparse %.3g adds/s" % (dense_bps, sparse_adds))
    assert 1e10 < dense_bps < 2e13 and 1e9 < sparse_adds < 4e13
    outs = eng.solve_batch(probs, p, want_state=True)
    paths = q.qpa_batch_paths(eng.ctx, len(insts))
    for k, inst in enumerate(insts):
        np_ = -(-inst.n // 128) * 128
        jb = 4.0 * inst.csr.nnz if inst.csr.nnz <= 0.1 * np_ * np_ else 2.0 * np_ * np_
        dense_cost = (jb + 16.0 * R * np_) / dense_bps
        sparse_cost = inst.csr.nnz * R / sparse_adds
        exact = int(np.abs(inst.csr.w).max(initial=0)) <= 256
        want_dense = exact and dense_cost < sparse_cost
        assert (paths[k] != q.QPA_PATH_BATCH_SPARSE) == want_dense, (k, paths[k])
    assert paths[-1] == q.QPA_PATH_BATCH_SPARSE
    lam = orc.lambda_linear(T, lam0)
    for k, (inst, out) in enumerate(zip(insts, outs)):
        x, m, _ = _oracle_instance(inst, R, T, lam, eta, alpha, seed=9 + k)
        assert np.array_equal(host(out["x"]), x) and np.array_equal(host(out["m"]), m), k


def test_batch_reports_the_failing_instance(q, eng):
    # An asymmetric instance in the middle of a batch is named in the error (it has 16 or
    # more entries per row, the batched canonicalisation's case); the context then solves
    # a valid batch to the oracle's bits.
    rng = np.random.default_rng(5)
    insts = [gen.er_qubo(int(n), 0.1, 100, rng) for n in (60, 90, 130, 70, 300, 80, 50)]
    assert insts[4].csr.col.size >= 16 * insts[4].n
    bad = insts[4]
    k0 = int(np.flatnonzero(bad.csr.col[bad.csr.rp[0]:bad.csr.rp[1]] != 0)[0])
    w = bad.csr.w.copy()
    w[k0] += 1
    bad.csr = gen.CSR(bad.n, bad.csr.rp, bad.csr.col, w)
    R, T, eta, alpha, lam0 = 8, 5, 0.0002, 0.8, 200.0
    p = _params(q, R, T, eta, alpha, lam0, seed=3)
    say("batch with an asymmetric instance")
    with pytest.raises(q.QpaError) as ei:
        eng.solve_batch([q.Problem.from_instance(i) for i in insts], p)
    assert ei.value.status == q.QPA_E_ASYM and "instance 4" in str(ei.value), str(ei.value)
    good = insts[:4] + insts[5:]
    say("valid batch after the error")
    outs = eng.solve_batch([q.Problem.from_instance(i) for i in good], p, want_state=True)
    lam = orc.lambda_linear(T, lam0)
    for k, (inst, out) in enumerate(zip(good, outs)):
        x, m, _ = _oracle_instance(inst, R, T, lam, eta, alpha, seed=3 + k)
        assert np.array_equal(host(out["x"]), x) and np.array_equal(host(out["m"]), m), k


def test_batch_scoring_size_limits(q, eng):
    # Dense-forced batch at the largest instance size of a batch (n = 4096, also the
    # largest of the bit-packed batched energies: 64 sign words per replica in LDS; int8
    # entry lists over 32 chunks), a small one, and one too dense for entry lists (int8
    # rows over 8 chunks, more than the 5 stages); R = 70 spans two replica groups.  A
    # larger instance is refused.
    rng = np.random.default_rng(21)
    insts = [gen.er_qubo(4096, 0.01, 100, rng), gen.er_qubo(300, 0.1, 100, rng),
             gen.er_qubo(1000, 0.3, 100, rng)]
    R, T, eta, alpha, lam0 = 70, 4, 0.0002, 0.8, 200.0
    p = _params(q, R, T, eta, alpha, lam0, seed=13, flags=q.QPA_BATCH_DENSE)
    with pytest.raises(q.QpaError) as ei:
        eng.solve_batch([q.Problem.from_instance(gen.er_qubo(4097, 0.01, 100, rng))], p)
    assert ei.value.status == q.QPA_E_UNSUPPORTED, str(ei.value)
    say("batch at the size limit, n=4096/300, R=70")
    outs = eng.solve_batch([q.Problem.from_instance(i) for i in insts], p, want_state=True)
    assert list(q.qpa_batch_paths(eng.ctx, len(insts))) == [
        q.QPA_PATH_BATCH_SPARSE_I8, q.QPA_PATH_BATCH_SPARSE_I8, q.QPA_PATH_BATCH_DENSE_I8]
    lam = orc.lambda_linear(T, lam0)
    for k, (inst, out) in enumerate(zip(insts, outs)):
        x, m, canon = _oracle_instance(inst, R, T, lam, eta, alpha, seed=13 + k)
        assert np.array_equal(host(out["x"]), x) and np.array_equal(host(out["m"]), m), k
        s = np.where(x >= 0, 1, -1).astype(np.int8)
        assert np.array_equal(host(out["spins"]), s), k
        e = _energies_csr_int(canon, inst.kind, s)
        assert np.array_equal(host(out["energy_i64"]), e), k
        assert int(host(out["best"])[0]) == int(np.flatnonzero(e == e.min())[0]), k


def test_er512_full_workload_sampled(q, eng):
    wl = WORKLOADS["er512"]
    say("er512 generation")
    insts = wl.make()
    probs = [q.Problem.from_instance(i) for i in insts]
    p = _params(q, wl.replicas, wl.steps, wl.eta, wl.alpha, wl.lambda0, seed=wl.seed)
    say("er512 full workload solve")
    outs = eng.solve_batch(probs, p, want_state=True)
    assert (q.qpa_batch_paths(eng.ctx, len(insts)) == q.QPA_PATH_BATCH_SPARSE_I8).all()
    lam = orc.lambda_linear(wl.steps, wl.lambda0)
    sizes = np.array([i.n for i in insts])
    for k in [int(np.argmin(sizes)), int(np.argmax(sizes)), 137]:
        inst = insts[k]
        for r0 in [0, wl.replicas - 1]:
            x, m, canon = _oracle_instance(inst, 1, wl.steps, lam, wl.eta, wl.alpha,
                                           seed=wl.seed + k, r0=r0)
            assert np.array_equal(host(outs[k]["x"])[r0], x[0]), (k, r0)
        s = host(outs[k]["spins"])
        e = _energies_csr_int(orc.qubo_to_ising_csr_int(inst.csr.rp, inst.csr.col, inst.csr.w,
                                                        inst.lin), "qubo", s)
        assert np.array_equal(host(outs[k]["energy_i64"]), e), k


# ------------------------------------------------------------------ relaxed adjoint
def _rel_case(which):
    if which == "dense":
        inst = gen.sk_ising(64, 0.1, seed=21)
        J = inst.dense.astype(np.float64)
        return inst, lambda x0, T, lam, eta, alpha, grads: orc.relaxed_grad_dense(
            J, inst.lin, x0, T, lam, eta, alpha, grads=grads)
    inst = gen.chimera_ising(3, seed=22)
    c = inst.csr
    return inst, lambda x0, T, lam, eta, alpha, grads: orc.relaxed_grad_csr(
        c.rp, c.col, c.w.astype(np.float64), inst.lin, x0, T, lam, eta, alpha, grads=grads)


@pytest.mark.parametrize("which", ["dense", "csr"])
def test_relaxed_adjoint_matches_fp64_oracle_and_fd(q, eng, which):
    inst, oracle_fn = _rel_case(which)
    # a regime where the relaxed trajectories stay inside [-1, 1] long enough for the loss
    # to be smooth in (eta, alpha): finite differences are meaningless across clip kinks
    R, T, eta, alpha, lam0, k = 8, 30, 0.01, 0.5, 4.0, 7
    prob = q.Problem.from_instance(inst)
    lam = orc.lambda_linear(T, lam0)
    p = q.make_params(R, T, eta, alpha, lam0, 0.1, 3, lambda_table=lam)
    say("relaxed adjoint %s R=%d T=%d k=%d" % (which, R, T, k))
    L, de, da, dl = [host(v) for v in eng.relaxed_grad(prob, p, k)]
    x0, _ = orc.pa_init(inst.n, R, 3, np.float32(0.1))
    Lo, deo, dao, dlo = oracle_fn(x0, T, lam.astype(np.float64), float(np.float32(eta)),
                                  float(np.float32(alpha)), True)
    assert abs(deo) > 1.0 and abs(dao) > 0.1          # a non-trivial gradient is checked
    assert abs(L[0] - Lo) <= 1e-4 * max(1.0, abs(Lo))
    assert abs(de[0] - deo) <= 2e-3 * max(1.0, abs(deo))
    assert abs(da[0] - dao) <= 2e-3 * max(1.0, abs(dao))
    assert np.max(np.abs(dl - dlo)) <= 2e-3 * max(1.0, np.max(np.abs(dlo)))
    # central differences of the GPU loss itself (steps of 1% of eta and 0.2% of alpha)
    def loss_at(eta_, alpha_):
        pp = q.make_params(R, T, eta_, alpha_, lam0, 0.1, 3, lambda_table=lam)
        return float(host(eng.relaxed_grad(prob, pp, k)[0])[0])
    he, ha = 1e-2 * eta, 1e-3
    fd_e = (loss_at(eta + he, alpha) - loss_at(eta - he, alpha)) / (2 * he)
    fd_a = (loss_at(eta, alpha + ha) - loss_at(eta, alpha - ha)) / (2 * ha)
    assert abs(de[0] - fd_e) <= 1e-2 * max(1.0, abs(fd_e))
    assert abs(da[0] - fd_a) <= 1e-2 * max(1.0, abs(fd_a))


def test_relaxed_adjoint_independent_of_checkpoint_interval(q, eng):
    inst = gen.chimera_ising(2, seed=9)
    prob = q.Problem.from_instance(inst)
    R, T = 5, 50
    p = q.make_params(R, T, 0.05, 0.6, 2.0, 0.1, 4)
    say("relaxed adjoint checkpoint invariance")
    ref = [host(v) for v in eng.relaxed_grad(prob, p, 1)]
    for k in [3, 50, 64]:
        got = [host(v) for v in eng.relaxed_grad(prob, p, k)]
        for a_, b_ in zip(ref, got):
            assert np.array_equal(a_, b_), k


def test_relaxed_energy_autograd_function(q, eng):
    import torch
    inst = gen.sk_ising(48, 0.1, seed=5)
    prob = q.Problem.from_instance(inst)
    T = 40
    eta = torch.tensor(0.05, dtype=torch.float64, requires_grad=True)
    alpha = torch.tensor(0.7, dtype=torch.float64, requires_grad=True)
    lam0 = torch.tensor(1.5, dtype=torch.float64, requires_grad=True)
    lam = lam0 * (1.0 - torch.arange(T, dtype=torch.float64) / T)
    say("relaxed energy autograd")
    L = q.RelaxedEnergy.apply(eta, alpha, lam, eng, prob, 6, 0.1, 2, 10)
    L.backward()
    p = q.make_params(6, T, 0.05, 0.7, 1.5, 0.1, 2,
                      lambda_table=lam.detach().numpy().astype(np.float32))
    _, de, da, dl = [host(v) for v in eng.relaxed_grad(prob, p, 10)]
    assert abs(eta.grad.item() - de[0]) <= 1e-12 * max(1.0, abs(de[0]))
    assert abs(alpha.grad.item() - da[0]) <= 1e-12 * max(1.0, abs(da[0]))
    dlam0 = float(np.dot(dl, 1.0 - np.arange(T) / T))
    assert abs(lam0.grad.item() - dlam0) <= 1e-9 * max(1.0, abs(dlam0))


# ------------------------------------------------------------------ planted 3-regular, n = 1e8
def test_planted3r_full_workload_sampled(q, eng):
    import time
    import torch
    wl = WORKLOADS["planted3r"]
    t0 = time.time()
    say("planted3r: generating n=1e8 (about a minute)")
    inst = wl.make()
    c = inst.csr
    say("planted3r: generated in %.0f s, nnz=%d" % (time.time() - t0, c.nnz))
    prob = q.Problem.from_instance(inst)
    R, n = wl.replicas, inst.n
    # one-step check from a mid-trajectory state, sampled rows computed one by one
    p = _params(q, R, wl.steps, wl.eta, wl.alpha, wl.lambda0, seed=wl.seed)
    x0, m0 = orc.pa_init(n, R, wl.seed, np.float32(wl.sigma0))
    xd, md = torch.from_numpy(x0).cuda(), torch.from_numpy(m0).cuda()
    del x0, m0
    say("planted3r: 40 steps on the GPU")
    eng.steps(prob, p, 0, 40, xd, md)
    xs, ms = host(xd), host(md)
    say("planted3r: step 40 with fields")
    h = host(eng.steps(prob, p, 40, 41, xd, md, want_h=True))
    lam = orc.lambda_linear(wl.steps, wl.lambda0)
    rng = np.random.default_rng(0)
    rows = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, 2000)]))
    b = np.zeros(n, np.int64)
    gx, gm = host(xd), host(md)
    for r in range(R):
        hr, xr, mr = orc.pa_step_rows_csr_int(c.rp, c.col, c.w, b, xs[r], ms[r], rows, lam[40],
                                              wl.eta, wl.alpha)
        assert np.array_equal(h[r, rows], hr), r
        assert np.array_equal(gx[r, rows], xr), r
        assert np.array_equal(gm[r, rows], mr), r
    del xs, ms, gx, gm, h, xd, md
    # the full solve: exact energies of every returned replica, planted optimum as bound
    say("planted3r: full solve")
    out = eng.solve(prob, p)
    spins = host(out["spins"])
    e_star = -int(np.abs(c.w.astype(np.int64)).sum()) // 2
    say("planted3r: oracle energies")
    for r in range(R):
        e = orc.ising_energy_csr_int(c.rp, c.col, c.w, b, spins[r])
        assert int(host(out["energy_i64"])[r]) == e
        assert e >= e_star
    best = int(host(out["best"])[0])
    say("planted3r: best energy %d, planted optimum %d, gap %.4f%%"
        % (int(host(out["energy_i64"])[best]), e_star,
           100.0 * (int(host(out["energy_i64"])[best]) - e_star) / abs(e_star)))


# ------------------------------------------------------------------ HIP-graph step loops
@pytest.mark.parametrize("which", ["mfma", "dense-tiled", "csr-streamed"])
def test_graph_step_loop_matches_plain_launches(q, eng, which):
    """QPA_SOLVE_GRAPH replays a captured step loop: every replay, with other work on
    the stream in between, gives the bits of the plain launches."""
    import torch
    if which == "csr-streamed":
        inst, prec, flags = gen.chimera_ising(4, seed=3), "fp32", q.QPA_SOLVE_STREAMED
    else:
        inst, prec, flags = gen.dense_int_ising(300, seed=4), \
            ("bf16" if which == "mfma" else "fp32"), 0
    prob = q.Problem.from_instance(inst)
    R, T = 70, 40
    say("graph step loop %s" % which)
    ref = eng.solve(prob, _params(q, R, T, 0.05, 0.8, 3.0, prec=prec, flags=flags),
                    want_state=True)
    pg = _params(q, R, T, 0.05, 0.8, 3.0, prec=prec, flags=flags | q.QPA_SOLVE_GRAPH)
    for rep in range(3):
        out = eng.solve(prob, pg, want_state=True)
        torch.cuda.synchronize()
        assert np.array_equal(host(out["x"]), host(ref["x"]))
        assert np.array_equal(host(out["m"]), host(ref["m"]))
        assert np.array_equal(host(out["energy"]), host(ref["energy"]))
        # eager work between the replays
        eng.energy(prob, _params(q, R, T, 0.05, 0.8, 3.0, prec=prec), out["spins"])
        torch.cuda.synchronize()


def test_graph_batch_step_loop_matches_plain_launches(q, eng):
    """qpa_solve_batch with QPA_SOLVE_GRAPH: the captured per-step loop of the dense tiles
    (int8 entry-list, int8 and BF16 tiles in one batch, beside a sparse instance) replayed
    three times with eager work in between, then replayed for a second batch of the same
    shapes but other couplings, gives the bits of the plain launches every time."""
    import torch

    def batch(seed):
        rng = np.random.default_rng(seed)
        return [gen.er_qubo(180, 0.1, 100, rng), gen.er_qubo(200, 0.4, 100, rng),
                gen.er_qubo(300, 0.1, 200, rng),
                gen.er_qubo(260, 0.1, 300, rng)]          # the last is never densified
    R, T, eta, alpha, lam0 = 70, 30, 0.0002, 0.8, 200.0
    for seed in (1, 2):
        probs = [q.Problem.from_instance(i) for i in batch(seed)]
        say("graph batch step loop, batch seed %d" % seed)
        ref = eng.solve_batch(probs, _params(q, R, T, eta, alpha, lam0, seed=4,
                                             flags=q.QPA_BATCH_DENSE), want_state=True)
        paths = q.qpa_batch_paths(eng.ctx, len(probs))
        assert list(paths) == [q.QPA_PATH_BATCH_SPARSE_I8, q.QPA_PATH_BATCH_DENSE_I8,
                               q.QPA_PATH_BATCH_DENSE, q.QPA_PATH_BATCH_SPARSE]
        pg = _params(q, R, T, eta, alpha, lam0, seed=4,
                     flags=q.QPA_BATCH_DENSE | q.QPA_SOLVE_GRAPH)
        for rep in range(3 if seed == 1 else 1):
            outs = eng.solve_batch(probs, pg, want_state=True)
            torch.cuda.synchronize()
            for a_, b_ in zip(outs, ref):
                for key in ("x", "m", "energy_i64", "best"):
                    assert np.array_equal(host(a_[key]), host(b_[key])), (seed, rep, key)
            eng.energy(probs[0], _params(q, R, T, eta, alpha, lam0), outs[0]["spins"])
            torch.cuda.synchronize()


def test_graph_steps_split_equals_oracle(q, eng):
    import torch
    inst = gen.chimera_ising(3, seed=5)
    R, T = 5, 30
    prob = q.Problem.from_instance(inst)
    p = _params(q, R, T, 0.2, 0.8, 5.0, flags=q.QPA_SOLVE_STREAMED | q.QPA_SOLVE_GRAPH)
    x0, _ = orc.pa_init(inst.n, R, 1, np.float32(0.1))
    xd = torch.from_numpy(x0.copy()).cuda()
    md = torch.zeros_like(xd)
    for t0, t1 in [(0, 11), (11, 30)]:
        eng.steps(prob, p, t0, t1, xd, md)
    x, m, _ = _oracle_csr(inst, R, T, orc.lambda_linear(T, 5.0), 0.2, 0.8)
    assert np.array_equal(host(xd), x) and np.array_equal(host(md), m)


# ------------------------------------------------------------------ sparse kernel choice
def test_sparse_kernel_choices_and_autotune_give_identical_bits(q, eng):
    inst = gen.chimera_ising(6, seed=7)
    R, T = 100, 60
    prob = q.Problem.from_instance(inst)
    p = _params(q, R, T, 0.2, 0.8, 5.0)
    x, m, _ = _oracle_csr(inst, R, T, orc.lambda_linear(T, 5.0), 0.2, 0.8)
    for choice in (0, 1, 2, 4, 8):
        say("sparse kernel choice %d" % choice)
        eng.tune_set(prob, p, choice)
        out = eng.solve(prob, p, want_state=True)
        assert np.array_equal(host(out["x"]), x) and np.array_equal(host(out["m"]), m)
    choice, ms = eng.autotune(prob, p, 30)
    say("autotune choice %d, ms %s" % (choice, ms))
    assert choice in (0, 1, 2, 4, 8)
    assert ms[0] > 0 and ms[[0, 1, 2, 4, 8].index(choice)] == min(v for v in ms if v >= 0)
    out = eng.solve(prob, p, want_state=True)
    assert np.array_equal(host(out["x"]), x) and np.array_equal(host(out["m"]), m)
    with pytest.raises(q.QpaError) as ei:
        eng.tune_set(prob, p, 3)
    assert ei.value.status == q.QPA_E_ARG
    dense = q.Problem.from_instance(gen.dense_int_ising(20, seed=1))
    with pytest.raises(q.QpaError) as ei:
        eng.autotune(dense, p, 10)
    assert ei.value.status == q.QPA_E_UNSUPPORTED


def test_schedule_tuning_lowers_the_relaxed_energy(q, eng):
    """A few Adam steps on (eta, alpha, lambda) through the adjoint lower the relaxed
    final energy (the adjoint used to tune schedules)."""
    import torch
    rng = np.random.default_rng(4)
    inst = gen.er_qubo(150, 0.1, 100, rng)
    prob = q.Problem.from_instance(inst)
    T, R = 100, 16
    log_eta = torch.tensor(np.log(2e-4), dtype=torch.float64, requires_grad=True)
    log_lam0 = torch.tensor(np.log(200.0), dtype=torch.float64, requires_grad=True)
    alpha = torch.tensor(0.8, dtype=torch.float64)
    frac = 1.0 - torch.arange(T, dtype=torch.float64) / T
    opt = torch.optim.Adam([log_eta, log_lam0], lr=0.1)
    losses = []
    say("schedule tuning")
    for _ in range(8):
        L = q.RelaxedEnergy.apply(torch.exp(log_eta), alpha, torch.exp(log_lam0) * frac, eng,
                                  prob, R, 0.1, 3, 10)
        opt.zero_grad()
        L.backward()
        opt.step()
        losses.append(float(L.detach()))
    assert losses[-1] < losses[0]
