"""Parity of the HIP Simulated Bifurcation path (App. B) with the CPU oracle.

The SBM kernels sum every field with one fused multiply-add per term in ascending
column order and round each update operation separately, exactly as the oracle does, so
positions, momenta, fields, spins and integer energies must match bit for bit.  The
power method runs in FP64 with a different reduction order: its estimate is compared
within 1e-9 relative.
"""
import sys

import numpy as np
import pytest

import oracle as orc
from paper_2501_19221_amd import instances as gen

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-sbm] " + msg, flush=True)
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


def _canon(inst):
    """Ising form (J, b) the dynamics run on, as float32, plus a dense copy of J."""
    if inst.csr is not None:
        c = inst.csr
        if inst.kind == "qubo":
            rp, col, w, b, _ = orc.qubo_to_ising_csr_int(c.rp, c.col, c.w, inst.lin)
        else:
            rp, col, w = c.rp, c.col, c.w
            b = np.zeros(inst.n) if inst.lin is None else inst.lin
        D = gen.CSR(inst.n, np.asarray(rp), np.asarray(col), np.asarray(w)).to_dense(np.float64)
        return ("csr", (np.asarray(rp), np.asarray(col), np.asarray(w, np.float32)),
                np.asarray(b, np.float32), D)
    if inst.kind == "qubo":
        if np.issubdtype(inst.dense.dtype, np.integer):
            J, b, _ = orc.qubo_to_ising_int(inst.dense, inst.lin)
        else:
            J, b, _ = orc.qubo_to_ising_float(inst.dense, inst.lin)
    else:
        J, b = inst.dense, inst.lin
    J = np.asarray(J, np.float32)
    return "dense", J, np.asarray(b, np.float32), J.astype(np.float64)


def _oracle_run(inst, R, T, a0, c0, dt, seed, sigma0, t_end=None, r0=0, want_g=False):
    fmt, J, b, _ = _canon(inst)
    qv, _ = orc.pa_init(inst.n, R, seed, np.float32(sigma0), r0=r0)
    p = np.zeros_like(qv)
    t_end = T if t_end is None else t_end
    if fmt == "dense":
        g = orc.sbm_steps_dense(J, b, qv, p, 0, t_end, T, a0, c0, dt, want_g=want_g)
    else:
        rp, col, w = J
        g = orc.sbm_steps_csr(rp, col, w, b, qv, p, 0, t_end, T, a0, c0, dt, want_g=want_g)
    return qv, p, g


def _energies(inst, s):
    if inst.csr is not None:
        c = inst.csr
        if inst.kind == "qubo":
            D = c.to_dense(np.int64)
            return np.array([orc.qubo_energy_int(D.astype(np.int32), inst.lin,
                                                 (s[r] > 0).astype(np.int8))
                             for r in range(len(s))])
        b = np.zeros(inst.n, np.int64) if inst.lin is None else inst.lin
        if np.issubdtype(c.w.dtype, np.floating):
            return np.array([orc.ising_energy_csr_float(c.rp, c.col, c.w, b, s[r])
                             for r in range(len(s))])
        return np.array([orc.ising_energy_csr_int(c.rp, c.col, c.w, b, s[r])
                         for r in range(len(s))])
    if inst.kind == "qubo":
        return np.array([orc.qubo_energy_int(inst.dense, inst.lin, (s[r] > 0).astype(np.int8))
                         for r in range(len(s))])
    return np.array([orc.ising_energy_float(inst.dense.astype(np.float64),
                                            inst.lin.astype(np.float64), s[r])
                     for r in range(len(s))])


def _check_solve(q, eng, inst, R, T, a0=1.0, c0=0.05, dt=0.5, seed=3, sigma0=0.1):
    prob = q.Problem.from_instance(inst)
    sp = q.make_sbm_params(R, T, dt, a0=a0, c0=c0, sigma0=sigma0, seed=seed)
    say("sbm solve %s n=%d R=%d T=%d" % (inst.kind, inst.n, R, T))
    out = eng.sbm_solve(prob, sp, want_state=True)
    qv, p, _ = _oracle_run(inst, R, T, a0, c0, dt, seed, sigma0)
    assert np.array_equal(host(out["x"]), qv)
    assert np.array_equal(host(out["m"]), p)
    s = np.where(qv >= 0, 1, -1).astype(np.int8)
    assert np.array_equal(host(out["spins"]), s)
    e = _energies(inst, s)
    if np.issubdtype(e.dtype, np.integer):
        assert np.array_equal(host(out["energy_i64"]), e)
        assert int(host(out["best"])[0]) == int(np.flatnonzero(e == e.min())[0])
    else:
        np.testing.assert_allclose(host(out["energy"]), e, rtol=1e-12, atol=1e-9)
        assert int(host(out["best"])[0]) == int(np.argmin(e))
    return out


# ------------------------------------------------------------------ dense
@pytest.mark.parametrize("n,R,T", [(300, 70, 60), (129, 3, 40), (1, 1, 5), (256, 130, 20)])
def test_sbm_dense_float_bit_exact(q, eng, n, R, T):
    _check_solve(q, eng, gen.sk_ising(n, 0.1, seed=n), R, T, c0=0.5 / np.sqrt(n))


def test_sbm_dense_int_qubo_bit_exact(q, eng):
    _check_solve(q, eng, gen.dense_int_qubo(50, -10, 10, seed=7), 10, 80, c0=0.01, dt=0.25)


# ------------------------------------------------------------------ CSR
@pytest.mark.parametrize("m_,R,T", [(4, 70, 100), (2, 1, 30), (3, 64, 50), (3, 5, 40)])
def test_sbm_csr_chimera_bit_exact(q, eng, m_, R, T):
    _check_solve(q, eng, gen.chimera_ising(m_, seed=m_), R, T, c0=0.2)


def test_sbm_csr_float_weights_bit_exact(q, eng):
    inst = gen.chimera_ising(3, seed=4)
    rng = np.random.default_rng(0)
    c = inst.csr
    D = c.to_dense(np.int32).astype(np.float32)
    W = np.triu(rng.standard_normal(D.shape).astype(np.float32) * (D != 0), 1)
    W = W + W.T
    rows, cols = np.nonzero(D)
    inst.csr = gen.CSR(inst.n, c.rp, c.col, W[rows, cols].astype(np.float32))
    inst.lin = rng.standard_normal(inst.n).astype(np.float32) * 0.3
    _check_solve(q, eng, inst, 3, 80, c0=0.3)


def test_sbm_csr_er_qubo_int16_with_diagonal_bit_exact(q, eng):
    """QUBO CSR with stored diagonal entries: they fold into b and are skipped in J q."""
    rng = np.random.default_rng(9)
    inst = gen.er_qubo(300, 0.05, 20, rng)
    D = inst.csr.to_dense(np.int32)
    D[np.arange(300), np.arange(300)] = rng.integers(-20, 21, 300)
    rows, cols = np.nonzero(D)
    rp = np.r_[0, np.cumsum(np.bincount(rows, minlength=300))].astype(np.int32)
    inst.csr = gen.CSR(300, rp, cols.astype(np.int16), D[rows, cols].astype(np.int16))
    _check_solve(q, eng, inst, 9, 60, c0=0.02, dt=0.25)


# ------------------------------------------------------------------ steps, resume, c0
@pytest.mark.parametrize("which", ["dense", "csr"])
def test_sbm_steps_split_equals_uninterrupted(q, eng, which):
    import torch
    inst = gen.sk_ising(200, 0.1, seed=5) if which == "dense" else gen.chimera_ising(4, seed=6)
    R, T, a0, c0, dt, seed = 6, 50, 1.0, 0.1, 0.5, 11
    prob = q.Problem.from_instance(inst)
    sp = q.make_sbm_params(R, T, dt, a0=a0, c0=c0, seed=seed)
    x0, _ = orc.pa_init(inst.n, R, seed, np.float32(0.1))
    qd = torch.from_numpy(x0.copy()).cuda()
    pd = torch.zeros_like(qd)
    say("sbm steps split %s" % which)
    for t0, t1 in [(0, 17), (17, 17), (17, 49), (49, 50)]:
        g = eng.sbm_steps(prob, sp, t0, t1, qd, pd, want_g=True)
    qv, p, gref = _oracle_run(inst, R, T, a0, c0, dt, seed, 0.1, want_g=True)
    assert np.array_equal(host(qd), qv) and np.array_equal(host(pd), p)
    assert np.array_equal(host(g), gref)


@pytest.mark.parametrize("which", ["dense-float", "dense-qubo", "csr-bipartite"])
def test_spectral_radius_matches_oracle(q, eng, which):
    inst = {"dense-float": lambda: gen.sk_ising(300, 0.1, seed=1),
            "dense-qubo": lambda: gen.dense_int_qubo(40, -10, 10, seed=2),
            "csr-bipartite": lambda: gen.chimera_ising(4, seed=1)}[which]()
    _, _, _, D = _canon(inst)
    iters, seed = 300, 5
    sp = q.make_sbm_params(1, 0, 0.5, seed=seed, power_iters=iters)
    say("spectral radius %s" % which)
    rho = float(host(eng.spectral_radius(q.Problem.from_instance(inst), sp))[0])
    ref = orc.spectral_radius_power(D, iters, seed)
    assert rho == pytest.approx(ref, rel=1e-9)
    ev = np.linalg.eigvalsh(D)
    assert rho == pytest.approx(max(-ev[0], ev[-1]), rel=5e-3)


def test_sbm_c0_from_power_method(q, eng):
    """c0 = 0 runs the power method and uses float32(1 / rho).  The oracle's own power
    method gives the same float32 c0 (FP64 reduction-order differences are far below its
    rounding), so the trajectories match the oracle's bit for bit."""
    inst = gen.sk_ising(256, 0.1, seed=8)
    R, T = 4, 40
    prob = q.Problem.from_instance(inst)
    sp0 = q.make_sbm_params(R, T, 0.5, c0=0.0, seed=2, power_iters=80)
    say("sbm c0 from power method")
    rho = float(host(eng.spectral_radius(prob, sp0))[0])
    out0 = eng.sbm_solve(prob, sp0, want_state=True)
    out1 = eng.sbm_solve(prob, q.make_sbm_params(R, T, 0.5, c0=float(np.float32(1.0 / rho)),
                                                 seed=2), want_state=True)
    assert np.array_equal(host(out0["x"]), host(out1["x"]))
    c0 = np.float32(1.0 / orc.spectral_radius_power(inst.dense, 80, 2))
    assert c0 == np.float32(1.0 / rho)
    qv, _, _ = _oracle_run(inst, R, T, 1.0, float(c0), 0.5, 2, 0.1)
    assert np.array_equal(host(out0["x"]), qv)


def test_sbm_zero_steps_scores_initial_positions(q, eng):
    inst = gen.chimera_ising(2, seed=3)
    _check_solve(q, eng, inst, 5, 0)


def test_sbm_invalid_params_rejected(q, eng):
    inst = gen.chimera_ising(2, seed=3)
    prob = q.Problem.from_instance(inst)
    for kw in ({"a0": 0.0}, {"dt": -1.0}, {"c0": -1.0}, {"flags": 1}, {"power_iters": -1}):
        args = dict(a0=1.0, c0=0.1, dt=0.5, flags=0, power_iters=10)
        args.update(kw)
        dt = args.pop("dt")
        sp = q.make_sbm_params(2, 10, dt, **args)
        with pytest.raises(q.QpaError) as ei:
            eng.sbm_solve(prob, sp)
        assert ei.value.status == q.QPA_E_ARG


# ------------------------------------------------------------------ full-size workloads
def test_sbm_sk4096_full_workload_sampled(q, eng):
    """The benchmark's dense SBM workload at full size (n = 4096, 1024 replicas, schedule of
    1000 steps): the first 120 steps of every replica on the GPU, replicas 0 and 1023
    (first and last of the padded tiles) against the oracle."""
    import torch
    from paper_2501_19221_amd.configs import SBM_WORKLOADS
    wl = SBM_WORKLOADS["sbm_sk4096"]
    inst = wl.make()
    c0 = float(np.float32(1.0 / orc.spectral_radius_power(inst.dense, wl.power_iters,
                                                           wl.seed)))
    prob = q.Problem.from_instance(inst)
    sp = q.make_sbm_params(wl.replicas, wl.steps, wl.dt, wl.a0, c0, wl.sigma0, wl.seed)
    x0, _ = orc.pa_init(inst.n, wl.replicas, wl.seed, np.float32(wl.sigma0))
    qd = torch.from_numpy(x0).cuda()
    pd = torch.zeros_like(qd)
    say("sbm sk4096 full size, 120 steps")
    eng.sbm_steps(prob, sp, 0, 120, qd, pd)
    qg, pg = host(qd), host(pd)
    J, b = inst.dense.astype(np.float32), inst.lin.astype(np.float32)
    for r in (0, wl.replicas - 1):
        qv, _ = orc.pa_init(inst.n, 1, wl.seed, np.float32(wl.sigma0), r0=r)
        p = np.zeros_like(qv)
        orc.sbm_steps_dense(J, b, qv, p, 0, 120, wl.steps, wl.a0, c0, wl.dt)
        assert np.array_equal(qg[r], qv[0]) and np.array_equal(pg[r], p[0])


def test_sbm_chimera16_full_workload_sampled(q, eng):
    """The benchmark's sparse SBM workload, whole solve: replicas 0, 517 and 1023 against
    the oracle's full trajectories; every replica's energy against the oracle's energy of
    the spins it returned; the best replica is the first minimum."""
    from paper_2501_19221_amd.configs import SBM_WORKLOADS
    wl = SBM_WORKLOADS["sbm_chimera16"]
    inst = wl.make()
    c = inst.csr
    c0 = float(np.float32(1.0 / orc.spectral_radius_power(c.to_dense(np.float64),
                                                           wl.power_iters, wl.seed)))
    prob = q.Problem.from_instance(inst)
    sp = q.make_sbm_params(wl.replicas, wl.steps, wl.dt, wl.a0, c0, wl.sigma0, wl.seed)
    say("sbm chimera16 full solve")
    out = eng.sbm_solve(prob, sp, want_state=True)
    qg = host(out["x"])
    b = np.zeros(inst.n, np.float32)
    for r in (0, 517, wl.replicas - 1):
        qv, _ = orc.pa_init(inst.n, 1, wl.seed, np.float32(wl.sigma0), r0=r)
        p = np.zeros_like(qv)
        orc.sbm_steps_csr(c.rp, c.col, c.w.astype(np.float32), b, qv, p, 0, wl.steps, wl.steps,
                          wl.a0, c0, wl.dt)
        assert np.array_equal(qg[r], qv[0])
    s = host(out["spins"])
    assert np.array_equal(s, np.where(qg >= 0, 1, -1))
    e = np.array([orc.ising_energy_csr_int(c.rp, c.col, c.w, np.zeros(inst.n, np.int64), s[r])
                  for r in range(wl.replicas)])
    assert np.array_equal(host(out["energy_i64"]), e)
    assert int(host(out["best"])[0]) == int(np.flatnonzero(e == e.min())[0])


@pytest.mark.parametrize("which", ["dense", "csr"])
def test_sbm_graph_matches_plain(q, eng, which):
    import torch
    inst = gen.sk_ising(200, 0.1, seed=2) if which == "dense" else gen.chimera_ising(3, seed=2)
    prob = q.Problem.from_instance(inst)
    say("sbm graph %s" % which)
    ref = eng.sbm_solve(prob, q.make_sbm_params(9, 31, 0.5, c0=0.1, seed=4), want_state=True)
    pg = q.make_sbm_params(9, 31, 0.5, c0=0.1, seed=4, flags=q.QPA_SOLVE_GRAPH)
    for rep in range(3):
        out = eng.sbm_solve(prob, pg, want_state=True)
        torch.cuda.synchronize()
        assert np.array_equal(host(out["x"]), host(ref["x"]))
        assert np.array_equal(host(out["m"]), host(ref["m"]))
        eng.spectral_radius(prob, pg)
        torch.cuda.synchronize()


@pytest.mark.parametrize("R", [512, 1024, 2048, 3])
def test_sbm_resident_groups_match_streamed_and_oracle(q, eng, R):
    """The resident sparse SBM kernel (replica groups 2, 4, 8 at these sizes, 1 for small
    R) gives the bits of the per-step kernel and of the oracle."""
    inst = gen.chimera_ising(16, seed=2)
    c = inst.csr
    T, c0, dt = 60, 0.2, 0.5
    prob = q.Problem.from_instance(inst)
    say("sbm resident R=%d" % R)
    out = eng.sbm_solve(prob, q.make_sbm_params(R, T, dt, c0=c0, seed=5), want_state=True)
    ref = eng.sbm_solve(prob, q.make_sbm_params(R, T, dt, c0=c0, seed=5,
                                                flags=q.QPA_SOLVE_STREAMED), want_state=True)
    assert np.array_equal(host(out["x"]), host(ref["x"]))
    assert np.array_equal(host(out["m"]), host(ref["m"]))
    qg = host(out["x"])
    for r in sorted({0, R // 2, R - 1}):
        qv, _ = orc.pa_init(inst.n, 1, 5, np.float32(0.1), r0=r)
        p = np.zeros_like(qv)
        orc.sbm_steps_csr(c.rp, c.col, c.w.astype(np.float32), np.zeros(inst.n, np.float32), qv,
                          p, 0, T, T, 1.0, c0, dt)
        assert np.array_equal(qg[r], qv[0])


def test_sbm_resident_split_steps_and_fields(q, eng):
    import torch
    inst = gen.chimera_ising(5, seed=9)
    R, T, c0, dt, seed = 300, 40, 0.2, 0.5, 3
    prob = q.Problem.from_instance(inst)
    sp = q.make_sbm_params(R, T, dt, c0=c0, seed=seed)
    x0, _ = orc.pa_init(inst.n, R, seed, np.float32(0.1))
    qd = torch.from_numpy(x0.copy()).cuda()
    pd = torch.zeros_like(qd)
    say("sbm resident split")
    for t0, t1 in [(0, 13), (13, 13), (13, 40)]:
        g = eng.sbm_steps(prob, sp, t0, t1, qd, pd, want_g=True)
    qv, p, gref = _oracle_run(inst, R, T, 1.0, c0, dt, seed, 0.1, want_g=True)
    assert np.array_equal(host(qd), qv) and np.array_equal(host(pd), p)
    assert np.array_equal(host(g), gref)
