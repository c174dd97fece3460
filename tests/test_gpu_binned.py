"""Parity of the binned sparse PA step (QPA_SOLVE_BINNED) with the CPU oracle.

The binned kernels sum the integer couplings of a row in an order fixed by their entry
layout, not by column; integer sums are exact, so positions, momenta and energies must
equal the oracle's (which sums in column order) bit for bit.  The instances span several
source chunks and destination bins with ragged last ones (chunk 2^20 / G variables, bin
2^14 / G rows for a replica group of G lanes), QUBO diagonals, int16 weights and empty
rows.
"""
import sys

import numpy as np
import pytest

import oracle as orc
from paper_2501_19221_amd import instances as gen

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-binned] " + msg, flush=True)
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


def _params(q, R, T, eta, alpha, lam0, flags, seed=1):
    return q.make_params(R, T, eta, alpha, lam0, 0.1, seed, q.QPA_PREC_FP32, flags=flags)


def _sparse_qubo(n, deg, wmax, diag_frac, active_frac, seed):
    """Random sparse QUBO: about deg*n/2 distinct pairs among a random subset of
    active_frac*n variables (the other rows are empty), int16 weights in [-wmax, wmax],
    diagonal entries on a random diag_frac of the variables, int16 linear terms."""
    rng = np.random.default_rng(seed)
    act = np.flatnonzero(rng.random(n) < active_frac)
    m = int(deg * len(act) / 2)
    u = act[rng.integers(0, len(act), m)]
    v = act[rng.integers(0, len(act), m)]
    keep = u != v
    lo, hi = np.minimum(u[keep], v[keep]), np.maximum(u[keep], v[keep])
    key = np.unique(lo.astype(np.int64) * n + hi)
    lo, hi = key // n, key % n
    w = rng.integers(-wmax, wmax + 1, size=len(lo)).astype(np.int16)
    d = np.flatnonzero(rng.random(n) < diag_frac)
    wd = rng.integers(-wmax, wmax + 1, size=len(d)).astype(np.int16)
    rows = np.concatenate([lo, hi, d])
    cols = np.concatenate([hi, lo, d])
    ws = np.concatenate([w, w, wd])
    order = np.lexsort((cols, rows))
    rows, cols, ws = rows[order], cols[order], ws[order]
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    csr = gen.CSR(n, rp.astype(np.int32), cols.astype(np.int32), ws)
    lin = rng.integers(-wmax, wmax + 1, size=n).astype(np.int16)
    return gen.Instance("qubo", n, csr=csr, lin=lin, meta={})


def _oracle(inst, R, T, lam, eta, alpha):
    c = inst.csr
    if inst.kind == "qubo":
        rp, col, w, b, K = orc.qubo_to_ising_csr_int(c.rp, c.col, c.w, inst.lin)
    else:
        rp, col, w, b, K = c.rp, c.col, c.w, inst.lin, 0
    x, m = orc.pa_init(inst.n, R, 1, np.float32(0.1))
    orc.pa_steps_csr_int(rp, col, w, b, x, m, 0, T, lam, eta, alpha)
    return x, m, (rp, col, w, b, K)


def _paths(q, eng, fn):
    q.qpa_profile_read(eng.ctx, reset=True)
    q.qpa_profile_enable(eng.ctx, True)
    try:
        res = fn()
    finally:
        q.qpa_profile_enable(eng.ctx, False)
    out = {}
    for code in range(0, q.QPA_PATH_CSR_BINNED + 1):
        _, n = q.qpa_profile_read_path(eng.ctx, code)
        if n:
            out[code] = n
    q.qpa_profile_read(eng.ctx, reset=True)
    return res, out


CASES = [
    # name, instance builder, R, T
    ("3reg n=300k R=8 (G=8: 3 chunks, 147 bins)",
     lambda: gen.planted_3regular(300_000, 1, 7, seed=11), 8, 12),
    ("3reg n=1.2M R=1 (G=1: 2 chunks, 74 bins)",
     lambda: gen.planted_3regular(1_200_000, 1, 7, seed=12), 1, 8),
    ("qubo n=300k R=3 (G=4: 2 chunks, 74 bins, diagonals, empty rows)",
     lambda: _sparse_qubo(300_000, 4, 300, 0.1, 0.6, seed=13), 3, 10),
    ("qubo n=5000 R=2 (G=2: one chunk, one bin)",
     lambda: _sparse_qubo(5000, 6, 1000, 0.3, 0.9, seed=14), 2, 30),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_binned_bit_exact(q, eng, case):
    name, build, R, T = CASES[case]
    say("binned: " + name)
    inst = build()
    prob = q.Problem.from_instance(inst)
    p = _params(q, R, T, 0.1, 0.8, 6.0, q.QPA_SOLVE_BINNED)
    out, paths = _paths(q, eng, lambda: eng.solve(prob, p, want_state=True))
    assert paths == {q.QPA_PATH_CSR_BINNED: 2 * T}, paths
    x, m, canon = _oracle(inst, R, T, orc.lambda_linear(T, 6.0), 0.1, 0.8)
    assert np.array_equal(host(out["x"]), x)
    assert np.array_equal(host(out["m"]), m)
    rp, col, w, b, K = canon
    spins = host(out["spins"])
    for r in range(R):
        H = orc.ising_energy_csr_int(rp, col, w, b, spins[r])
        e = (H + K) // 2 if inst.kind == "qubo" else H
        assert int(host(out["energy_i64"])[r]) == e, r


def test_binned_steps_split_and_fields(q, eng):
    """qpa_steps over [0, 7) then [7, 19) with the binned step equals the oracle, and
    the fields of the last step equal the streamed kernel's."""
    import torch
    inst = gen.planted_3regular(300_000, 1, 7, seed=15)
    R, T = 4, 19
    prob = q.Problem.from_instance(inst)
    lam = orc.lambda_linear(T, 4.0)
    x0, _ = orc.pa_init(inst.n, R, 1, np.float32(0.1))
    outs = {}
    for name, flags in (("binned", q.QPA_SOLVE_BINNED), ("streamed", q.QPA_SOLVE_STREAMED)):
        say("binned split steps: " + name)
        p = _params(q, R, T, 0.15, 0.8, 4.0, flags)
        xd = torch.from_numpy(x0.copy()).cuda()
        md = torch.zeros_like(xd)
        eng.steps(prob, p, 0, 7, xd, md)
        h = eng.steps(prob, p, 7, T, xd, md, want_h=True)
        outs[name] = (host(xd), host(md), host(h))
    x, m, _ = _oracle(inst, R, T, lam, 0.15, 0.8)
    assert np.array_equal(outs["binned"][0], x) and np.array_equal(outs["binned"][1], m)
    assert np.array_equal(outs["binned"][2], outs["streamed"][2])


def test_binned_default_choice_tuning_and_errors(q, eng):
    """Integer instances whose spin words exceed 4 MiB take the binned step by default;
    QPA_TUNE_BINNED and the autotuner cover it; inapplicable instances and flag mixes
    are refused."""
    R, T = 4, 6
    p = _params(q, R, T, 0.1, 0.8, 4.0, 0)
    # G = 4: n / 16 spin words of 8 bytes; 4 MiB <=> n = 8388608
    for n, want in ((8_388_608, q.QPA_PATH_CSR), (8_388_624, q.QPA_PATH_CSR_BINNED)):
        say("binned default choice n=%d" % n)
        pb = q.Problem.from_instance(gen.planted_3regular(n, 1, 7, seed=16))
        _, paths = _paths(q, eng, lambda: eng.solve(pb, p))
        assert list(paths) == [want], paths
        del pb
    inst = gen.planted_3regular(300_000, 1, 7, seed=17)
    prob = q.Problem.from_instance(inst)
    x, m, _ = _oracle(inst, R, T, orc.lambda_linear(T, 4.0), 0.1, 0.8)
    say("binned tune_set / autotune")
    eng.tune_set(prob, p, q.QPA_TUNE_BINNED)
    out2, paths = _paths(q, eng, lambda: eng.solve(prob, p, want_state=True))
    assert paths == {q.QPA_PATH_CSR_BINNED: 2 * T}, paths
    assert np.array_equal(host(out2["x"]), x) and np.array_equal(host(out2["m"]), m)
    choice, ms = eng.autotune(prob, p, 4)
    say("autotune choice %d ms %s" % (choice, ms))
    assert ms[0] > 0 and ms[5] > 0 and ms[1:5] == [-1.0] * 4
    assert choice == (q.QPA_TUNE_BINNED if ms[5] < ms[0] else 0)
    # refusals
    fl = gen.chimera_ising(2, seed=1)
    fl.csr.w = fl.csr.w.astype(np.float32)
    for bad, why in ((gen.chimera_ising(2, seed=1), 9), (fl, 4)):
        with pytest.raises(q.QpaError) as ei:
            eng.solve(q.Problem.from_instance(bad), _params(q, why, 3, 0.1, 0.8, 4.0,
                                                            q.QPA_SOLVE_BINNED))
        assert ei.value.status == q.QPA_E_UNSUPPORTED
    with pytest.raises(q.QpaError) as ei:
        eng.solve(prob, _params(q, R, T, 0.1, 0.8, 4.0,
                                q.QPA_SOLVE_BINNED | q.QPA_SOLVE_STREAMED))
    assert ei.value.status == q.QPA_E_ARG


def test_binned_graph_replays_match_plain_launches(q, eng):
    """QPA_SOLVE_GRAPH with the binned step: the entry order is built eagerly per call,
    the captured step loop replays with the plain launches' bits."""
    import torch
    inst = _sparse_qubo(120_000, 5, 500, 0.2, 0.8, seed=18)
    prob = q.Problem.from_instance(inst)
    R, T = 5, 9
    say("binned graph replays")
    ref = eng.solve(prob, _params(q, R, T, 0.1, 0.8, 6.0, q.QPA_SOLVE_BINNED), want_state=True)
    pg = _params(q, R, T, 0.1, 0.8, 6.0, q.QPA_SOLVE_BINNED | q.QPA_SOLVE_GRAPH)
    for rep in range(3):
        out = eng.solve(prob, pg, want_state=True)
        torch.cuda.synchronize()
        assert np.array_equal(host(out["x"]), host(ref["x"]))
        assert np.array_equal(host(out["m"]), host(ref["m"]))
        assert np.array_equal(host(out["energy_i64"]), host(ref["energy_i64"]))
        eng.energy(prob, _params(q, R, T, 0.1, 0.8, 6.0, 0), out["spins"])
        torch.cuda.synchronize()


@pytest.mark.parametrize("kind", ["no-edges", "diagonal-only-qubo"])
def test_binned_without_entries(q, eng, kind):
    """An instance with no off-diagonal couplings leaves the binned entry order empty;
    the fields are the linear terms alone, as in the oracle."""
    n = 70_000
    rng = np.random.default_rng(21)
    if kind == "no-edges":
        csr = gen.CSR(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int8))
        inst = gen.Instance("ising", n, csr=csr,
                            lin=rng.integers(-5, 6, size=n).astype(np.int8), meta={})
    else:
        d = np.flatnonzero(rng.random(n) < 0.5)
        rp = np.zeros(n + 1, np.int64)
        rp[1:] = np.cumsum(np.isin(np.arange(n), d))
        csr = gen.CSR(n, rp.astype(np.int32), d.astype(np.int32),
                      rng.integers(-9, 10, size=len(d)).astype(np.int16))
        inst = gen.Instance("qubo", n, csr=csr,
                            lin=rng.integers(-9, 10, size=n).astype(np.int16), meta={})
    prob = q.Problem.from_instance(inst)
    R, T = 6, 7
    say("binned without entries: " + kind)
    out, paths = _paths(q, eng, lambda: eng.solve(
        prob, _params(q, R, T, 0.1, 0.8, 3.0, q.QPA_SOLVE_BINNED), want_state=True))
    assert paths == {q.QPA_PATH_CSR_BINNED: 2 * T}, paths
    x, m, canon = _oracle(inst, R, T, orc.lambda_linear(T, 3.0), 0.1, 0.8)
    assert np.array_equal(host(out["x"]), x) and np.array_equal(host(out["m"]), m)
    rp, col, w, b, K = canon
    spins = host(out["spins"])
    for r in range(R):
        H = orc.ising_energy_csr_int(rp, col, w, b, spins[r])
        e = (H + K) // 2 if inst.kind == "qubo" else H
        assert int(host(out["energy_i64"])[r]) == e, r
