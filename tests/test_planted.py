"""Pins of the planted-instance generators (Sec. VIII) against brute force and the
oracle's energy functions: the planted state is a ground state and its energy is the one
each construction promises."""
import itertools

import numpy as np
import pytest

import oracle as orc
from paper_2501_19221_amd import instances as gen


def _all_states(n):
    return np.array(list(itertools.product((-1, 1), repeat=n)), np.int8)


# ------------------------------------------------------------------ Wishart (Sec. VIII.C)
@pytest.mark.parametrize("alpha,seed", [(0.3, 1), (1.0, 2), (0.6, 3)])
def test_wishart_planted_state_is_the_bruteforce_ground_state(alpha, seed):
    n = 14
    inst = gen.wishart_planted(n, alpha, seed)
    J = inst.dense.astype(np.float64)
    S = _all_states(n).astype(np.float64)
    E = 0.5 * np.einsum("ri,ij,rj->r", S, J, S)
    s_star = inst.meta["planted_state"]
    e_star = orc.ising_energy_float(J, np.zeros(n), s_star)
    assert E.min() == pytest.approx(e_star, rel=1e-12, abs=1e-12)
    # only the planted pair attains it (W^T s = 0 has no other +-1 solution here)
    winners = S[np.isclose(E, E.min(), rtol=0, atol=1e-9)]
    assert len(winners) == 2 and {tuple(w) for w in winners} == {tuple(s_star),
                                                               tuple(-s_star)}
    # the section's closed form E0 = (1/2) Tr J~, within the float32 rounding of J
    assert e_star == pytest.approx(inst.meta["planted_energy"], rel=1e-5)


def test_wishart_shape_and_symmetry():
    inst = gen.wishart_planted(200, 0.5, 4)
    J = inst.dense
    assert J.shape == (200, 200) and J.dtype == np.float32
    assert np.array_equal(J, J.T) and not np.any(np.diag(J))
    assert inst.meta["M"] == 100


# ------------------------------------------------------------------ tile planting (VIII.B)
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_tile_types_have_k_ground_state_pairs(k):
    """Tile type k (edges around a plaquette a-b-c-d-a, H = -sum J_e s s) has exactly k
    ground-state pairs, the all-up pair among them, in every rotation."""
    base = np.array(gen.TILE_TYPES[k])
    S = _all_states(4).astype(np.int64)
    for r in range(4):
        Je = np.roll(base, r)
        E = -(Je[0] * S[:, 0] * S[:, 1] + Je[1] * S[:, 1] * S[:, 2]
              + Je[2] * S[:, 2] * S[:, 3] + Je[3] * S[:, 3] * S[:, 0])
        mins = S[E == E.min()]
        assert len(mins) == 2 * k
        assert any(np.all(m == 1) for m in mins)


@pytest.mark.parametrize("probs,seed", [((0, 0.2, 0, 0.8), 1), ((0, 0.8, 0, 0.2), 2),
                                        ((0.25, 0.25, 0.25, 0.25), 3)])
def test_tile_planted_state_is_the_bruteforce_ground_state(probs, seed):
    inst = gen.tile_planted(4, probs, seed)
    D = inst.csr.to_dense(np.int32)
    b = np.zeros(inst.n, np.int64)
    Hmin, _ = orc.bruteforce_ising_int(D, b)
    assert Hmin == inst.meta["planted_energy"]
    assert orc.ising_energy_int(D, b, inst.meta["planted_state"]) == Hmin


def test_tile_lattice_structure():
    L = 10
    inst = gen.tile_planted(L, seed=5)
    c = inst.csr
    assert np.all(np.diff(c.rp) == 4)                      # square lattice, periodic
    assert len(inst.meta["tile_types"]) == L * L // 2      # checkerboard of plaquettes
    D = c.to_dense(np.int32)
    assert np.array_equal(D, D.T)
    for v in range(inst.n):
        x, y = v % L, v // L
        nb = {y * L + (x + 1) % L, y * L + (x - 1) % L, ((y + 1) % L) * L + x,
              ((y - 1) % L) * L + x}
        assert set(np.flatnonzero(D[v])) == nb


# ------------------------------------------------------------------ 3R3X (VIII.A, VI.A)
def test_3r3x_structure_and_planted_solution():
    n = 60
    inst = gen.xorsat_3r3x(n, seed=6)
    eqs, rhs = inst.meta["equations"], inst.meta["rhs"]
    assert eqs.shape == (n, 3)
    assert np.all(np.bincount(eqs.ravel(), minlength=n) == 3)           # 3-regular
    assert np.all((eqs[:, 0] != eqs[:, 1]) & (eqs[:, 1] != eqs[:, 2]))
    x = (1 - inst.meta["planted_state"][:n]) // 2
    assert np.array_equal(x[eqs].sum(axis=1) % 2, rhs)                  # A x* = b
    D = inst.csr.to_dense(np.int32)
    e = orc.ising_energy_int(D, inst.lin.astype(np.int64), inst.meta["planted_state"])
    assert e == inst.meta["planted_energy"] == -4 * n


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_3r3x_reduction_reproduces_the_cubic_cost(seed):
    """For every assignment of the original spins, the two-body instance minimised over
    the auxiliary spins equals the XORSAT cost -sum_e (-1)^{b_e} s_i s_j s_k minus the
    dropped constant 3 per equation (brute force over all 2^(n+m) states)."""
    n = 6
    inst = gen.xorsat_3r3x(n, seed=seed)
    eqs, rhs = inst.meta["equations"], inst.meta["rhs"]
    D = inst.csr.to_dense(np.int64)
    b = inst.lin.astype(np.int64)
    S = _all_states(2 * n).astype(np.int64)
    E = 0.5 * np.einsum("ri,ij,rj->r", S, D, S) + S @ b
    orig = S[:, :n]
    cubic = -((1 - 2 * rhs)[None, :] * orig[:, eqs[:, 0]] * orig[:, eqs[:, 1]]
              * orig[:, eqs[:, 2]]).sum(axis=1)
    key = ((orig + 1) // 2) @ (1 << np.arange(n))
    for kv in np.unique(key):
        sel = key == kv
        assert E[sel].min() == cubic[sel][0] - 3 * n
    Hmin, _ = orc.bruteforce_ising_int(D.astype(np.int32), b)
    assert Hmin == -4 * n == inst.meta["planted_energy"]
