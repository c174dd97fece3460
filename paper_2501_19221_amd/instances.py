"""Seeded synthetic instance generators shaped like the paper's workloads.

This module holds random-instance construction only: no step of the annealing method,
no energy evaluation and no canonicalisation.  Both the HIP path's tests/benchmarks and
the CPU oracle's tests draw their inputs from here.  Every generator is a pure function
of its arguments and a numpy ``default_rng(seed)`` stream.

Families (paper sections they stand in for):
  * ``dense_int_qubo``    -- small all-to-all instances with integer couplings
                             (Sec. VII.A uses brute-forceable all-to-all instances).
  * ``chimera_ising``     -- Chimera C_{m,m} graphs of K_{4,4} cells with +-1 couplings
                             (Sec. VII.B, random Chimera instances).
  * ``sk_ising``          -- dense Sherrington-Kirkpatrick couplings N(0, 1/n) with
                             Gaussian fields (dense pseudo-random instances, Sec. IX).
  * ``er_qubo_batch``     -- many uneven Erdos-Renyi QUBOs with integer weights (the
                             many-instances-per-size protocol of Secs. V and VIII).
  * ``planted_3regular``  -- gauge-transformed random 3-regular Ising graph with a planted
                             ground state (planted families of Sec. VIII; size of the
                             largest sparse instances the paper solves, ~1e8 variables).
  * ``wishart_planted``   -- dense Wishart-planted instances (Sec. VIII.C).
  * ``tile_planted``      -- tile-planted square lattices (Sec. VIII.B).
  * ``xorsat_3r3x``       -- 3-regular 3-XORSAT, planted, reduced to two-body form
                             (Sec. VIII.A with the cubic reduction of Sec. VI.A).
  * ``sdk_toy``           -- the four-term spin model of the SDK listing in Sec. V.C.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class CSR:
    """Symmetric sparse couplings: row i holds (col[k], w[k]) for k in [rp[i], rp[i+1])."""
    n: int
    rp: np.ndarray      # int32 [n+1] (int64 if nnz >= 2^31)
    col: np.ndarray     # int32 or int16 [nnz]
    w: np.ndarray       # int8 / int16 / int32 / float32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rp[-1])

    def to_dense(self, dtype=None) -> np.ndarray:
        d = np.zeros((self.n, self.n), dtype or self.w.dtype)
        rows = np.repeat(np.arange(self.n), np.diff(self.rp.astype(np.int64)))
        np.add.at(d, (rows, self.col.astype(np.int64)), self.w)
        return d


@dataclass
class Instance:
    """One problem. kind 'qubo': minimise x^T Q x + c^T x (Q symmetric);
    kind 'ising': minimise sum_{i<j} J_ij s_i s_j + sum_i b_i s_i."""
    kind: str
    n: int
    dense: np.ndarray | None = None    # [n, n] symmetric
    csr: CSR | None = None
    lin: np.ndarray | None = None      # c (qubo) or b (ising), length n
    meta: dict = field(default_factory=dict)


def dense_int_qubo(n: int = 20, lo: int = -10, hi: int = 10, seed: int = 1) -> Instance:
    """Q_ij (i <= j) uniform integers in [lo, hi] mirrored to a symmetric int32 matrix,
    linear terms uniform integers in [lo, hi]."""
    rng = np.random.default_rng(seed)
    U = rng.integers(lo, hi + 1, size=(n, n), dtype=np.int32)
    Q = np.triu(U)
    Q = Q + np.triu(Q, 1).T
    c = rng.integers(lo, hi + 1, size=n, dtype=np.int32)
    return Instance("qubo", n, dense=np.ascontiguousarray(Q, np.int32), lin=c)


def dense_int_ising(n: int, lo: int = -10, hi: int = 10, seed: int = 1) -> Instance:
    rng = np.random.default_rng(seed)
    U = rng.integers(lo, hi + 1, size=(n, n), dtype=np.int32)
    J = np.triu(U, 1)
    J = J + J.T
    b = rng.integers(lo, hi + 1, size=n, dtype=np.int32)
    return Instance("ising", n, dense=np.ascontiguousarray(J, np.int32), lin=b)


def _csr_from_edges(n, u, v, w, idx_dtype=np.int32):
    """Symmetric CSR (both directions stored), rows sorted by column."""
    rows = np.concatenate([u, v]).astype(np.int64)
    cols = np.concatenate([v, u]).astype(np.int64)
    ws = np.concatenate([w, w])
    order = np.lexsort((cols, rows))
    rows, cols, ws = rows[order], cols[order], ws[order]
    counts = np.bincount(rows, minlength=n)
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=rp[1:])
    rp_dtype = np.int32 if rp[-1] < 2**31 else np.int64
    return CSR(n, rp.astype(rp_dtype), cols.astype(idx_dtype), ws)


def chimera_ising(m: int = 16, L: int = 4, seed: int = 2) -> Instance:
    """Chimera C_{m,m}: an m x m grid of K_{L,L} cells.  Vertex (row, col, side, k) has
    index ((row*m + col)*2 + side)*L + k.  Inside a cell every side-0 vertex couples to
    every side-1 vertex; side-0 vertex k couples to side-0 vertex k of the cell below,
    side-1 vertex k to side-1 vertex k of the cell to the right.  Couplings are +-1
    uniform, fields zero, weights stored as int8."""
    rng = np.random.default_rng(seed)
    n = m * m * 2 * L

    def vid(r, c, side, k):
        return ((r * m + c) * 2 + side) * L + k

    us, vs = [], []
    for r in range(m):
        for c in range(m):
            for a in range(L):
                for b_ in range(L):
                    us.append(vid(r, c, 0, a))
                    vs.append(vid(r, c, 1, b_))
            for k in range(L):
                if r + 1 < m:
                    us.append(vid(r, c, 0, k))
                    vs.append(vid(r + 1, c, 0, k))
                if c + 1 < m:
                    us.append(vid(r, c, 1, k))
                    vs.append(vid(r, c + 1, 1, k))
    u = np.array(us, np.int64)
    v = np.array(vs, np.int64)
    w = (2 * rng.integers(0, 2, size=len(u)) - 1).astype(np.int8)
    csr = _csr_from_edges(n, u, v, w)
    return Instance("ising", n, csr=csr, lin=np.zeros(n, np.int8),
                    meta={"edges": len(u), "cells": m * m})


def sk_ising(n: int = 4096, field_var: float = 0.1, seed: int = 3) -> Instance:
    """Sherrington-Kirkpatrick couplings: J_ij (i<j) ~ N(0, 1/n) mirrored, zero diagonal,
    FP32; fields b_i ~ N(0, field_var) (variance)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n), dtype=np.float32) * np.float32(1.0 / np.sqrt(n))
    J = np.triu(G, 1)
    J = J + J.T
    b = (rng.standard_normal(n, dtype=np.float32) * np.float32(np.sqrt(field_var)))
    return Instance("ising", n, dense=np.ascontiguousarray(J, np.float32),
                    lin=b.astype(np.float32))


def er_qubo(n: int, p: float, wmax: int, rng, idx_dtype=np.int16) -> Instance:
    """Erdos-Renyi QUBO: each unordered pair i<j present with probability p, weight
    uniform in [-wmax, wmax] (zero allowed), Q_ii = 0, c_i uniform in [-wmax, wmax]."""
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(len(iu)) < p
    u, v = iu[keep], ju[keep]
    w = rng.integers(-wmax, wmax + 1, size=len(u)).astype(np.int16)
    csr = _csr_from_edges(n, u, v, w, idx_dtype=idx_dtype)
    c = rng.integers(-wmax, wmax + 1, size=n).astype(np.int16)
    return Instance("qubo", n, csr=csr, lin=c, meta={"edges": len(u)})


def er_qubo_batch(count: int = 512, nmin: int = 100, nmax: int = 2000, p: float = 0.1,
                  wmax: int = 100, seed: int = 4) -> list[Instance]:
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=count)
    return [er_qubo(int(n), p, wmax, rng) for n in sizes]


def planted_3regular(n: int, wmin: int = 1, wmax: int = 7, seed: int = 5) -> Instance:
    """Random 3-regular graph as a Hamiltonian cycle through a random vertex order plus a
    random perfect matching (re-drawn locally until no matching edge repeats a cycle edge,
    so the graph is simple).  Edge magnitudes |w| uniform in [wmin, wmax]; a random
    planted state s* gauges every coupling to J_ij = -s*_i s*_j |w_ij| (int8), fields zero.
    Every coupling is then satisfied by s*, which is a ground state.  Rows have exactly
    three entries, sorted by column."""
    if n % 2 or n < 6:
        raise ValueError("n must be even and >= 6")
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n).astype(np.int64)
    # cycle edges perm[k] -- perm[k+1]
    cu = perm
    cv = np.roll(perm, -1)
    # matching edges
    mperm = rng.permutation(n).astype(np.int64)
    mu = mperm[0::2].copy()
    mv = mperm[1::2].copy()
    pos = np.empty(n, np.int64)
    pos[perm] = np.arange(n)
    for _ in range(64):
        d = (pos[mu] - pos[mv]) % n
        bad = np.flatnonzero((d == 1) | (d == n - 1))
        if len(bad) == 0:
            break
        for k in bad:                      # one swap at a time: indices may be adjacent
            j = (int(k) + 1 + int(rng.integers(0, len(mu) - 1))) % len(mu)
            mv[k], mv[j] = mv[j], mv[k]
    else:
        raise RuntimeError("matching repair did not converge")
    s_star = (2 * rng.integers(0, 2, size=n) - 1).astype(np.int8)
    wc = rng.integers(wmin, wmax + 1, size=n).astype(np.int8)
    wm = rng.integers(wmin, wmax + 1, size=n // 2).astype(np.int8)
    # three neighbours per vertex, with their magnitudes
    nb = np.empty((n, 3), np.int64)
    mag = np.empty((n, 3), np.int8)
    nb[cu, 0] = cv
    mag[cu, 0] = wc
    nb[cv, 1] = cu
    mag[cv, 1] = wc
    nb[mu, 2] = mv
    mag[mu, 2] = wm
    nb[mv, 2] = mu
    mag[mv, 2] = wm
    del perm, cu, cv, mperm, mu, mv, pos, wc, wm
    order = np.argsort(nb, axis=1, kind="stable")
    nb = np.take_along_axis(nb, order, axis=1)
    mag = np.take_along_axis(mag, order, axis=1)
    del order
    sgn = (-(s_star[:, None].astype(np.int8) * s_star[nb].astype(np.int8))).astype(np.int8)
    w = (sgn * mag).astype(np.int8)
    del sgn, mag
    rp = (np.arange(n + 1, dtype=np.int64) * 3)
    rp = rp.astype(np.int32 if rp[-1] < 2**31 else np.int64)
    csr = CSR(n, rp, nb.reshape(-1).astype(np.int32), w.reshape(-1))
    return Instance("ising", n, csr=csr, lin=np.zeros(n, np.int8),
                    meta={"planted_state": s_star})


def _csr_from_pairs(n, u, v, w, dtype=np.int8):
    """Symmetric CSR from unordered pairs (u < v or u > v) with weights; repeated pairs
    are summed, zero sums dropped."""
    a = np.minimum(u, v).astype(np.int64)
    b = np.maximum(u, v).astype(np.int64)
    key = a * n + b
    uk, inv = np.unique(key, return_inverse=True)
    ws = np.zeros(len(uk), np.int64)
    np.add.at(ws, inv, np.asarray(w, np.int64))
    keep = ws != 0
    uk, ws = uk[keep], ws[keep]
    return _csr_from_edges(n, uk // n, uk % n, ws.astype(dtype))


def wishart_planted(n: int, alpha: float, seed: int = 7) -> Instance:
    """Wishart planting (Sec. VIII.C).  M = max(1, round(alpha n)) columns w of W are
    drawn from N(0, Sigma), Sigma = n/(n-1) (I - t t^T / n) with t = (1, ..., 1), as
    sqrt(n/(n-1)) (z - mean(z)) with z ~ N(0, I) (so W^T t = 0 up to rounding).  With
    J~ = -(1/n) W W^T, the section's Hamiltonian -(1/2) sum_ij J_ij s_i s_j on
    J = J~ - diag(J~) is, in the convention of eq. (2), the dense float32 coupling matrix
    (1/n) W W^T with its diagonal removed, gauged by a random planted state s*
    (J_ij -> J_ij s*_i s*_j).  s* is a ground state with energy (1/2) Tr J~ (exactly so
    for the float64 matrix; the float32 couplings move it by rounding only).  Zero fields.
    meta: planted_state, alpha, M, planted_energy = (1/2) Tr J~ (float64)."""
    rng = np.random.default_rng(seed)
    M = max(1, int(round(alpha * n)))
    z = rng.standard_normal((n, M))
    W = np.sqrt(n / (n - 1.0)) * (z - z.mean(axis=0, keepdims=True))
    J = (W @ W.T) / n
    np.fill_diagonal(J, 0.0)
    E0 = -0.5 * float(np.sum(W * W)) / n           # (1/2) Tr J~
    s_star = (2 * rng.integers(0, 2, size=n) - 1).astype(np.int8)
    J = J * np.outer(s_star, s_star)
    J = (J + J.T) / 2
    return Instance("ising", n, dense=np.ascontiguousarray(J, np.float32),
                    lin=np.zeros(n, np.float32),
                    meta={"planted_state": s_star, "alpha": alpha, "M": M,
                          "planted_energy": E0})


# Tiles of the tile-planted square lattice: |J| of the four plaquette edges in cyclic
# order, the last one antiferromagnetic.  With H_tile = -sum J_e s_a s_b, the all-up state
# leaves only the negative edge unsatisfied; type k has exactly k ground-state pairs
# (the unsatisfied edge may be the negative one or any of the k - 1 unit positive ones).
TILE_TYPES = {1: (2, 2, 2, -1), 2: (2, 2, 1, -1), 3: (2, 1, 1, -1), 4: (1, 1, 1, -1)}


def tile_planted(L: int, probs=(0.0, 0.2, 0.0, 0.8), seed: int = 8) -> Instance:
    """Tile planting on an L x L square lattice with periodic boundaries (Sec. VIII.B).
    Vertex (x, y) has index y L + x.  The tiles are the plaquettes with lower-left corner
    (x, y), x + y even (a checkerboard: every edge lies in exactly one tile, every vertex
    in two); each draws its type k from `probs` = (p1, p2, p3, p4) and the edge weights
    TILE_TYPES[k] in a random rotation around its edges (bottom, right, top, left).  The
    all-up state minimises every tile, hence the sum; a random planted state s* gauges the
    couplings.  Stored in the convention of eq. (2): J'_ab = -J_e s*_a s*_b (int8), zero
    fields; the planted energy is -sum_e J_e.  meta: planted_state, tile_types."""
    if L % 2 or L < 4:
        raise ValueError("L must be even and >= 4")
    rng = np.random.default_rng(seed)
    xs, ys = np.meshgrid(np.arange(L), np.arange(L), indexing="xy")
    black = ((xs + ys) % 2 == 0)
    x0, y0 = xs[black].ravel(), ys[black].ravel()
    T = len(x0)
    v00 = y0 * L + x0
    v10 = y0 * L + (x0 + 1) % L
    v11 = ((y0 + 1) % L) * L + (x0 + 1) % L
    v01 = ((y0 + 1) % L) * L + x0
    eu = np.stack([v00, v10, v01, v00], axis=1)       # bottom, right, top, left
    ev = np.stack([v10, v11, v11, v01], axis=1)
    p = np.asarray(probs, np.float64)
    kinds = rng.choice(4, size=T, p=p / p.sum()) + 1
    table = np.array([TILE_TYPES[k] for k in (1, 2, 3, 4)], np.int64)
    rot = rng.integers(0, 4, size=T)
    idx = (np.arange(4)[None, :] - rot[:, None]) % 4
    Je = np.take_along_axis(table[kinds - 1], idx, axis=1)
    s_star = (2 * rng.integers(0, 2, size=L * L) - 1).astype(np.int8)
    u, v, je = eu.ravel(), ev.ravel(), Je.ravel()
    w = -je * s_star[u].astype(np.int64) * s_star[v].astype(np.int64)
    csr = _csr_from_pairs(L * L, u, v, w, np.int8)
    return Instance("ising", L * L, csr=csr, lin=np.zeros(L * L, np.int8),
                    meta={"planted_state": s_star, "tile_types": kinds,
                          "planted_energy": int(-je.sum())})


def xorsat_3r3x(n: int, seed: int = 9) -> Instance:
    """3-regular 3-XORSAT with a planted solution (Sec. VIII.A), reduced to two-body form.
    m = n equations over GF(2), each on three distinct variables, each variable in three
    equations (configuration model; triples with a repeated variable are repaired by
    random swaps).  A random x* fixes the right-hand sides b = A x* mod 2, so the Ising
    cost -sum_e (-1)^{b_e} s_i s_j s_k (s = (-1)^x) has minimum -m at s* = (-1)^{x*}.
    Every cubic term sigma s_i s_j s_k (sigma = -(-1)^{b_e}) is replaced by the two-body
    form of the cubic-term reduction of Sec. VI.A, with its own auxiliary spin a_e
    (variable n + e):
        3 + sigma (s_i + s_j + s_k + 2 a) + 2 a (s_i + s_j + s_k) + s_i s_j + s_j s_k + s_i s_k,
    whose minimum over a equals the cubic term.  The stored Ising instance (int8 couplings
    and fields) drops the constant 3 per equation, so its minimum is -4m.
    meta: planted_state (n + m spins: s* and the minimising a), equations, rhs."""
    if n < 3:
        raise ValueError("n must be >= 3")
    rng = np.random.default_rng(seed)
    m = n
    stubs = rng.permutation(np.repeat(np.arange(n), 3)).reshape(m, 3)
    for _ in range(10000):
        bad = np.flatnonzero((stubs[:, 0] == stubs[:, 1]) | (stubs[:, 1] == stubs[:, 2])
                             | (stubs[:, 0] == stubs[:, 2]))
        if len(bad) == 0:
            break
        for e in bad:
            f = int(rng.integers(0, m))
            c1, c2 = int(rng.integers(0, 3)), int(rng.integers(0, 3))
            stubs[e, c1], stubs[f, c2] = stubs[f, c2], stubs[e, c1]
    else:
        raise RuntimeError("3-regular repair did not converge")
    eqs = np.sort(stubs, axis=1)
    x_star = rng.integers(0, 2, size=n)
    rhs = x_star[eqs].sum(axis=1) % 2
    s = (1 - 2 * x_star).astype(np.int64)
    sigma = -(1 - 2 * rhs)                       # -(-1)^b
    i, j, k = eqs[:, 0], eqs[:, 1], eqs[:, 2]
    aux = n + np.arange(m)
    S = s[i] + s[j] + s[k]
    # minimising auxiliary spin of each equation at the planted state (ties: +1)
    f_up = sigma * (S + 2) + 2 * S
    f_dn = sigma * (S - 2) - 2 * S
    a_star = np.where(f_up <= f_dn, 1, -1)
    u = np.concatenate([i, j, i, aux, aux, aux])
    v = np.concatenate([j, k, k, i, j, k])
    w = np.concatenate([np.ones(3 * m, np.int64), np.full(3 * m, 2, np.int64)])
    N = n + m
    csr = _csr_from_pairs(N, u, v, w, np.int8)
    lin = np.zeros(N, np.int64)
    np.add.at(lin, i, sigma)
    np.add.at(lin, j, sigma)
    np.add.at(lin, k, sigma)
    lin[aux] += 2 * sigma
    planted = np.concatenate([s, a_star]).astype(np.int8)
    return Instance("ising", N, csr=csr, lin=lin.astype(np.int8),
                    meta={"planted_state": planted, "equations": eqs, "rhs": rhs,
                          "planted_energy": -4 * m})


def sdk_toy() -> Instance:
    """The spin-type model built in the SDK listing of Sec. V.C: linear biases
    {0: 1, 2: -1}, quadratic couplings {(0,1): -1, (1,2): 0.5}, offset 0."""
    J = np.zeros((3, 3), np.float32)
    J[0, 1] = J[1, 0] = -1.0
    J[1, 2] = J[2, 1] = 0.5
    b = np.array([1.0, 0.0, -1.0], np.float32)
    return Instance("ising", 3, dense=J, lin=b)
