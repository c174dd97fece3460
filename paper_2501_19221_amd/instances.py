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


def sdk_toy() -> Instance:
    """The spin-type model built in the SDK listing of Sec. V.C: linear biases
    {0: 1, 2: -1}, quadratic couplings {(0,1): -1, (1,2): 0.5}, offset 0."""
    J = np.zeros((3, 3), np.float32)
    J[0, 1] = J[1, 0] = -1.0
    J[1, 2] = J[2, 1] = 0.5
    b = np.array([1.0, 0.0, -1.0], np.float32)
    return Instance("ising", 3, dense=J, lin=b)
