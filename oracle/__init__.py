"""CPU oracle for replica-batched Parallel Annealing -- test infrastructure only.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
import this package.  It wraps the plain C reference in ``qpa_oracle.c`` (compiled with
gcc, no FMA contraction) with numpy-friendly functions and adds the end-to-end
``solve_*`` drivers that string the primitives together in the order of App. B of the
paper (initialise, T synchronous PA steps, binarise, exact energies, best replica).
It also holds the Simulated Bifurcation steps of App. B, a float64 power method for
the spectral radius that sets SBM's c0, and the low-energy spectrum of a sample set
(distinct states by energy, Sec. V.A).
It shares no code with the HIP library and never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qpa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_F32 = ctypes.c_float
_F64 = ctypes.c_double


def build(force: bool = False) -> str:
    """Compile qpa_oracle.c into liboracle.so (plain gcc, -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
               "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        sig = {
            "orc_sm64_output": (_U64, [_U64, _U64]),
            "orc_pa_init": (None, [_I64, _I64, _I64, _U64, _F32, _P, _P]),
            "orc_lambda_linear": (None, [_I64, _F32, _P]),
            "orc_qubo_to_ising_i64": (None, [_I64, _P, _P, _P, _P, _P]),
            "orc_qubo_to_ising_f64": (None, [_I64, _P, _P, _P, _P, _P]),
            "orc_ising_energy_i64": (_I64, [_I64, _P, _P, _P]),
            "orc_ising_energy_f64": (_F64, [_I64, _P, _P, _P]),
            "orc_qubo_energy_i64": (_I64, [_I64, _P, _P, _P]),
            "orc_qubo_energy_f64": (_F64, [_I64, _P, _P, _P]),
            "orc_ising_energy_csr_i64": (_I64, [_I64, _P, _P, _P, _P, _P]),
            "orc_ising_energy_csr_f64": (_F64, [_I64, _P, _P, _P, _P, _P]),
            "orc_bruteforce_ising_i64": (_I64, [_I64, _P, _P, _P]),
            "orc_pa_steps_dense_i64": (None, [_I64, _P, _P, _I64, _P, _P, _I64, _I64, _P,
                                              _F32, _F32, _P]),
            "orc_pa_steps_dense_f32": (None, [_I64, _P, _P, _I64, _P, _P, _I64, _I64, _P,
                                              _F32, _F32, _P]),
            "orc_pa_steps_csr_i64": (None, [_I64, _P, _P, _P, _P, _I64, _P, _P, _I64, _I64,
                                            _P, _F32, _F32, _P]),
            "orc_pa_steps_csr_f32": (None, [_I64, _P, _P, _P, _P, _I64, _P, _P, _I64, _I64,
                                            _P, _F32, _F32, _P]),
            "orc_pa_step_rows_csr_i64": (None, [_I64, _P, _P, _P, _P, _P, _P, _I64, _P, _F32,
                                                _F32, _F32, _P, _P, _P]),
            "orc_pa_update_f32": (None, [_I64, _P, _F32, _F32, _F32, _P, _P]),
            "orc_bf16_scale_exponent": (ctypes.c_int32, [_I64, _P]),
            "orc_bf16_quantise": (None, [_I64, _P, ctypes.c_int32, _P]),
            "orc_relaxed_grad_dense_f64": (_F64, [_I64, _P, _P, _I64, _P, _P, _I64, _P, _F64,
                                                  _F64, _F64, _P, _P, _P, _P]),
            "orc_relaxed_grad_csr_f64": (_F64, [_I64, _P, _P, _P, _P, _I64, _P, _P, _I64, _P,
                                                _F64, _F64, _F64, _P, _P, _P, _P]),
            "orc_relaxed_grad_dense_f32": (_F64, [_I64, _P, _P, _I64, _P, _I64, _P, _F32,
                                                  _F32, _F64, _P, _P, _P, _P]),
            "orc_relaxed_grad_csr_f32": (_F64, [_I64, _P, _P, _P, _P, _I64, _P, _I64, _P,
                                                _F32, _F32, _F64, _P, _P, _P, _P]),
            "orc_sbm_steps_dense_f32": (None, [_I64, _P, _P, _I64, _P, _P, _I64, _I64, _I64,
                                               _F32, _F32, _F32, _P]),
            "orc_sbm_steps_csr_f32": (None, [_I64, _P, _P, _P, _P, _I64, _P, _P, _I64, _I64,
                                             _I64, _F32, _F32, _F32, _P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = _Lib(lib)
    return _lib


class _Lib:
    """Calls into the C oracle with numpy arrays converted to pointers at call time, so
    that every (possibly freshly converted) array stays referenced during the call."""

    def __init__(self, lib):
        self._lib = lib

    def __getattr__(self, name):
        fn = getattr(self._lib, name)

        def call(*args):
            return fn(*[a.ctypes.data if isinstance(a, np.ndarray) else a for a in args])
        return call


def _ptr(a):
    return a


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ------------------------------------------------------------------------------------
# Counter RNG, initial state and schedule
# ------------------------------------------------------------------------------------
def sm64_output(seed: int, k: int) -> int:
    """k-th output (k >= 1) of SplitMix64 seeded with ``seed``."""
    return int(_load().orc_sm64_output(seed & (2**64 - 1), k & (2**64 - 1)))


def pa_init(n: int, nrep: int, seed: int, sigma0: float, r0: int = 0):
    """Initial analog spins x0 (FP32, [nrep, n]) and zero momentum for replicas r0.."""
    x = np.empty((nrep, n), np.float32)
    m = np.empty((nrep, n), np.float32)
    _load().orc_pa_init(n, r0, nrep, seed & (2**64 - 1), sigma0, _ptr(x), _ptr(m))
    return x, m


def lambda_linear(T: int, lambda0: float) -> np.ndarray:
    lam = np.empty(T, np.float32)
    _load().orc_lambda_linear(T, lambda0, _ptr(lam))
    return lam


# ------------------------------------------------------------------------------------
# App. A canonicalisation and energies
# ------------------------------------------------------------------------------------
def qubo_to_ising_int(Q, c):
    Q = _c(Q, np.int32)
    c = _c(c, np.int64)
    n = Q.shape[0]
    J = np.empty_like(Q)
    b = np.empty(n, np.int64)
    K = np.zeros(1, np.int64)
    _load().orc_qubo_to_ising_i64(n, _ptr(Q), _ptr(c), _ptr(J), _ptr(b), _ptr(K))
    return J, b, int(K[0])


def qubo_to_ising_float(Q, c):
    Q = _c(Q, np.float64)
    c = _c(c, np.float64)
    n = Q.shape[0]
    J = np.empty_like(Q)
    b = np.empty(n, np.float64)
    K = np.zeros(1, np.float64)
    _load().orc_qubo_to_ising_f64(n, _ptr(Q), _ptr(c), _ptr(J), _ptr(b), _ptr(K))
    return J, b, float(K[0])


def ising_energy_int(J, b, s) -> int:
    J = _c(J, np.int32)
    return int(_load().orc_ising_energy_i64(J.shape[0], _ptr(J), _ptr(_c(b, np.int64)),
                                             _ptr(_c(s, np.int8))))


def ising_energy_float(J, b, s) -> float:
    J = _c(J, np.float64)
    return float(_load().orc_ising_energy_f64(J.shape[0], _ptr(J), _ptr(_c(b, np.float64)),
                                               _ptr(_c(s, np.int8))))


def qubo_energy_int(Q, c, x) -> int:
    Q = _c(Q, np.int32)
    return int(_load().orc_qubo_energy_i64(Q.shape[0], _ptr(Q), _ptr(_c(c, np.int64)),
                                            _ptr(_c(x, np.int8))))


def qubo_energy_float(Q, c, x) -> float:
    Q = _c(Q, np.float64)
    return float(_load().orc_qubo_energy_f64(Q.shape[0], _ptr(Q), _ptr(_c(c, np.float64)),
                                              _ptr(_c(x, np.int8))))


def ising_energy_csr_int(rp, col, w, b, s) -> int:
    rp = _c(rp, np.int64)
    return int(_load().orc_ising_energy_csr_i64(len(rp) - 1, _ptr(rp), _ptr(_c(col, np.int32)),
                                                 _ptr(_c(w, np.int32)), _ptr(_c(b, np.int64)),
                                                 _ptr(_c(s, np.int8))))


def ising_energy_csr_float(rp, col, w, b, s) -> float:
    rp = _c(rp, np.int64)
    return float(_load().orc_ising_energy_csr_f64(len(rp) - 1, _ptr(rp),
                                                   _ptr(_c(col, np.int32)),
                                                   _ptr(_c(w, np.float64)),
                                                   _ptr(_c(b, np.float64)),
                                                   _ptr(_c(s, np.int8))))


def bruteforce_ising_int(J, b):
    """Exact minimum of eq. (2) over all 2^n spin states (Gray-code walk)."""
    J = _c(J, np.int32)
    n = J.shape[0]
    if np.any(np.diag(J) != 0):
        raise ValueError("Ising couplings must have a zero diagonal")
    best = np.empty(n, np.int8)
    e = _load().orc_bruteforce_ising_i64(n, _ptr(J), _ptr(_c(b, np.int64)), _ptr(best))
    return int(e), best


# ------------------------------------------------------------------------------------
# PA steps (App. B)
# ------------------------------------------------------------------------------------
def pa_steps_dense_int(J, b, x, m, t0, t1, lam, eta, alpha, want_h=False):
    """Advance (x, m) in place through steps t0..t1-1 with integer dense couplings."""
    J = _c(J, np.int32)
    n = J.shape[0]
    assert x.dtype == np.float32 and x.flags.c_contiguous and m.flags.c_contiguous
    h = np.empty_like(x) if want_h else None
    _load().orc_pa_steps_dense_i64(n, _ptr(J), _ptr(_c(b, np.int64)), x.shape[0], _ptr(x),
                                   _ptr(m), t0, t1, _ptr(_c(lam, np.float32)), eta, alpha,
                                   _ptr(h))
    return h


def pa_steps_dense_float(J, b, x, m, t0, t1, lam, eta, alpha, want_h=False):
    J = _c(J, np.float32)
    n = J.shape[0]
    assert x.dtype == np.float32 and x.flags.c_contiguous and m.flags.c_contiguous
    h = np.empty_like(x) if want_h else None
    _load().orc_pa_steps_dense_f32(n, _ptr(J), _ptr(_c(b, np.float32)), x.shape[0], _ptr(x),
                                   _ptr(m), t0, t1, _ptr(_c(lam, np.float32)), eta, alpha,
                                   _ptr(h))
    return h


def pa_steps_csr_int(rp, col, w, b, x, m, t0, t1, lam, eta, alpha, want_h=False):
    rp = _c(rp, np.int64)
    assert x.dtype == np.float32 and x.flags.c_contiguous and m.flags.c_contiguous
    h = np.empty_like(x) if want_h else None
    _load().orc_pa_steps_csr_i64(len(rp) - 1, _ptr(rp), _ptr(_c(col, np.int32)),
                                 _ptr(_c(w, np.int32)), _ptr(_c(b, np.int64)), x.shape[0],
                                 _ptr(x), _ptr(m), t0, t1, _ptr(_c(lam, np.float32)), eta,
                                 alpha, _ptr(h))
    return h


def pa_steps_csr_float(rp, col, w, b, x, m, t0, t1, lam, eta, alpha, want_h=False):
    rp = _c(rp, np.int64)
    assert x.dtype == np.float32 and x.flags.c_contiguous and m.flags.c_contiguous
    h = np.empty_like(x) if want_h else None
    _load().orc_pa_steps_csr_f32(len(rp) - 1, _ptr(rp), _ptr(_c(col, np.int32)),
                                 _ptr(_c(w, np.float32)), _ptr(_c(b, np.float32)), x.shape[0],
                                 _ptr(x), _ptr(m), t0, t1, _ptr(_c(lam, np.float32)), eta,
                                 alpha, _ptr(h))
    return h


def pa_step_rows_csr_int(rp, col, w, b, x, m, rows, lam_t, eta, alpha):
    """One step of one replica evaluated only at ``rows`` (full state x, m given)."""
    rp = _c(rp, np.int64)
    rows = _c(rows, np.int64)
    x = _c(x, np.float32)
    m = _c(m, np.float32)
    h = np.empty(len(rows), np.float32)
    xo = np.empty(len(rows), np.float32)
    mo = np.empty(len(rows), np.float32)
    _load().orc_pa_step_rows_csr_i64(len(rp) - 1, _ptr(rp), _ptr(_c(col, np.int32)),
                                     _ptr(_c(w, np.int32)), _ptr(_c(b, np.int64)), _ptr(x),
                                     _ptr(m), len(rows), _ptr(rows), lam_t, eta, alpha,
                                     _ptr(h), _ptr(xo), _ptr(mo))
    return h, xo, mo


def pa_update(h, x, m, lam_t, eta, alpha):
    """The PA update of App. B alone (momentum, position, clip), in place on FP32 x, m
    from given fields h of the same shape: the update every step function applies."""
    assert x.dtype == np.float32 and x.flags.c_contiguous and m.flags.c_contiguous
    assert x.shape == m.shape == np.shape(h)
    _load().orc_pa_update_f32(x.size, _ptr(_c(h, np.float32)), lam_t, eta, alpha, _ptr(x),
                              _ptr(m))


# ------------------------------------------------------------------------------------
# BF16 storage of float couplings
# ------------------------------------------------------------------------------------
def bf16_scale_exponent(J) -> int:
    J = _c(J, np.float32)
    return int(_load().orc_bf16_scale_exponent(J.size, _ptr(J)))


def bf16_quantise(J, e: int) -> np.ndarray:
    """2^e * RNE_bf16(J / 2^e) as FP32 (the couplings a scaled-BF16 field sees)."""
    J = _c(J, np.float32)
    out = np.empty_like(J)
    _load().orc_bf16_quantise(J.size, _ptr(J), e, _ptr(out))
    return out


# ------------------------------------------------------------------------------------
# Relaxed PA and its adjoint (FP64)
# ------------------------------------------------------------------------------------
def relaxed_grad_dense(J, b, x0, T, lam, eta, alpha, norm=None, grads=True, m0=None):
    """Returns (L, d_eta, d_alpha, d_lam[T]) of the mean relaxed final energy."""
    J = _c(J, np.float64)
    x0 = _c(x0, np.float64)
    nrep, n = x0.shape
    norm = 1.0 / nrep if norm is None else norm
    de = np.zeros(1)
    da = np.zeros(1)
    dl = np.zeros(T)
    L = _load().orc_relaxed_grad_dense_f64(
        n, _ptr(J), _ptr(_c(b, np.float64)), nrep, _ptr(x0),
        _ptr(None if m0 is None else _c(m0, np.float64)), T, _ptr(_c(lam, np.float64)), eta,
        alpha, norm, _ptr(de) if grads else None, _ptr(da) if grads else None,
        _ptr(dl) if grads else None, None)
    return float(L), float(de[0]), float(da[0]), dl


def relaxed_grad_csr(rp, col, w, b, x0, T, lam, eta, alpha, norm=None, grads=True, m0=None):
    rp = _c(rp, np.int64)
    x0 = _c(x0, np.float64)
    nrep, n = x0.shape
    norm = 1.0 / nrep if norm is None else norm
    de = np.zeros(1)
    da = np.zeros(1)
    dl = np.zeros(T)
    L = _load().orc_relaxed_grad_csr_f64(
        n, _ptr(rp), _ptr(_c(col, np.int32)), _ptr(_c(w, np.float64)),
        _ptr(_c(b, np.float64)), nrep, _ptr(x0),
        _ptr(None if m0 is None else _c(m0, np.float64)), T, _ptr(_c(lam, np.float64)), eta,
        alpha, norm, _ptr(de) if grads else None, _ptr(da) if grads else None,
        _ptr(dl) if grads else None, None)
    return float(L), float(de[0]), float(da[0]), dl


def relaxed_grad32_dense(J, b, x0, T, lam, eta, alpha, norm=None, grads=True):
    """The single-precision pass (state, adjoint vectors and products in FP32, one fused
    multiply-add per product term in ascending column order; sums in FP64).  Returns
    (L, d_eta, d_alpha, d_lam[T], x_T [nrep, n] float32)."""
    J = _c(J, np.float32)
    x0 = _c(x0, np.float32)
    nrep, n = x0.shape
    norm = 1.0 / nrep if norm is None else norm
    de, da, dl = np.zeros(1), np.zeros(1), np.zeros(T)
    xT = np.empty((nrep, n), np.float32)
    L = _load().orc_relaxed_grad_dense_f32(
        n, _ptr(J), _ptr(_c(b, np.float32)), nrep, _ptr(x0), T, _ptr(_c(lam, np.float32)),
        float(np.float32(eta)), float(np.float32(alpha)), norm, _ptr(de) if grads else None,
        _ptr(da) if grads else None, _ptr(dl) if grads else None, _ptr(xT))
    return float(L), float(de[0]), float(da[0]), dl, xT


def relaxed_grad32_csr(rp, col, w, b, x0, T, lam, eta, alpha, norm=None, grads=True):
    """relaxed_grad32_dense for CSR couplings (entries summed in stored order, which is
    ascending column order for a valid instance)."""
    x0 = _c(x0, np.float32)
    nrep, n = x0.shape
    norm = 1.0 / nrep if norm is None else norm
    de, da, dl = np.zeros(1), np.zeros(1), np.zeros(T)
    xT = np.empty((nrep, n), np.float32)
    L = _load().orc_relaxed_grad_csr_f32(
        n, _ptr(_c(rp, np.int64)), _ptr(_c(col, np.int32)), _ptr(_c(w, np.float32)),
        _ptr(_c(b, np.float32)), nrep, _ptr(x0), T, _ptr(_c(lam, np.float32)),
        float(np.float32(eta)), float(np.float32(alpha)), norm, _ptr(de) if grads else None,
        _ptr(da) if grads else None, _ptr(dl) if grads else None, _ptr(xT))
    return float(L), float(de[0]), float(da[0]), dl, xT


# ------------------------------------------------------------------------------------
# End-to-end drivers: what a solve returns, computed the slow way
# ------------------------------------------------------------------------------------
@dataclass
class OracleResult:
    x: np.ndarray          # final analog spins [R, n] FP32
    m: np.ndarray          # final momenta [R, n] FP32
    spins: np.ndarray      # sign(x_T) in {-1,+1} [R, n] int8
    energy: np.ndarray     # objective of each replica's final spins (int64 or float64)
    best: int              # lowest replica index attaining the minimum energy


def _sign(x):
    return np.where(x >= 0, 1, -1).astype(np.int8)


def _argmin_first(e):
    return int(np.flatnonzero(e == e.min())[0])


def solve_dense_int(Jq, lin, kind, R, T, lam, eta, alpha, seed, sigma0, r0=0):
    """PA on a dense integer instance.  kind 'qubo': (Jq, lin) = (Q, c) and the energy is
    x^T Q x + c^T x of x = (1+s)/2; kind 'ising': (Jq, lin) = (J, b) and the energy is
    H(s) of eq. (2)."""
    Jq = _c(Jq, np.int32)
    n = Jq.shape[0]
    if kind == "qubo":
        J, b, _ = qubo_to_ising_int(Jq, lin)
    else:
        J, b = Jq, _c(lin, np.int64)
    x, m = pa_init(n, R, seed, sigma0, r0)
    pa_steps_dense_int(J, b, x, m, 0, T, lam, eta, alpha)
    s = _sign(x)
    if kind == "qubo":
        e = np.array([qubo_energy_int(Jq, lin, (s[r] > 0).astype(np.int8)) for r in range(R)],
                     np.int64)
    else:
        e = np.array([ising_energy_int(J, b, s[r]) for r in range(R)], np.int64)
    return OracleResult(x, m, s, e, _argmin_first(e))


def solve_csr_int(rp, col, w, lin, R, T, lam, eta, alpha, seed, sigma0, r0=0):
    """PA on an Ising CSR instance with integer couplings (energy = eq. (2))."""
    n = len(rp) - 1
    x, m = pa_init(n, R, seed, sigma0, r0)
    pa_steps_csr_int(rp, col, w, lin, x, m, 0, T, lam, eta, alpha)
    s = _sign(x)
    e = np.array([ising_energy_csr_int(rp, col, w, lin, s[r]) for r in range(R)], np.int64)
    return OracleResult(x, m, s, e, _argmin_first(e))


def track_best(x, m, T, every, step, energy):
    """Best sampled state of a PA trajectory (Sec. VIII: many states are evolved and the
    best one found is what the solver reports, not necessarily where a replica ends).
    step(x, m, t0, t1) advances the state in place through steps t0 .. t1-1; energy(s)
    gives the objective of spins s [R, n].  The state after each segment of `every` steps
    and after step T (the initial state when T == 0) is binarised (+1 where x >= 0) and
    scored; per replica the lowest energy is kept, the earliest state on ties.
    Returns (best_energy [R], best_step [R] int32, best_spins [R, n] int8)."""
    best_e = best_t = best_s = None
    t0 = 0
    while True:
        t1 = min(t0 + every, T)
        if t1 > t0:
            step(x, m, t0, t1)
        s = _sign(x)
        e = np.asarray(energy(s))
        if best_e is None:
            best_e, best_t, best_s = e.copy(), np.full(len(e), t1, np.int32), s.copy()
        else:
            better = e < best_e
            best_e = np.where(better, e, best_e)
            best_t[better] = t1
            best_s[better] = s[better]
        t0 = t1
        if t0 >= T:
            return best_e, best_t, best_s


def qubo_to_ising_csr_int(rp, col, w, c):
    """App. A for a CSR QUBO with integer weights: J = the off-diagonal entries,
    b_i = (sum of row i, diagonal included) + c_i, K = (1/2) 1^T Q 1 + (1/2) tr Q + 1^T c."""
    rp = np.asarray(rp, np.int64)
    col = np.asarray(col, np.int64)
    w = np.asarray(w, np.int64)
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    rowsum = np.zeros(n, np.int64)
    np.add.at(rowsum, rows, w)
    diag = np.zeros(n, np.int64)
    on = rows == col
    np.add.at(diag, rows[on], w[on])
    keep = ~on
    rp2 = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows[keep], minlength=n), out=rp2[1:])
    b = rowsum + np.asarray(c, np.int64)
    K = (int(rowsum.sum()) + int(diag.sum())) // 2 + int(np.asarray(c, np.int64).sum())
    return rp2, col[keep].astype(np.int32), w[keep].astype(np.int32), b, K


# ---- Simulated Bifurcation Machine (App. B, SBM) ---------------------------------------
def sbm_steps_dense(J, b, q, p, t0, t1, T, a0, c0, dt, want_g=False):
    """Symplectic-Euler SBM steps t0..t1-1 on float32 q, p [R][n] in place (problem in
    the PA convention; see orc_sbm_steps_dense_f32).  Returns the last step's g = J q + b
    when want_g."""
    J = _c(J, np.float32)
    n = J.shape[0]
    assert q.dtype == np.float32 and q.flags.c_contiguous and p.flags.c_contiguous
    g = np.empty_like(q) if want_g else None
    _load().orc_sbm_steps_dense_f32(n, _ptr(J), _ptr(_c(b, np.float32)), q.shape[0], _ptr(q),
                                    _ptr(p), t0, t1, T, a0, c0, dt, _ptr(g))
    return g


def sbm_steps_csr(rp, col, w, b, q, p, t0, t1, T, a0, c0, dt, want_g=False):
    """As sbm_steps_dense for CSR couplings (any numeric weights, used as float32)."""
    rp = _c(rp, np.int64)
    assert q.dtype == np.float32 and q.flags.c_contiguous and p.flags.c_contiguous
    g = np.empty_like(q) if want_g else None
    _load().orc_sbm_steps_csr_f32(len(rp) - 1, _ptr(rp), _ptr(_c(col, np.int32)),
                                  _ptr(_c(w, np.float32)), _ptr(_c(b, np.float32)), q.shape[0],
                                  _ptr(q), _ptr(p), t0, t1, T, a0, c0, dt, _ptr(g))
    return g


def power_start_vector(n, seed):
    """Start vector of the power method: v_i = 2u - 1, u the top 24 bits of SplitMix64
    output number i + 1 of `seed` (the draw of the initial state, replica 0)."""
    k = np.arange(1, n + 1, dtype=np.uint64)
    return np.array([2.0 * (sm64_output(seed, int(i)) >> 40) / 16777216.0 - 1.0 for i in k])


def spectral_radius_power(J, iters, seed):
    """Power method in float64 on the symmetric matrix J (dense): v <- J v / ||J v|| from
    power_start_vector; returns ||J v|| after `iters` normalised iterations, which tends
    to the spectral radius max |lambda| (also when +-lambda_max both occur)."""
    J = np.asarray(J, np.float64)
    v = power_start_vector(J.shape[0], seed)
    v = v / np.linalg.norm(v)
    for _ in range(iters):
        w = J @ v
        v = w / np.linalg.norm(w)
    return float(np.linalg.norm(J @ v))


# ---- low-energy spectrum (Sec. V.A: the sample set of many low-energy states) ----------
def spectrum(spins, energy, k):
    """Distinct states among the R samples, ordered by energy and then by the lowest
    replica index holding the state; the first k of them.  Returns (states [m][n] int8,
    energies [m], counts [m] (replicas holding the state), first [m] (lowest such
    replica index), distinct (number of distinct states)), m = min(k, distinct).  Each
    state's energy is the energy its first replica reports (equal states have equal
    energies)."""
    spins = np.asarray(spins, np.int8)
    energy = np.asarray(energy)
    uniq, first, counts = np.unique(spins, axis=0, return_index=True, return_counts=True)
    E = energy[first]
    order = np.lexsort((first, E))[:k]
    return uniq[order], E[order], counts[order].astype(np.int32), \
        first[order].astype(np.int32), len(uniq)
