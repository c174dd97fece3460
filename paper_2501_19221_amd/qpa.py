"""Thin ctypes binding of libqpa (include/qpa.h).

The functions named like the C entry points (``qpa_solve``, ``qpa_steps``, ...) only
marshal arguments: torch tensors supply device memory and the current HIP stream, and
every step of the method runs in the library's kernels.  Importing this module fails
loudly if the built library is missing -- there is no fallback path.

Convenience layer: ``Problem`` wraps device tensors of one instance and ``solve`` /
``steps`` / ``energy`` allocate outputs and the workspace with torch and call the C ABI.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqpa.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libqpa.so is not built: run `python -m paper_2501_19221_amd.build` "
                      "(expected at %s)" % LIB_PATH)
# torch brings its own HIP runtime; loading it first makes libqpa bind to that same copy
# (a process must hold a single HIP runtime -- a second one finds no device).
import torch  # noqa: E402,F401

from .abi import *  # noqa: E402,F401,F403  (enums, structs, EXPORTED)
from .abi import _P, _S, load as _load_abi  # noqa: E402

_lib = _load_abi(LIB_PATH)


class QpaError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        name = _lib.qpa_status_string(status).decode()
        super().__init__("%s: %s" % (name, message))


# ---- C entry points under their own names --------------------------------------------
def qpa_create(device: int = 0):
    h = _P()
    st = _lib.qpa_create(ctypes.byref(h), device)
    if st != QPA_OK:
        raise QpaError(st, "qpa_create(device=%d) failed: %s" % (device, qpa_last_error(None)))
    return h


def qpa_destroy(ctx):
    _lib.qpa_destroy(ctx)


def qpa_last_error(ctx) -> str:
    return _lib.qpa_last_error(ctx).decode()


def qpa_status_string(status: int) -> str:
    return _lib.qpa_status_string(status).decode()


def qpa_version() -> str:
    return _lib.qpa_version().decode()


def _check(ctx, st):
    if st != QPA_OK:
        raise QpaError(st, qpa_last_error(ctx))


def qpa_workspace_size(ctx, problem: qpa_problem, params: qpa_params) -> int:
    nbytes = ctypes.c_size_t()
    _check(ctx, _lib.qpa_workspace_size(ctx, ctypes.byref(problem), ctypes.byref(params),
                                        ctypes.byref(nbytes)))
    return nbytes.value


def qpa_solve(ctx, problem, params, workspace, workspace_bytes, stream, outputs):
    _check(ctx, _lib.qpa_solve(ctx, ctypes.byref(problem), ctypes.byref(params), workspace,
                               workspace_bytes, stream, ctypes.byref(outputs)))


def qpa_solve_noalloc(ctx, problem, params, stream, outputs):
    _check(ctx, _lib.qpa_solve_noalloc(ctx, ctypes.byref(problem), ctypes.byref(params), stream,
                                       ctypes.byref(outputs)))


def qpa_solve_track(ctx, problem, params, every, workspace, workspace_bytes, stream, outputs,
                    track):
    _check(ctx, _lib.qpa_solve_track(ctx, ctypes.byref(problem), ctypes.byref(params), every,
                                     workspace, workspace_bytes, stream, ctypes.byref(outputs),
                                     ctypes.byref(track)))


def qpa_steps(ctx, problem, params, t0, t1, x, m, h_last, workspace, workspace_bytes, stream):
    _check(ctx, _lib.qpa_steps(ctx, ctypes.byref(problem), ctypes.byref(params), t0, t1, x, m,
                               h_last, workspace, workspace_bytes, stream))


def qpa_energy(ctx, problem, params, spins, energy, energy_i64, best, workspace,
               workspace_bytes, stream):
    _check(ctx, _lib.qpa_energy(ctx, ctypes.byref(problem), ctypes.byref(params), spins, energy,
                                energy_i64, best, workspace, workspace_bytes, stream))


def qpa_workspace_size_batch(ctx, problems, params) -> int:
    """problems: a ctypes array of qpa_problem."""
    nbytes = ctypes.c_size_t()
    _check(ctx, _lib.qpa_workspace_size_batch(ctx, len(problems), problems, ctypes.byref(params),
                                              ctypes.byref(nbytes)))
    return nbytes.value


def qpa_solve_batch(ctx, problems, params, workspace, workspace_bytes, stream, outputs):
    """problems / outputs: ctypes arrays of qpa_problem / qpa_outputs of equal length."""
    _check(ctx, _lib.qpa_solve_batch(ctx, len(problems), problems, ctypes.byref(params),
                                     workspace, workspace_bytes, stream, outputs))


def qpa_workspace_size_relaxed(ctx, problem, params, ckpt_every) -> int:
    nbytes = ctypes.c_size_t()
    _check(ctx, _lib.qpa_workspace_size_relaxed(ctx, ctypes.byref(problem), ctypes.byref(params),
                                                ckpt_every, ctypes.byref(nbytes)))
    return nbytes.value


def qpa_relaxed_grad(ctx, problem, params, ckpt_every, scale, workspace, workspace_bytes,
                     stream, loss, d_eta, d_alpha, d_lambda):
    _check(ctx, _lib.qpa_relaxed_grad(ctx, ctypes.byref(problem), ctypes.byref(params),
                                      ckpt_every, scale, workspace, workspace_bytes, stream,
                                      loss, d_eta, d_alpha, d_lambda))


def qpa_workspace_size_relaxed_batch(ctx, problems, params, ckpt_every) -> int:
    """problems: a ctypes array of qpa_problem."""
    nbytes = ctypes.c_size_t()
    _check(ctx, _lib.qpa_workspace_size_relaxed_batch(ctx, len(problems), problems,
                                                      ctypes.byref(params), ckpt_every,
                                                      ctypes.byref(nbytes)))
    return nbytes.value


def qpa_relaxed_grad_batch(ctx, problems, params, ckpt_every, scale, workspace,
                           workspace_bytes, stream, loss, d_eta, d_alpha, d_lambda):
    _check(ctx, _lib.qpa_relaxed_grad_batch(ctx, len(problems), problems, ctypes.byref(params),
                                            ckpt_every, scale, workspace, workspace_bytes,
                                            stream, loss, d_eta, d_alpha, d_lambda))


def qpa_profile_enable(ctx, enable: bool):
    _check(ctx, _lib.qpa_profile_enable(ctx, 1 if enable else 0))


def qpa_profile_read(ctx, reset: bool = True):
    """Returns (summed step-kernel milliseconds, step-kernel launches)."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(ctx, _lib.qpa_profile_read(ctx, ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
    return ms.value, n.value


def qpa_profile_read_path(ctx, path: int, reset: bool = False):
    """(milliseconds, launches) of the step kernels of one path (QPA_PATH_*)."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(ctx, _lib.qpa_profile_read_path(ctx, path, ctypes.byref(ms), ctypes.byref(n),
                                           1 if reset else 0))
    return ms.value, n.value


def qpa_batch_paths(ctx, count: int) -> np.ndarray:
    """Path (QPA_PATH_BATCH_SPARSE / _DENSE) of each instance of the last batch solve."""
    out = np.zeros(count, np.int32)
    _check(ctx, _lib.qpa_batch_paths(ctx, count, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return out


def qpa_workspace_size_sbm(ctx, problem, params) -> int:
    nbytes = ctypes.c_size_t()
    _check(ctx, _lib.qpa_workspace_size_sbm(ctx, ctypes.byref(problem), ctypes.byref(params),
                                            ctypes.byref(nbytes)))
    return nbytes.value


def qpa_sbm_solve(ctx, problem, params, workspace, workspace_bytes, stream, outputs):
    _check(ctx, _lib.qpa_sbm_solve(ctx, ctypes.byref(problem), ctypes.byref(params), workspace,
                                   workspace_bytes, stream, ctypes.byref(outputs)))


def qpa_sbm_steps(ctx, problem, params, t0, t1, q, p, g_last, workspace, workspace_bytes,
                  stream):
    _check(ctx, _lib.qpa_sbm_steps(ctx, ctypes.byref(problem), ctypes.byref(params), t0, t1, q,
                                   p, g_last, workspace, workspace_bytes, stream))


def qpa_spectral_radius(ctx, problem, params, workspace, workspace_bytes, stream, rho):
    _check(ctx, _lib.qpa_spectral_radius(ctx, ctypes.byref(problem), ctypes.byref(params),
                                         workspace, workspace_bytes, stream, rho))


def qpa_autotune(ctx, problem, params, probe_steps, workspace, workspace_bytes, stream):
    """Returns (choice, [ms of streamed, G=1, 2, 4, 8, binned], -1 where not applicable)."""
    choice = ctypes.c_int32()
    ms = (ctypes.c_double * 6)()
    _check(ctx, _lib.qpa_autotune(ctx, ctypes.byref(problem), ctypes.byref(params), probe_steps,
                                  workspace, workspace_bytes, stream, ctypes.byref(choice), ms))
    return choice.value, list(ms)


def qpa_autotune_batch(ctx, problems, params, probe_steps, stream):
    """Returns the batch path rates now in effect: (dense bytes/s, sparse adds/s)."""
    rates = (ctypes.c_double * 2)()
    _check(ctx, _lib.qpa_autotune_batch(ctx, len(problems), problems, ctypes.byref(params),
                                        probe_steps, stream, rates))
    return rates[0], rates[1]


def qpa_tune_set(ctx, problem, params, choice):
    _check(ctx, _lib.qpa_tune_set(ctx, ctypes.byref(problem), ctypes.byref(params), choice))


def qpa_workspace_size_spectrum(ctx, n, R) -> int:
    nbytes = ctypes.c_size_t()
    _check(ctx, _lib.qpa_workspace_size_spectrum(ctx, n, R, ctypes.byref(nbytes)))
    return nbytes.value


def qpa_spectrum(ctx, n, R, spins, energy, k, flags, workspace, workspace_bytes, stream,
                 out_spins, out_energy, out_count, out_first, out_distinct):
    _check(ctx, _lib.qpa_spectrum(ctx, n, R, spins, energy, k, flags, workspace,
                                  workspace_bytes, stream, out_spins, out_energy, out_count,
                                  out_first, out_distinct))


# ---- convenience layer (torch supplies memory and streams) ---------------------------
_DT = {"int8": QPA_I8, "int16": QPA_I16, "int32": QPA_I32, "float32": QPA_F32}


def _dt_code(t):
    name = str(t.dtype).replace("torch.", "")
    if name not in _DT:
        raise TypeError("unsupported dtype %s" % t.dtype)
    return _DT[name]


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class Problem:
    """One instance held in device tensors (kept referenced here while in use)."""
    kind: int
    n: int
    dense: object = None
    row_ptr: object = None
    col: object = None
    weights: object = None
    linear: object = None

    def struct(self) -> qpa_problem:
        p = qpa_problem()
        p.n = self.n
        p.kind = self.kind
        if self.dense is not None:
            p.format = QPA_FMT_DENSE
            p.coupling_dtype = _dt_code(self.dense)
            p.dense = self.dense.data_ptr()
        else:
            p.format = QPA_FMT_CSR
            p.coupling_dtype = _dt_code(self.weights)
            p.index_dtype = _dt_code(self.col)
            p.nnz = int(self.col.numel())
            p.row_ptr = self.row_ptr.data_ptr()
            p.col = self.col.data_ptr() if self.col.numel() else None
            p.weights = self.weights.data_ptr() if self.weights.numel() else None
        if self.linear is not None:
            p.linear_dtype = _dt_code(self.linear)
            p.linear = self.linear.data_ptr()
        return p

    @staticmethod
    def from_instance(inst, device="cuda"):
        """Upload a paper_2501_19221_amd.instances.Instance to device tensors."""
        import torch
        kind = QPA_KIND_QUBO if inst.kind == "qubo" else QPA_KIND_ISING
        lin = None if inst.lin is None else torch.from_numpy(
            np.ascontiguousarray(inst.lin)).to(device)
        if inst.dense is not None:
            return Problem(kind, inst.n, dense=torch.from_numpy(
                np.ascontiguousarray(inst.dense)).to(device), linear=lin)
        c = inst.csr
        return Problem(kind, inst.n,
                       row_ptr=torch.from_numpy(c.rp.astype(np.int32)).to(device),
                       col=torch.from_numpy(np.ascontiguousarray(c.col)).to(device),
                       weights=torch.from_numpy(np.ascontiguousarray(c.w)).to(device),
                       linear=lin)


def make_params(replicas, steps, eta, alpha, lambda0, sigma0=0.1, seed=1, precision=QPA_PREC_FP32,
                lambda_table=None, flags=0):
    p = qpa_params()
    p.replicas = replicas
    p.steps = steps
    p.eta = eta
    p.alpha = alpha
    p.lambda0 = lambda0
    p.sigma0 = sigma0
    p.seed = seed & (2**64 - 1)
    p.precision = precision
    p.flags = flags
    keep = None
    if lambda_table is not None:
        keep = np.ascontiguousarray(lambda_table, dtype=np.float32)
        assert keep.shape == (steps,)
        p.lambda_table = keep.ctypes.data
    p._keep = keep            # host table must outlive the call
    return p


def make_sbm_params(replicas, steps, dt, a0=1.0, c0=0.0, sigma0=0.1, seed=1, power_iters=100,
                    flags=0):
    p = qpa_sbm_params()
    p.replicas = replicas
    p.steps = steps
    p.a0 = a0
    p.c0 = c0
    p.dt = dt
    p.sigma0 = sigma0
    p.seed = seed & (2**64 - 1)
    p.power_iters = power_iters
    p.flags = flags
    return p


class Engine:
    """A context on one device plus a reusable torch workspace."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.device = device
        torch.cuda.init()                 # one HIP runtime per process: let torch set it up
        torch.cuda.set_device(device)
        self.ctx = qpa_create(device)
        self._ws = None

    def close(self):
        if self.ctx:
            qpa_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, problem: qpa_problem, params: qpa_params):
        nbytes = qpa_workspace_size(self.ctx, problem, params)
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = self.torch.empty(max(nbytes, 256), dtype=self.torch.uint8,
                                        device="cuda:%d" % self.device)
        return self._ws, nbytes

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def solve(self, prob: Problem, params: qpa_params, want_state=False, noalloc=False):
        """Returns dict(spins [R,n] int8, energy [R] f64, energy_i64 [R] or None,
        best int tensor [1], x, m) -- device tensors.  noalloc: run qpa_solve_noalloc
        (the library's static workspace) instead of qpa_solve with a torch workspace."""
        torch = self.torch
        dev = "cuda:%d" % self.device
        R, n = params.replicas, prob.n
        ps = prob.struct()
        if not noalloc:
            ws, nbytes = self.workspace(ps, params)
        out = {"spins": torch.empty((R, n), dtype=torch.int8, device=dev),
               "energy": torch.empty(R, dtype=torch.float64, device=dev),
               "best": torch.empty(1, dtype=torch.int32, device=dev),
               "energy_i64": torch.empty(R, dtype=torch.int64, device=dev),
               "x": torch.empty((R, n), dtype=torch.float32, device=dev) if want_state else None,
               "m": torch.empty((R, n), dtype=torch.float32, device=dev) if want_state else None}
        o = qpa_outputs()
        o.spins = out["spins"].data_ptr()
        o.energy = out["energy"].data_ptr()
        o.energy_i64 = out["energy_i64"].data_ptr()
        o.best = out["best"].data_ptr()
        o.x = out["x"].data_ptr() if want_state else None
        o.m = out["m"].data_ptr() if want_state else None
        if noalloc:
            qpa_solve_noalloc(self.ctx, ps, params, self._stream(), o)
        else:
            qpa_solve(self.ctx, ps, params, ctypes.c_void_p(ws.data_ptr()), nbytes,
                      self._stream(), o)
        return out

    def solve_track(self, prob: Problem, params: qpa_params, every: int, want_state=False):
        """qpa_solve_track: the solve() outputs plus each replica's best sampled state --
        best_energy [R] f64, best_step [R] int32, best_spins [R,n] int8 (device tensors)."""
        torch = self.torch
        dev = "cuda:%d" % self.device
        R, n = params.replicas, prob.n
        ps = prob.struct()
        ws, nbytes = self.workspace(ps, params)
        out = {"spins": torch.empty((R, n), dtype=torch.int8, device=dev),
               "energy": torch.empty(R, dtype=torch.float64, device=dev),
               "best": torch.empty(1, dtype=torch.int32, device=dev),
               "energy_i64": torch.empty(R, dtype=torch.int64, device=dev),
               "x": torch.empty((R, n), dtype=torch.float32, device=dev) if want_state else None,
               "m": torch.empty((R, n), dtype=torch.float32, device=dev) if want_state else None,
               "best_energy": torch.empty(R, dtype=torch.float64, device=dev),
               "best_step": torch.empty(R, dtype=torch.int32, device=dev),
               "best_spins": torch.empty((R, n), dtype=torch.int8, device=dev)}
        o = qpa_outputs()
        o.spins = out["spins"].data_ptr()
        o.energy = out["energy"].data_ptr()
        o.energy_i64 = out["energy_i64"].data_ptr()
        o.best = out["best"].data_ptr()
        o.x = out["x"].data_ptr() if want_state else None
        o.m = out["m"].data_ptr() if want_state else None
        tr = qpa_track_outputs()
        tr.best_energy = out["best_energy"].data_ptr()
        tr.best_step = out["best_step"].data_ptr()
        tr.best_spins = out["best_spins"].data_ptr()
        qpa_solve_track(self.ctx, ps, params, int(every), ctypes.c_void_p(ws.data_ptr()), nbytes,
                        self._stream(), o, tr)
        return out

    def solve_batch(self, probs, params: qpa_params, want_state=False):
        """Solve a list of CSR Problems in one launch; returns one output dict per problem."""
        torch = self.torch
        dev = "cuda:%d" % self.device
        R = params.replicas
        pa = (qpa_problem * len(probs))(*[p.struct() for p in probs])
        nbytes = qpa_workspace_size_batch(self.ctx, pa, params)
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
        outs = []
        oa = (qpa_outputs * len(probs))()
        for k, p in enumerate(probs):
            o = {"spins": torch.empty((R, p.n), dtype=torch.int8, device=dev),
                 "energy": torch.empty(R, dtype=torch.float64, device=dev),
                 "energy_i64": torch.empty(R, dtype=torch.int64, device=dev),
                 "best": torch.empty(1, dtype=torch.int32, device=dev),
                 "x": torch.empty((R, p.n), dtype=torch.float32, device=dev) if want_state else None,
                 "m": torch.empty((R, p.n), dtype=torch.float32, device=dev) if want_state else None}
            oa[k].spins = o["spins"].data_ptr()
            oa[k].energy = o["energy"].data_ptr()
            oa[k].energy_i64 = o["energy_i64"].data_ptr()
            oa[k].best = o["best"].data_ptr()
            oa[k].x = o["x"].data_ptr() if want_state else None
            oa[k].m = o["m"].data_ptr() if want_state else None
            outs.append(o)
        qpa_solve_batch(self.ctx, pa, params, ctypes.c_void_p(self._ws.data_ptr()), nbytes,
                        self._stream(), oa)
        return outs

    def relaxed_grad(self, prob, params: qpa_params, ckpt_every: int, scale=None,
                     grads=True):
        """Loss and gradients of the relaxed final energy (device float64 tensors):
        (loss [1], d_eta [1], d_alpha [1], d_lambda [T]).  `prob` is one Problem or a list
        of them (a batch sharing params; instance k starts from seed + k); the default
        scale is the mean over all replicas of all instances.  grads=False runs the
        forward pass only and returns (loss, None, None, None)."""
        torch = self.torch
        dev = "cuda:%d" % self.device
        probs = list(prob) if isinstance(prob, (list, tuple)) else [prob]
        pa = (qpa_problem * len(probs))(*[p.struct() for p in probs])
        nbytes = qpa_workspace_size_relaxed_batch(self.ctx, pa, params, ckpt_every)
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
        scale = 1.0 / (params.replicas * len(probs)) if scale is None else scale
        out = [torch.empty(1, dtype=torch.float64, device=dev) for _ in range(3)]
        dl = torch.empty(max(params.steps, 1), dtype=torch.float64, device=dev)
        qpa_relaxed_grad_batch(self.ctx, pa, params, ckpt_every, scale,
                               ctypes.c_void_p(self._ws.data_ptr()), nbytes, self._stream(),
                               _ptr(out[0]), _ptr(out[1]) if grads else None,
                               _ptr(out[2]) if grads else None, _ptr(dl) if grads else None)
        if not grads:
            return out[0], None, None, None
        return out[0], out[1], out[2], dl[:params.steps]

    def steps(self, prob: Problem, params: qpa_params, t0: int, t1: int, x, m, want_h=False):
        """Advance device tensors x, m ([R,n] float32, contiguous) in place; returns h or None."""
        torch = self.torch
        assert x.is_contiguous() and m.is_contiguous() and x.dtype == torch.float32
        ps = prob.struct()
        ws, nbytes = self.workspace(ps, params)
        h = torch.empty_like(x) if want_h else None
        qpa_steps(self.ctx, ps, params, t0, t1, _ptr(x), _ptr(m), _ptr(h),
                  ctypes.c_void_p(ws.data_ptr()), nbytes, self._stream())
        return h

    def _grow(self, nbytes):
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = self.torch.empty(max(nbytes, 256), dtype=self.torch.uint8,
                                        device="cuda:%d" % self.device)
        return self._ws

    def sbm_solve(self, prob: Problem, params: qpa_sbm_params, want_state=False):
        """SBM solve; returns the dict of solve() with x = q_T and m = p_T."""
        torch = self.torch
        dev = "cuda:%d" % self.device
        R, n = params.replicas, prob.n
        ps = prob.struct()
        nbytes = qpa_workspace_size_sbm(self.ctx, ps, params)
        ws = self._grow(nbytes)
        out = {"spins": torch.empty((R, n), dtype=torch.int8, device=dev),
               "energy": torch.empty(R, dtype=torch.float64, device=dev),
               "best": torch.empty(1, dtype=torch.int32, device=dev),
               "energy_i64": torch.empty(R, dtype=torch.int64, device=dev),
               "x": torch.empty((R, n), dtype=torch.float32, device=dev) if want_state else None,
               "m": torch.empty((R, n), dtype=torch.float32, device=dev) if want_state else None}
        o = qpa_outputs()
        o.spins = out["spins"].data_ptr()
        o.energy = out["energy"].data_ptr()
        o.energy_i64 = out["energy_i64"].data_ptr()
        o.best = out["best"].data_ptr()
        o.x = out["x"].data_ptr() if want_state else None
        o.m = out["m"].data_ptr() if want_state else None
        qpa_sbm_solve(self.ctx, ps, params, ctypes.c_void_p(ws.data_ptr()), nbytes,
                      self._stream(), o)
        return out

    def sbm_steps(self, prob: Problem, params: qpa_sbm_params, t0: int, t1: int, q, p,
                  want_g=False):
        """Advance device tensors q, p ([R,n] float32) in place; returns g or None."""
        torch = self.torch
        assert q.is_contiguous() and p.is_contiguous() and q.dtype == torch.float32
        ps = prob.struct()
        nbytes = qpa_workspace_size_sbm(self.ctx, ps, params)
        ws = self._grow(nbytes)
        g = torch.empty_like(q) if want_g else None
        qpa_sbm_steps(self.ctx, ps, params, t0, t1, _ptr(q), _ptr(p), _ptr(g),
                      ctypes.c_void_p(ws.data_ptr()), nbytes, self._stream())
        return g

    def spectral_radius(self, prob: Problem, params: qpa_sbm_params):
        """Power-method estimate of max |lambda(J)| (device float64 tensor [1])."""
        torch = self.torch
        ps = prob.struct()
        nbytes = qpa_workspace_size_sbm(self.ctx, ps, params)
        ws = self._grow(nbytes)
        rho = torch.empty(1, dtype=torch.float64, device="cuda:%d" % self.device)
        qpa_spectral_radius(self.ctx, ps, params, ctypes.c_void_p(ws.data_ptr()), nbytes,
                            self._stream(), _ptr(rho))
        return rho

    def autotune(self, prob: Problem, params: qpa_params, probe_steps=50):
        """Time the sparse kernel configurations and record the fastest on the context."""
        ps = prob.struct()
        ws, nbytes = self.workspace(ps, params)
        return qpa_autotune(self.ctx, ps, params, probe_steps, ctypes.c_void_p(ws.data_ptr()),
                            nbytes, self._stream())

    def tune_set(self, prob: Problem, params: qpa_params, choice):
        qpa_tune_set(self.ctx, prob.struct(), params, choice)

    def autotune_batch(self, probs, params: qpa_params, probe_steps=20):
        """Measure both batch paths for these instances; the context keeps the rates.
        Returns (dense bytes/s, sparse adds/s)."""
        pa = (qpa_problem * len(probs))(*[p.struct() for p in probs])
        return qpa_autotune_batch(self.ctx, pa, params, probe_steps, self._stream())

    def spectrum(self, spins, energy, k, flags=0):
        """Low-energy spectrum of device samples spins [R,n] int8 / energy [R] float64:
        dict(spins [m,n], energy [m], count [m], first [m], distinct), m = min(k, distinct)."""
        torch = self.torch
        R, n = spins.shape
        dev = spins.device
        assert spins.dtype == torch.int8 and energy.dtype == torch.float64
        spins, energy = spins.contiguous(), energy.contiguous()
        nbytes = qpa_workspace_size_spectrum(self.ctx, n, R)
        ws = self._grow(nbytes)
        kk = max(1, min(k, R))
        out = {"spins": torch.empty((kk, n), dtype=torch.int8, device=dev),
               "energy": torch.empty(kk, dtype=torch.float64, device=dev),
               "count": torch.empty(kk, dtype=torch.int32, device=dev),
               "first": torch.empty(kk, dtype=torch.int32, device=dev)}
        nd = torch.empty(1, dtype=torch.int32, device=dev)
        qpa_spectrum(self.ctx, n, R, _ptr(spins), _ptr(energy), k, flags,
                     ctypes.c_void_p(ws.data_ptr()), nbytes, self._stream(),
                     _ptr(out["spins"]), _ptr(out["energy"]), _ptr(out["count"]),
                     _ptr(out["first"]), _ptr(nd))
        m = min(k, int(nd.cpu()[0]))
        res = {key: v[:m] for key, v in out.items()}
        res["distinct"] = int(nd.cpu()[0])
        return res

    def energy(self, prob: Problem, params: qpa_params, spins):
        torch = self.torch
        R = spins.shape[0]
        dev = spins.device
        ps = prob.struct()
        ws, nbytes = self.workspace(ps, params)
        e = torch.empty(R, dtype=torch.float64, device=dev)
        ei = torch.empty(R, dtype=torch.int64, device=dev)
        best = torch.empty(1, dtype=torch.int32, device=dev)
        qpa_energy(self.ctx, ps, params, _ptr(spins), _ptr(e), _ptr(ei), _ptr(best),
                   ctypes.c_void_p(ws.data_ptr()), nbytes, self._stream())
        return e, ei, best


class RelaxedEnergy:
    """Mean relaxed final energy as a differentiable function of (eta, alpha, lambda_t).

    ``RelaxedEnergy.apply(eta, alpha, lam, engine, problem, replicas, sigma0, seed,
    ckpt_every)`` with 0-d float64 tensors eta, alpha and a 1-d float64 tensor lam of
    length T returns the loss -- the mean over the replicas (and over the instances when
    `problem` is a list of Problems, instance k starting from seed + k).  Its backward is
    the library's hand-written adjoint (qpa_relaxed_grad_batch), so gradients flow into
    whatever produced eta, alpha and lam (e.g. lam = lambda0 * (1 - t/T)); when no input
    needs a gradient only the forward pass runs."""

    @staticmethod
    def _fn():
        import torch

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, eta, alpha, lam, engine, problem, replicas, sigma0, seed, ckpt):
                T = int(lam.numel())
                table = lam.detach().cpu().numpy().astype(np.float32)
                p = make_params(replicas, T, float(eta), float(alpha), 0.0, sigma0, seed,
                                QPA_PREC_FP32, lambda_table=table)
                grads = any(ctx.needs_input_grad[:3])
                loss, de, da, dl = engine.relaxed_grad(problem, p, ckpt, grads=grads)
                if grads:
                    ctx.save_for_backward(de.to(eta.device), da.to(alpha.device),
                                          dl.to(lam.device))
                return loss[0].to(eta.device)

            @staticmethod
            def backward(ctx, g):
                de, da, dl = ctx.saved_tensors
                return (g * de[0], g * da[0], g * dl, None, None, None, None, None, None)

        return _F

    @classmethod
    def apply(cls, *args):
        return cls._fn().apply(*args)
