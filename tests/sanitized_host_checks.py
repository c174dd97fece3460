"""Host-side paths of libqpa run under AddressSanitizer and UndefinedBehaviorSanitizer.

Run by tests/test_abi.py in a subprocess with the sanitizer runtime preloaded, against the
copy built by `python -m paper_2501_19221_amd.build --sanitize`:

    python tests/sanitized_host_checks.py <path of libqpa_san.so>

No GPU is used: every call below is argument validation, workspace planning (single,
batch, relaxed, SBM, spectrum), status strings and the failure of qpa_create without a
device.  A sanitizer finding aborts the process; a wrong status fails an assertion."""
import ctypes
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2501_19221_amd import abi  # noqa: E402  (ctypes declarations only, no torch)

lib = abi.load(sys.argv[1])
FAKE = 0x1000          # never dereferenced by host-side checks


def dense(n, dt=abi.QPA_I32, kind=abi.QPA_KIND_QUBO):
    p = abi.qpa_problem()
    p.n, p.kind, p.format, p.coupling_dtype, p.dense = n, kind, abi.QPA_FMT_DENSE, dt, FAKE
    return p


def csr(n, nnz, wdt=abi.QPA_I16, idt=abi.QPA_I16, kind=abi.QPA_KIND_QUBO):
    p = abi.qpa_problem()
    p.n, p.kind, p.format, p.coupling_dtype, p.index_dtype = n, kind, abi.QPA_FMT_CSR, wdt, idt
    p.nnz, p.row_ptr, p.col, p.weights = nnz, FAKE, FAKE, FAKE
    p.linear_dtype, p.linear = abi.QPA_I16, FAKE
    return p


def params(R, T, prec=abi.QPA_PREC_FP32, flags=0):
    a = abi.qpa_params()
    a.replicas, a.steps, a.eta, a.alpha, a.lambda0, a.sigma0 = R, T, 0.1, 0.8, 4.0, 0.1
    a.seed, a.precision, a.flags = 1, prec, flags
    return a


def ws(p, a):
    n = ctypes.c_size_t()
    return lib.qpa_workspace_size(None, ctypes.byref(p), ctypes.byref(a), ctypes.byref(n)), n.value


def arr(ps):
    return (abi.qpa_problem * len(ps))(*ps)


n = ctypes.c_size_t()
# single-instance planning on every path
for p, a in [(dense(20), params(256, 2000)), (dense(300), params(70, 10)),
             (dense(4096, abi.QPA_F32), params(1024, 10, abi.QPA_PREC_BF16)),
             (csr(2048, 12032, abi.QPA_I8, abi.QPA_I32, abi.QPA_KIND_ISING), params(1024, 10)),
             (csr(3_000_000, 9_000_000, abi.QPA_I8, abi.QPA_I32, abi.QPA_KIND_ISING),
              params(4, 10, flags=abi.QPA_SOLVE_BINNED)),
             (csr(1000, 0), params(3, 0))]:
    st, size = ws(p, a)
    assert st == abi.QPA_OK and size > 0, (st, size)
# invalid arguments
bad = dense(10)
bad.n = 0
assert ws(bad, params(4, 10))[0] == abi.QPA_E_SHAPE
bad = dense(10)
bad.kind = 7
assert ws(bad, params(4, 10))[0] == abi.QPA_E_ARG
assert ws(dense(10), params(0, 10))[0] == abi.QPA_E_ARG
assert ws(dense(10), params(4, -1))[0] == abi.QPA_E_ARG
assert ws(dense(10), params(4, 10, flags=3))[0] == abi.QPA_E_ARG
assert ws(csr(40000, 10), params(4, 10))[0] == abi.QPA_E_SHAPE
assert ws(csr(100, -1), params(4, 10))[0] == abi.QPA_E_SHAPE
assert lib.qpa_workspace_size(None, None, None, ctypes.byref(n)) == abi.QPA_E_ARG
assert len(lib.qpa_last_error(None)) > 0
# batches, with and without the graph flag, and an instance over the size limit
probs = [csr(1000, 100_000), csr(1000, 2_000), csr(150, 2_000)]
for fl in (0, abi.QPA_BATCH_SPARSE, abi.QPA_BATCH_DENSE,
           abi.QPA_BATCH_DENSE | abi.QPA_SOLVE_GRAPH):
    assert lib.qpa_workspace_size_batch(None, 3, arr(probs), ctypes.byref(params(64, 10, flags=fl)),
                                        ctypes.byref(n)) == abi.QPA_OK and n.value > 0
assert lib.qpa_workspace_size_batch(None, 1, arr([csr(5000, 10, idt=abi.QPA_I32)]),
                                    ctypes.byref(params(64, 10)),
                                    ctypes.byref(n)) == abi.QPA_E_UNSUPPORTED
assert lib.qpa_workspace_size_batch(None, 0, arr(probs), ctypes.byref(params(64, 10)),
                                    ctypes.byref(n)) == abi.QPA_E_ARG
# relaxed gradient of a mixed batch, checkpoint intervals
mixed = [csr(900, 80_000), dense(300, abi.QPA_F32, abi.QPA_KIND_ISING), csr(100, 900)]
for k in (1, 7, 50, 600):
    assert lib.qpa_workspace_size_relaxed_batch(None, 3, arr(mixed), ctypes.byref(params(20, 500)),
                                                k, ctypes.byref(n)) == abi.QPA_OK
assert lib.qpa_workspace_size_relaxed_batch(None, 3, arr(mixed), ctypes.byref(params(20, 500)),
                                            0, ctypes.byref(n)) == abi.QPA_E_ARG
assert lib.qpa_workspace_size_relaxed(None, ctypes.byref(dense(64, abi.QPA_F32)),
                                      ctypes.byref(params(8, 0)), 1,
                                      ctypes.byref(n)) == abi.QPA_OK
# SBM and spectrum planning
sp = abi.qpa_sbm_params()
sp.replicas, sp.steps, sp.a0, sp.c0, sp.dt, sp.sigma0, sp.power_iters = 64, 100, 1.0, 0.0, 0.5, 0.1, 10
assert lib.qpa_workspace_size_sbm(None, ctypes.byref(dense(200, abi.QPA_F32, abi.QPA_KIND_ISING)),
                                  ctypes.byref(sp), ctypes.byref(n)) == abi.QPA_OK
sp.dt = -1.0
assert lib.qpa_workspace_size_sbm(None, ctypes.byref(dense(200, abi.QPA_F32, abi.QPA_KIND_ISING)),
                                  ctypes.byref(sp), ctypes.byref(n)) == abi.QPA_E_ARG
assert lib.qpa_workspace_size_spectrum(None, 1000, 1024, ctypes.byref(n)) == abi.QPA_OK
assert lib.qpa_workspace_size_spectrum(None, 1000, 5000, ctypes.byref(n)) != abi.QPA_OK
# contexts: no device here, and every call refuses a NULL context
h = ctypes.c_void_p()
assert lib.qpa_create(ctypes.byref(h), 0) == abi.QPA_E_DEVICE
o = abi.qpa_outputs()
assert lib.qpa_solve(None, ctypes.byref(dense(10)), ctypes.byref(params(4, 10)), None, 0, None,
                     ctypes.byref(o)) == abi.QPA_E_ARG
assert lib.qpa_solve_noalloc(None, ctypes.byref(dense(10)), ctypes.byref(params(4, 10)), None,
                             ctypes.byref(o)) == abi.QPA_E_ARG
lib.qpa_destroy(None)
for s in range(9):
    assert lib.qpa_status_string(s)
assert lib.qpa_version().startswith(b"qpa")
print("sanitized host checks ok", flush=True)
