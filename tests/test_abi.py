"""Host-side checks of the C ABI library (no GPU needed): it loads, exports every symbol
include/qpa.h declares, and its argument validation and workspace planning behave as
documented.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qpa.h")


@pytest.fixture(scope="module")
def q():
    from paper_2501_19221_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_2501_19221_amd import qpa
    return qpa


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qpa_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ["qpa_create", "qpa_solve", "qpa_steps", "qpa_energy", "qpa_workspace_size"]:
        assert must in names


def test_library_exports_every_declared_symbol(q):
    lib = ctypes.CDLL(q.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(q.EXPORTED)


def test_status_strings(q):
    assert q.qpa_status_string(q.QPA_OK) == "QPA_OK"
    assert q.qpa_status_string(q.QPA_E_ASYM) == "QPA_E_ASYM"
    assert q.qpa_version().startswith("qpa")


def _dense_problem(q, n=10, dt=None):
    p = q.qpa_problem()
    p.n = n
    p.kind = q.QPA_KIND_QUBO
    p.format = q.QPA_FMT_DENSE
    p.coupling_dtype = q.QPA_I32 if dt is None else dt
    p.dense = 0x1000          # never dereferenced by the host-side checks
    return p


def _ws(q, p, a):
    n = ctypes.c_size_t()
    st = q._lib.qpa_workspace_size(None, ctypes.byref(p), ctypes.byref(a), ctypes.byref(n))
    return st, n.value


def test_workspace_size_paths(q):
    a = q.make_params(256, 2000, 0.002, 0.9, 30.0)
    st, small = _ws(q, _dense_problem(q, 20), a)
    assert st == q.QPA_OK and small > 0
    st, tiled = _ws(q, _dense_problem(q, 300), a)
    assert st == q.QPA_OK and tiled > 300 * 300 * 4
    a16 = q.make_params(1024, 10, 0.1, 0.8, 4.0, precision=q.QPA_PREC_BF16)
    st, mf = _ws(q, _dense_problem(q, 4096, q.QPA_F32), a16)
    assert st == q.QPA_OK and mf >= 4096 * 4096 * 2 + 3 * 1024 * 4096 * 4


def test_argument_validation(q):
    a = q.make_params(4, 10, 0.1, 0.5, 1.0)
    p = _dense_problem(q)
    p.n = 0
    assert _ws(q, p, a)[0] == q.QPA_E_SHAPE
    p = _dense_problem(q)
    p.dense = None
    assert _ws(q, p, a)[0] == q.QPA_E_ARG
    p = _dense_problem(q)
    p.kind = 7
    assert _ws(q, p, a)[0] == q.QPA_E_ARG
    bad = q.make_params(0, 10, 0.1, 0.5, 1.0)
    assert _ws(q, _dense_problem(q), bad)[0] == q.QPA_E_ARG
    bad = q.make_params(4, -1, 0.1, 0.5, 1.0)
    assert _ws(q, _dense_problem(q), bad)[0] == q.QPA_E_ARG
    bad = q.make_params(4, 10, 0.1, 0.5, 1.0)
    bad.flags = 3
    assert _ws(q, _dense_problem(q), bad)[0] == q.QPA_E_ARG
    c = q.qpa_problem()
    c.n = 40000
    c.format = q.QPA_FMT_CSR
    c.kind = q.QPA_KIND_ISING
    c.coupling_dtype = q.QPA_I8
    c.index_dtype = q.QPA_I16
    c.row_ptr = 0x1000
    c.col = 0x1000
    c.weights = 0x1000
    c.nnz = 10
    assert _ws(q, c, a)[0] == q.QPA_E_SHAPE       # int16 indices cannot address 40000 rows
    c.index_dtype = q.QPA_I32
    assert _ws(q, c, a)[0] == q.QPA_OK
    c.nnz = -1
    assert _ws(q, c, a)[0] == q.QPA_E_SHAPE


def _csr_problem(q, n, nnz, wdt):
    c = q.qpa_problem()
    c.n = n
    c.format = q.QPA_FMT_CSR
    c.kind = q.QPA_KIND_ISING
    c.coupling_dtype = wdt
    c.index_dtype = q.QPA_I32
    c.row_ptr = 0x1000
    c.col = 0x1000
    c.weights = 0x1000
    c.nnz = nnz
    return c


def test_binned_workspace_and_flags(q):
    """Integer CSR problems with at most 8 replicas carry the binned entry arrays (block
    offsets, 9 bytes per entry); other problems do not; flag mixes are refused."""
    n, nnz = 3_000_000, 9_000_000
    ws = {}
    for R in (4, 9):
        for wdt in (q.QPA_I8, q.QPA_F32):
            st, ws[R, wdt] = _ws(q, _csr_problem(q, n, nnz, wdt), q.make_params(R, 10, 0.1, 0.8, 4.0))
            assert st == q.QPA_OK
    # G = 4: chunks of 2^18 variables, bins of 2^12 rows
    blocks = ((n + 2**18 - 1) // 2**18) * ((n + 2**12 - 1) // 2**12)
    assert ws[4, q.QPA_I8] - ws[4, q.QPA_F32] >= 9 * nnz + 8 * blocks
    assert ws[9, q.QPA_I8] - ws[9, q.QPA_F32] < 9 * nnz
    both = q.make_params(4, 10, 0.1, 0.8, 4.0, flags=q.QPA_SOLVE_BINNED | q.QPA_SOLVE_STREAMED)
    assert _ws(q, _csr_problem(q, n, nnz, q.QPA_I8), both)[0] == q.QPA_E_ARG
    one = q.make_params(4, 10, 0.1, 0.8, 4.0, flags=q.QPA_SOLVE_BINNED | q.QPA_SOLVE_GRAPH)
    assert _ws(q, _csr_problem(q, n, nnz, q.QPA_I8), one)[0] == q.QPA_OK


def test_solve_rejects_null_context_and_bad_workspace(q):
    a = q.make_params(4, 10, 0.1, 0.5, 1.0)
    p = _dense_problem(q)
    o = q.qpa_outputs()
    st = q._lib.qpa_solve(None, ctypes.byref(p), ctypes.byref(a), None, 0, None, ctypes.byref(o))
    assert st == q.QPA_E_ARG
    st = q._lib.qpa_solve_noalloc(None, ctypes.byref(p), ctypes.byref(a), None, ctypes.byref(o))
    assert st == q.QPA_E_ARG


def test_create_without_device_fails_cleanly(q):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert q._lib.qpa_create(ctypes.byref(h), 0) == q.QPA_E_DEVICE


def _fake_csr(q, n, nnz):
    c = q.qpa_problem()
    c.n = n
    c.format = q.QPA_FMT_CSR
    c.kind = q.QPA_KIND_QUBO
    c.coupling_dtype = q.QPA_I16
    c.index_dtype = q.QPA_I16
    c.linear_dtype = q.QPA_I16
    c.row_ptr = 0x1000
    c.col = 0x1000
    c.weights = 0x1000
    c.nnz = nnz
    return c


def _ws_batch(q, probs, a):
    arr = (q.qpa_problem * len(probs))(*probs)
    n = ctypes.c_size_t(0)
    st = q._lib.qpa_workspace_size_batch(None, len(probs), arr, ctypes.byref(a), ctypes.byref(n))
    return st, n.value


def test_batch_path_flags(q):
    # a dense-friendly instance (n=1000, 10% of pairs) and a very sparse one
    probs = [_fake_csr(q, 1000, 100_000), _fake_csr(q, 1000, 200)]
    sizes = {}
    for name, fl in [("auto", 0), ("sparse", q.QPA_BATCH_SPARSE), ("dense", q.QPA_BATCH_DENSE)]:
        a = q.make_params(64, 10, 0.1, 0.8, 4.0, flags=fl)
        st, sizes[name] = _ws_batch(q, probs, a)
        assert st == q.QPA_OK, name
    # the dense path adds a 1024x1024 BF16 matrix per densified instance
    bf16 = 1024 * 1024 * 2
    assert sizes["dense"] >= sizes["sparse"] + 2 * bf16
    assert sizes["sparse"] + bf16 <= sizes["auto"] < sizes["sparse"] + 2 * bf16
    bad = q.make_params(64, 10, 0.1, 0.8, 4.0, flags=3)
    assert _ws_batch(q, probs, bad)[0] == q.QPA_E_ARG
    # single-instance solves take no flags
    one = q.make_params(4, 10, 0.1, 0.5, 1.0, flags=q.QPA_BATCH_SPARSE)
    assert _ws(q, _dense_problem(q), one)[0] == q.QPA_E_ARG


def _ws_sbm(q, p, s):
    n = ctypes.c_size_t()
    st = q._lib.qpa_workspace_size_sbm(None, ctypes.byref(p), ctypes.byref(s), ctypes.byref(n))
    return st, n.value


def test_sbm_workspace_and_validation(q):
    s = q.make_sbm_params(1024, 1000, 0.5)
    st, dense = _ws_sbm(q, _dense_problem(q, 4096, q.QPA_F32), s)
    # canonical FP32 couplings + q0, q1, p, g of [n][1024]
    assert st == q.QPA_OK and dense >= 4096 * 4096 * 4 + 4 * 1024 * 4096 * 4
    s3 = q.make_sbm_params(3, 10, 0.5)
    st, small = _ws_sbm(q, _dense_problem(q, 100), s3)
    assert st == q.QPA_OK and small >= 4 * 128 * 100 * 4       # replicas padded to the tile
    for kw in ({"a0": 0.0}, {"a0": float("nan")}, {"c0": -0.5}, {"flags": 2},
               {"power_iters": -3}):
        args = dict(a0=1.0, c0=0.0, flags=0, power_iters=10)
        args.update(kw)
        bad = q.make_sbm_params(4, 10, 0.5, **args)
        assert _ws_sbm(q, _dense_problem(q), bad)[0] == q.QPA_E_ARG
    assert _ws_sbm(q, _dense_problem(q), q.make_sbm_params(4, 10, 0.0))[0] == q.QPA_E_ARG
    assert _ws_sbm(q, _dense_problem(q), q.make_sbm_params(0, 10, 0.5))[0] == q.QPA_E_ARG
    assert _ws_sbm(q, _dense_problem(q), q.make_sbm_params(4, -1, 0.5))[0] == q.QPA_E_ARG


def test_spectrum_workspace_and_limits(q):
    n = ctypes.c_size_t()
    assert q._lib.qpa_workspace_size_spectrum(None, 130, 1024, ctypes.byref(n)) == q.QPA_OK
    assert n.value >= 1024 * 3 * 8 + 1024 * 8
    assert q._lib.qpa_workspace_size_spectrum(None, 10, q.QPA_SPECTRUM_MAX_R + 1,
                                              ctypes.byref(n)) == q.QPA_E_UNSUPPORTED
    assert q._lib.qpa_workspace_size_spectrum(None, 0, 10, ctypes.byref(n)) == q.QPA_E_SHAPE
    assert q._lib.qpa_workspace_size_spectrum(None, 10, 0, ctypes.byref(n)) == q.QPA_E_ARG


def test_host_code_under_sanitizers():
    """The library's host code built with AddressSanitizer and UndefinedBehaviorSanitizer
    (device code unchanged) runs tests/sanitized_host_checks.py -- validation and planning
    of every entry point -- without a finding."""
    import subprocess
    import sys
    from paper_2501_19221_amd import build
    lib = build.build(sanitize=True)
    rt = build.sanitizer_runtime()
    assert os.path.exists(rt), rt
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitized_host_checks.py"),
                        lib], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "sanitized host checks ok" in r.stdout
