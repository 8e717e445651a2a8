"""The C-ABI library builds, loads and exports every entry point declared in
include/stablel1.h (no compute call: these run without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stablel1.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sl1_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1812_06635_amd import _lib
    return _lib.load()


def test_header_declares_the_expected_entry_points():
    names = _declared()
    for n in ["sl1_dict_dense", "sl1_dict_kron", "sl1_dict_free", "sl1_solve", "sl1_lambda_max", "sl1_grad",
              "sl1_measure_rc", "sl1_status_str", "sl1_version", "sl1_opts_default"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1812_06635_amd.build import lib_path
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path()], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    for n in _declared():
        assert n in exported, n
        assert hasattr(lib, n)
    # nothing but the C ABI is exported
    assert all(e.startswith("sl1_") for e in exported)


def test_binding_covers_every_declared_symbol():
    from paper_1812_06635_amd import _lib
    bound = {s[0] for s in _lib.SIGNATURES}
    assert bound == set(_declared())


def test_host_only_calls(lib):
    from paper_1812_06635_amd import _lib
    assert lib.sl1_version().decode().startswith("stablel1")
    assert lib.sl1_status_str(0).decode() == "ok"
    assert "singular" in lib.sl1_status_str(-6).decode()
    o = _lib.Opts()
    assert ctypes.sizeof(o) == 72          # the library checks sizeof(sl1_opts) == 72 at build time
    assert lib.sl1_opts_default(ctypes.byref(o)) == 0
    assert (o.Gamma, o.tol, o.max_iter, o.chunk, o.y_dtype) == (0.5, 1e-6, 100000, 16, _lib.F32)
    assert (o.screen_every, o.gemm_signals, o.x0) == (1, 64, None)
    assert lib.sl1_opts_default(None) == _lib.EINVAL
    assert lib.sl1_dict_free(None) == 0


def test_argument_validation_without_device(lib):
    from paper_1812_06635_amd import _lib
    h = _lib.c_dict()
    # NULL pointers and bad sizes are refused on the host before any HIP call
    assert lib.sl1_dict_dense(ctypes.byref(h), _lib.F32, 256, 1024, None, None, None, 2.0, None) == _lib.EINVAL
    assert lib.sl1_dict_kron(ctypes.byref(h), _lib.F32, 0, 16, 16, 16, 16, None, None, None, 2.0, None) == _lib.EINVAL
    assert lib.sl1_dict_kron(ctypes.byref(h), 7, 1, 16, 16, 16, 16, 1, 1, 1, 2.0, None) == _lib.EDTYPE
    assert lib.sl1_dict_kron(ctypes.byref(h), _lib.F32, 1, 15, 16, 16, 16, 1, 1, 1, 2.0, None) == _lib.ELIMIT
    assert lib.sl1_dict_dense(ctypes.byref(h), _lib.F32, 258, 16, 1, None, 1, 2.0, None) == _lib.ELIMIT
    assert lib.sl1_dict_dense(ctypes.byref(h), 9, 256, 16, 1, None, 1, 2.0, None) == _lib.EDTYPE
    # the norm q of the error bounds: 1 <= q <= inf, NaN refused (checked before the limits)
    inf, nan = float("inf"), float("nan")
    for q in (0.5, 0.0, -2.0, nan):
        assert lib.sl1_dict_dense(ctypes.byref(h), _lib.F32, 256, 16, 1, None, 1, q, None) == _lib.EINVAL
        assert lib.sl1_dict_kron(ctypes.byref(h), _lib.F32, 1, 16, 16, 16, 16, 1, 1, 1, q, None) == _lib.EINVAL
    for q in (1.0, 1.5, 3.0, inf):
        assert lib.sl1_dict_dense(ctypes.byref(h), _lib.F32, 258, 16, 1, None, 1, q, None) == _lib.ELIMIT
        assert lib.sl1_dict_kron(ctypes.byref(h), _lib.F32, 1, 15, 16, 16, 16, 1, 1, 1, q, None) == _lib.ELIMIT
    # FAuST: sizes, dtype and the CSR arrays are checked on the host
    import numpy as np
    dims = (_lib.c_i64 * 3)(8, 4, 5)
    nnz = (_lib.c_i64 * 2)(2, 2)
    rp = np.array([0, 1, 2, 2, 2, 2, 2, 2, 2, 0, 1, 1, 2, 2], dtype=np.int32)
    ci = np.array([0, 3, 1, 4], dtype=np.int32)
    va = np.ones(4, dtype=np.float32)
    fa = lambda dt, J, d, r, c: lib.sl1_dict_faust(ctypes.byref(h), dt, J, d, nnz, r.ctypes.data, c.ctypes.data,
                                                   va.ctypes.data, 1, 2.0, None)
    assert lib.sl1_dict_faust(ctypes.byref(h), _lib.F32, 0, dims, nnz, None, None, None, None, 2.0,
                              None) == _lib.EINVAL
    assert lib.sl1_dict_faust(ctypes.byref(h), _lib.F32, 2, dims, nnz, rp.ctypes.data, ci.ctypes.data,
                              va.ctypes.data, 1, 0.9, None) == _lib.EINVAL
    assert fa(_lib.BF16, 2, dims, rp, ci) == _lib.EDTYPE
    assert fa(_lib.F32, 9, dims, rp, ci) == _lib.ELIMIT
    assert fa(_lib.F32, 2, (_lib.c_i64 * 3)(6, 4, 5), rp, ci) == _lib.ELIMIT        # N not a multiple of 4
    assert fa(_lib.F32, 2, (_lib.c_i64 * 3)(8, 2000, 5), rp, ci) == _lib.ELIMIT     # inner size above 1024
    bad = ci.copy(); bad[1] = 4                                                    # column out of range
    assert fa(_lib.F32, 2, dims, rp, bad) == _lib.EINVAL
    bad = rp.copy(); bad[8] = 1                                                    # rows do not end at nnz
    assert fa(_lib.F32, 2, dims, bad, ci) == _lib.EINVAL
    assert lib.sl1_solve(None, 1, None, None, None, 1, None, None, None, None, None, None, None, None, None,
                         None) == _lib.EINVAL
    assert lib.sl1_lambda_max(None, 1, None, 1, None, None) == _lib.EINVAL
    assert lib.sl1_grad(None, 1, None, None, None, None, None, None, 1, None) == _lib.EINVAL


def test_bench_refuses_more_than_one_gpu():
    # the benchmark measures one GPU; asked for more it says so and exits with status 2
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
