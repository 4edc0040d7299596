"""The C ABI on the CPU: the library loads, exports every declared symbol,
and validates arguments before touching the GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bsm.h")


def _lib_path():
    from paper_1401_3733_amd import bsm
    if not os.path.exists(bsm.LIB_PATH):
        from paper_1401_3733_amd import build
        build.build()
    return bsm.LIB_PATH


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bsm_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    path = _lib_path()
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (bsm_[a-z0-9_]+)\b", out))
    declared = declared_functions()
    assert declared, "no declarations found"
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    L = C.CDLL(path)
    for f in declared:
        getattr(L, f)


def test_binding_covers_the_header():
    from paper_1401_3733_amd import bsm
    assert set(declared_functions()) == set(bsm.exported_symbols())


def test_argument_validation_without_gpu():
    from paper_1401_3733_amd import bsm
    _lib_path()
    L = bsm.lib()
    assert L.bsm_rep_dim(4, 1) == 15 and L.bsm_rep_dim(5, 2) == 15 and L.bsm_rep_dim(6, 3) == 15
    assert L.bsm_rep_dim(3, 9) == -1
    h = C.c_void_p()
    lat = bsm.Lattice((C.c_int32 * 4)(4, 3, 4, 4), (C.c_int32 * 4)(-1, 1, 1, 1))
    assert L.bsm_ctx_create(C.byref(lat), C.byref(h)) == bsm.ERR_ARG
    assert b"even" in L.bsm_last_error()
    lat = bsm.Lattice((C.c_int32 * 4)(4, 4, 4, 4), (C.c_int32 * 4)(-1, 2, 1, 1))
    assert L.bsm_ctx_create(C.byref(lat), C.byref(h)) == bsm.ERR_ARG
    d = bsm.FieldDesc(3, 0, 3, 0, 0)
    assert L.bsm_dslash_apply(None, C.byref(d), None, 0.1, 0, None, None, None) == bsm.ERR_ARG
    assert L.bsm_gauge_bytes(None, C.byref(d)) == 0


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; --gpus N > 1 exits with status 2 and a
    message, before touching a device"""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
