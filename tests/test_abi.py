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


def _lat(T, LX, LY, LZ):
    from paper_1401_3733_amd import bsm
    return bsm.Lattice((C.c_int32 * 4)(T, LX, LY, LZ), (C.c_int32 * 4)(-1, 1, 1, 1))


@pytest.mark.parametrize("dims,N,rep,prec,expect", [
    # FP64 colour split (four threads per site, 64 sites per workgroup) at d_R = 15
    ((96, 48, 48, 48), 4, 1, 0, 2 * (48 ** 3 * 96 // 2) // 64),
    # one thread per site, 256 sites per workgroup
    ((128, 64, 64, 64), 3, 0, 0, 2 * (64 ** 3 * 128 // 2) // 256),
    ((128, 64, 64, 64), 3, 0, 1, 2 * (64 ** 3 * 128 // 2) // 256),
    ((64, 32, 32, 32), 3, 0, 1, 2 * (32 ** 3 * 64 // 2) // 256),
])
def test_fused_norm_hops_fit_the_context_reduction_slots(dims, N, rep, prec, expect):
    """Every fused-norm hop writes one FP64 partial per workgroup; the context
    must hold that many for the largest lattices a GPU holds (a fixed 65 536
    slots did not: 165 888 are needed for SU(4) adjoint FP64 on 48^3 x 96,
    131 072 for SU(3) on 64^3 x 128)."""
    from paper_1401_3733_amd import bsm
    _lib_path()
    L = bsm.lib()
    lat = _lat(*dims)
    d = bsm.FieldDesc(N, rep, L.bsm_rep_dim(N, rep), prec, prec)
    need = L.bsm_hop_norm_slots(C.byref(lat), C.byref(d))
    have = L.bsm_reduction_slots(C.byref(lat))
    assert need == expect
    assert need <= have
    # every representation and precision on this lattice fits too
    for n, r in ((2, 0), (3, 0), (3, 1), (3, 2), (4, 1), (5, 2), (6, 3), (15, 0)):
        for p in (0, 1, 2):
            dd = bsm.FieldDesc(n, r, L.bsm_rep_dim(n, r), p, min(p, 1) if p == 2 else p)
            assert 0 < L.bsm_hop_norm_slots(C.byref(lat), C.byref(dd)) <= have


def test_slot_queries_reject_bad_arguments():
    from paper_1401_3733_amd import bsm
    _lib_path()
    L = bsm.lib()
    assert L.bsm_reduction_slots(C.byref(_lat(4, 3, 4, 4))) == -1
    assert L.bsm_reduction_slots(None) == -1
    assert L.bsm_reduction_slots(C.byref(_lat(4, 4, 4, 4))) == 1 << 16
    bad = bsm.FieldDesc(3, 0, 4, 0, 0)
    assert L.bsm_hop_norm_slots(C.byref(_lat(4, 4, 4, 4)), C.byref(bad)) == -1
