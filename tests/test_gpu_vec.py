"""Krylov vector operations (bsm_vec_axpby, bsm_vec_dot) against numpy on the
unpacked fields."""
import numpy as np
import pytest

from oracle import quant
from paper_1401_3733_amd import bsm
from paper_1401_3733_amd import inputs as gen
from tests.gpu_util import Setup, note, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("d", [2, 3, 6])
def test_axpby_and_dot(prec, d):
    note(f"vec ops {prec} d={d}")
    N = {2: 2, 3: 3, 6: 6}[d]
    lat = gen.Lattice(8, 6, 4, 6)
    S = Setup(lat, N, "fund", gen.gauge_links(lat, N, "haar", 1), prec=prec)
    x = gen.gaussian_spinor(lat, d, 2)
    y = gen.gaussian_spinor(lat, d, 3)
    X, Y = S.pack(x), S.pack(y)
    xs, ys = S.unpack(X), S.unpack(Y)      # the stored (rounded) values
    out = S.ctx.new_spinor(S.desc)
    S.ctx.bsm_vec_axpby(S.desc, 2, 0.5, X, -1.25, Y, out)
    ref = 0.5 * xs - 1.25 * ys
    tol = {"f64": 1e-15, "f32": 1e-7, "f16s": 1e-3}[prec]
    assert rel(S.unpack(out), ref) < tol
    # norms and dots accumulate in FP64 over the stored values
    n2 = S.ctx.bsm_vec_dot(S.desc, 2, X)
    assert abs(n2 - np.vdot(xs, xs).real) / n2 < 1e-13
    dt = S.ctx.bsm_vec_dot(S.desc, 2, X, Y)
    assert abs(dt - np.vdot(xs, ys).real) < 1e-12 * np.sqrt(n2 * np.vdot(ys, ys).real)
    # one parity block
    nb = S.ctx.spinor_bytes(S.desc, 1, 1)
    par = __import__("oracle").parity_mask(lat)
    n2e = S.ctx.bsm_vec_dot(S.desc, 1, X[:nb])
    assert abs(n2e - np.vdot(xs[par == 0], xs[par == 0]).real) / n2e < 1e-13


def test_conversions():
    lat = gen.Lattice(8, 6, 4, 6)
    S = Setup(lat, 3, "fund", gen.gauge_links(lat, 3, "haar", 1))
    d32 = bsm.desc(3, "fund", "f32")
    d16 = bsm.desc(3, "fund", "f16s")
    x = gen.gaussian_spinor(lat, 3, 5)
    X = S.pack(x)
    o32 = S.ctx.new_spinor(d32)
    S.ctx.bsm_vec_axpby(S.desc, 2, 1.0, X, 0.0, None, o32, prec_out="f32")
    ref = (x.real.astype(np.float32) + 1j * x.imag.astype(np.float32)).astype(complex)
    assert np.array_equal(S.unpack(o32, desc=d32), ref)
    o16 = S.ctx.new_spinor(d16)
    S.ctx.bsm_vec_axpby(S.desc, 2, 1.0, X, 0.0, None, o16, prec_out="f16s")
    q, s = quant.quantise(x)
    assert np.array_equal(S.unpack(o16, desc=d16), quant.dequantise(q, s, 3))


@pytest.mark.parametrize("nbytes", [1 << 20, (1 << 20) + 4096 * 16 + 48])
@pytest.mark.parametrize("blocks", [1, 7, 2048, 65536])
def test_stream_copy_and_read(nbytes, blocks):
    """the bandwidth calibration kernels: the copy is exact, including a
    ragged chunk per workgroup and a tail, and the read sweep's per-workgroup
    sums add up to the buffer's sum"""
    import torch
    n = nbytes // 4
    src = (torch.arange(n, dtype=torch.float32, device="cuda") % 7) - 3.0
    dst = torch.zeros_like(src)
    for nt in (0, 1):
        dst.zero_()
        bsm.bsm_stream_copy(src, dst, nontemporal=nt, blocks=blocks)
        torch.cuda.synchronize()
        assert torch.equal(dst, src)
    for nt in (0, 1):
        part = torch.zeros(blocks, dtype=torch.float32, device="cuda")
        bsm.bsm_stream_read(src, part, blocks=blocks, nontemporal=nt)
        torch.cuda.synchronize()
        assert abs(part.double().sum().item() - src.double().sum().item()) <= 1e-3 * n ** 0.5
    with pytest.raises(bsm.BsmError):
        bsm.bsm_stream_read(src, part, nbytes=nbytes - 4, blocks=blocks)
