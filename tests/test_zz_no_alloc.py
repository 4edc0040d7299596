"""The allocation-free collapsed network (bsm_precond_apply_collapsed_noalloc)
against the allocating entry point (bsm_precond_apply_collapsed) through the
C ABI: identical kernels on identical inputs, so the outputs must agree bit
for bit, also on a second call with a smaller lattice that finds the first
call's contents in the shared static scratch."""
import numpy as np
import pytest

import oracle
from oracle import ptc
from paper_1401_3733_amd import bsm
from paper_1401_3733_amd import inputs as gen
from tests.gpu_util import Setup, note

pytestmark = pytest.mark.gpu


def _case(lat, seed, link_prec="f32"):
    import torch
    Uf = gen.gauge_links(lat, 3, "near_identity", seed, eps=0.5)
    S = Setup(lat, 3, "fund", Uf, prec="f32", link_prec="f32")
    desc = S.desc
    U = S.U
    if link_prec == "f16s":
        desc = bsm.desc(3, "fund", "f32", "f16s")
        U = S.ctx.new_gauge(desc)
        S.ctx.bsm_gauge_represent(desc, S.Uf_dev, U)
    C = 8
    W1, W2 = ptc.init_weights(C, gen.SEED_NET + seed)
    g = np.random.Generator(np.random.Philox(seed))
    W1 = W1 + 0.05 * (g.standard_normal(W1.shape) + 1j * g.standard_normal(W1.shape))
    W2 = W2 + 0.05 * (g.standard_normal(W2.shape) + 1j * g.standard_normal(W2.shape))
    net = torch.cat([torch.from_numpy(np.ascontiguousarray(W.astype(np.complex64))).reshape(-1)
                     for W in (W1, W2)]).cuda()
    r = S.pack(gen.gaussian_spinor(lat, 3, seed + 1), desc=desc)
    return S, Uf, desc, U, C, net, r


def _both(S, desc, U, C, net, r):
    import torch
    z_ref = torch.zeros_like(r)
    z_new = torch.zeros_like(r)
    S.ctx.bsm_precond_apply_collapsed(desc, U, C, net, r, z_ref)
    S.ctx.bsm_precond_apply_collapsed_noalloc(desc, U, C, net, r, z_new)
    torch.cuda.synchronize()
    return z_ref, z_new


@pytest.mark.parametrize("link_prec", ["f32", "f16s"])
def test_noalloc_matches_allocating_entry_point_twice(link_prec):
    import torch
    # first call: the cfg5-sized lattice, near the static array's limit
    big = gen.Lattice(32, 16, 16, 16)
    note(f"noalloc collapsed net, first call 16^3x32 ({link_prec} links)")
    S1, _, d1, U1, C, net1, r1 = _case(big, 41, link_prec)
    z_ref, z_new = _both(S1, d1, U1, C, net1, r1)
    assert torch.isfinite(z_ref).all() and z_ref.abs().max() > 0
    assert torch.equal(z_ref, z_new)
    # second call: a smaller lattice with a ragged tail (576 sites per parity)
    small = gen.Lattice(8, 6, 4, 6)
    note(f"noalloc collapsed net, second call 8x6x4x6 ({link_prec} links)")
    S2, Uf2, d2, U2, C, net2, r2 = _case(small, 42, link_prec)
    z_ref2, z_new2 = _both(S2, d2, U2, C, net2, r2)
    assert torch.equal(z_ref2, z_new2)
    # and the result is still the network: against the oracle's FP64 net
    if link_prec == "f32":
        W = net2.cpu().numpy().astype(np.complex128)
        n1 = C * 9 * 16
        W1, W2 = W[:n1].reshape(C, 1, 9, 4, 4), W[n1:].reshape(1, C, 9, 4, 4)
        UR = oracle.represent(Uf2, "fund").astype(np.complex64).astype(np.complex128)
        rin = S2.unpack(r2, desc=d2)
        ref = ptc.net_apply(small, UR, W1, W2, rin)
        got = S2.unpack(z_new2, desc=d2)
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        print(f"noalloc net vs oracle: rel err {err:.2e} (FP16 mixing bound 8 * 2^-11)", flush=True)
        assert err < 8 * 2.0 ** -11


def test_noalloc_refuses_a_lattice_beyond_the_static_array():
    import torch
    lat = gen.Lattice(32, 24, 24, 24)   # needs about 2.9 x the 64 MiB
    note("noalloc collapsed net, oversize lattice refused")
    ctx = bsm.Context(lat.dims, lat.bc)
    d = bsm.desc(3, "fund", "f32", "f32")
    U = ctx.new_gauge(d)
    r = ctx.new_spinor(d)
    z = ctx.new_spinor(d)
    net = torch.zeros(bsm.lib().bsm_net_bytes(8) // 8, dtype=torch.complex64, device="cuda")
    with pytest.raises(bsm.BsmError) as e:
        ctx.bsm_precond_apply_collapsed_noalloc(d, U, 8, net, r, z)
    assert e.value.status == bsm.ERR_ARG
