"""GPU parity: libbsm (through its C ABI) against the FP64 oracle.

Tolerances: FP64 operator rel. L2 <= 1e-13, FP32 <= 1e-6 (inputs are the
FP64 fields rounded by the library), F16S is stated and held to a loose
sanity bound only.  Lattices span several 256-site workgroups with a ragged
tail, use unequal extents (axis order), and include extent-2 directions
where the forward and backward neighbour coincide.
"""
import numpy as np
import pytest

import oracle
from oracle import quant
from paper_1401_3733_amd import inputs as gen
from tests.gpu_util import Setup, note, rel
from tests.helpers import valid_reps

pytestmark = pytest.mark.gpu

KAPPA = 0.13
# T, LX, LY, LZ: Vh = 576 = 2 x 256 + 64 (ragged tail), all extents distinct
DIMS_MAIN = (8, 6, 4, 6)
DIMS_TINY = (2, 2, 2, 2)
DIMS_SMALL = (4, 2, 6, 4)


def _links(lat, N, seed, kind="haar"):
    return gen.gauge_links(lat, N, kind, seed, eps=0.4)


@pytest.mark.parametrize("N,rep,d", valid_reps())
def test_represent_matches_oracle(N, rep, d):
    note(f"represent N={N} rep={rep}")
    lat = gen.Lattice(*DIMS_SMALL)
    Uf = _links(lat, N, 100 + N)
    S = Setup(lat, N, rep, Uf)
    import torch
    out = torch.zeros((lat.V, 4, d, d), dtype=torch.complex128, device="cuda")
    S.ctx.bsm_unpack_gauge(S.desc, S.U, out)
    torch.cuda.synchronize()
    ref = oracle.represent(Uf, rep)
    if rep == "adj":
        ref = ref.real.astype(np.complex128)   # stored as real d x d matrices
    assert np.abs(out.cpu().numpy() - ref).max() < 1e-13


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_pack_round_trip(prec):
    note(f"pack {prec}")
    lat = gen.Lattice(*DIMS_MAIN)
    Uf = _links(lat, 3, 1)
    S = Setup(lat, 3, "fund", Uf, prec=prec)
    psi = gen.gaussian_spinor(lat, 3, 2)
    psi[7] = 0
    back = S.unpack(S.pack(psi))
    if prec == "f64":
        assert np.array_equal(back, psi)
    elif prec == "f32":
        ref = psi.real.astype(np.float32) + 1j * psi.imag.astype(np.float32)
        assert np.array_equal(back, ref.astype(np.complex128))
    else:
        q, s = quant.quantise(psi)
        ref = quant.dequantise(q, s, 3)
        # the stored code of every component is decided in float32/binary16
        # exactly as the oracle quantiser does it
        assert np.array_equal(back, ref)


@pytest.mark.parametrize("N,rep,d", valid_reps())
@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_dslash_full_all_reps(N, rep, d, prec, tol):
    note(f"dslash_apply N={N} rep={rep} prec={prec}")
    lat = gen.Lattice(*DIMS_MAIN)
    Uf = _links(lat, N, 200 + N)
    S = Setup(lat, N, rep, Uf, prec=prec)
    UR = oracle.represent(Uf, rep)
    if rep == "adj":
        UR = UR.real.astype(np.complex128)
    psi = gen.gaussian_spinor(lat, d, 300 + d)
    inp = S.pack(psi)
    for dag in (0, 1):
        out = S.ctx.new_spinor(S.desc)
        S.ctx.bsm_dslash_apply(S.desc, S.U, KAPPA, dag, inp, out)
        got = S.unpack(out)
        ref = oracle.dslash(lat, UR, KAPPA, psi, dagger=bool(dag))
        assert rel(got, ref) <= tol, (N, rep, prec, dag, rel(got, ref))


@pytest.mark.parametrize("dims", [DIMS_TINY, (2, 4, 2, 2), (4, 2, 2, 6)])
@pytest.mark.parametrize("bc", [(-1, 1, 1, 1), (1, -1, 1, -1)])
def test_dslash_extent_two_and_boundaries(dims, bc):
    note(f"dslash dims={dims} bc={bc}")
    lat = gen.Lattice(*dims, bc=bc)
    Uf = _links(lat, 3, 7)
    S = Setup(lat, 3, "fund", Uf)
    psi = gen.gaussian_spinor(lat, 3, 8)
    out = S.ctx.new_spinor(S.desc)
    S.ctx.bsm_dslash_apply(S.desc, S.U, KAPPA, 0, S.pack(psi), out)
    assert rel(S.unpack(out), oracle.dslash(lat, Uf, KAPPA, psi)) <= 1e-13


@pytest.mark.parametrize("N,rep", [(3, "fund"), (3, "sym"), (4, "adj"), (6, "asym")])
@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_dslash_eo_blocks(N, rep, prec, tol):
    note(f"dslash_eo N={N} rep={rep} prec={prec}")
    lat = gen.Lattice(*DIMS_MAIN)
    Uf = _links(lat, N, 400 + N)
    S = Setup(lat, N, rep, Uf, prec=prec)
    UR = oracle.represent(Uf, rep)
    if rep == "adj":
        UR = UR.real.astype(np.complex128)
    d = S.d
    par = oracle.parity_mask(lat)
    psi = gen.gaussian_spinor(lat, d, 500)
    xf = gen.gaussian_spinor(lat, d, 501)
    inp, xin = S.pack(psi), S.pack(xf)
    a, b = 0.7, -0.3
    for p in (0, 1):
        for dag in (0, 1):
            out = S.ctx.new_spinor(S.desc)
            S.ctx.bsm_dslash_eo(S.desc, S.U, p, dag, a, S.block(xin, p), b, S.block(inp, 1 - p),
                                S.block(out, p))
            got = S.unpack(out)
            ref = a * xf + b * oracle.hop(lat, UR, psi, dagger=bool(dag), parity=p)
            m = par == p
            assert rel(got[m], ref[m]) <= tol
            assert np.all(got[~m] == 0)
    # a = 0 with a null x, and x aliasing out
    out = S.pack(xf)
    S.ctx.bsm_dslash_eo(S.desc, S.U, 0, 0, a, S.block(out, 0), b, S.block(inp, 1), S.block(out, 0))
    ref = a * xf + b * oracle.hop(lat, UR, psi, parity=0)
    m = par == 0
    assert rel(S.unpack(out)[m], ref[m]) <= tol
    out = S.ctx.new_spinor(S.desc)
    S.ctx.bsm_dslash_eo(S.desc, S.U, 1, 0, 0.0, None, 1.0, S.block(inp, 0), S.block(out, 1))
    ref = oracle.hop(lat, UR, psi, parity=1)
    assert rel(S.unpack(out)[par == 1], ref[par == 1]) <= tol


@pytest.mark.parametrize("link_prec", ["f32", "f16s"])
def test_dslash_f16s_error_stated(link_prec):
    note(f"dslash f16s links={link_prec}")
    lat = gen.Lattice(*DIMS_MAIN)
    Uf = gen.gauge_links(lat, 3, "near_identity", 9, eps=0.3)
    S = Setup(lat, 3, "sym", Uf, prec="f16s", link_prec=link_prec)
    UR = oracle.represent(Uf, "sym")
    psi = gen.gaussian_spinor(lat, 6, 10)
    out = S.ctx.new_spinor(S.desc)
    S.ctx.bsm_dslash_apply(S.desc, S.U, 0.125, 0, S.pack(psi), out)
    err = rel(S.unpack(out), oracle.dslash(lat, UR, 0.125, psi))
    print(f"F16S spinor, {link_prec} links: rel L2 error vs FP64 oracle = {err:.3e}")
    assert err < 2e-3


def test_dslash_deterministic():
    lat = gen.Lattice(*DIMS_MAIN)
    S = Setup(lat, 3, "fund", _links(lat, 3, 11), prec="f32")
    inp = S.pack(gen.gaussian_spinor(lat, 3, 12))
    o1, o2 = S.ctx.new_spinor(S.desc), S.ctx.new_spinor(S.desc)
    S.ctx.bsm_dslash_apply(S.desc, S.U, KAPPA, 0, inp, o1)
    S.ctx.bsm_dslash_apply(S.desc, S.U, KAPPA, 0, inp, o2)
    import torch
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-6), ("f16s", 2e-3)])
@pytest.mark.parametrize("order,tchunk", [(0, 1), (1, 1), (1, 2), (1, 4), (2, 1), (3, 1), (3, 2), (3, 4)])
@pytest.mark.parametrize("bc", [(-1, 1, 1, 1), (-1, -1, 1, 1)])
def test_every_traversal_plan_gives_the_same_operator(prec, tol, order, tchunk, bc):
    note(f"plan order={order} tchunk={tchunk} prec={prec} bc={bc}")
    lat = gen.Lattice(4, 8, 8, 8, bc=bc)      # LX*LY*LZ/2 = 256: one tile per time slice
    Uf = _links(lat, 3, 600)
    S = Setup(lat, 3, "fund", Uf, prec=prec)
    S.ctx.bsm_set_hop_plan(S.desc, order, tchunk)
    assert S.ctx.bsm_get_hop_plan(S.desc)["order"] == order
    psi = gen.gaussian_spinor(lat, 3, 601)
    for dag in (0, 1):
        # D_W parity by parity through the even-odd hop, which follows the
        # plan (bsm_dslash_apply takes the one-pass kernel on this lattice)
        inp = S.pack(psi)
        out = S.ctx.new_spinor(S.desc)
        for p in (0, 1):
            S.ctx.bsm_dslash_eo(S.desc, S.U, p, dag, 1.0, S.block(inp, p), -KAPPA, S.block(inp, 1 - p),
                                S.block(out, p))
        assert rel(S.unpack(out), oracle.dslash(lat, Uf, KAPPA, psi, dagger=bool(dag))) <= tol
    # even-odd block with the norm fused (the CG path) under this plan
    par = oracle.parity_mask(lat)
    inp = S.pack(psi)
    out = S.ctx.new_spinor(S.desc)
    S.ctx.bsm_dslash_eo(S.desc, S.U, 1, 0, 0.5, S.block(inp, 1), 2.0, S.block(inp, 0), S.block(out, 1))
    ref = 0.5 * psi + 2.0 * oracle.hop(lat, Uf, psi, parity=1)
    assert rel(S.unpack(out)[par == 1], ref[par == 1]) <= tol


def test_autotune_and_plan_validation():
    lat = gen.Lattice(4, 8, 8, 8)
    S = Setup(lat, 3, "fund", _links(lat, 3, 602), prec="f32")
    plan = S.ctx.bsm_autotune(S.desc, S.U)
    assert plan["us"] > 0
    from paper_1401_3733_amd import bsm as _b
    with pytest.raises(_b.BsmError):
        S.ctx.bsm_set_hop_plan(S.desc, 1, 3)         # T = 4 is not a multiple of 3
    lat2 = gen.Lattice(4, 6, 4, 6)                     # 72 sites per slice: does not tile
    S2 = Setup(lat2, 3, "fund", _links(lat2, 3, 603))
    with pytest.raises(_b.BsmError):
        S2.ctx.bsm_set_hop_plan(S2.desc, 3, 1)


_FULL = {}


def _full_fields(cfg):
    """Links and a source of a full-size workload (generated once per run)."""
    if cfg not in _FULL:
        _FULL.clear()
        lat = gen.config_lattice(cfg)
        d = oracle.rep_dim(3, gen.CONFIGS[cfg]["rep"])
        _FULL[cfg] = (lat, gen.config_links(cfg, lat), gen.gaussian_spinor(lat, d, 900 + cfg))
    return _FULL[cfg]


@pytest.mark.parametrize("cfg,prec,lprec,tol", [(2, "f32", "f32", 1e-6), (2, "f64", "f64", 1e-13),
                                                (3, "f32", "f32", 1e-6), (3, "f16s", "f32", 2e-3),
                                                (3, "f16s", "f16s", 2e-3)])
def test_hop_full_size_sampled(cfg, prec, lprec, tol):
    """32^3 x 64 lattices at full size, in the launch configuration bench.py
    times (autotuned plan, even-odd block with out = x - H in, i.e. D at
    kappa = 1 on the output parity): sampled sites against the oracle."""
    note(f"full-size hop cfg{cfg} {prec}/{lprec}")
    lat, Uf, psi = _full_fields(cfg)
    rep = gen.CONFIGS[cfg]["rep"]
    S = Setup(lat, 3, rep, Uf, prec=prec, link_prec=lprec)
    UR = oracle.represent(Uf, rep)
    S.ctx.bsm_autotune(S.desc, S.U)
    inp = S.pack(psi)
    par = oracle.parity_mask(lat)
    rng = np.random.default_rng(cfg)
    for p in (0, 1):
        out = S.ctx.new_spinor(S.desc)
        S.ctx.bsm_dslash_eo(S.desc, S.U, p, 0, 1.0, S.block(inp, p), -1.0, S.block(inp, 1 - p), S.block(out, p))
        got = S.unpack(out)
        sites = np.flatnonzero(par == p)
        sample = np.concatenate([sites[:256], sites[-256:], rng.choice(sites, 2048, replace=False)])
        ref = oracle.dslash_sites(lat, UR, 1.0, psi, sample)
        err = rel(got[sample], ref)
        print(f"cfg{cfg} {prec}/{lprec} parity {p}: sampled rel L2 error {err:.3e}")
        assert err <= tol


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-6), ("f16s", 2e-3)])
@pytest.mark.parametrize("bc", [(-1, 1, 1, 1), (1, -1, -1, 1)])
def test_xcd_band_plan_gives_the_same_operator(prec, tol, bc):
    note(f"plan order=4 prec={prec} bc={bc}")
    lat = gen.Lattice(4, 16, 16, 16, bc=bc)   # 2048 sites per parity and time slice: 8 bands of one tile
    Uf = _links(lat, 3, 610)
    S = Setup(lat, 3, "fund", Uf, prec=prec)
    S.ctx.bsm_set_hop_plan(S.desc, 4, 1)
    assert S.ctx.bsm_get_hop_plan(S.desc)["order"] == 4
    psi = gen.gaussian_spinor(lat, 3, 611)
    for dag in (0, 1):
        out = S.ctx.new_spinor(S.desc)
        S.ctx.bsm_dslash_apply(S.desc, S.U, KAPPA, dag, S.pack(psi), out)
        assert rel(S.unpack(out), oracle.dslash(lat, Uf, KAPPA, psi, dagger=bool(dag))) <= tol
    par = oracle.parity_mask(lat)
    inp = S.pack(psi)
    out = S.ctx.new_spinor(S.desc)
    S.ctx.bsm_dslash_eo(S.desc, S.U, 0, 1, 0.5, S.block(inp, 0), 2.0, S.block(inp, 1), S.block(out, 0))
    ref = 0.5 * psi + 2.0 * oracle.hop(lat, Uf, psi, dagger=True, parity=0)
    assert rel(S.unpack(out)[par == 0], ref[par == 0]) <= tol
    if prec == "f64":
        # the fused norms of the CG path under this plan: a Schur solve
        from paper_1401_3733_amd import bsm as _b
        import torch
        x = torch.zeros_like(inp)
        st, stats = S.ctx.bsm_cg_solve(S.desc, S.U, S.U, _b.solver_params(KAPPA, 1e-10, schur=True), inp, x)
        assert st == 0 and oracle.true_residual(lat, Uf, KAPPA, psi, S.unpack(x)) <= 1e-10


def test_xcd_band_plan_needs_whole_bands():
    lat = gen.Lattice(4, 8, 8, 8)                      # 256 sites per slice: no 8 bands
    S = Setup(lat, 3, "fund", _links(lat, 3, 612), prec="f32")
    from paper_1401_3733_amd import bsm as _b
    with pytest.raises(_b.BsmError):
        S.ctx.bsm_set_hop_plan(S.desc, 4, 1)
