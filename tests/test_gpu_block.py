"""Multi-RHS block path: the matrix-core hop of 16 right-hand sides and the
batched solver, against the FP64 oracle applied to each RHS."""
import numpy as np
import pytest

import oracle
from paper_1401_3733_amd import bsm
from paper_1401_3733_amd import inputs as gen
from tests.gpu_util import Setup, c128, note, rel

pytestmark = pytest.mark.gpu

# FP32 operator against the FP64 oracle on the same FP64 fields (inputs
# rounded to FP32 on the GPU)
FP32_TOL = 1e-6


def _block_setup(lat, N, seed):
    Uf = gen.gauge_links(lat, N, "haar", seed)
    S = Setup(lat, N, "adj", Uf, prec="f64")
    UR = oracle.represent(Uf, "adj").real.astype(np.complex128)
    Ub = S.ctx.new_block_gauge(S.desc)
    S.ctx.bsm_gauge_to_block(S.desc, S.U, Ub)
    return S, UR, Ub


def _unpack_block(S, blk, n):
    import torch
    out = torch.zeros((n, S.lat.V, 4, S.d), dtype=torch.complex128, device="cuda")
    S.ctx.bsm_unpack_block(S.desc, blk, out, n)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("N", [2, 3, 4])
@pytest.mark.parametrize("n_rhs", [16, 5])
def test_block_hop_matches_oracle_per_rhs(N, n_rhs):
    note(f"block hop N={N} n_rhs={n_rhs}")
    lat = gen.Lattice(8, 6, 4, 6)
    S, UR, Ub = _block_setup(lat, N, 700 + N)
    d = S.d
    psi = gen.gaussian_spinor(lat, d, 701, n_rhs=n_rhs)
    xs = gen.gaussian_spinor(lat, d, 702, n_rhs=n_rhs)
    A, X = S.ctx.new_block(S.desc), S.ctx.new_block(S.desc)
    S.ctx.bsm_pack_block(S.desc, c128(psi), A, n_rhs)
    S.ctx.bsm_pack_block(S.desc, c128(xs), X, n_rhs)
    # pack/unpack round trip is the FP32 rounding of the input
    back = _unpack_block(S, A, n_rhs)
    assert rel(back, psi) < 1e-7
    nb = S.ctx.block_bytes(S.desc) // 2
    par = oracle.parity_mask(lat)
    a = np.linspace(0.5, 1.5, 16)
    b = -np.linspace(0.01, 0.02, 16)
    worst = 0.0
    for p in (0, 1):
        for dag in (0, 1):
            out = S.ctx.new_block(S.desc)
            S.ctx.bsm_dslash_eo_block(S.desc, Ub, p, dag, a, X[p * nb:(p + 1) * nb], b,
                                      A[(1 - p) * nb:(2 - p) * nb], out[p * nb:(p + 1) * nb])
            got = _unpack_block(S, out, n_rhs)
            for r in range(n_rhs):
                ref = a[r] * xs[r] + b[r] * oracle.hop(lat, UR, psi[r], dagger=bool(dag), parity=p)
                m = par == p
                worst = max(worst, rel(got[r][m], ref[m]))
                assert rel(got[r][m], ref[m]) < FP32_TOL, (p, dag, r, rel(got[r][m], ref[m]))
                assert np.all(got[r][~m] == 0)
    print(f"block hop N={N} n_rhs={n_rhs}: max rel err {worst:.2e}", flush=True)


def test_block_hop_without_x():
    lat = gen.Lattice(4, 4, 4, 4)
    S, UR, Ub = _block_setup(lat, 4, 710)
    psi = gen.gaussian_spinor(lat, 15, 711, n_rhs=16)
    A = S.ctx.new_block(S.desc)
    S.ctx.bsm_pack_block(S.desc, c128(psi), A, 16)
    nb = S.ctx.block_bytes(S.desc) // 2
    out = S.ctx.new_block(S.desc)
    S.ctx.bsm_dslash_eo_block(S.desc, Ub, 0, 0, None, None, np.ones(16), A[nb:], out[:nb])
    got = _unpack_block(S, out, 16)
    par = oracle.parity_mask(lat)
    for r in (0, 7, 15):
        ref = oracle.hop(lat, UR, psi[r], parity=0)
        err = rel(got[r][par == 0], ref[par == 0])
        print(f"block hop without x, rhs {r}: rel err {err:.2e}", flush=True)
        assert err < FP32_TOL


@pytest.mark.parametrize("n_rhs", [16, 7, 3, 1])
def test_batched_solve_adjoint(n_rhs):
    """16 and 7 RHS retire together and take the block operator's FP64 true
    residual (and odd-site rebuild); 3 RHS and a single one take the per-RHS
    one"""
    note(f"batched solve adjoint n_rhs={n_rhs}")
    lat = gen.Lattice(8, 4, 4, 6)
    Uf = gen.gauge_links(lat, 4, "haar", 720)
    S = Setup(lat, 4, "adj", Uf, prec="f64")
    UR = oracle.represent(Uf, "adj").real.astype(np.complex128)
    kappas = list(np.linspace(0.10, 0.125, 16))[:n_rhs]
    b = gen.gaussian_spinor(lat, 15, 721, n_rhs=n_rhs)
    bb = S.pack(b, n_rhs=n_rhs)
    import torch
    x = torch.zeros_like(bb)
    prm = bsm.solver_params(0.1, 1e-10, schur=True, check_every=8)
    status, stats = S.ctx.bsm_batched_solve(S.desc, S.U, prm, kappas, bb, x)
    xs = S.unpack(x, n_rhs=n_rhs).reshape(b.shape)
    print(stats[0], stats[-1])
    assert status == 0
    for r in range(n_rhs):
        assert stats[r]["converged"]
        tr = oracle.true_residual(lat, UR, kappas[r], b[r], xs[r])
        assert tr <= 1e-10, (r, tr)
        assert abs(tr - stats[r]["true_rel_res"]) < 1e-12
    for r in (0, n_rhs - 1):
        xo, _ = oracle.solve(lat, UR, kappas[r], b[r], tol=1e-13, schur=True)
        assert rel(xs[r], xo) <= 1e-9


@pytest.mark.parametrize("prec", ["f32", "f16s"])
def test_batched_solve_widely_spread_kappas(prec):
    """Light and heavy members in one block (kappa 0.01 ... 0.125): the light
    ones meet their trigger replays before the heavy ones and wait (at most a
    few replays, then judged alone); every member must still meet tol and
    match the oracle."""
    note(f"batched solve spread kappas {prec}")
    lat = gen.Lattice(8, 4, 4, 6)
    Uf = gen.gauge_links(lat, 4, "haar", 725)
    S = Setup(lat, 4, "adj", Uf, prec="f64")
    UR = oracle.represent(Uf, "adj").real.astype(np.complex128)
    kappas = [0.01, 0.02, 0.04] + list(np.linspace(0.10, 0.125, 13))
    n_rhs = len(kappas)
    b = gen.gaussian_spinor(lat, 15, 726, n_rhs=n_rhs)
    bb = S.pack(b, n_rhs=n_rhs)
    import torch
    x = torch.zeros_like(bb)
    d = S.desc if prec == "f32" else _half_desc(4)   # an F64 descriptor runs the FP32 recurrence
    prm = bsm.solver_params(0.1, 1e-10, schur=True, check_every=2)
    status, stats = S.ctx.bsm_batched_solve(d, S.U, prm, kappas, bb, x)
    xs = S.unpack(x, n_rhs=n_rhs).reshape(b.shape)
    print([s["iters"] for s in stats], [s["reliable_updates"] for s in stats], flush=True)
    assert status == 0
    for r in range(n_rhs):
        assert stats[r]["converged"]
        tr = oracle.true_residual(lat, UR, kappas[r], b[r], xs[r])
        assert tr <= 1e-10, (r, tr)
        assert abs(tr - stats[r]["true_rel_res"]) < 1e-12
    for r in (0, n_rhs - 1):
        xo, _ = oracle.solve(lat, UR, kappas[r], b[r], tol=1e-13, schur=True)
        assert rel(xs[r], xo) <= 1e-9


def test_batched_solve_complex_links_fallback():
    note("batched solve fund fallback")
    lat = gen.Lattice(8, 4, 4, 4)
    Uf = gen.gauge_links(lat, 3, "near_identity", 730, eps=0.3)
    S = Setup(lat, 3, "fund", Uf, prec="f64")
    S32 = Setup(lat, 3, "fund", Uf, prec="f32")
    kappas = [0.11, 0.12, 0.125]
    b = gen.gaussian_spinor(lat, 3, 731, n_rhs=3)
    bb = S.pack(b, n_rhs=3)
    import torch
    x = torch.zeros_like(bb)
    status, stats = S32.ctx.bsm_batched_solve(S32.desc, S.U, bsm.solver_params(0.1, 1e-10), kappas, bb, x)
    xs = S.unpack(x, n_rhs=3)
    assert status == 0
    for r in range(3):
        assert oracle.true_residual(lat, Uf, kappas[r], b[r], xs[r]) <= 1e-10


def test_block_hop_full_size_sampled():
    """24^3x48 SU(4) adjoint, 16 RHS, the launch configuration of the batched
    solver: out_r = x_r - H in_r with x = in = psi_r gives D(kappa=1) psi_r on
    the output parity; compared at sampled sites with the oracle."""
    note("block hop full size sampled")
    lat = gen.config_lattice(4)
    Uf = gen.config_links(4, lat)
    S = Setup(lat, 4, "adj", Uf, prec="f64")
    UR = oracle.represent(Uf, "adj").real.astype(np.complex128)
    Ub = S.ctx.new_block_gauge(S.desc)
    S.ctx.bsm_gauge_to_block(S.desc, S.U, Ub)
    n_rhs = 4
    psi = gen.gaussian_spinor(lat, 15, 740, n_rhs=n_rhs)
    A = S.ctx.new_block(S.desc)
    S.ctx.bsm_pack_block(S.desc, c128(psi), A, n_rhs)
    nb = S.ctx.block_bytes(S.desc) // 2
    par = oracle.parity_mask(lat)
    rng = np.random.default_rng(5)
    for p in (0, 1):
        out = S.ctx.new_block(S.desc)
        S.ctx.bsm_dslash_eo_block(S.desc, Ub, p, 0, np.ones(16), A[p * nb:(p + 1) * nb], -np.ones(16),
                                  A[(1 - p) * nb:(2 - p) * nb], out[p * nb:(p + 1) * nb])
        got = _unpack_block(S, out, n_rhs)
        sites = np.flatnonzero(par == p)
        sample = np.concatenate([sites[:64], sites[-64:], rng.choice(sites, 256, replace=False)])
        for r in range(n_rhs):
            ref = oracle.dslash_sites(lat, UR, 1.0, psi[r], sample)
            err = rel(got[r][sample], ref)
            print(f"full-size block hop p={p} rhs {r}: rel err {err:.2e}", flush=True)
            assert err < FP32_TOL, (p, r, err)


PLANS = [(s, w) for s in (1, 2) for w in (1, 2, 4)]


@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("xchunk", [0, 1, 5])
@pytest.mark.parametrize("tiled", [0, 1])
@pytest.mark.parametrize("spw,wpb", PLANS)
def test_every_block_plan_gives_the_same_operator(N, spw, wpb, tiled, xchunk):
    """every site is visited once under every plan: the tiled order (tiles of
    4 x 2 x 4 rows here, t x z x y) and the plain one, and every order of the
    workgroups over the XCDs (runs of 5 leave a tail of the grid outside the
    runs), give the same operator"""
    note(f"block plan spw={spw} wpb={wpb} tiled={tiled} xchunk={xchunk} N={N}")
    lat = gen.Lattice(8, 6, 4, 6)
    S, UR, Ub = _block_setup(lat, N, 760 + N)
    S.ctx.bsm_set_block_plan(S.desc, spw, wpb, tiled, xchunk)
    plan = S.ctx.bsm_get_block_plan(S.desc)
    assert plan["sites_per_wave"] == spw and plan["tiled"] == tiled and plan["xcd_chunk"] == xchunk
    d = S.d
    psi = gen.gaussian_spinor(lat, d, 761, n_rhs=16)
    A = S.ctx.new_block(S.desc)
    S.ctx.bsm_pack_block(S.desc, c128(psi), A, 16)
    nb = S.ctx.block_bytes(S.desc) // 2
    par = oracle.parity_mask(lat)
    for p in (0, 1):
        out = S.ctx.new_block(S.desc)
        S.ctx.bsm_dslash_eo_block(S.desc, Ub, p, 1, np.ones(16), A[p * nb:(p + 1) * nb], -0.1 * np.ones(16),
                                  A[(1 - p) * nb:(2 - p) * nb], out[p * nb:(p + 1) * nb])
        got = _unpack_block(S, out, 16)
        for r in (0, 9, 15):
            ref = psi[r] - 0.1 * oracle.hop(lat, UR, psi[r], dagger=True, parity=p)
            m = par == p
            assert rel(got[r][m], ref[m]) < FP32_TOL, (p, r, rel(got[r][m], ref[m]))


@pytest.mark.parametrize("xchunk", [0, 3])
@pytest.mark.parametrize("tiled", [0, 1])
@pytest.mark.parametrize("spw,wpb", PLANS)
def test_batched_solve_under_every_block_plan(spw, wpb, tiled, xchunk):
    """the fused per-RHS norms of the block hop depend on the plan's workgroup
    shape, site order and workgroup order; the FP64 block hop follows the
    site and workgroup orders"""
    import torch
    note(f"batched solve plan spw={spw} wpb={wpb} tiled={tiled} xchunk={xchunk}")
    lat = gen.Lattice(4, 4, 4, 6)
    Uf = gen.gauge_links(lat, 3, "haar", 770)
    S = Setup(lat, 3, "adj", Uf, prec="f64")
    S.ctx.bsm_set_block_plan(S.desc, spw, wpb, tiled, xchunk)
    UR = oracle.represent(Uf, "adj").real.astype(np.complex128)
    kappas = [0.11, 0.12, 0.125]
    b = gen.gaussian_spinor(lat, 8, 771, n_rhs=3)
    bb = S.pack(b, n_rhs=3)
    x = torch.zeros_like(bb)
    status, stats = S.ctx.bsm_batched_solve(S.desc, S.U, bsm.solver_params(0.1, 1e-10), kappas, bb, x)
    assert status == 0
    assert S.ctx.bsm_get_block_plan(S.desc)["us"] == -1.0     # a hand-set plan is kept
    xs = S.unpack(x, n_rhs=3)
    for r in range(3):
        assert oracle.true_residual(lat, UR, kappas[r], b[r], xs[r]) <= 1e-10


def test_block_autotune_picks_a_plan():
    lat = gen.Lattice(8, 6, 4, 6)
    S, UR, Ub = _block_setup(lat, 4, 780)
    plan = S.ctx.bsm_block_autotune(S.desc, Ub)
    assert plan["us"] > 0 and (plan["sites_per_wave"], plan["waves_per_group"]) in PLANS
    assert plan["tiled"] in (0, 1) and plan["xcd_chunk"] in (0, 1, 16)
    with pytest.raises(bsm.BsmError):
        S.ctx.bsm_set_block_plan(S.desc, 1, 4, 2)
    with pytest.raises(bsm.BsmError):
        S.ctx.bsm_set_block_plan(S.desc, 1, 4, 0, -1)
    with pytest.raises(bsm.BsmError):
        S.ctx.bsm_set_block_plan(S.desc, 1, 4, 0, 4097)
    with pytest.raises(bsm.BsmError):
        S.ctx.bsm_set_block_plan(S.desc, 3, 4)
    with pytest.raises(bsm.BsmError):
        S.ctx.bsm_set_block_plan(S.desc, 1, 8)


def test_batched_solve_two_stage_reduction_and_staggered_padding():
    """16 RHS on 16 x 16 x 8 x 8 SU(2) adjoint: V/2 = 8192 sites per parity, so
    the planes get 256 staggering sites (four whole 64-site tiles of padding)
    and the block vector kernels run 6336 workgroups, beyond the 4096 partials
    summed in one stage: the per-RHS sums take the two-stage reduction.  Every
    RHS against the oracle's FP64 solve to 1e-13."""
    import torch
    note("batched solve 16x16x8x8 SU(2) adj, 16 RHS (two-stage per-RHS sums)")
    lat = gen.Lattice(16, 16, 8, 8)
    Uf = gen.gauge_links(lat, 2, "haar", 790)
    S = Setup(lat, 2, "adj", Uf, prec="f64")
    UR = oracle.represent(Uf, "adj").real.astype(np.complex128)
    kappas = list(np.linspace(0.10, 0.125, 16))
    b = gen.gaussian_spinor(lat, 3, 791, n_rhs=16)
    bb = S.pack(b, n_rhs=16)
    x = torch.zeros_like(bb)
    status, stats = S.ctx.bsm_batched_solve(S.desc, S.U, bsm.solver_params(0.1, 1e-10), kappas, bb, x)
    assert status == 0
    xs = S.unpack(x, n_rhs=16)
    worst = 0.0
    for r in range(16):
        assert stats[r]["converged"]
        tr = oracle.true_residual(lat, UR, kappas[r], b[r], xs[r])
        assert tr <= 1e-10, (r, tr)
        xo, _ = oracle.solve(lat, UR, kappas[r], b[r], tol=1e-13, schur=True)
        worst = max(worst, rel(xs[r], xo))
        assert rel(xs[r], xo) <= 1e-9, (r, rel(xs[r], xo))
    print(f"two-stage batched: iters {[s['iters'] for s in stats]}, max |x - x_oracle| / |x_oracle| {worst:.2e}",
          flush=True)


def test_cg_solve_batched_variant_forwards():
    """bsm_cg_solve with the BATCHED variant gives bsm_batched_solve's result"""
    import torch
    note("cg_solve BATCHED variant")
    lat = gen.Lattice(4, 4, 4, 6)
    Uf = gen.gauge_links(lat, 3, "haar", 792)
    S = Setup(lat, 3, "adj", Uf, prec="f64")
    kappas = [0.11, 0.125, 0.1]
    b = gen.gaussian_spinor(lat, 8, 793, n_rhs=3)
    bb = S.pack(b, n_rhs=3)
    x1, x2 = torch.zeros_like(bb), torch.zeros_like(bb)
    st1, s1 = S.ctx.bsm_batched_solve(S.desc, S.U, bsm.solver_params(0.1, 1e-10), kappas, bb, x1)
    prm = bsm.solver_params(0.1, 1e-10, variant=bsm.SOLVER_BATCHED, kappas=kappas)
    st2, s2 = S.ctx.bsm_cg_solve(S.desc, S.U, S.U, prm, bb, x2)
    assert st1 == st2 == 0 and len(s2) == 3
    assert [a["iters"] for a in s1] == [a["iters"] for a in s2]
    assert torch.equal(x1, x2)


# ---------------------------------------------------------------- FP16 blocks
# F16S bar (as for the single-RHS F16S operator): FP16 links (relative 2^-11
# per element), the projected half spinor rounded to FP16 (2^-11) and the
# output rounded to FP16 with its site scale (2^-12 of the largest component)
F16_TOL = 2e-3


def _half_desc(N):
    return bsm.desc(N, "adj", "f16s", "f64")


def _quantised(psi):
    """the FP16 block storage of each RHS: the oracle's per-site F16S rounding"""
    from oracle import quant
    d = psi.shape[-1]
    return np.stack([quant.dequantise(*quant.quantise(p), d) for p in psi])


@pytest.mark.parametrize("N", [2, 3, 4])
def test_half_block_pack_matches_oracle_quantisation(N):
    """pack rounds each site and RHS exactly as the oracle's F16S quantiser
    (bit for bit); padding RHS slots and unused colours stay zero"""
    note(f"half block pack N={N}")
    lat = gen.Lattice(4, 4, 6, 4)
    S, UR, Ub = _block_setup(lat, N, 790 + N)
    dh = _half_desc(N)
    psi = gen.gaussian_spinor(lat, S.d, 791, n_rhs=11) * np.exp(np.linspace(-3, 3, lat.V))[None, :, None, None]
    A = S.ctx.new_block(dh)
    S.ctx.bsm_pack_block(dh, c128(psi), A, 11)
    import torch
    back = torch.zeros((11, lat.V, 4, S.d), dtype=torch.complex128, device="cuda")
    S.ctx.bsm_unpack_block(dh, A, back, 11)
    torch.cuda.synchronize()
    got = back.cpu().numpy()
    assert np.array_equal(got, _quantised(psi))
    assert S.ctx.block_bytes(dh) < S.ctx.block_bytes(S.desc) // 2 + S.ctx.block_bytes(S.desc) // 8


@pytest.mark.parametrize("N", [2, 3, 4])
@pytest.mark.parametrize("n_rhs", [16, 5])
def test_half_block_hop_matches_oracle_per_rhs(N, n_rhs):
    """FP16 block hop against the FP64 oracle on the decoded FP16 inputs"""
    note(f"half block hop N={N} n_rhs={n_rhs}")
    lat = gen.Lattice(8, 6, 4, 6)
    S, UR, _ = _block_setup(lat, N, 800 + N)
    dh = _half_desc(N)
    Uh = S.ctx.new_block_gauge(dh)
    S.ctx.bsm_gauge_to_block(dh, S.U, Uh)
    d = S.d
    psi = gen.gaussian_spinor(lat, d, 801, n_rhs=n_rhs)
    xs = gen.gaussian_spinor(lat, d, 802, n_rhs=n_rhs)
    A, X = S.ctx.new_block(dh), S.ctx.new_block(dh)
    S.ctx.bsm_pack_block(dh, c128(psi), A, n_rhs)
    S.ctx.bsm_pack_block(dh, c128(xs), X, n_rhs)
    psi_q, xs_q = _quantised(psi), _quantised(xs)
    nb = S.ctx.block_bytes(dh) // 2
    par = oracle.parity_mask(lat)
    a = np.linspace(0.5, 1.5, 16)
    b = -np.linspace(0.01, 0.02, 16)
    worst = 0.0
    for p in (0, 1):
        for dag in (0, 1):
            out = S.ctx.new_block(dh)
            S.ctx.bsm_dslash_eo_block(dh, Uh, p, dag, a, X[p * nb:(p + 1) * nb], b,
                                      A[(1 - p) * nb:(2 - p) * nb], out[p * nb:(p + 1) * nb])
            got = _unpack_block_as(S, dh, out, n_rhs)
            for r in range(n_rhs):
                ref = a[r] * xs_q[r] + b[r] * oracle.hop(lat, UR, psi_q[r], dagger=bool(dag), parity=p)
                m = par == p
                err = rel(got[r][m], ref[m])
                worst = max(worst, err)
                assert err < F16_TOL, (p, dag, r, err)
                assert np.all(got[r][~m] == 0)
    print(f"half block hop N={N} n_rhs={n_rhs}: max rel err {worst:.2e}", flush=True)


def test_half_block_hop_full_size_sampled():
    """24^3x48 SU(4) adjoint, FP16 blocks and links, under the plan the F16S
    batched solver tunes: out_r = x_r - H in_r with x = in = the FP16 storage
    of psi_r gives D(kappa=1) on the output parity, compared at sampled sites
    with the oracle applied to the decoded FP16 input."""
    note("half block hop full size sampled")
    lat = gen.config_lattice(4)
    Uf = gen.config_links(4, lat)
    S = Setup(lat, 4, "adj", Uf, prec="f64")
    UR = oracle.represent(Uf, "adj").real.astype(np.complex128)
    dh = _half_desc(4)
    Uh = S.ctx.new_block_gauge(dh)
    S.ctx.bsm_gauge_to_block(dh, S.U, Uh)
    S.ctx.bsm_block_autotune(dh, Uh)
    n_rhs = 3
    psi = gen.gaussian_spinor(lat, 15, 745, n_rhs=n_rhs)
    A = S.ctx.new_block(dh)
    S.ctx.bsm_pack_block(dh, c128(psi), A, n_rhs)
    psi_q = _quantised(psi)
    del psi
    nb = S.ctx.block_bytes(dh) // 2
    par = oracle.parity_mask(lat)
    rng = np.random.default_rng(6)
    for p in (0, 1):
        out = S.ctx.new_block(dh)
        S.ctx.bsm_dslash_eo_block(dh, Uh, p, 0, np.ones(16), A[p * nb:(p + 1) * nb], -np.ones(16),
                                  A[(1 - p) * nb:(2 - p) * nb], out[p * nb:(p + 1) * nb])
        got = _unpack_block_as(S, dh, out, n_rhs)
        sites = np.flatnonzero(par == p)
        sample = np.concatenate([sites[:64], sites[-64:], rng.choice(sites, 256, replace=False)])
        for r in range(n_rhs):
            ref = oracle.dslash_sites(lat, UR, 1.0, psi_q[r], sample)
            err = rel(got[r][sample], ref)
            print(f"full-size FP16 block hop p={p} rhs {r}: rel err {err:.2e}", flush=True)
            assert err < F16_TOL, (p, r, err)


def _unpack_block_as(S, d, blk, n):
    import torch
    out = torch.zeros((n, S.lat.V, 4, S.d), dtype=torch.complex128, device="cuda")
    S.ctx.bsm_unpack_block(d, blk, out, n)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("xchunk", [0, 1, 5])
@pytest.mark.parametrize("tiled", [0, 1])
@pytest.mark.parametrize("wpb", [1, 2, 4])
def test_every_half_block_plan_gives_the_same_operator(wpb, tiled, xchunk):
    note(f"half block plan wpb={wpb} tiled={tiled} xchunk={xchunk}")
    lat = gen.Lattice(8, 6, 4, 6)
    S, UR, _ = _block_setup(lat, 4, 810)
    dh = _half_desc(4)
    Uh = S.ctx.new_block_gauge(dh)
    S.ctx.bsm_gauge_to_block(dh, S.U, Uh)
    S.ctx.bsm_set_block_plan(dh, 1, wpb, tiled, xchunk)
    assert S.ctx.bsm_get_block_plan(dh)["waves_per_group"] == wpb
    assert S.ctx.bsm_get_block_plan(S.desc)["us"] != -1.0   # the FP32 plan is separate
    psi = gen.gaussian_spinor(lat, 15, 811, n_rhs=16)
    A = S.ctx.new_block(dh)
    S.ctx.bsm_pack_block(dh, c128(psi), A, 16)
    psi_q = _quantised(psi)
    nb = S.ctx.block_bytes(dh) // 2
    par = oracle.parity_mask(lat)
    for p in (0, 1):
        out = S.ctx.new_block(dh)
        S.ctx.bsm_dslash_eo_block(dh, Uh, p, 1, np.ones(16), A[p * nb:(p + 1) * nb], -0.1 * np.ones(16),
                                  A[(1 - p) * nb:(2 - p) * nb], out[p * nb:(p + 1) * nb])
        got = _unpack_block_as(S, dh, out, 16)
        for r in (0, 9, 15):
            ref = psi_q[r] - 0.1 * oracle.hop(lat, UR, psi_q[r], dagger=True, parity=p)
            m = par == p
            assert rel(got[r][m], ref[m]) < F16_TOL, (p, r, rel(got[r][m], ref[m]))
    with pytest.raises(bsm.BsmError):
        S.ctx.bsm_set_block_plan(dh, 2, 4)


def test_half_block_autotune_picks_a_plan():
    lat = gen.Lattice(8, 6, 4, 6)
    S, UR, _ = _block_setup(lat, 3, 815)
    dh = _half_desc(3)
    Uh = S.ctx.new_block_gauge(dh)
    S.ctx.bsm_gauge_to_block(dh, S.U, Uh)
    plan = S.ctx.bsm_block_autotune(dh, Uh)
    assert plan["us"] > 0 and plan["sites_per_wave"] == 1 and plan["waves_per_group"] in (1, 2, 4)


@pytest.mark.parametrize("n_rhs", [16, 3, 1])
def test_batched_solve_adjoint_f16(n_rhs):
    """F16S inner recurrence (FP16 block fields, links and matrix cores) with
    FP64 reliable updates: every RHS to a 1e-10 FP64 true residual"""
    note(f"batched solve adjoint f16s n_rhs={n_rhs}")
    import torch
    lat = gen.Lattice(8, 4, 4, 6)
    Uf = gen.gauge_links(lat, 4, "haar", 820)
    S = Setup(lat, 4, "adj", Uf, prec="f64")
    UR = oracle.represent(Uf, "adj").real.astype(np.complex128)
    kappas = list(np.linspace(0.10, 0.125, 16))[:n_rhs]
    b = gen.gaussian_spinor(lat, 15, 821, n_rhs=n_rhs)
    bb = S.pack(b, n_rhs=n_rhs)
    x = torch.zeros_like(bb)
    prm = bsm.solver_params(0.1, 1e-10, schur=True, check_every=0)   # the F16S default replay length
    status, stats = S.ctx.bsm_batched_solve(_half_desc(4), S.U, prm, kappas, bb, x)
    xs = S.unpack(x, n_rhs=n_rhs).reshape(b.shape)
    print(stats[0], stats[-1], flush=True)
    assert status == 0
    for r in range(n_rhs):
        assert stats[r]["converged"]
        tr = oracle.true_residual(lat, UR, kappas[r], b[r], xs[r])
        assert tr <= 1e-10, (r, tr)
        assert abs(tr - stats[r]["true_rel_res"]) < 1e-12
    xo, _ = oracle.solve(lat, UR, kappas[-1], b[-1], tol=1e-13, schur=True)
    assert rel(xs[-1], xo) <= 1e-9
    assert S.ctx.bsm_get_block_plan(_half_desc(4))["us"] > 0   # tuned on the first call
    # the FP16 recurrence costs at most a few replays more than the FP32 one
    # (a recurrence that ran ahead of the true residual is restarted)
    x32 = torch.zeros_like(bb)
    st32, stats32 = S.ctx.bsm_batched_solve(S.desc, S.U, prm, kappas, bb, x32)
    assert st32 == 0
    for r in range(n_rhs):
        assert stats[r]["iters"] <= 2 * stats32[r]["iters"] + 16, (r, stats[r]["iters"], stats32[r]["iters"])


def test_batched_solve_f16_two_stage_reduction():
    """16 x 16 x 8 x 8 SU(2) adjoint, 16 RHS, F16S: V/2 = 8192, so a
    one-site-per-workgroup FP16 hop writes 8192 norm partials and the per-RHS
    sums take the two-stage path"""
    note("batched solve f16s two-stage")
    import torch
    lat = gen.Lattice(16, 16, 8, 8)
    Uf = gen.gauge_links(lat, 2, "haar", 830)
    S = Setup(lat, 2, "adj", Uf, prec="f64")
    UR = oracle.represent(Uf, "adj").real.astype(np.complex128)
    dh = _half_desc(2)
    S.ctx.bsm_set_block_plan(dh, 1, 1, 0, 0)
    kappas = list(np.linspace(0.10, 0.125, 16))
    b = gen.gaussian_spinor(lat, 3, 831, n_rhs=16)
    bb = S.pack(b, n_rhs=16)
    x = torch.zeros_like(bb)
    status, stats = S.ctx.bsm_batched_solve(dh, S.U, bsm.solver_params(0.1, 1e-10, schur=True), kappas, bb, x)
    assert status == 0
    xs = S.unpack(x, n_rhs=16)
    for r in (0, 7, 15):
        assert oracle.true_residual(lat, UR, kappas[r], b[r], xs[r]) <= 1e-10
