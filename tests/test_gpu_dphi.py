"""The one-pass full-lattice Wilson operator behind bsm_dslash_apply (FP32,
d_R <= 3; both parities in one launch, most links read once; lanes of a
wavefront hold whole x-rows, threads march over time slices) against the
FP64 oracle, on lattices that exercise every sharing path: 2 to 16 rows per
wavefront, 1 to 4 wavefronts per workgroup, time chunks of 2 and 4 slices,
extent-2 directions, antiperiodic boundaries in every direction.  FP64 and
larger d_R take the even-odd hop over both parities (checked here too)."""
import numpy as np
import pytest

import oracle
from paper_1401_3733_amd import inputs as gen
from tests.gpu_util import Setup, note, rel

pytestmark = pytest.mark.gpu

KAPPA = 0.13
TOL = {"f64": 1e-13, "f32": 1e-6}

# (T, LX, LY, LZ): rows per wavefront 64 / LX, wavefronts per workgroup, time chunk
LATTICES = [
    (4, 8, 8, 4),      # 8 rows per wavefront, one wavefront per workgroup, chunk 4
    (6, 16, 8, 2),     # 4 rows, two wavefronts, chunk 2 (T = 6), z extent 2
    (4, 32, 8, 2),     # 2 rows, four wavefronts
    (2, 4, 16, 2),     # 16 rows, t extent 2 (forward and backward time neighbour coincide)
    (6, 32, 2, 4),     # 2 rows = the whole y extent (both y neighbours inside the wavefront)
]
BCS = [(-1, 1, 1, 1), (1, -1, -1, 1), (-1, -1, -1, -1)]


@pytest.mark.parametrize("dims", LATTICES)
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_dphi_one_pass_matches_oracle(dims, bc, prec):
    note(f"dphi dims={dims} bc={bc} {prec}")
    lat = gen.Lattice(*dims, bc=bc)
    Uf = gen.gauge_links(lat, 3, "haar", 940)
    S = Setup(lat, 3, "fund", Uf, prec=prec)
    psi = gen.gaussian_spinor(lat, 3, 941)
    for dag in (0, 1):
        out = S.ctx.new_spinor(S.desc)
        S.ctx.bsm_dslash_apply(S.desc, S.U, KAPPA, dag, S.pack(psi), out)
        err = rel(S.unpack(out), oracle.dslash(lat, Uf, KAPPA, psi, dagger=bool(dag)))
        assert err <= TOL[prec], (dag, err)


# the one-pass kernel: FP32, d_R 2 and 3 (complex and real links); the rest
# takes the even-odd path on the same lattice
REPS = [(2, "fund", "f32"), (2, "adj", "f32"), (3, "fund", "f32"), (2, "sym", "f32"), (3, "asym", "f32"),
        (3, "fund", "f64"), (4, "fund", "f32"), (3, "sym", "f32")]


@pytest.mark.parametrize("N,rep,prec", REPS)
def test_dphi_one_pass_every_representation(N, rep, prec):
    note(f"dphi N={N} {rep} {prec}")
    lat = gen.Lattice(4, 16, 4, 2, bc=(-1, 1, -1, 1))
    Uf = gen.gauge_links(lat, N, "haar", 950 + N)
    S = Setup(lat, N, rep, Uf, prec=prec)
    UR = oracle.represent(Uf, rep)
    psi = gen.gaussian_spinor(lat, S.d, 951)
    for dag in (0, 1):
        out = S.ctx.new_spinor(S.desc)
        S.ctx.bsm_dslash_apply(S.desc, S.U, KAPPA, dag, S.pack(psi), out)
        err = rel(S.unpack(out), oracle.dslash(lat, UR, KAPPA, psi, dagger=bool(dag)))
        assert err <= TOL[prec], (dag, err)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_dphi_one_pass_full_size_sampled(prec):
    """32^3 x 64 SU(3), the paper-task configuration: sampled sites of both
    parities against the oracle"""
    note(f"dphi full size {prec}")
    lat = gen.Lattice(64, 32, 32, 32)
    Uf = gen.gauge_links(lat, 3, "near_identity", 960, eps=0.3)
    S = Setup(lat, 3, "fund", Uf, prec=prec)
    psi = gen.gaussian_spinor(lat, 3, 961)
    out = S.ctx.new_spinor(S.desc)
    S.ctx.bsm_dslash_apply(S.desc, S.U, KAPPA, 0, S.pack(psi), out)
    got = S.unpack(out)
    rng = np.random.default_rng(7)
    sample = np.concatenate([np.arange(64), np.arange(lat.V - 64, lat.V), rng.choice(lat.V, 512, replace=False)])
    ref = oracle.dslash_sites(lat, Uf, KAPPA, psi, sample)
    err = rel(got[sample], ref)
    print(f"one-pass D_W 32^3x64 {prec}: sampled rel err {err:.2e}", flush=True)
    assert err <= TOL[prec]
