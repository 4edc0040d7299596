"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module draws random numbers and shapes them into gauge links, spinors
and gauge transforms.  It holds none of the operator's arithmetic (no
representation maps, no Dirac operator, no solver): it only produces the
fields that both sides consume, as complex128 numpy arrays in the canonical
user-facing layout.

Canonical layouts (complex interleaved, lexicographic site order, x fastest):
  site index  s = ((t*LZ + z)*LY + y)*LX + x
  spinor      [V][4 spin][d colour]
  gauge link  [V][4 mu][N][N]     (mu = 0 is time, 1..3 are x, y, z)
  block of RHS spinors: [n_rhs][V][4][d]

The paper fills its fields with random numbers (Section III); the
distributions below are the synthetic workloads of the five benchmark
configurations (Haar SU(N), near-identity exp(i eps H), Gaussian spinors).

Random source: numpy's Philox4x32-10 counter-based bit generator
(Salmon et al., SC'11), one independent stream per seed.
"""
from __future__ import annotations

import concurrent.futures as _cf
import numpy as np

__all__ = [
    "Lattice", "rng", "gaussian_spinor", "haar_su2_quaternion", "haar_sun",
    "near_identity_sun", "random_gauge_transform", "unit_links",
    "SEED_GAUGE", "SEED_SOURCE", "SEED_NET", "SEED_TRAIN",
]

# seed offsets per configuration k: gauge 1000+k, source 2000+k, net 3000+k,
# training data 4000+k
SEED_GAUGE, SEED_SOURCE, SEED_NET, SEED_TRAIN = 1000, 2000, 3000, 4000


class Lattice:
    """Extents and boundary signs; dims[mu] with mu = 0 time, 1..3 = x, y, z."""

    def __init__(self, T, LX, LY, LZ, bc=(-1, 1, 1, 1)):
        self.dims = (int(T), int(LX), int(LY), int(LZ))
        self.bc = tuple(int(b) for b in bc)

    @property
    def T(self):
        return self.dims[0]

    @property
    def V(self):
        T, X, Y, Z = self.dims
        return T * X * Y * Z

    def __repr__(self):
        T, X, Y, Z = self.dims
        return f"Lattice({X}x{Y}x{Z}x{T}, bc={self.bc})"


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(int(seed)))


def _cgauss(g: np.random.Generator, shape) -> np.ndarray:
    """Complex Gaussian with Re, Im ~ N(0, 1/2), so E|z|^2 = 1."""
    z = g.standard_normal(tuple(shape) + (2,))
    z *= np.sqrt(0.5)
    return z[..., 0] + 1j * z[..., 1]


def gaussian_spinor(lat: Lattice, d: int, seed: int, n_rhs: int | None = None) -> np.ndarray:
    """i.i.d. complex Gaussian spinor field(s), [V][4][d] or [n_rhs][V][4][d]."""
    g = rng(seed)
    shape = (lat.V, 4, d) if n_rhs is None else (n_rhs, lat.V, 4, d)
    return np.ascontiguousarray(_cgauss(g, shape))


def unit_links(lat: Lattice, N: int) -> np.ndarray:
    U = np.zeros((lat.V, 4, N, N), dtype=np.complex128)
    U[..., np.arange(N), np.arange(N)] = 1.0
    return U


def haar_su2_quaternion(n: int, seed: int) -> np.ndarray:
    """Haar SU(2): a0 + i a.sigma with a a normalised 4-d Gaussian vector."""
    g = rng(seed)
    a = g.standard_normal((n, 4))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    U = np.empty((n, 2, 2), dtype=np.complex128)
    U[:, 0, 0] = a[:, 0] + 1j * a[:, 3]
    U[:, 0, 1] = a[:, 2] + 1j * a[:, 1]
    U[:, 1, 0] = -a[:, 2] + 1j * a[:, 1]
    U[:, 1, 1] = a[:, 0] - 1j * a[:, 3]
    return U


def _fix_det(U: np.ndarray) -> np.ndarray:
    N = U.shape[-1]
    det = np.linalg.det(U)
    return U / (det ** (1.0 / N))[:, None, None]


def _chunks(n, size=1 << 18):
    return [(i, min(n, i + size)) for i in range(0, n, size)]


def _par_map(fn, *arrays):
    """Apply fn to row chunks of the arrays in threads (LAPACK drops the GIL).
    The random draws happen before this, so the result is independent of the
    thread count."""
    n = arrays[0].shape[0]
    out = [None] * len(_chunks(n))
    with _cf.ThreadPoolExecutor(max_workers=8) as ex:
        futs = {ex.submit(fn, *[a[i:j] for a in arrays]): k
                for k, (i, j) in enumerate(_chunks(n))}
        for f in futs:
            out[futs[f]] = f.result()
    return np.concatenate(out, axis=0) if out else np.zeros((0,) + arrays[0].shape[1:], np.complex128)


def _haar_from_gauss(Z):
    Q, R = np.linalg.qr(Z)
    diag = np.diagonal(R, axis1=1, axis2=2)
    ph = diag / np.abs(diag)
    Q = Q * ph[:, None, :]
    return _fix_det(Q)


def haar_sun(n: int, N: int, seed: int) -> np.ndarray:
    """Haar-random SU(N) (Mezzadri 2007): QR of a complex Gaussian matrix,
    column phases fixed by the diagonal of R, then det divided out."""
    if N == 2:
        return haar_su2_quaternion(n, seed)
    Z = _cgauss(rng(seed), (n, N, N))
    return _par_map(_haar_from_gauss, Z)


def _mgs_rows(U):
    """Modified Gram-Schmidt on the rows of each matrix (re-unitarise)."""
    U = U.copy()
    N = U.shape[-1]
    for i in range(N):
        for j in range(i):
            c = np.sum(U[:, j, :].conj() * U[:, i, :], axis=1)
            U[:, i, :] -= c[:, None] * U[:, j, :]
        U[:, i, :] /= np.linalg.norm(U[:, i, :], axis=1)[:, None]
    return U


def _expm_herm(H, eps):
    w, v = np.linalg.eigh(H)
    E = (v * np.exp(1j * eps * w)[:, None, :]) @ v.conj().transpose(0, 2, 1)
    return _fix_det(_mgs_rows(E))


def _expm_su3_cayley_hamilton(Q):
    """exp(i Q) for traceless Hermitian 3x3 Q as f0 + f1 Q + f2 Q^2, with the
    coefficients from the invariants c0 = det Q, c1 = Tr Q^2 / 2
    (Morningstar & Peardon, Phys. Rev. D 69 (2004) 054501, eqs. 19-34)."""
    Q2 = Q @ Q
    c1 = 0.5 * np.trace(Q2, axis1=1, axis2=2).real
    c0 = np.trace(Q2 @ Q, axis1=1, axis2=2).real / 3.0
    neg = c0 < 0
    c0a = np.abs(c0)
    c0max = 2.0 * (c1 / 3.0) ** 1.5
    theta = np.arccos(np.clip(c0a / np.where(c0max > 0, c0max, 1.0), -1.0, 1.0))
    u = np.sqrt(c1 / 3.0) * np.cos(theta / 3.0)
    w = np.sqrt(c1) * np.sin(theta / 3.0)
    xi0 = np.where(np.abs(w) > 0.05, np.sin(w) / np.where(w != 0, w, 1.0),
                   1 - w ** 2 / 6 * (1 - w ** 2 / 20 * (1 - w ** 2 / 42)))
    e2iu, emiu = np.exp(2j * u), np.exp(-1j * u)
    cw = np.cos(w)
    h0 = (u ** 2 - w ** 2) * e2iu + emiu * (8 * u ** 2 * cw + 2j * u * (3 * u ** 2 + w ** 2) * xi0)
    h1 = 2 * u * e2iu - emiu * (2 * u * cw - 1j * (3 * u ** 2 - w ** 2) * xi0)
    h2 = e2iu - emiu * (cw + 3j * u * xi0)
    den = 9 * u ** 2 - w ** 2
    f0, f1, f2 = h0 / den, h1 / den, h2 / den
    # c0 < 0: f_j(-c0) = (-1)^j conj(f_j(c0))
    f0 = np.where(neg, np.conj(f0), f0)
    f1 = np.where(neg, -np.conj(f1), f1)
    f2 = np.where(neg, np.conj(f2), f2)
    E = f1[:, None, None] * Q + f2[:, None, None] * Q2
    E[:, [0, 1, 2], [0, 1, 2]] += f0[:, None]
    return E


def near_identity_sun(n: int, N: int, eps: float, seed: int) -> np.ndarray:
    """U = exp(i eps H), H random traceless Hermitian with E Tr H^2 = (N^2-1)/2
    (the isotropic Gaussian on su(N) with unit-normal coefficients on a basis
    normalised to Tr T_a T_b = delta_ab / 2); exponentiated in closed form
    for N = 3 (Cayley-Hamilton) and through the Hermitian eigendecomposition
    otherwise, re-unitarised by modified Gram-Schmidt and the determinant
    divided out."""
    G = _cgauss(rng(seed), (n, N, N))
    H = 0.5 * (G + G.conj().transpose(0, 2, 1))
    tr = np.trace(H, axis1=1, axis2=2).real / N
    H[:, np.arange(N), np.arange(N)] -= tr[:, None]
    if N == 3:
        return _par_map(lambda h: _fix_det(_mgs_rows(_expm_su3_cayley_hamilton(eps * h))), H)
    return _par_map(lambda h: _expm_herm(h, eps), H)


def random_gauge_transform(lat: Lattice, N: int, seed: int) -> np.ndarray:
    """Omega(x) Haar SU(N) per site, [V][N][N]."""
    return haar_sun(lat.V, N, seed)


def gauge_links(lat: Lattice, N: int, kind: str, seed: int, eps: float = 0.0) -> np.ndarray:
    """Fundamental links [V][4][N][N]: kind 'haar', 'near_identity' or 'unit'."""
    n = lat.V * 4
    if kind == "haar":
        U = haar_sun(n, N, seed)
    elif kind == "near_identity":
        U = near_identity_sun(n, N, eps, seed)
    elif kind == "unit":
        return unit_links(lat, N)
    else:
        raise ValueError(kind)
    return np.ascontiguousarray(U.reshape(lat.V, 4, N, N))


# The five benchmark workloads: lattice, gauge group and representation,
# link distribution, hopping parameter(s), solver form.
CONFIGS = {
    1: dict(name="cfg1 4^4 SU(2) fund FP64 CGNR", dims=(4, 4, 4, 4), N=2, rep="fund",
            links=("haar", 0.0), kappa=0.12, solve="cgnr_full"),
    2: dict(name="cfg2 32^3x64 SU(3) fund even-odd", dims=(64, 32, 32, 32), N=3, rep="fund",
            links=("near_identity", 0.3), kappa=0.13, solve="schur_cg"),
    3: dict(name="cfg3 32^3x64 SU(3) 2S mixed RU-CG", dims=(64, 32, 32, 32), N=3, rep="sym",
            links=("near_identity", 0.3), kappa=0.125, solve="ru_cg"),
    4: dict(name="cfg4 24^3x48 SU(4) adj 16-RHS batched", dims=(48, 24, 24, 24), N=4, rep="adj",
            links=("haar", 0.0), kappa=list(np.linspace(0.10, 0.125, 16)), solve="batched"),
    5: dict(name="cfg5 16^3x32 SU(3) fund FGCR+net", dims=(32, 16, 16, 16), N=3, rep="fund",
            links=("near_identity", 0.5), kappa=0.1335, solve="fgcr_net"),
}


def config_lattice(k: int, dims=None) -> Lattice:
    T, X, Y, Z = dims if dims is not None else CONFIGS[k]["dims"]
    return Lattice(T, X, Y, Z, bc=(-1, 1, 1, 1))


def config_links(k: int, lat: Lattice | None = None) -> np.ndarray:
    c = CONFIGS[k]
    lat = lat or config_lattice(k)
    kind, eps = c["links"]
    return gauge_links(lat, c["N"], kind, SEED_GAUGE + k, eps)


def config_source(k: int, d: int, lat: Lattice | None = None, n_rhs=None) -> np.ndarray:
    lat = lat or config_lattice(k)
    return gaussian_spinor(lat, d, SEED_SOURCE + k, n_rhs)
