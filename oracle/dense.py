"""Dense brute force of the Wilson-Dirac operator on tiny lattices.

TEST INFRASTRUCTURE ONLY.  Builds D as an explicit (4 d V) x (4 d V) matrix
block by block from the operator's definition (paper, Section II.B: a matrix
coupling every fermion component to every other, nonzero only between nearest
neighbours), with spin projectors built as Kronecker products.  When the
lattice is 2 sites long in some direction, the forward and backward neighbour
are the same site and both hops add into one block: the dense form catches
an implementation that overwrites instead of accumulating.

Also the free-field closed form: with U = 1 a plane wave exp(i p.x) u is an
eigenvector family of D with
    D(p) = 1 - 2 kappa sum_mu cos p_mu + 2 i kappa sum_mu gamma_mu sin p_mu,
p_mu = (2 pi n_mu + pi [mu antiperiodic]) / L_mu.
"""
from __future__ import annotations

import itertools

import numpy as np

SIGMA = [np.eye(2, dtype=complex),
         np.array([[0, 1], [1, 0]], dtype=complex),
         np.array([[0, -1j], [1j, 0]], dtype=complex),
         np.array([[1, 0], [0, -1]], dtype=complex)]


def gammas():
    """Euclidean chiral basis, g_0 = [[0,1],[1,0]], g_k = [[0,-i s_k],[i s_k,0]]."""
    Z = np.zeros((2, 2), complex)
    g = [np.block([[Z, SIGMA[0]], [SIGMA[0], Z]])]
    for k in (1, 2, 3):
        g.append(np.block([[Z, -1j * SIGMA[k]], [1j * SIGMA[k], Z]]))
    return g


def gamma5():
    g = gammas()
    return g[1] @ g[2] @ g[3] @ g[0]


def _coords(dims):
    T, X, Y, Z = dims
    out = []
    for t in range(T):
        for z in range(Z):
            for y in range(Y):
                for x in range(X):
                    out.append((t, x, y, z))
    return out


def _index(dims, c):
    T, X, Y, Z = dims
    t, x, y, z = c
    return ((t * Z + z) * Y + y) * X + x


def dense_dirac(lat, U, kappa, dagger=False):
    """Dense D (or D^dag built from the stencil with g -> -g) from the links
    U [V][4][d][d] in the fermion representation."""
    dims, bc = lat.dims, lat.bc
    V = lat.V
    d = U.shape[-1]
    n = 4 * d
    g = gammas()
    eta = -1.0 if dagger else 1.0
    Dm = np.eye(V * n, dtype=complex)
    for s, c in enumerate(_coords(dims)):
        for mu in range(4):
            for step in (+1, -1):
                cc = list(c)
                cc[mu] += step
                sign = 1.0
                if cc[mu] == dims[mu]:
                    cc[mu] = 0
                    sign = bc[mu]
                if cc[mu] < 0:
                    cc[mu] = dims[mu] - 1
                    sign = bc[mu]
                y = _index(dims, cc)
                link = U[s, mu] if step > 0 else U[y, mu].conj().T
                P = np.eye(4) - step * eta * g[mu]
                Dm[s * n:(s + 1) * n, y * n:(y + 1) * n] -= kappa * sign * np.kron(P, link)
    return Dm


def free_field_symbol(lat, kappa, nvec, d):
    """D(p) (a 4d x 4d matrix, spin (x) colour identity) for integer momenta
    nvec (per mu), and the momentum vector p."""
    g = gammas()
    p = np.array([(2 * np.pi * nvec[mu] + (np.pi if lat.bc[mu] < 0 else 0.0)) / lat.dims[mu]
                  for mu in range(4)])
    M = (1 - 2 * kappa * np.sum(np.cos(p))) * np.eye(4, dtype=complex)
    for mu in range(4):
        M = M + 2j * kappa * np.sin(p[mu]) * g[mu]
    return np.kron(M, np.eye(d)), p


def plane_wave(lat, p, u):
    """psi(x) = exp(i p.x) u for every site, [V][4][d] with u [4][d]."""
    coords = np.array(_coords(lat.dims), dtype=float)  # (t, x, y, z) = mu order
    ph = np.exp(1j * coords @ p)
    return ph[:, None, None] * u[None, :, :]


def all_momenta(lat):
    return itertools.product(*[range(L) for L in lat.dims])
