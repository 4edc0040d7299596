"""Test-side helpers: lattice shifts, gauge transformations, norms.

These are used only to build the pins (gauge covariance and the like); they
are not part of either implementation.
"""
import numpy as np

# axis of the [T][Z][Y][X] grid that each direction mu runs along
MU_AXIS = {0: 0, 1: 3, 2: 2, 3: 1}


def grid(lat, a):
    T, X, Y, Z = lat.dims
    return a.reshape((T, Z, Y, X) + a.shape[1:])


def flat(lat, a):
    return a.reshape((lat.V,) + a.shape[4:])


def shift_forward(lat, a, mu):
    """a(x + mu) as a field of x (periodic wrap, no sign)."""
    return flat(lat, np.roll(grid(lat, a), -1, axis=MU_AXIS[mu]))


def gauge_transform_links(lat, U, Om):
    """U_mu(x) -> Om(x) U_mu(x) Om(x+mu)^dag  (fundamental links)."""
    out = np.empty_like(U)
    for mu in range(4):
        Oy = shift_forward(lat, Om, mu)
        out[:, mu] = Om @ U[:, mu] @ Oy.conj().transpose(0, 2, 1)
    return out


def rel(a, b):
    """relative L2 distance ||a - b|| / ||b||"""
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def vdot(a, b):
    return np.vdot(a.ravel(), b.ravel())


# every (N, rep) with representation dimension d_R in [2, 15]
def valid_reps():
    out = []
    for N in range(2, 16):
        out.append((N, "fund", N))
    for N in (2, 3, 4):
        out.append((N, "adj", N * N - 1))
    for N in (2, 3, 4, 5):
        out.append((N, "sym", N * (N + 1) // 2))
    for N in (3, 4, 5, 6):
        out.append((N, "asym", N * (N - 1) // 2))
    return out
