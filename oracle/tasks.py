"""The benchmark's two elementary tasks, and its flop model, in plain numpy.

TEST INFRASTRUCTURE ONLY: the tests and the CPU-baseline leg of the
benchmark are the only callers; the GPU library never imports, links or
executes anything here.

Section III of the paper times three tasks on random fields: an elementary
vector operation, a matrix-vector operation and the full Dirac operator.  It
names neither the two elementary operations nor the flop counts, so they are
read here as:
  vector   out = a x + b y on a whole spinor field (the solver's update);
  mat-vec  out(x)_s = sum_mu U_mu(x) psi(x)_s for each of the 4 spin
           components: the link algebra of the Dirac operator with no
           neighbour access;
and the Dirac task is the operator of oracle.dslash.

Fields are complex128 in the canonical layout: spinor [V][4][d], links
[V][4][d][d] with U_mu(x) at [x][mu].
"""
from __future__ import annotations

import numpy as np


def axpby(a: float, x: np.ndarray, b: float, y: np.ndarray) -> np.ndarray:
    """Section III's vector task: a x + b y, element by element."""
    return a * np.asarray(x, np.complex128) + b * np.asarray(y, np.complex128)


def link_matvec(U: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Section III's matrix-vector task: every site's four forward links
    applied to each spin component of the site's own spinor, summed over the
    four directions.  A batched matrix product (numpy's matmul) per
    direction, accumulated in direction order."""
    U = np.asarray(U, np.complex128)
    psi = np.asarray(psi, np.complex128)
    V, nmu, d, _ = U.shape
    assert nmu == 4 and psi.shape == (V, 4, d)
    col = psi.transpose(0, 2, 1)            # [V][d][spin]: spin components as columns
    out = np.zeros_like(col)
    for mu in range(4):
        out += U[:, mu] @ col
    return np.ascontiguousarray(out.transpose(0, 2, 1))


def task_flops_per_site(task: str, d: int, real: bool) -> int:
    """Flop model of one repetition per lattice site (the paper calibrates its
    counts but does not print them).  A complex multiply is 6 flops, a
    complex add 2, a real x complex multiply 2.
      vector: 8d reals, each 2 multiplies and 1 add;
      mat-vec: per spin, 4 matrix-vector products (d rows of d multiplies and
        d - 1 adds) and 3 adds of d-vectors;
      Dirac: 8 hops of the Wilson stencil, each spin-projected to 2d
        components (2d complex adds), 2 d-dimensional matrix-vector products,
        and 4d complex adds to reconstruct and accumulate (less the 4d of the
        first, which is a store), plus 1 multiply and 1 add per real for
        psi - kappa H psi."""
    if task == "vector":
        return 24 * d
    mul, add = (2, 2) if real else (6, 2)
    matvec = d * (d * mul + (d - 1) * add)
    if task == "matvec":
        return 4 * (4 * matvec + 3 * 2 * d)
    if task == "dphi":
        hop = 8 * (2 * d * add + 2 * matvec + 4 * d * add) - 4 * d * add
        return hop + 2 * 8 * d
    raise ValueError(task)
