"""Learned preconditioner and flexible GCR, step by step (FP64).

TEST INFRASTRUCTURE ONLY.

Network: two parallel-transport convolution layers (1 -> C -> 1 channels,
9 paths each: stay, and one hop along +-mu carried by the links), linear, no
bias.  A layer maps channel fields v_j to
    out_i(x) = sum_j sum_p W_p^{ij} (T_p v_j)(x)
with W_p^{ij} a complex 4 x 4 spin matrix; the hop paths make it covariant
under gauge transformations.  The layer with W_0 = 1,
W_{+mu} = -kappa (1 - g_mu), W_{-mu} = -kappa (1 + g_mu) is exactly the
Wilson-Dirac operator.

Training: pairs (r, e) with r = D e; loss = mean over a batch of
|M(r) - e|^2 / |e|^2; gradients by the adjoint of each layer (the input
gradient) and the outer-product weight gradient; Adam (Kingma & Ba 2014) on
the real and imaginary parts.

FGCR(m) (flexible GCR, with z_k = M(r_k) possibly changing every step):
    r = b - D x
    for k = 0..m-1:  z_k = M(r); w_k = D z_k
                     for j < k: c = <w_j, w_k>; w_k -= c w_j; z_k -= c z_j
                     n = |w_k|; w_k /= n; z_k /= n
                     a = <w_k, r>; x += a z_k; r -= a w_k
    then restart with the recomputed r = b - D x.
"""
from __future__ import annotations

import numpy as np

import oracle

NPATH = 9


def wilson_weights(kappa: float) -> np.ndarray:
    """Layer weights [1][1][9][4][4] that reproduce D_W exactly."""
    W = np.zeros((1, 1, NPATH, 4, 4), np.complex128)
    W[0, 0, 0] = np.eye(4)
    for mu in range(4):
        g = oracle.gamma(mu)
        W[0, 0, 1 + mu] = -kappa * (np.eye(4) - g)
        W[0, 0, 5 + mu] = -kappa * (np.eye(4) + g)
    return W


def init_weights(channels: int, seed: int):
    """W1 [C][1][9][4][4], W2 [1][C][9][4][4]: stay path ~ identity / sqrt(C),
    hops ~ N(0, 1e-2) complex."""
    g = np.random.Generator(np.random.Philox(seed))

    def cg(shape, s):
        z = g.standard_normal(shape + (2,)) * s
        return z[..., 0] + 1j * z[..., 1]

    W1 = cg((channels, 1, NPATH, 4, 4), 1e-2)
    W2 = cg((1, channels, NPATH, 4, 4), 1e-2)
    W1[:, 0, 0] += np.eye(4) / np.sqrt(channels)
    W2[0, :, 0] += np.eye(4) / np.sqrt(channels)
    return W1, W2


def net_apply(lat, U, W1, W2, r):
    """M(r) for a single field r [V][4][d]."""
    h = oracle.ptc_layer(lat, U, W1, r[None])
    return oracle.ptc_layer(lat, U, W2, h)[0]


def loss_and_grad(lat, U, W1, W2, rs, es):
    """Batch loss mean_b |M(r_b) - e_b|^2 / |e_b|^2 and its gradients
    (dL/dRe W + i dL/dIm W) by backpropagation through the two layers."""
    B = len(rs)
    C = W1.shape[0]
    loss = 0.0
    g1 = np.zeros_like(W1)
    g2 = np.zeros_like(W2)
    for r, e in zip(rs, es):
        h = oracle.ptc_layer(lat, U, W1, r[None])          # [C][V][4][d]
        y = oracle.ptc_layer(lat, U, W2, h)[0]
        ne = np.vdot(e, e).real
        diff = y - e
        loss += np.vdot(diff, diff).real / ne / B
        Gy = 2.0 * diff / ne / B                             # dL/dRe y + i dL/dIm y
        g2 += oracle.ptc_weight_grad(lat, U, Gy[None], h, C, 1)
        Gh = oracle.ptc_layer_adjoint(lat, U, W2, Gy[None])   # [C][V][4][d]
        g1 += oracle.ptc_weight_grad(lat, U, Gh, r[None], 1, C)
    return loss, g1, g2


class Adam:
    """Adam on complex parameters, real and imaginary parts as separate
    coordinates: m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
    w <- w - lr mhat / (sqrt(vhat) + eps), with bias correction."""

    def __init__(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = None
        self.v = None

    def step(self, w, g):
        wr = np.stack([w.real, w.imag])
        gr = np.stack([g.real, g.imag])
        if self.m is None:
            self.m = np.zeros_like(wr)
            self.v = np.zeros_like(wr)
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * gr
        self.v = self.b2 * self.v + (1 - self.b2) * gr * gr
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        wr = wr - self.lr * mh / (np.sqrt(vh) + self.eps)
        return wr[0] + 1j * wr[1]


def fgcr(apply_D, apply_M, b, x0=None, tol=1e-10, m=16, maxit=1000):
    """Flexible GCR(m) on D x = b with preconditioner M.  Returns
    (x, iterations, |r|/|b| history at every iteration)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bn = np.linalg.norm(b)
    r = b - apply_D(x)
    hist = [np.linalg.norm(r) / bn]
    it = 0
    while it < maxit and hist[-1] > tol:
        Z, Wv = [], []
        for k in range(m):
            z = apply_M(r)
            w = apply_D(z)
            for zj, wj in zip(Z, Wv):
                c = np.vdot(wj, w)
                w = w - c * wj
                z = z - c * zj
            n = np.linalg.norm(w)
            w, z = w / n, z / n
            a = np.vdot(w, r)
            x = x + a * z
            r = r - a * w
            Z.append(z)
            Wv.append(w)
            it += 1
            hist.append(np.linalg.norm(r) / bn)
            if hist[-1] <= tol or it >= maxit:
                break
        r = b - apply_D(x)
        hist[-1] = np.linalg.norm(r) / bn
    return x, it, hist
