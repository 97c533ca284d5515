"""Oracle of the learned per-cell preconditioner (test infrastructure only).

Network: 276 -> 256 -> 256 -> 125 with ReLU, parameters stored flat as
[W1, b1, W2, b2, W3, b3] with W row-major [out, in].  Working precision of the
GPU path: BF16 weights and activations, FP32 accumulation; this oracle does the
arithmetic in FP64 on BF16-rounded operands (``bf16=True``) or entirely in FP64
(``bf16=False``, used for finite-difference gradient checks).

BF16 rounding is round-to-nearest-even from FP32, done by bit manipulation.

Features of a cell K (all divided by s = RMS(r_K); zero when s = 0):
  [ r_K (n^3, local lexicographic order),
    for each face -x,+x,-y,+y,-z,+z: the neighbour's residual on its n^2
    Gauss-Lobatto nodes of the shared face (lexicographic in the two
    tangential directions, lower direction fastest; zeros on a boundary),
    log(beta_bar / (alpha_bar * ell^2)) with ell = (lx ly lz)^(1/3) ]
The preconditioner is z = BJ(r) + w_K MLP(features)_K per cell, with w_K the
RMS of the block-Jacobi output BJ(r)_K.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    nan = np.isnan(f)
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def unpack(params: np.ndarray, n_in=276, hidden=256, n_out=None):
    """[(W1, b1), (W2, b2), (W3, b3)] from the flat vector; n_out (the
    cell's dof count) follows from the vector's length when not given."""
    p = np.asarray(params, dtype=np.float64)
    if n_out is None:
        n_out = (p.size - hidden * (n_in + 1) - hidden * (hidden + 1)) // (hidden + 1)
    shapes = [(hidden, n_in), (hidden, hidden), (n_out, hidden)]
    out, o = [], 0
    for (r, c) in shapes:
        W = p[o:o + r * c].reshape(r, c); o += r * c
        bvec = p[o:o + r]; o += r
        out.append((W, bvec))
    assert o == p.size
    return out


def layer(W, bvec, a, bf16=True):
    """Pre-activation a W^T + b of one layer whose input activations a are
    already in working precision (the weights are rounded here)."""
    rnd = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    return np.asarray(a, dtype=np.float64) @ rnd(W).T + bvec


def layer_grads(W, d, a, bf16=True):
    """Back-propagation through one layer: d = d loss / d pre-activation
    [B, out], a = the layer's input activations [B, in].  Returns
    (d loss / d W, d loss / d b, d loss / d a); with ``bf16`` d enters the
    two products rounded, as on the GPU, and the bias gradient takes it
    unrounded."""
    rnd = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    d = np.asarray(d, dtype=np.float64)
    dr = rnd(d)
    return dr.T @ np.asarray(a, dtype=np.float64), d.sum(axis=0), dr @ rnd(W)


def forward(params, X, bf16=True):
    """X: [B, n_in].  Returns (output [B, n_out], cache)."""
    layers = unpack(params, X.shape[1])
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    a = rnd(X)
    cache = [a]
    pre = []
    for li, (W, bv) in enumerate(layers):
        z = layer(W, bv, a, bf16)
        pre.append(z)
        if li < len(layers) - 1:
            a = rnd(np.maximum(z, 0.0))
            cache.append(a)
        else:
            a = z
    return a, (cache, pre)


def mse(out, target):
    return float(np.mean((out - target) ** 2))


def backward(params, X, target, bf16=True):
    """Gradient of the MSE loss (mean over batch and outputs).

    With ``bf16`` the output gradient and back-propagated activation gradients
    are rounded to BF16 before they enter the next product, as the GPU does."""
    layers = unpack(params, X.shape[1])
    out, (acts, pre) = forward(params, X, bf16)
    B, n_out = out.shape
    loss = mse(out, target)
    d = 2.0 * (out - target) / (B * n_out)
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        gW, gb, da = layer_grads(W, d, acts[li], bf16)
        grads.append((gW, gb))
        if li > 0:
            d = da * (pre[li - 1] > 0)
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam_step(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def face_layer(rK: np.ndarray, n: int, f: int) -> np.ndarray:
    """Residual of a neighbour on the layer touching the shared face.

    ``f`` is the face of the *owner* cell (0..5 = -x,+x,-y,+y,-z,+z); the
    neighbour across it touches with its opposite layer."""
    u = rK.reshape(n, n, n)          # [l][j][i]
    d, plus = divmod(f, 2)
    idx = 0 if plus else n - 1
    if d == 0:
        return u[:, :, idx].ravel()  # (j, l), j fastest
    if d == 1:
        return u[:, idx, :].ravel()  # (i, l), i fastest
    return u[idx, :, :].ravel()      # (i, j), i fastest


def features(r: np.ndarray, nbr: np.ndarray, n: int, coef: np.ndarray):
    """Feature matrix [n_cells, n^3 + 6 n^2 + 1] and the per-cell scale s."""
    nd = n ** 3
    nc = nbr.shape[0]
    R = r.reshape(nc, nd)
    s = np.sqrt(np.mean(R * R, axis=1))
    F = np.zeros((nc, nd + 6 * n * n + 1))
    inv = np.where(s > 0, 1.0 / np.where(s > 0, s, 1.0), 0.0)
    F[:, :nd] = R * inv[:, None]
    for c in range(nc):
        for f in range(6):
            nb = nbr[c, f]
            if nb >= 0:
                F[c, nd + f * n * n: nd + (f + 1) * n * n] = face_layer(R[nb], n, f) * inv[c]
    F[:, -1] = np.where(s > 0, coef, 0.0)
    return F, s


def precondition(p, params, r, coef):
    """z = BJ(r) + w_K net(features(r))_K with w_K = RMS(BJ(r)_K); p is an
    oracle Problem (its separable block Jacobi), coef the per-cell coefficient
    feature."""
    z = p.bj_apply(r)
    F, _ = features(r, p.nbr, p.n, coef)
    out, _ = forward(params, F, bf16=True)
    Z = z.reshape(p.n_cells, -1)
    w = np.sqrt(np.mean(Z * Z, axis=1))
    return (Z + w[:, None] * out).ravel()
