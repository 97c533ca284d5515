"""Pins of the network oracle (CPU): BF16 rounding, gradients against central
finite differences, the closed form of a first Adam step, and the feature
layout against the geometry (the neighbour's face layer sits at the same
physical points as the owner's)."""
import numpy as np
import pytest

import oracle
import synth_inputs as si
from oracle import mlp


def test_bf16_rounding_pins():
    one = 1.0
    ulp = 2.0 ** -7                     # spacing of bf16 at 1
    vals = np.array([1.0, 1.0 + ulp / 2, 1.0 + 3 * ulp / 2, 1.0 + 0.74 * ulp, -2.5, 0.0,
                     3.0e38, 1e-40], dtype=np.float64)
    got = mlp.bf16_round(vals)
    exp = [1.0, 1.0, 1.0 + 2 * ulp, 1.0 + ulp, -2.5, 0.0]
    np.testing.assert_array_equal(got[:6], exp)   # ties go to the even mantissa
    assert np.isfinite(got[6]) and got[7] >= 0
    assert np.isnan(mlp.bf16_round(np.array([np.nan]))[0])
    # idempotent, and a bf16 number has at most 8 significant bits
    r = mlp.bf16_round(np.random.default_rng(0).normal(size=1000))
    np.testing.assert_array_equal(mlp.bf16_round(r), r)
    m, e = np.frexp(r)
    assert np.all(np.abs(m * 256 - np.round(m * 256)) == 0)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    n_in, n_out = 276, 125
    w = si.mlp_init(3, n_in=n_in, n_out=n_out).astype(np.float64)
    w[rng.integers(0, w.size, 2000)] += 0.01 * rng.normal(size=2000)   # nonzero biases too
    X = rng.normal(size=(6, n_in))
    T = rng.normal(size=(6, n_out))
    loss, g = mlp.backward(w, X, T, bf16=False)
    layers = mlp.unpack(w)
    # probe coordinates in every block (weights and biases of each layer)
    sizes = [W.size + b.size for W, b in layers]
    starts = np.cumsum([0] + sizes[:-1])
    probe = []
    for s0, sz in zip(starts, sizes):
        probe += list(s0 + rng.integers(0, sz, 8))
        probe.append(s0 + sz - 1)      # last bias entry
    eps = 1e-6
    for i in probe:
        wp = w.copy(); wp[i] += eps
        wm = w.copy(); wm[i] -= eps
        fd = (mlp.mse(mlp.forward(wp, X, False)[0], T) - mlp.mse(mlp.forward(wm, X, False)[0], T)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g).max()) + 1e-6 * abs(fd), (i, fd, g[i])


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(2)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    lr = 1e-3
    p1, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr)
    # m_hat = g, v_hat = g^2 after bias correction: the step is lr * sign(g)
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_feature_layout_matches_geometry():
    """With r a linear function of position on a non-periodic mesh, the
    neighbour's face-layer residual equals the owner's own face-layer values at
    the same tangential positions."""
    m = si.box_mesh(3, 2, 2, periodic=(False,) * 3, mapping=si.random_affine_mapping(4))
    k = 3
    n = k + 1
    p = oracle.Problem(m, k)
    x, y, z = p.dof_coords()
    r = 1.0 + x + 2 * y + 3 * z
    F, s = mlp.features(r, m.nbr, n, np.zeros(m.n_cells))
    R = r.reshape(m.n_cells, n, n, n)     # [c][l][j][i]
    nd, nf = n ** 3, n * n
    checked = 0
    for c in range(m.n_cells):
        for f in range(6):
            if m.nbr[c, f] < 0:
                assert np.all(F[c, nd + f * nf: nd + (f + 1) * nf] == 0)
                continue
            d, plus = divmod(f, 2)
            own = n - 1 if plus else 0
            if d == 0:
                layer = R[c][:, :, own]
            elif d == 1:
                layer = R[c][:, own, :]
            else:
                layer = R[c][own, :, :]
            got = F[c, nd + f * nf: nd + (f + 1) * nf] * s[c]
            np.testing.assert_allclose(got, layer.ravel(), rtol=1e-12, atol=1e-12)
            checked += 1
    assert checked > 10
    np.testing.assert_allclose(F[:, :nd] * s[:, None], r.reshape(m.n_cells, nd), rtol=1e-12)
    np.testing.assert_allclose(np.sqrt(np.mean((F[:, :nd]) ** 2, axis=1)), 1.0, rtol=1e-12)
