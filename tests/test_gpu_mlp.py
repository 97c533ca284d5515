"""GPU parity of the learned preconditioner's inference and training kernels
with the network oracle on the same BF16-rounded weights, plus the solver policy
around it: FGMRES with the network converges, a poisoned network is replaced
by block Jacobi, a zero network reproduces block Jacobi, and training on the
solver's own iterates lowers the loss.

Tolerances: end to end, hidden activations are BF16, so an activation that
sits on a rounding boundary may round differently when the FP32 (GPU) and
FP64 (oracle) pre-activations differ in their last bits; normwise 2e-3
covers a handful of such flips, and gradients, which pass through one more
BF16 rounding (the back-propagated signal), 1e-2.  Layer by layer on the
GPU's own BF16 operands (exported after a training step) only the FP32
accumulation differs from the oracle's FP64: 1e-5 normwise per block."""
import numpy as np
import pytest

import oracle
import synth_inputs as si
from helpers import gpu_context, problem, to_dev
from oracle import mlp

pytestmark = pytest.mark.gpu


def _hx():
    import paper_2505_00384_amd as hx
    return hx


def _rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def terrain():
    p = problem(si.terrain_mesh(6, 2, 3, g=4), 4, coef="terrain")
    ctx = gpu_context(p)
    yield p, ctx
    ctx.close()


def _oracle_coef(p):
    c = np.zeros(p.n_cells)
    for i in range(p.n_cells):
        ell, ab, bb, _ = p.bj_cell_data(i)
        l2 = np.cbrt(ell.prod()) ** 2
        c[i] = np.log(bb / (ab * l2))
    return c


def test_features_parity(terrain):
    p, ctx = terrain
    r = si.rhs_terrain(2)(*p.dof_coords()) + 0.1 * si.random_vector(p.n_dofs, 5)
    F, s = ctx.gather_features(to_dev(r))
    Fo, so = mlp.features(r, p.nbr, p.n, _oracle_coef(p))
    np.testing.assert_allclose(s.cpu().numpy(), so, rtol=1e-6)
    assert _rel(F.cpu().numpy(), Fo) <= 1e-6
    # zero residual: zero features and scale
    F0, s0 = ctx.gather_features(to_dev(np.zeros(p.n_dofs)))
    assert float(F0.abs().max()) == 0.0 and float(s0.abs().max()) == 0.0


def test_forward_parity(terrain):
    import torch
    p, ctx = terrain
    hx = _hx()
    w = si.mlp_init(7)
    ctx.set_network(w)
    np.testing.assert_array_equal(ctx.get_network(), w)
    for B in (1, 37, 300):                       # ragged against the 64-row tiles
        X = np.random.default_rng(B).normal(size=(B, ctx.n_features())).astype(np.float32)
        out = ctx.network_forward(to_dev(X)).cpu().numpy()
        ref, _ = mlp.forward(w.astype(np.float64), X.astype(np.float64), bf16=True)
        assert _rel(out, ref) <= 2e-3, (B, _rel(out, ref))


def test_backward_and_adam_parity(terrain):
    import torch
    p, ctx = terrain
    w = si.mlp_init(8)
    w[-125:] = 0.05                              # nonzero output bias
    ctx.set_network(w)
    rng = np.random.default_rng(3)
    B = 200
    X = rng.normal(size=(B, ctx.n_features())).astype(np.float32)
    T = rng.normal(size=(B, 125)).astype(np.float32)
    loss, g = ctx.train_step(to_dev(X), to_dev(T), 0.0, want_grad=True)
    lo, go = mlp.backward(w.astype(np.float64), X.astype(np.float64), T.astype(np.float64), bf16=True)
    assert abs(loss - lo) <= 1e-3 * lo
    g = g.cpu().numpy()
    # per parameter block
    o = 0
    for (W, bvec) in mlp.unpack(go):
        for blk in (W.ravel(), bvec):
            assert _rel(g[o:o + blk.size], blk) <= 1e-2, o
            o += blk.size
    np.testing.assert_array_equal(ctx.get_network(), w)      # lr = 0: no update
    # one Adam step matches the oracle's update of the GPU gradient
    lr = 1e-3
    ctx.train_step(to_dev(X), to_dev(T), lr)
    w1 = ctx.get_network()
    ref, _, _ = mlp.adam_step(w.astype(np.float64), g.astype(np.float64), 0.0, 0.0, 1, lr)
    np.testing.assert_allclose(w1, ref, rtol=0, atol=2e-6)


def test_layers_on_exact_operands(terrain):
    """Each product of the forward and backward pass against the oracle's
    layer on the operands the GPU used: the exported BF16 inputs and the FP32
    activations and back-propagated signals, rounded to BF16 by the oracle
    where the next product rounds them."""
    hx = _hx()
    p, ctx = terrain
    w = si.mlp_init(12)
    w[-125:] = 0.03
    ctx.set_network(w)
    rng = np.random.default_rng(4)
    B = 173                                      # ragged against the 64/128-row tiles
    X = rng.normal(size=(B, ctx.n_features())).astype(np.float32)
    T = rng.normal(size=(B, 125)).astype(np.float32)
    with pytest.raises(hx.HXError):
        ctx.network_trace(hx.HX_TRACE_H1, B + 1)             # wrong size
    _, g = ctx.train_step(to_dev(X), to_dev(T), 0.0, want_grad=True)
    g = g.cpu().numpy().astype(np.float64)
    tr = {k: ctx.network_trace(getattr(hx, "HX_TRACE_" + k), B).astype(np.float64)
          for k in ("INPUT", "H1", "H2", "OUT", "DOUT", "DH2", "DH1")}
    (W1, b1), (W2, b2), (W3, b3) = mlp.unpack(w.astype(np.float64))
    rb = mlp.bf16_round
    tol = 1e-5
    np.testing.assert_array_equal(tr["INPUT"], rb(X))
    assert _rel(tr["H1"], np.maximum(mlp.layer(W1, b1, tr["INPUT"]), 0)) <= tol
    assert _rel(tr["H2"], np.maximum(mlp.layer(W2, b2, rb(tr["H1"])), 0)) <= tol
    assert _rel(tr["OUT"], mlp.layer(W3, b3, rb(tr["H2"]))) <= tol
    assert _rel(tr["DOUT"], 2.0 * (tr["OUT"] - T) / T.size) <= tol
    gW3, gb3, dA2 = mlp.layer_grads(W3, tr["DOUT"], rb(tr["H2"]))
    assert _rel(tr["DH2"], dA2 * (tr["H2"] > 0)) <= tol
    gW2, gb2, dA1 = mlp.layer_grads(W2, tr["DH2"], rb(tr["H1"]))
    assert _rel(tr["DH1"], dA1 * (tr["H1"] > 0)) <= tol
    gW1, gb1, _ = mlp.layer_grads(W1, tr["DH1"], tr["INPUT"])
    o = 0
    for name, blk in (("W1", gW1), ("b1", gb1), ("W2", gW2), ("b2", gb2), ("W3", gW3), ("b3", gb3)):
        assert _rel(g[o:o + blk.size], blk.ravel()) <= tol, name
        o += blk.size
    assert o == g.size
    # a forward call reuses the work buffers: the trace is gone
    ctx.network_forward(to_dev(X))
    with pytest.raises(hx.HXError) as e:
        ctx.network_trace(hx.HX_TRACE_H1, B)
    assert e.value.status == hx.HX_ERR_STATE


def test_learned_preconditioner_parity(terrain):
    """The whole learned preconditioner, BJ + w_K net(features), against the
    oracle's composition of the same steps."""
    hx = _hx()
    p, ctx = terrain
    w = si.mlp_init(11, out_scale=0.5)
    ctx.set_network(w)
    r = si.rhs_terrain(3)(*p.dof_coords()) + 0.2 * si.random_vector(p.n_dofs, 8)
    z = ctx.apply_preconditioner(to_dev(r), kind=hx.HX_PC_LEARNED).cpu().numpy()
    zr = mlp.precondition(p, w.astype(np.float64), r, _oracle_coef(p))
    zb = p.bj_apply(r)
    # the block-Jacobi part is exact to 1e-11; the correction carries BF16 error
    assert np.linalg.norm(z - zr) <= 2e-3 * np.linalg.norm(zr - zb) + 1e-11 * np.linalg.norm(zb)
    assert np.linalg.norm(zr - zb) > 0.01 * np.linalg.norm(zb)      # the correction is not trivial


@pytest.mark.parametrize("k", [2, 6])
def test_learned_preconditioner_parity_other_degrees(k):
    """The whole learned preconditioner at degree 2 (one launch: block
    Jacobi inside the network kernel) and at degree 6 (two launches: block
    Jacobi, then the network kernel) against the oracle's composition, on a
    terrain channel of 16 cells."""
    hx = _hx()
    p = problem(si.terrain_mesh(4, 2, 2, g=4), k, coef="terrain")
    ctx = gpu_context(p)
    try:
        n = k + 1
        w = si.mlp_init(13, n_in=n ** 3 + 6 * n * n + 1, n_out=n ** 3, out_scale=0.5)
        ctx.set_network(w)
        r = si.rhs_terrain(3)(*p.dof_coords()) + 0.2 * si.random_vector(p.n_dofs, 8)
        z = ctx.apply_preconditioner(to_dev(r), kind=hx.HX_PC_LEARNED).cpu().numpy()
        zr = mlp.precondition(p, w.astype(np.float64), r, _oracle_coef(p))
        zb = p.bj_apply(r)
        print(f"[learned] k={k}: |z - zr| / |zr - zb| = "
              f"{np.linalg.norm(z - zr) / np.linalg.norm(zr - zb):.2e}", flush=True)
        assert np.linalg.norm(z - zr) <= 2e-3 * np.linalg.norm(zr - zb) + 1e-11 * np.linalg.norm(zb)
        assert np.linalg.norm(zr - zb) > 0.01 * np.linalg.norm(zb)
    finally:
        ctx.close()


def test_learned_preconditioner_two_launch_form():
    """On 4,352 cells (272 workgroups of 16 cells, more than one per compute
    unit of a 256-CU device) block Jacobi and the network kernel run as two
    launches instead of one.  Parity with the oracle on sampled cells (a
    cell's output depends only on its own and its neighbours' residual values
    and on its own coefficient feature), and a zero network reproduces block
    Jacobi bit for bit, also inside FGMRES, where the preconditioner launch
    also normalises the Krylov vector."""
    import torch
    hx = _hx()
    p = problem(si.terrain_mesh(34, 8, 16, g=4), 4, coef="terrain")
    ctx = gpu_context(p)
    try:
        w = si.mlp_init(11, out_scale=0.5)
        ctx.set_network(w)
        r = si.rhs_terrain(3)(*p.dof_coords()) + 0.2 * si.random_vector(p.n_dofs, 8)
        z = ctx.apply_preconditioner(to_dev(r), kind=hx.HX_PC_LEARNED).cpu().numpy()
        cells = np.random.default_rng(5).choice(p.n_cells, 256, replace=False)
        coef = np.zeros(p.n_cells)
        for i in cells:
            ell, ab, bb, _ = p.bj_cell_data(int(i))
            coef[i] = np.log(bb / (ab * np.cbrt(ell.prod()) ** 2))
        zr = mlp.precondition(p, w.astype(np.float64), r, coef).reshape(p.n_cells, -1)[cells]
        zb = p.bj_apply(r).reshape(p.n_cells, -1)[cells]
        zg = z.reshape(p.n_cells, -1)[cells]
        assert np.linalg.norm(zg - zr) <= 2e-3 * np.linalg.norm(zr - zb) + 1e-11 * np.linalg.norm(zb)
        assert np.linalg.norm(zr - zb) > 0.01 * np.linalg.norm(zb)
        ctx.set_network(si.mlp_init(9, out_scale=0.0))
        rd = to_dev(si.random_vector(p.n_dofs, 6))
        assert torch.equal(ctx.apply_preconditioner(rd, kind=hx.HX_PC_LEARNED),
                           ctx.apply_preconditioner(rd, kind=hx.HX_PC_BLOCK_JACOBI))
        b = to_dev(si.rhs_terrain(4)(*p.dof_coords()))
        x_l, i_l = ctx.solve(b, params=hx.default_params(method=1, pc=hx.HX_PC_LEARNED))
        x_b, i_b = ctx.solve(b, params=hx.default_params(method=1, pc=hx.HX_PC_BLOCK_JACOBI))
        assert i_l["status"] == hx.HX_OK and i_l["iters"] == i_b["iters"]
        assert torch.equal(x_l, x_b)
    finally:
        ctx.close()


def test_zero_network_is_block_jacobi_and_poisoned_network_falls_back(terrain):
    import torch
    hx = _hx()
    p, ctx = terrain
    b = to_dev(si.rhs_terrain(4)(*p.dof_coords()))
    w = si.mlp_init(9, out_scale=0.0)            # W3 = 0, b3 = 0: correction 0
    ctx.set_network(w)
    r = to_dev(si.random_vector(p.n_dofs, 6))
    z_l = ctx.apply_preconditioner(r, kind=hx.HX_PC_LEARNED)
    z_b = ctx.apply_preconditioner(r, kind=hx.HX_PC_BLOCK_JACOBI)
    assert torch.equal(z_l, z_b)
    _, i_l = ctx.solve(b, params=hx.default_params(method=1, pc=hx.HX_PC_LEARNED))
    _, i_b = ctx.solve(b, params=hx.default_params(method=1, pc=hx.HX_PC_BLOCK_JACOBI))
    assert i_l["iters"] == i_b["iters"] and i_l["status"] == hx.HX_OK
    # NaN in the output bias: non-finite preconditioned vectors -> block Jacobi
    wn = w.copy(); wn[-1] = np.nan
    ctx.set_network(wn)
    x, info = ctx.solve(b, params=hx.default_params(method=1, pc=hx.HX_PC_LEARNED))
    assert info["status"] == hx.HX_FALLBACK_USED and info["fallback_used"]
    assert info["true_rel_res"] <= 1e-8
    assert np.isfinite(x.cpu().numpy()).all()
    # a network that points the wrong way stalls FGMRES -> stall rule -> BJ
    wb = si.mlp_init(10, out_scale=50.0)
    ctx.set_network(wb)
    x, info = ctx.solve(b, params=hx.default_params(method=1, pc=hx.HX_PC_LEARNED,
                                                     stall_window=3, stall_ratio=0.9))
    assert info["true_rel_res"] <= 1e-8 and info["status"] in (hx.HX_OK, hx.HX_FALLBACK_USED)


def test_training_on_solver_iterates_lowers_loss():
    import torch
    hx = _hx()
    from paper_2505_00384_amd import learned
    F, T = learned.generate_pairs(8000, seed=1, log=lambda *a: None, source="iterates")
    assert F.shape == (8000, 276) and torch.isfinite(F).all() and torch.isfinite(T).all()
    p = problem(si.cube_mesh(4), 4, coef="const")
    ctx = gpu_context(p)
    ctx.set_network(learned.init_weights(ctx, seed=0))
    hist = learned.train(ctx, F, T, steps=400, batch=1024, lr=1e-3, log=lambda *a: None,
                         log_every=399)
    assert hist[-1][1] < 0.7 * hist[0][1], hist
    ctx.close()


def test_learned_gain_over_block_jacobi():
    """Train on 10^5 pairs from the unit cube (Q4; error fields and solver
    iterates, the library's defaults), then solve with FGMRES(30) to 1e-8
    with and without the network.  On the 32x8x16 terrain channel (Q4) the
    learned preconditioner must converge without the fallback in fewer
    iterations and less wall time than block Jacobi, the same solver without
    the network; on held-out cube problems it must not need more iterations
    on average."""
    import torch
    hx = _hx()
    from paper_2505_00384_amd import learned
    F, T = learned.generate_pairs(100000, seed=0, log=print)
    p = problem(si.cube_mesh(4), 4, coef="const")
    ctx = gpu_context(p)
    ctx.set_network(learned.init_weights(ctx, seed=0))
    hist = learned.train(ctx, F, T, steps=3000, batch=2048, lr=1e-3, log=print, log_every=1000)
    assert hist[-1][1] < 0.5 * hist[0][1]
    xyz = p.dof_coords()
    gains = []
    for tau in (0.01, 0.001):
        ctx.set_coefficients(np.ones(p.n_dofs), tau * np.ones(p.n_dofs), 2.0)
        for seed in (101, 102):
            b = to_dev(si.rhs_cube(seed)(*xyz))
            r = learned.compare(ctx, b)
            bj, le = r["block_jacobi"], r["learned"]
            print(f"[gain] cube tau={tau} seed={seed}: BJ {bj['iters']} it {bj['wall_ms']:.1f} ms, "
                  f"learned {le['iters']} it {le['wall_ms']:.1f} ms, fallback {le['fallback_used']}",
                  flush=True)
            assert le["true_rel_res"] <= 1e-8 and bj["true_rel_res"] <= 1e-8
            gains.append(bj["iters"] / le["iters"])
    assert np.mean(gains) >= 1.0, gains
    w = ctx.get_network()
    ctx.close()
    p2 = problem(si.terrain_mesh(32, 8, 16, g=4), 4, coef="terrain")
    c2 = gpu_context(p2)
    c2.set_network(w)
    b2 = to_dev(si.rhs_terrain(0)(*p2.dof_coords()))
    learned.compare(c2, b2)                      # warm-up of both paths
    r = learned.compare(c2, b2)
    bj, le = r["block_jacobi"], r["learned"]
    print(f"[gain] terrain 32x8x16: BJ {bj['iters']} it {bj['wall_ms']:.1f} ms, learned "
          f"{le['iters']} it {le['wall_ms']:.1f} ms, fallback {le['fallback_used']}", flush=True)
    assert le["status"] == hx.HX_OK and not le["fallback_used"]
    assert le["true_rel_res"] <= 1e-8
    assert le["iters"] < bj["iters"] and le["wall_ms"] < bj["wall_ms"], (le, bj)
    c2.close()
