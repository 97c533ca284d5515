"""The allocation-free forward pass of the network (work buffers in a static
device array) against the allocating entry point, through the C ABI: equal bit
for bit on two calls in a row, the second with a smaller batch, and a batch
above the stated maximum rejected before any launch."""
import numpy as np
import pytest

import synth_inputs as si
from helpers import gpu_context, problem, to_dev

pytestmark = pytest.mark.gpu


def test_forward_noalloc_equals_forward():
    import paper_2505_00384_amd as hx
    p = problem(si.terrain_mesh(4, 2, 2, g=4), 4, coef="terrain")
    ctx = gpu_context(p)
    try:
        ctx.set_network(si.mlp_init(21, out_scale=0.5))
        bmax = ctx.network_noalloc_max_batch()
        n_in = ctx.n_features()
        assert bmax == (16 << 20) // (2 * (((n_in + 31) // 32) * 32 + 512))
        rng = np.random.default_rng(5)
        for B in (300, 37):                       # the second call smaller: stale rows remain
            print(f"[noalloc] batch {B}", flush=True)
            X = to_dev(rng.normal(size=(B, n_in)).astype(np.float32))
            ref = ctx.network_forward(X).cpu().numpy()
            out = ctx.network_forward_noalloc(X).cpu().numpy()
            assert out.shape == ref.shape
            np.testing.assert_array_equal(out, ref)
            assert np.isfinite(out).all() and np.abs(out).max() > 0
        with pytest.raises(hx.HXError) as e:
            import torch
            ctx.network_forward_noalloc(torch.zeros(bmax + 1, n_in, dtype=torch.float32,
                                                    device="cuda:0"))
        assert e.value.status == hx.HX_ERR_ARG
    finally:
        ctx.close()
