"""dd_apply_D_block_noalloc (the operator with the library's preallocated per-device scratch
instead of workspaces) against dd_apply_D_block: two calls in a row, the second on a smaller
input, in FP64 and FP32; both run the same kernels, so the outputs agree bit for bit (which is
within the FP64 1e-12 / FP32 1e-5 bars).  Requests beyond the scratch size are refused."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_06902_amd import dd

    c = dd.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_matches_apply_twice_then_smaller(ctx, prec):
    import torch

    cases = [((8, 8, 8, 8), [[4, 4]] * 4, 3, 501), ((8, 4, 4, 8), [[4, 4], [4], [4], [4, 4]], 2, 502)]
    for L, segs, n_rhs, seed in cases:  # the second call is the smaller input
        blk = ctx.make_blocks(L, -1, segs)
        U = synth.gauge_field(L, 0.3, seed)
        g = ctx.load_gauge(blk, _dev(U), "f32")
        x = _dev(synth.gaussian_complex((n_rhs, blk.total_sites, 4, 3), seed + 1))
        ref = ctx.apply_D_block(blk, g, 0.1355, prec, x).cpu().numpy()
        y = torch.full_like(x, float("nan"))
        ctx.apply_D_block_noalloc(blk, g, 0.1355, prec, x, y)
        got = y.cpu().numpy()
        assert np.array_equal(got, ref)
        assert np.linalg.norm(got - ref) <= (1e-12 if prec == "f64" else 1e-5) * np.linalg.norm(ref)
        g.close()
        blk.close()


def test_noalloc_refuses_requests_beyond_its_scratch(ctx):
    import torch

    from paper_2211_06902_amd import dd

    L = (16, 16, 16, 16)  # 65 536 sites x 8 rhs x 48 x 8 bytes = 201 MB > 128 MiB
    blk = ctx.make_blocks(L, -1, [[8, 8]] * 4)
    U = torch.zeros((16**4, 4, 3, 3), dtype=torch.complex128, device="cuda")
    for a in range(3):
        U[:, :, a, a] = 1
    g = ctx.load_gauge(blk, U, "f32")
    x = torch.zeros((8, blk.total_sites, 4, 3), dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(dd.DDError):
        ctx.apply_D_block_noalloc(blk, g, 0.1355, "f64", x, y)
    # the same call fits in FP32 with 4 rhs (50 MB)
    ctx.apply_D_block_noalloc(blk, g, 0.1355, "f32", x[:4], y[:4])
    assert float(y[:4].abs().max()) == 0.0
    g.close()
    blk.close()
