"""The BiCGStab autotuner (dd_autotune_bicgstab): every candidate is timed, the fastest is kept, the
JSON cache is written and a second call takes the stored configuration without timing; solves under
the chosen configuration meet the tolerance and agree with the default configuration's solution."""
import json

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

L = (16, 16, 16, 16)
KAPPA = 0.1355


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_06902_amd import dd

    c = dd.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("inner,ncand", [("f32", 10), ("f64", 4)])
def test_bicgstab_autotuner_and_cache(ctx, tmp_path, inner, ncand):
    from paper_2211_06902_amd import dd

    blk = ctx.make_blocks(L, -1, [[8, 8]] * 4)
    g = ctx.load_gauge(blk, _dev(synth.gauge_field(L, 0.2, 7101)), "f32")
    b = _dev(synth.gaussian_complex((4, blk.total_sites, 4, 3), 7102))
    prm = dd.solve_params(inner_prec=inner)
    x0, info0, st0 = ctx.block_solve(blk, g, KAPPA, b, params=prm)
    assert st0 == dd.DD_OK
    cache = str(tmp_path / "bicg_tune.json")
    try:
        res, hit = ctx.autotune_bicgstab(blk, g, KAPPA, b, params=prm, cache=cache)
        assert not hit and len(res) == ncand and all(r[4] > 0 for r in res)
        best = min(res, key=lambda r: r[4])
        with open(cache) as f:
            stored = json.load(f)
        assert len(stored) == 1
        (key, val), = stored.items()
        assert ("inner=" + inner) in key and "rhs=4" in key
        assert (val["rhs_group"], val["dhat_walk"], val["dhat_rhs"], val["bicg_fuse"]) == best[:4]
        # the chosen configuration solves to the tolerance and agrees with the default's solution
        x1, info1, st1 = ctx.block_solve(blk, g, KAPPA, b, params=prm)
        assert st1 == dd.DD_OK and np.all(info1["true_relres"] <= 1e-10)
        x0n, x1n = x0.cpu().numpy(), x1.cpu().numpy()
        assert np.linalg.norm(x1n - x0n) <= 1e-8 * np.linalg.norm(x0n)
        # a second call takes the stored entry without timing
        res2, hit2 = ctx.autotune_bicgstab(blk, g, KAPPA, b, params=prm, cache=cache)
        assert hit2 and len(res2) == 1 and res2[0][:4] == best[:4]
        # GMRES is not this tuner's
        with pytest.raises(dd.DDError):
            ctx.autotune_bicgstab(blk, g, KAPPA, b, params=dd.solve_params(method=dd.GMRES, inner_prec="f32"))
    finally:
        for what in (dd.TUNE_RHS_GROUP_F32, dd.TUNE_RHS_GROUP_F64, dd.TUNE_DHAT_WALK, dd.TUNE_DHAT_RHS,
                     dd.TUNE_BICG_FUSE):
            ctx.tune_set(what, 0)
    g.close()
    blk.close()
