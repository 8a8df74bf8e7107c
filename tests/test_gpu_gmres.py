"""GPU parity of the persistent batched GMRES(m) inner solver (method DD_GMRES).

The outer FP64 defect correction is shared with BiCGStab, so every accepted
pair must again reach an FP64 true relative residual <= 1e-10, recomputed here
by the oracle's operator, and its solution must match the oracle's (dense LU
on the tiny blocks, the oracle's FP64 block solve elsewhere).
"""
import numpy as np
import pytest

import synth
from oracle import dense, geometry, wilson
from tests import _cfg

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_06902_amd import dd

    c = dd.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _true_relres(L, kappa, U, bx, x, b):
    r = b - wilson.dirac_box(L, -1, kappa, U, bx[:4], bx[4:8], x)
    return np.linalg.norm(r) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def c1(ctx):
    c = _cfg.C1
    L = c["L"]
    U = synth.gauge_field(L, c["eps"], c["seed_u"])
    boxes = _cfg.c1_boxes()
    b = synth.spinor_field(L, c["nrhs"], c["seed_src"])[:, _cfg.block_sites(L, boxes)]
    blk = ctx.make_blocks_boxes(L, -1, boxes)
    xs = []
    for k, bx in enumerate(boxes):
        M = dense.dense_dirac_box(L, -1, c["kappa"], U, bx[:4], bx[4:8])
        xs.append(np.linalg.solve(M, b[:, 16 * k:16 * (k + 1)].reshape(c["nrhs"], -1).T).T.reshape(c["nrhs"], 16, 4, 3))
    return dict(L=L, U=U, boxes=boxes, b=b, blk=blk, x_lu=np.concatenate(xs, axis=1), kappa=c["kappa"])


@pytest.mark.parametrize("inner,restart", [("f64", 16), ("f32", 16), ("bf16", 16), ("f32", 3), ("f64", 2)])
def test_c1_gmres_vs_dense_lu(ctx, c1, inner, restart):
    from paper_2211_06902_amd import dd

    g = ctx.load_gauge(c1["blk"], _dev(c1["U"]), "bf16" if inner == "bf16" else "f32")
    x, info, st = ctx.block_solve(c1["blk"], g, c1["kappa"], _dev(c1["b"]),
                                  params=dd.solve_params(method=dd.GMRES, restart=restart, inner_prec=inner, tol=TOL))
    print("C1 gmres(%d) %s: outer %d, max steps %d" % (restart, inner, info["outer_cycles"], info["inner_iterations"]))
    assert st == dd.DD_OK
    assert np.all(info["true_relres"] <= TOL) and np.all(info["flags"] & 1)
    x = x.cpu().numpy()
    for k, bx in enumerate(c1["boxes"]):
        for r in range(x.shape[0]):
            sl = slice(16 * k, 16 * (k + 1))
            assert _true_relres(c1["L"], c1["kappa"], c1["U"], bx, x[r, sl], c1["b"][r, sl]) <= TOL
    assert _cfg.rel_err(x, c1["x_lu"]) <= 1e-9
    g.close()


def test_gmres_graph_replay_is_bit_identical(ctx, c1):
    from paper_2211_06902_amd import dd

    g = ctx.load_gauge(c1["blk"], _dev(c1["U"]), "f32")
    b = _dev(c1["b"])
    p = dict(method=dd.GMRES, restart=8)
    x1, i1, _ = ctx.block_solve(c1["blk"], g, c1["kappa"], b, params=dd.solve_params(use_graph=1, **p))
    x2, i2, _ = ctx.block_solve(c1["blk"], g, c1["kappa"], b, params=dd.solve_params(use_graph=0, **p))
    x3, i3, _ = ctx.block_solve(c1["blk"], g, c1["kappa"], b, params=dd.solve_params(use_graph=1, **p))
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    assert np.array_equal(x1.cpu().numpy(), x3.cpu().numpy())
    assert np.array_equal(i1["iters"], i2["iters"]) and np.array_equal(i1["iters"], i3["iters"])
    g.close()


def test_gmres_zero_and_nan_sources_are_isolated(ctx, c1):
    from paper_2211_06902_amd import dd

    g = ctx.load_gauge(c1["blk"], _dev(c1["U"]), "f32")
    b = c1["b"][:3].copy()
    b[0, 0:16] = 0.0
    b[1, 16 * 5 + 3, 2, 1] = np.nan
    x, info, st = ctx.block_solve(c1["blk"], g, c1["kappa"], _dev(b), params=dd.solve_params(method=dd.GMRES))
    assert st == dd.DD_ENOCONV
    x = x.cpu().numpy()
    assert np.all(x[0, 0:16] == 0) and info["flags"][0, 0] & 1
    assert info["flags"][1, 5] & 4 and not info["flags"][1, 5] & 1
    ok = np.ones_like(info["flags"], dtype=bool)
    ok[1, 5] = False
    assert np.all(info["true_relres"][ok] <= TOL)
    for r in range(3):
        for k in range(len(c1["boxes"])):
            if (r, k) == (1, 5):
                continue
            sl = slice(16 * k, 16 * (k + 1))
            ref = np.zeros_like(x[r, sl]) if (r, k) == (0, 0) else c1["x_lu"][r, sl]
            assert np.linalg.norm(x[r, sl] - ref) <= 1e-9 * max(np.linalg.norm(ref), 1.0)
    g.close()


@pytest.fixture(scope="module")
def uneven(ctx):
    """Blocks of 12 x 8^3 and 8^4 sites (the two shapes of the 48^3 x 96 decomposition), 3 rhs."""
    L = (20, 8, 8, 16)
    segs = [[12, 8], [8], [8], [8, 8]]
    kappa = 0.1355
    U = synth.gauge_field(L, 0.3, 3101)
    boxes = geometry.tile_boxes(L, segs)
    b = synth.spinor_field(L, 3, 3102)[:, _cfg.block_sites(L, boxes)]
    blk = ctx.make_blocks(L, -1, segs)
    return dict(L=L, U=U, boxes=boxes, b=b, blk=blk, kappa=kappa, off=_cfg.site_offsets(boxes))


def _check_uneven(u, x, info, nrhs):
    x = x.cpu().numpy()
    assert np.all(info["true_relres"] <= TOL)
    for k, bx in enumerate(u["boxes"]):
        sl = slice(u["off"][k], u["off"][k + 1])
        for r in range(nrhs):
            assert _true_relres(u["L"], u["kappa"], u["U"], bx, x[r, sl], u["b"][r, sl]) <= TOL
            xo, _, _ = wilson.solve_box(u["L"], -1, u["kappa"], u["U"], bx[:4], bx[4:8], u["b"][r, sl], tol=1e-12)
            assert _cfg.rel_err(x[r, sl], xo) <= 1e-8


@pytest.mark.parametrize("inner,walk", [("bf16", 0), ("f32", 0), ("f64", 0), ("bf16", -1), ("f64", -1)])
def test_uneven_blocks_gmres(ctx, uneven, inner, walk):
    """walk 0: the kernel's hops walk the x0-slices; -1: the kernel whose hops read every neighbour
    from global memory."""
    from paper_2211_06902_amd import dd

    g = ctx.load_gauge(uneven["blk"], _dev(uneven["U"]), "bf16" if inner == "bf16" else "f32")
    try:
        ctx.tune_set(dd.TUNE_HOP_WALK, walk)
        x, info, st = ctx.block_solve(uneven["blk"], g, uneven["kappa"], _dev(uneven["b"]),
                                      params=dd.solve_params(method=dd.GMRES, inner_prec=inner))
    finally:
        ctx.tune_set(dd.TUNE_HOP_WALK, 0)
    print("uneven %s: outer %d, max steps %d" % (inner, info["outer_cycles"], info["inner_iterations"]))
    assert st == dd.DD_OK
    _check_uneven(uneven, x, info, 3)
    g.close()


@pytest.mark.parametrize("threads,queues,wpc", [(512, 1, 0), (256, 8, 1), (512, 8, 2), (256, 1, 0)])
def test_gmres_schedules_agree(ctx, uneven, threads, queues, wpc):
    """Every launch schedule the tuner may choose gives a converged, oracle-matching solve."""
    from paper_2211_06902_amd import dd

    g = ctx.load_gauge(uneven["blk"], _dev(uneven["U"]), "bf16")
    try:
        ctx.tune_set(dd.TUNE_GMRES_THREADS, threads)
        ctx.tune_set(dd.TUNE_GMRES_QUEUES, queues)
        ctx.tune_set(dd.TUNE_GMRES_WG_PER_CU, wpc)
        x, info, st = ctx.block_solve(uneven["blk"], g, uneven["kappa"], _dev(uneven["b"]),
                                      params=dd.solve_params(method=dd.GMRES, inner_prec="bf16"))
    finally:
        for k in (dd.TUNE_GMRES_THREADS, dd.TUNE_GMRES_QUEUES, dd.TUNE_GMRES_WG_PER_CU):
            ctx.tune_set(k, 0)
    assert st == dd.DD_OK
    _check_uneven(uneven, x, info, 3)
    g.close()


def test_gmres_and_bicgstab_agree(ctx, uneven):
    from paper_2211_06902_amd import dd

    g = ctx.load_gauge(uneven["blk"], _dev(uneven["U"]), "f32")
    b = _dev(uneven["b"])
    x1, _, s1 = ctx.block_solve(uneven["blk"], g, uneven["kappa"], b, params=dd.solve_params(method=dd.GMRES))
    x2, _, s2 = ctx.block_solve(uneven["blk"], g, uneven["kappa"], b, params=dd.solve_params(method=dd.BICGSTAB))
    assert s1 == dd.DD_OK and s2 == dd.DD_OK
    assert _cfg.rel_err(x1.cpu().numpy(), x2.cpu().numpy()) <= 1e-8
    g.close()


def test_bad_restart_is_rejected(ctx, c1):
    from paper_2211_06902_amd import dd

    g = ctx.load_gauge(c1["blk"], _dev(c1["U"]), "f32")
    for m in (0, 17):
        with pytest.raises(dd.DDError):
            ctx.block_solve(c1["blk"], g, c1["kappa"], _dev(c1["b"][:1]),
                            params=dd.solve_params(method=dd.GMRES, restart=m))
    g.close()


def test_autotuner_picks_a_working_schedule(ctx, uneven):
    from paper_2211_06902_amd import dd

    g = ctx.load_gauge(uneven["blk"], _dev(uneven["U"]), "bf16")
    b = _dev(uneven["b"])
    p = dd.solve_params(method=dd.GMRES, inner_prec="bf16")
    try:
        tried, best = ctx.autotune_gmres(uneven["blk"], g, uneven["kappa"], b, params=p)
        assert len(tried) >= 4 and all(r[3] > 0 for r in tried)
        assert best in tried and best[3] == min(r[3] for r in tried)
        x, info, st = ctx.block_solve(uneven["blk"], g, uneven["kappa"], b, params=p)
    finally:
        for k in (dd.TUNE_GMRES_THREADS, dd.TUNE_GMRES_QUEUES, dd.TUNE_GMRES_WG_PER_CU):
            ctx.tune_set(k, 0)
    assert st == dd.DD_OK
    _check_uneven(uneven, x, info, 3)
    g.close()


def test_c3_full_size_bf16_gmres(ctx):
    """The 48^3 x 96 workload at full size: 2160 uneven blocks x 12 rhs, BF16 links, GMRES(16).
    Every pair's FP64 true residual is checked by the library; sampled pairs of both block shapes
    against the oracle's FP64 solve."""
    import torch

    from paper_2211_06902_amd import dd

    c = _cfg.C3
    L = c["L"]
    U = synth.gauge_field(L, c["eps"], c["seed_u"])
    boxes = geometry.tile_boxes(L, c["segs"])
    off = _cfg.site_offsets(boxes)
    b = synth.spinor_field_device(c["nrhs"], int(off[-1]), c["seed_src"])
    blk = ctx.make_blocks(L, -1, c["segs"])
    g = ctx.load_gauge(blk, _dev(U), "bf16")
    x, info, st = ctx.block_solve(blk, g, c["kappa"], b,
                                  params=dd.solve_params(method=dd.GMRES, restart=16, inner_prec="bf16"))
    print("C3: outer cycles %d, max GMRES steps %d, %.3f s" % (info["outer_cycles"], info["inner_iterations"],
                                                               info["seconds"]))
    assert st == dd.DD_OK
    assert np.all(info["true_relres"] <= TOL)
    shapes = [tuple(bx[4:8]) for bx in boxes]
    picks = [0, shapes.index((8, 8, 8, 8)), len(boxes) - 1, 1000]
    for k, r in zip(picks, [0, 5, 11, 7]):
        bx = boxes[k]
        sl = slice(int(off[k]), int(off[k + 1]))
        bk = b[r, sl].cpu().numpy()
        xk = x[r, sl].cpu().numpy()
        assert _true_relres(L, c["kappa"], U, bx, xk, bk) <= TOL
        xo, _, rel = wilson.solve_box(L, -1, c["kappa"], U, bx[:4], bx[4:8], bk, tol=1e-12)
        assert rel <= 1e-12
        assert _cfg.rel_err(xk, xo) <= 1e-8
    del x, b
    torch.cuda.empty_cache()
    g.close()
    blk.close()


@pytest.mark.parametrize("reorth", [-1, 100, 40])
def test_gmres_reorthogonalization_thresholds(ctx, uneven, reorth):
    """Classical Gram-Schmidt once (-1), twice in every step (100) or twice when |w - V h| < 40 % of
    |w|: every setting converges to the oracle's solution."""
    from paper_2211_06902_amd import dd

    g = ctx.load_gauge(uneven["blk"], _dev(uneven["U"]), "f32")
    try:
        ctx.tune_set(dd.TUNE_GMRES_REORTH, reorth)
        x, info, st = ctx.block_solve(uneven["blk"], g, uneven["kappa"], _dev(uneven["b"]),
                                      params=dd.solve_params(method=dd.GMRES, inner_prec="f32"))
    finally:
        ctx.tune_set(dd.TUNE_GMRES_REORTH, 0)
    assert st == dd.DD_OK
    _check_uneven(uneven, x, info, 3)
    g.close()
