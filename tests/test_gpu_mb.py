"""GPU parity of the block-local multi-boson action (eq. localMB) against the oracle."""
import numpy as np
import pytest

import synth
from oracle import geometry, mb, roots, wilson
from tests import _cfg

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


def _setup(ctx, L, segs, inner_d, nf, seed):
    U = synth.gauge_field(L, 0.2, seed)
    boxes = geometry.tile_boxes(L, segs)
    blk = ctx.make_blocks(L, -1, segs, inner_d=inner_d)
    inner = blk.tables()[0][:, 8:16]
    bl = mb.boundary_lists(L, boxes, inner)
    return U, boxes, blk, inner, bl


def test_mb_closed_form(ctx):
    """xi = D_Omega eta with eta on dLambda_0: S^a = sum_k |u_k chi_k + eta_k|^2 exactly."""
    from paper_2211_06902_amd import dd

    L = (16, 16, 8, 8)
    kappa = 0.1365
    nf = 4
    U, boxes, blk, inner, bl = _setup(ctx, L, [[8, 8], [8, 8], [8], [8]], 1, nf, 5101)
    g = ctx.load_gauge(blk, _dev(U), "f32")
    u = roots.mb_roots(2 * nf, 0.5)[:nf]
    nbd = blk.total_bnd_sites
    chi = synth.gaussian_complex((nf, nbd, 4, 3), 5102)
    eta_b = synth.gaussian_complex((nf, nbd, 4, 3), 5103)
    off = _cfg.site_offsets(boxes)
    xi = np.zeros((nf, blk.total_sites, 4, 3), dtype=complex)
    expect = np.zeros(len(boxes))
    boff = 0
    for k, bx in enumerate(boxes):
        nb = bl[k].size
        for f in range(nf):
            eta = np.zeros((off[k + 1] - off[k], 4, 3), dtype=complex)
            eta[bl[k]] = eta_b[f, boff:boff + nb]
            xi[f, off[k]:off[k + 1]] = wilson.dirac_box(L, -1, kappa, U, bx[:4], bx[4:8], eta)
            expect[k] += np.sum(np.abs(u[f] * chi[f, boff:boff + nb] + eta_b[f, boff:boff + nb]) ** 2)
        boff += nb
    S, tot, info, st = ctx.multiboson_action(blk, g, kappa, u, _dev(chi), _dev(xi))
    assert st == dd.DD_OK
    S = S.cpu().numpy()
    assert np.max(np.abs(S - expect) / expect) <= 1e-9
    assert abs(tot - expect.sum()) <= 1e-9 * expect.sum()


@pytest.mark.parametrize("inner_prec", ["f64", "f32", "bf16"])
def test_mb_random_sources_vs_oracle(ctx, inner_prec):
    from paper_2211_06902_amd import dd

    L = (16, 8, 8, 16)
    kappa = 0.1365
    nf = 3
    U, boxes, blk, inner, bl = _setup(ctx, L, [[8, 8], [8], [8], [8, 8]], 1, nf, 77)
    g = ctx.load_gauge(blk, _dev(U), "bf16" if inner_prec == "bf16" else "f32")
    u = roots.mb_roots(2 * nf, 0.5)[:nf]
    chi = synth.gaussian_complex((nf, blk.total_bnd_sites, 4, 3), 78)
    xi = synth.gaussian_complex((nf, blk.total_sites, 4, 3), 79)
    S, tot, info, st = ctx.multiboson_action(blk, g, kappa, u, _dev(chi), _dev(xi),
                                             params=dd.solve_params(inner_prec=inner_prec))
    assert st == dd.DD_OK
    S_or, tot_or = mb.mb_local_action(L, -1, kappa, U, boxes, inner, u, chi, xi, tol=1e-12)
    assert np.max(np.abs(S.cpu().numpy() - S_or) / S_or) <= 1e-9
    assert abs(tot - tot_or) <= 1e-9 * tot_or


@pytest.mark.parametrize("fields_per_solve", [1, 2])
def test_mb_fields_in_groups_match_one_solve(ctx, fields_per_solve):
    """Solving the fields a few at a time (as on large lattices) gives the same action."""
    from paper_2211_06902_amd import dd

    L = (16, 8, 8, 16)
    kappa = 0.1365
    nf = 5
    U, boxes, blk, inner, bl = _setup(ctx, L, [[8, 8], [8], [8], [8, 8]], 1, nf, 81)
    g = ctx.load_gauge(blk, _dev(U), "f32")
    u = dd.mb_roots(2 * nf, 0.5)
    chi = _dev(synth.gaussian_complex((nf, blk.total_bnd_sites, 4, 3), 82))
    xi = _dev(synth.gaussian_complex((nf, blk.total_sites, 4, 3), 83))
    S1, tot1, i1, s1 = ctx.multiboson_action(blk, g, kappa, u, chi, xi)
    try:
        ctx.tune_set(dd.TUNE_MB_FIELDS, fields_per_solve)
        S2, tot2, i2, s2 = ctx.multiboson_action(blk, g, kappa, u, chi, xi)
    finally:
        ctx.tune_set(dd.TUNE_MB_FIELDS, 0)
    assert s1 == dd.DD_OK and s2 == dd.DD_OK
    assert np.all(i2["true_relres"] <= 1e-10)
    S1, S2 = S1.cpu().numpy(), S2.cpu().numpy()
    assert np.max(np.abs(S2 - S1) / S1) <= 1e-9
    assert abs(tot2 - tot1) <= 1e-9 * tot1
