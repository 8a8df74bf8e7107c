"""GPU parity of the multi-boson exterior source (dd_mb_exterior_source) and of the block-local
action of eq. (localMB) from the multi-boson fields alone, against the oracle (oracle/mb.py).

Geometries: paper-mode framed blocks (b = 4, d = 2 in every direction of a 12^4 lattice: 16
overlapping Omega of 8^4, some wrapping around the lattice; and decomposed in two directions
only), and 8^4 tiles with an inner box of 6^4 (the benchmark blocks) on a 16^4 lattice.
The source is FP64 arithmetic on FP64 links (a few products per site): compared to 1e-13.
"""
import numpy as np
import pytest

import synth
from oracle import mb

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


def _blocks(ctx, case):
    if case == "paper_4d":
        L = (12, 12, 12, 12)
        return L, ctx.make_blocks_paper(L, -1, [4, 2] * 4)
    if case == "paper_2d":
        L = (12, 12, 8, 8)
        return L, ctx.make_blocks_paper(L, -1, [4, 2, 4, 2, 0, 0, 0, 0])
    L = (16, 16, 16, 16)
    return L, ctx.make_blocks(L, -1, [[8, 8]] * 4, inner_d=1)


@pytest.mark.parametrize("case", ["paper_4d", "paper_2d", "tiles_inner"])
def test_exterior_source_matches_oracle(ctx, case):
    L, blk = _blocks(ctx, case)
    kappa = 0.1365
    U = synth.gauge_field(L, 0.3, 901)
    g = ctx.load_gauge(blk, _dev(U), "f32")
    bx = blk.tables()[0]
    nf = 3
    V = int(np.prod(L))
    chi = synth.gaussian_complex((nf, V, 4, 3), 902)
    xi0 = synth.gaussian_complex((nf, blk.total_sites, 4, 3), 903)
    chi_d = _dev(chi)
    for parts, name in ((1, "dPi1"), (2, "dLam0"), (3, "all")):
        xi = ctx.mb_exterior_source(blk, g, kappa, chi_d, _dev(xi0), parts=parts).cpu().numpy()
        ref = mb.exterior_source(L, -1, kappa, U, bx[:, :8], bx[:, 8:16], chi, name)
        # tiles with inner boxes do not overlap: no other block's dLambda_0 is outside a box
        assert np.abs(ref).max() > 0 or (case == "tiles_inner" and name == "dLam0")
        err = np.abs((xi - xi0) - ref).max()
        assert err <= 1e-13 * np.abs(ref).max(), (parts, err)
    g.close()
    blk.close()


@pytest.mark.parametrize("inner_prec", ["f64", "f32"])
def test_mb_action_from_chi_alone(ctx, inner_prec):
    """S^a of eq. (localMB) from chi alone: the exterior source of the whole dPi, then the
    D_Omega^{-1} solves and the boundary norms of dd_multiboson_action, against the oracle."""
    import torch

    from paper_2211_06902_amd import dd

    L, blk = _blocks(ctx, "paper_4d")
    kappa = 0.1365
    U = synth.gauge_field(L, 0.3, 911)
    g = ctx.load_gauge(blk, _dev(U), "f32")
    bx, sites, _, bnd = blk.tables()
    nf = 3
    V = int(np.prod(L))
    chi = synth.gaussian_complex((nf, V, 4, 3), 912)
    u = dd.mb_roots(2 * nf, 0.5)
    chi_d = _dev(chi)
    xi = torch.zeros((nf, blk.total_sites, 4, 3), dtype=torch.complex128, device="cuda")
    ctx.mb_exterior_source(blk, g, kappa, chi_d, xi, parts=3)
    # chi on each dLambda_0^a, in the layout of dd_multiboson_action (argument marshalling)
    soff = np.concatenate([[0], np.cumsum(np.prod(bx[:, 4:8], axis=1))])
    nb_per = [len(mb.boundary_lists(L, bx[k:k + 1, :8], bx[k:k + 1, 8:16])[0]) for k in range(blk.n_blocks)]
    boff = np.concatenate([[0], np.cumsum(nb_per)])
    gsite = np.concatenate([sites[soff[k] + bnd[boff[k]:boff[k + 1]]] for k in range(blk.n_blocks)])
    chib = chi_d[:, torch.from_numpy(gsite).cuda()].contiguous()
    S, tot, info, st = ctx.multiboson_action(blk, g, kappa, u, chib, xi, params=dd.solve_params(inner_prec=inner_prec))
    assert st == dd.DD_OK and np.all(info["true_relres"] <= 1e-10)
    S_or, tot_or = mb.mb_local_action_from_chi(L, -1, kappa, U, bx[:, :8], bx[:, 8:16], u, chi)
    S = S.cpu().numpy()
    assert np.max(np.abs(S - S_or) / S_or) <= 1e-9
    assert abs(tot - tot_or) <= 1e-9 * tot_or
    g.close()
    blk.close()
