"""GPU parity of the frame domains Phi_1^a = Omega_0^a minus Lambda_0^a (dd_make_frames): the
operator D_{Phi_1^a} (principal sub-matrix of D on the frame; the hole decoupled as the identity)
and the frame solves D_{Phi_1^a}^{-1} b, against the oracle (oracle.wilson.dirac_frame, dense LU).

Geometries: paper-mode blocks b = 4, d = 2 on 12^4 (8^4 boxes with 4^4 holes, some wrapping; the
x0-walk kernels run with the hole's hops dropped) and b = 2, d = 1 on 6 x 6 x 6 x 4 (4^4 boxes, the
last direction spanning the lattice, 2 x 2 x 2 x 4 holes; small enough for dense LU)."""
import numpy as np
import pytest

import synth
from oracle import dense, wilson

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


def _frames(ctx, case):
    if case == "paper_4d":
        L, bd = (12, 12, 12, 12), [4, 2] * 4
    else:
        L, bd = (6, 6, 6, 4), [2, 1, 2, 1, 2, 1, 0, 0]
    blk = ctx.make_blocks_paper(L, -1, bd)
    fr = ctx.make_frames(blk)
    blk.close()
    return L, fr


@pytest.mark.parametrize("case", ["paper_4d", "paper_3d"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_frame_operator_matches_oracle(ctx, case, prec):
    L, fr = _frames(ctx, case)
    kappa = 0.1355
    U = synth.gauge_field(L, 0.3, 951)
    g = ctx.load_gauge(fr, _dev(U), "f32")
    bx = fr.tables()[0]
    S = np.prod(bx[:, 4:8], axis=1)
    off = np.concatenate([[0], np.cumsum(S)])
    x = synth.gaussian_complex((2, fr.total_sites, 4, 3), 952)
    y = ctx.apply_D_block(fr, g, kappa, prec, _dev(x)).cpu().numpy()
    tol = 1e-12 if prec == "f64" else 1e-5
    for k, b in enumerate(bx):
        m = wilson.frame_mask(b[4:8], b[8:12], b[12:16])
        sl = slice(off[k], off[k + 1])
        for r in range(2):
            ref = wilson.dirac_frame(L, -1, kappa, U, b[:4], b[4:8], b[8:12], b[12:16], x[r, sl])
            got = y[r, sl]
            assert np.linalg.norm(got[m] - ref[m]) <= tol * np.linalg.norm(ref[m]), (k, r)
            # the hole is decoupled: D acts as the identity there
            assert np.linalg.norm(got[~m] - x[r, sl][~m]) <= tol * np.linalg.norm(x[r, sl][~m])
    g.close()
    fr.close()


@pytest.mark.parametrize("case", ["paper_4d", "paper_3d"])
def test_frame_solves_match_oracle(ctx, case):
    from paper_2211_06902_amd import dd

    L, fr = _frames(ctx, case)
    kappa = 0.1355
    U = synth.gauge_field(L, 0.3, 961)
    g = ctx.load_gauge(fr, _dev(U), "f32")
    bx = fr.tables()[0]
    S = np.prod(bx[:, 4:8], axis=1)
    off = np.concatenate([[0], np.cumsum(S)])
    n_rhs = 3
    b = synth.gaussian_complex((n_rhs, fr.total_sites, 4, 3), 962)
    masks = [wilson.frame_mask(bb[4:8], bb[8:12], bb[12:16]) for bb in bx]
    for k in range(len(bx)):
        b[:, off[k]:off[k + 1]][:, ~masks[k]] = 0.0
    x, info, st = ctx.block_solve(fr, g, kappa, _dev(b), params=dd.solve_params(inner_prec="f32"))
    assert st == dd.DD_OK and np.all(info["true_relres"] <= TOL)
    x = x.cpu().numpy()
    for k, bb in enumerate(bx):
        sl = slice(off[k], off[k + 1])
        m = masks[k]
        for r in range(n_rhs):
            assert np.all(x[r, sl][~m] == 0)
            res = b[r, sl] - wilson.dirac_frame(L, -1, kappa, U, bb[:4], bb[4:8], bb[8:12], bb[12:16], x[r, sl])
            assert np.linalg.norm(res) <= TOL * np.linalg.norm(b[r, sl]), (k, r)
    if case == "paper_3d":
        # two frames against dense LU of D_Phi
        for k in (0, len(bx) - 1):
            bb = bx[k]
            m = masks[k]
            Mb = dense.dense_dirac_box(L, -1, kappa, U, bb[:4], bb[4:8])
            fi = dense.dof(np.nonzero(m)[0])
            Mf = Mb[np.ix_(fi, fi)]
            sl = slice(off[k], off[k + 1])
            for r in range(n_rhs):
                ref = np.linalg.solve(Mf, b[r, sl].reshape(-1)[fi])
                got = x[r, sl].reshape(-1)[fi]
                assert np.linalg.norm(got - ref) <= 1e-8 * np.linalg.norm(ref), (k, r)
    g.close()
    fr.close()
