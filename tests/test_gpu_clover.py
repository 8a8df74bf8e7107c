"""GPU parity of the clover (Sheikholeslami-Wohlert) operator (dd_gauge_set_clover) against the oracle
(oracle.clover: the textbook term, pinned in test_oracle_clover.py).

* D_Lambda with the clover term (FP64 <= 1e-12, FP32 <= 1e-5 relative per block and rhs), on 4^4
  tiles of an 8^4 lattice and on the same tiling shifted by one site (blocks that wrap, including the
  antiperiodic time edge): A(x) of the whole lattice at every block site.
* Block solves (FP64 and FP32 inner even-odd BiCGStab on 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe inside
  FP64 defect correction), with the one-kernel Dhat walk (FP32 inner: A_oo^-1 on the intermediate in
  LDS, A_ee^-1 in the epilogue), two x0-walk hops, and the chunked hop kernel: every pair's true
  residual with the oracle's clover operator <= 1e-10, and two blocks' solutions against dense LU.
* Persistent GMRES with the term (FP64, FP32, BF16-link inner) against the same references.
* c_sw = 0 gives back the Wilson operator bit for bit; a kappa other than the clover term's, and GMRES
  without the walking hops, are refused (the log-determinants with the term are compared in
  test_gpu_logdet.py).
"""
import numpy as np
import pytest

import synth
from oracle import clover, geometry

pytestmark = pytest.mark.gpu

L = (8, 8, 8, 8)
KAPPA, CSW = 0.13, 1.6


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_06902_amd import dd

    c = dd.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def field():
    U = synth.gauge_field(L, 0.3, 4401)
    A = clover.clover_matrix(L, U, KAPPA, CSW)
    return U, A


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _boxes(shift):
    return geometry.tile_boxes(L, [[4, 4]] * 4, shift=(1, 1, 1, 1) if shift else (0, 0, 0, 0))


def _offsets(boxes):
    S = np.prod(boxes[:, 4:8], axis=1)
    return np.concatenate([[0], np.cumsum(S)])


@pytest.mark.parametrize("shift", [False, True])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_clover_operator_matches_oracle(ctx, field, shift, prec):
    U, A = field
    boxes = _boxes(shift)
    off = _offsets(boxes)
    blk = ctx.make_blocks_boxes(L, -1, boxes)
    g = ctx.load_gauge(blk, _dev(U), "f32").set_clover(_dev(U), KAPPA, CSW)
    x = synth.gaussian_complex((2, blk.total_sites, 4, 3), 4402)
    y = ctx.apply_D_block(blk, g, KAPPA, prec, _dev(x)).cpu().numpy()
    tol = 1e-12 if prec == "f64" else 1e-5
    for k, b in enumerate(boxes):
        sl = slice(off[k], off[k + 1])
        for r in range(2):
            ref = clover.dirac_clover_box(L, -1, KAPPA, CSW, U, b[:4], b[4:8], x[r, sl], A=A)
            assert np.linalg.norm(y[r, sl] - ref) <= tol * np.linalg.norm(ref), (k, r)
    if prec == "f64":
        # the no-alloc entry point takes the same path
        y2 = ctx.apply_D_block_noalloc(blk, g, KAPPA, prec, _dev(x), _dev(np.zeros_like(x))).cpu().numpy()
        assert np.array_equal(y, y2)
    g.close()
    blk.close()


def test_clover_off_is_wilson_bit_for_bit(ctx, field):
    U, _ = field
    boxes = _boxes(False)
    blk = ctx.make_blocks_boxes(L, -1, boxes)
    g = ctx.load_gauge(blk, _dev(U), "f32")
    x = _dev(synth.gaussian_complex((1, blk.total_sites, 4, 3), 4403))
    y0 = ctx.apply_D_block(blk, g, KAPPA, "f64", x).cpu().numpy()
    g.set_clover(_dev(U), KAPPA, CSW)
    y1 = ctx.apply_D_block(blk, g, KAPPA, "f64", x).cpu().numpy()
    assert np.max(np.abs(y1 - y0)) > 1e-3
    g.set_clover(None, KAPPA, 0.0)
    y2 = ctx.apply_D_block(blk, g, KAPPA, "f64", x).cpu().numpy()
    assert np.array_equal(y0, y2)
    g.close()
    blk.close()


def _relres(U, A, b, x, box):
    r = b - clover.dirac_clover_box(L, -1, KAPPA, CSW, U, box[:4], box[4:8], x, A=A)
    return np.linalg.norm(r) / np.linalg.norm(b)


@pytest.mark.parametrize("mode", ["dhat", "twohop", "chunked"])
@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_clover_solves_match_oracle(ctx, field, inner, mode):
    from paper_2211_06902_amd import dd

    U, A = field
    boxes = _boxes(True)
    off = _offsets(boxes)
    blk = ctx.make_blocks_boxes(L, -1, boxes)
    g = ctx.load_gauge(blk, _dev(U), "f32").set_clover(_dev(U), KAPPA, CSW)
    n_rhs = 3
    b = synth.gaussian_complex((n_rhs, blk.total_sites, 4, 3), 4404)
    try:
        # dhat: the one-kernel Dhat walk (FP32 inner); twohop: two walk hops per Dhat; chunked: the
        # walk off, every hop (the clover ones included) in the chunked kernel
        ctx.tune_set(dd.TUNE_DHAT_WALK, -1 if mode == "twohop" else 0)
        ctx.tune_set(dd.TUNE_HOP_WALK, -1 if mode == "chunked" else 0)
        x, info, st = ctx.block_solve(blk, g, KAPPA, _dev(b), params=dd.solve_params(inner_prec=inner))
    finally:
        ctx.tune_set(dd.TUNE_HOP_WALK, 0)
        ctx.tune_set(dd.TUNE_DHAT_WALK, 0)
    assert st == dd.DD_OK and np.all(info["true_relres"] <= 1e-10)
    x = x.cpu().numpy()
    for k, bx in enumerate(boxes):
        sl = slice(off[k], off[k + 1])
        for r in range(n_rhs):
            assert _relres(U, A, b[r, sl], x[r, sl], bx) <= 1e-10, (k, r)
    # two blocks against dense LU of the clover D_Lambda
    for k in (0, len(boxes) - 1):
        bx = boxes[k]
        S = int(np.prod(bx[4:8]))
        M = np.empty((12 * S, 12 * S), dtype=complex)
        e = np.zeros((S, 4, 3), dtype=complex)
        ef = e.reshape(-1)
        for j in range(12 * S):
            ef[j] = 1.0
            M[:, j] = clover.dirac_clover_box(L, -1, KAPPA, CSW, U, bx[:4], bx[4:8], e, A=A).reshape(-1)
            ef[j] = 0.0
        sl = slice(off[k], off[k + 1])
        for r in range(n_rhs):
            ref = np.linalg.solve(M, b[r, sl].reshape(-1))
            got = x[r, sl].reshape(-1)
            assert np.linalg.norm(got - ref) <= 1e-8 * np.linalg.norm(ref), (k, r)
    g.close()
    blk.close()


def test_clover_refusals(ctx, field):
    from paper_2211_06902_amd import dd

    U, _ = field
    boxes = _boxes(False)
    blk = ctx.make_blocks_boxes(L, -1, boxes)
    g = ctx.load_gauge(blk, _dev(U), "f32").set_clover(_dev(U), KAPPA, CSW)
    x = _dev(synth.gaussian_complex((1, blk.total_sites, 4, 3), 4405))
    with pytest.raises(dd.DDError):
        ctx.apply_D_block(blk, g, KAPPA + 0.01, "f64", x)
    try:  # GMRES takes the clover term only with the walking hops
        ctx.tune_set(dd.TUNE_HOP_WALK, -1)
        with pytest.raises(dd.DDError):
            ctx.block_solve(blk, g, KAPPA, x, params=dd.solve_params(method=dd.GMRES, inner_prec="f32"))
    finally:
        ctx.tune_set(dd.TUNE_HOP_WALK, 0)
    g.close()
    blk.close()


@pytest.mark.parametrize("inner", ["f64", "f32", "bf16"])
def test_clover_gmres_solves_match_oracle(ctx, field, inner):
    """Persistent GMRES(16) on 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe (A^-1 inside its walking hops; FP32
    spinors: the one-pass Dhat with A_oo^-1 on the intermediate), FP64 defect correction: every pair's
    true residual on the oracle's clover operator <= 1e-10, one block against dense LU."""
    from paper_2211_06902_amd import dd

    U, A = field
    boxes = _boxes(True)
    off = _offsets(boxes)
    blk = ctx.make_blocks_boxes(L, -1, boxes)
    g = ctx.load_gauge(blk, _dev(U), "bf16" if inner == "bf16" else "f32").set_clover(_dev(U), KAPPA, CSW)
    n_rhs = 2
    b = synth.gaussian_complex((n_rhs, blk.total_sites, 4, 3), 4406)
    x, info, st = ctx.block_solve(blk, g, KAPPA, _dev(b), params=dd.solve_params(method=dd.GMRES, inner_prec=inner))
    assert st == dd.DD_OK and np.all(info["true_relres"] <= 1e-10)
    x = x.cpu().numpy()
    for k, bx in enumerate(boxes):
        sl = slice(off[k], off[k + 1])
        for r in range(n_rhs):
            assert _relres(U, A, b[r, sl], x[r, sl], bx) <= 1e-10, (k, r)
    bx = boxes[0]
    S = int(np.prod(bx[4:8]))
    M = np.empty((12 * S, 12 * S), dtype=complex)
    e = np.zeros((S, 4, 3), dtype=complex)
    ef = e.reshape(-1)
    for j in range(12 * S):
        ef[j] = 1.0
        M[:, j] = clover.dirac_clover_box(L, -1, KAPPA, CSW, U, bx[:4], bx[4:8], e, A=A).reshape(-1)
        ef[j] = 0.0
    for r in range(n_rhs):
        ref = np.linalg.solve(M, b[r, off[0]:off[1]].reshape(-1))
        assert np.linalg.norm(x[r, off[0]:off[1]].reshape(-1) - ref) <= 1e-8 * np.linalg.norm(ref), r
    g.close()
    blk.close()
