"""Pins of the oracle's block solves: dense LU, even-odd determinant identity,
Neumann series, manufactured solutions."""
import numpy as np
import pytest

import synth
from oracle import dense, geometry, wilson


@pytest.fixture(scope="module")
def c1_field():
    # the 4^4 plain-FP64 configuration: kappa 0.12, eps 0.5, antiperiodic time
    L = (4, 4, 4, 4)
    return L, synth.gauge_field(L, 0.5, 1101)


def test_solve_matches_dense_lu(c1_field):
    L, U = c1_field
    kappa = 0.12
    for box in [((0, 0, 0, 0), (2, 2, 2, 2)), ((3, 3, 3, 3), (2, 2, 2, 2)), ((1, 0, 2, 0), (2, 4, 2, 2))]:
        S = int(np.prod(box[1]))
        b = synth.gaussian_complex((S, 4, 3), 17)
        x, it, rel = wilson.solve_box(L, -1, kappa, U, *box, b, tol=1e-13)
        M = dense.dense_dirac_box(L, -1, kappa, U, *box)
        xd = np.linalg.solve(M, b.reshape(-1)).reshape(S, 4, 3)
        assert rel <= 1e-13
        assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)


def test_even_odd_determinant(c1_field):
    """det D_Lambda = det(1 - kappa^2 H_eo H_oe) (diagonal blocks are the identity)."""
    L, U = c1_field
    kappa = 0.12
    box = ((1, 1, 1, 1), (2, 2, 2, 2))
    M = dense.dense_dirac_box(L, -1, kappa, U, *box)
    par = geometry.box_parity(L, *box)
    ev, od = np.nonzero(par == 0)[0], np.nonzero(par == 1)[0]
    Dee, Deo = dense.sub(M, ev), dense.sub(M, ev, od)
    Doe, Doo = dense.sub(M, od, ev), dense.sub(M, od)
    assert np.allclose(Dee, np.eye(Dee.shape[0]), atol=0)
    assert np.allclose(Doo, np.eye(Doo.shape[0]), atol=0)
    Heo, Hoe = -Deo / kappa, -Doe / kappa
    Dhat = np.eye(Dee.shape[0]) - kappa**2 * Heo @ Hoe
    assert abs(dense.logdet(M) - dense.logdet(Dhat)) < 1e-10
    # gamma_5-hermiticity makes the determinant real
    assert abs(np.sin(dense.logdet(M).imag)) < 1e-10


def test_neumann_series(c1_field):
    """kappa < 1/8 and |H| <= 8: x = sum_n (kappa H)^n b, error <= (8k)^(n+1)/(1-8k) |b|."""
    L, U = c1_field
    kappa = 0.12
    box = ((0, 2, 0, 2), (2, 2, 4, 2))
    S = int(np.prod(box[1]))
    b = synth.gaussian_complex((S, 4, 3), 23)
    x, _, _ = wilson.solve_box(L, -1, kappa, U, *box, b, tol=1e-13)
    term = b.copy()
    acc = b.copy()
    nterms = 400
    for _ in range(nterms):
        term = kappa * wilson.hop_box(L, -1, U, *box, term)
        acc += term
    bound = (8 * kappa) ** (nterms + 1) / (1 - 8 * kappa) * np.linalg.norm(b)
    assert np.linalg.norm(acc - x) <= bound + 1e-11 * np.linalg.norm(x)


def test_solve_many_manufactured_solution():
    """b = D_Lambda x* for known x*: solve_many returns x* and a true residual <= tol."""
    L = (8, 8, 8, 8)
    kappa = 0.1355
    U = synth.gauge_field(L, 0.3, 2101)
    boxes = geometry.tile_boxes(L, [[4, 4]] * 4)[:5]
    nrhs = 2
    S = [int(np.prod(bx[4:])) for bx in boxes]
    xs = synth.gaussian_complex((nrhs, sum(S), 4, 3), 2102)
    b = np.empty_like(xs)
    off = 0
    for k, bx in enumerate(boxes):
        for r in range(nrhs):
            b[r, off:off + S[k]] = wilson.dirac_box(L, -1, kappa, U, bx[:4], bx[4:], xs[r, off:off + S[k]])
        off += S[k]
    x, iters, rel, fails = wilson.solve_many(L, -1, kappa, U, boxes, b, tol=1e-12)
    assert fails == 0
    assert np.all(rel <= 1e-12)
    assert np.all(iters > 0)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_solve_zero_source():
    L = (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.5, 1101)
    x, it, rel = wilson.solve_box(L, -1, 0.12, U, (0, 0, 0, 0), (2, 2, 2, 2), np.zeros((16, 4, 3), complex))
    assert it == 0 and rel == 0.0 and np.all(x == 0)
