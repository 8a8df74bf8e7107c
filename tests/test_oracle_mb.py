"""Pins of the oracle's multi-boson roots and block-local action."""
import numpy as np
import pytest

import synth
from oracle import geometry, mb, roots, wilson


@pytest.mark.parametrize("N,c", [(10, 0.5), (24, 0.5), (12, 0.3)])
def test_roots_solve_remainder(N, c):
    u = roots.mb_roots(N, c)
    z = 1 - u
    assert np.max(np.abs(1 - roots.remainder(N, c, z))) < 1e-9
    # conjugate pairs k <-> N+1-k
    assert np.allclose(u[::-1], np.conj(u), atol=1e-15)
    # z = 0 is the extra root of 1 - R that P_N divides out
    assert abs(1 - roots.remainder(N, c, 0.0)) < 1e-15


@pytest.mark.parametrize("N,c", [(10, 0.5), (24, 0.5)])
def test_polynomial_product_form(N, c):
    """P_N(w) = c_N prod_{k<=N/2} |w - z_k|^2 for real w (roots come in conjugate pairs)."""
    z = 1 - roots.mb_roots(N, c)
    cN = roots.leading_coeff(N, c)
    for w in [0.3, 0.9, 1.0, 1.4]:
        lhs = roots.poly_P(N, c, w)
        rhs = cN * np.prod(np.abs(w - z[: N // 2]) ** 2)
        assert abs(lhs - rhs) < 1e-10 * abs(rhs)
        assert abs(lhs.imag) < 1e-12 * abs(lhs)


def test_remainder_bound_on_interval():
    N, c = 10, 0.5
    w = np.linspace(1 - c, 1 + c, 1001)
    bound = 1 / np.real(roots.chebyshev_T(N + 1, np.asarray(1 / c)))
    assert np.max(np.abs(roots.remainder(N, c, w))) <= bound * (1 + 1e-12)
    # and P_N approximates 1/w there
    assert np.max(np.abs(roots.poly_P(N, c, w) * w - 1)) <= bound + 1e-14


def _tile_setup(L, nf, seed):
    U = synth.gauge_field(L, 0.3, seed)
    boxes = geometry.tile_boxes(L, [[4, 4]] * 4)[:3]
    inner = np.array([[1, 1, 1, 1, 2, 2, 2, 2]] * len(boxes))
    bl = mb.boundary_lists(L, boxes, inner)
    return U, boxes, inner, bl


def test_mb_action_closed_form():
    """xi = D_Omega eta with eta supported on dLambda0 gives S = sum_k |u_k chi_k + eta_k|^2."""
    L = (8, 8, 8, 8)
    kappa = 0.13
    nf = 3
    U, boxes, inner, bl = _tile_setup(L, nf, 5101)
    u = roots.mb_roots(2 * nf, 0.5)[:nf]
    nbd = sum(b.size for b in bl)
    S_tot = sum(int(np.prod(b[4:])) for b in boxes)
    chi = synth.gaussian_complex((nf, nbd, 4, 3), 5102)
    eta_b = synth.gaussian_complex((nf, nbd, 4, 3), 5103)
    xi = np.zeros((nf, S_tot, 4, 3), dtype=complex)
    expect = np.zeros(len(boxes))
    soff = boff = 0
    for b, bx in enumerate(boxes):
        Sb = int(np.prod(bx[4:]))
        for k in range(nf):
            eta = np.zeros((Sb, 4, 3), dtype=complex)
            eta[bl[b]] = eta_b[k, boff:boff + bl[b].size]
            xi[k, soff:soff + Sb] = wilson.dirac_box(L, -1, kappa, U, bx[:4], bx[4:], eta)
            expect[b] += np.sum(np.abs(u[k] * chi[k, boff:boff + bl[b].size] + eta_b[k, boff:boff + bl[b].size]) ** 2)
        soff += Sb
        boff += bl[b].size
    S, tot = mb.mb_local_action(L, -1, kappa, U, boxes, inner, u, chi, xi, tol=1e-13)
    assert np.max(np.abs(S - expect) / expect) < 1e-10
    assert abs(tot - expect.sum()) < 1e-10 * expect.sum()


def test_mb_action_zero_source_is_chi_norm():
    L = (8, 8, 8, 8)
    U, boxes, inner, bl = _tile_setup(L, 2, 77)
    u = np.array([0.3 + 0.4j, -0.2 + 0.1j])
    nbd = sum(b.size for b in bl)
    chi = synth.gaussian_complex((2, nbd, 4, 3), 8)
    xi = np.zeros((2, sum(int(np.prod(b[4:])) for b in boxes), 4, 3), dtype=complex)
    S, tot = mb.mb_local_action(L, -1, 0.12, U, boxes, inner, u, chi, xi)
    expect = sum(abs(u[k]) ** 2 * np.sum(np.abs(chi[k]) ** 2) for k in range(2))
    assert abs(tot - expect) < 1e-12 * expect
