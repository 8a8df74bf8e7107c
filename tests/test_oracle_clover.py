"""Pins of the oracle's clover (Sheikholeslami-Wohlert) term against mathematics, not against itself.

* an abelian SU(3)-diagonal field with uniform flux B = 2 pi n / L_1 in the (1, 2) plane, where every
  plaquette of that plane is exp(i lambda_c B) and all others are 1: Fhat_12 = i sin(lambda_c B) per
  colour and A = 1 - kappa c_sw sin(lambda_c B) sigma_12 in closed form (a wrong leaf orientation,
  a misplaced dagger or a wrong sigma fails it);
* A hermitian and commuting with gamma_5 (block diagonal in the chiral basis);
* gauge covariance A[U^Omega](x) = Omega(x) A[U](x) Omega(x)^+;
* gamma_5-hermiticity of the full operator;
* the box operator as the principal sub-matrix of the full one (A taken from the whole lattice);
* the even-odd determinant identity det D = det A_oo det A_ee det(1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe)
  of the Schur form the library solves, on a small box.
"""
import numpy as np
import pytest

import synth
from oracle import clover, dense, geometry, wilson

LAM = np.array([1.0, 1.0, -2.0])


def _abelian(L, n):
    """U_2(x) = diag(exp(i lambda B x_1)), the other links 1; B = 2 pi n / L_1."""
    V = int(np.prod(L))
    B = 2 * np.pi * n / L[1]
    U = np.zeros((V, 4, 3, 3), dtype=complex)
    U[:, :] = np.eye(3)
    x1 = geometry.coords(L)[:, 1]
    U[:, 2] = 0
    for c in range(3):
        U[:, 2, c, c] = np.exp(1j * LAM[c] * B * x1)
    return U, B


@pytest.mark.parametrize("n", [1, 2])
def test_uniform_abelian_flux_closed_form(n):
    L = (4, 6, 4, 2)
    kappa, csw = 0.13, 1.7
    U, B = _abelian(L, n)
    F = clover.field_strength(L, U)
    for k, plane in enumerate(clover.PLANES):
        expect = np.diag(1j * np.sin(LAM * B)) if plane == (1, 2) else np.zeros((3, 3))
        assert np.max(np.abs(F[:, k] - expect[None])) < 1e-14, plane
    A = clover.clover_matrix(L, U, kappa, csw)
    s12 = clover.sigma(1, 2)
    expect = np.eye(12) - kappa * csw * np.kron(s12, np.diag(np.sin(LAM * B)))
    assert np.max(np.abs(A - expect[None])) < 1e-14


def test_sigma_is_hermitian_and_chiral():
    g5 = wilson.gamma(4)
    for mu, nu in clover.PLANES:
        s = clover.sigma(mu, nu)
        assert np.allclose(s, s.conj().T, atol=1e-15)
        assert np.allclose(s @ g5, g5 @ s, atol=1e-15)
        # sigma_{mu nu} = i gamma_mu gamma_nu for mu != nu
        assert np.allclose(s, 1j * wilson.gamma(mu) @ wilson.gamma(nu), atol=1e-15)


@pytest.fixture(scope="module")
def small():
    L = (4, 4, 2, 4)
    U = synth.gauge_field(L, 0.5, 21)
    return L, U


def test_clover_hermitian_block_diagonal_and_free_field_unit(small):
    L, U = small
    A = clover.clover_matrix(L, U, 0.12, 1.3)
    assert np.max(np.abs(A - np.conj(np.swapaxes(A, 1, 2)))) < 1e-14
    G5 = np.kron(wilson.gamma(4), np.eye(3))
    assert np.max(np.abs(A @ G5 - G5 @ A)) < 1e-14
    assert np.max(np.abs(A - np.eye(12)[None])) > 1e-3  # a non-trivial field
    A1 = clover.clover_matrix(L, synth.unit_gauge(L), 0.12, 1.3)
    assert np.max(np.abs(A1 - np.eye(12)[None])) == 0.0


def test_clover_gauge_covariance(small):
    L, U = small
    V = U.shape[0]
    Om = synth.gauge_field(L, 2.0, 22)[:, 0]  # a random SU(3) per site
    Ug = np.empty_like(U)
    for mu in range(4):
        p = clover._shift(L, mu, 1)
        Ug[:, mu] = Om @ U[:, mu] @ np.conj(np.swapaxes(Om[p], 1, 2))
    A = clover.clover_matrix(L, U, 0.12, 1.3)
    Ag = clover.clover_matrix(L, Ug, 0.12, 1.3)
    Omb = np.einsum("ab,vcd->vacbd", np.eye(4), Om).reshape(V, 12, 12)
    assert np.max(np.abs(Ag - Omb @ A @ np.conj(np.swapaxes(Omb, 1, 2)))) < 1e-13


def test_full_operator_gamma5_hermitian(small):
    L, U = small
    kappa, csw = 0.12, 1.3
    rng = np.random.default_rng(5)
    V = U.shape[0]
    phi = rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))
    psi = rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))
    g5 = wilson.gamma(4)
    lhs = np.vdot(phi, np.einsum("st,vtc->vsc", g5, clover.dirac_clover_full(L, -1, kappa, csw, U, psi)))
    rhs = np.vdot(np.einsum("st,vtc->vsc", g5, clover.dirac_clover_full(L, -1, kappa, csw, U, phi)), psi)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


@pytest.mark.parametrize("box", [((0, 0, 0, 0), (2, 2, 2, 2)), ((3, 1, 0, 1), (2, 4, 2, 2))])
def test_clover_box_is_principal_submatrix(small, box):
    L, U = small
    kappa, csw = 0.12, 1.3
    V = U.shape[0]
    # dense full clover operator, column by column
    M = np.empty((12 * V, 12 * V), dtype=complex)
    e = np.zeros((V, 4, 3), dtype=complex)
    ef = e.reshape(-1)
    A = clover.clover_matrix(L, U, kappa, csw)
    for j in range(12 * V):
        ef[j] = 1.0
        M[:, j] = clover.dirac_clover_full(L, -1, kappa, csw, U, e, A=A).reshape(-1)
        ef[j] = 0.0
    sites = geometry.box_sites(L, *box)
    S = len(sites)
    rng = np.random.default_rng(6)
    psi = rng.standard_normal((S, 4, 3)) + 1j * rng.standard_normal((S, 4, 3))
    got = clover.dirac_clover_box(L, -1, kappa, csw, U, *box, psi)
    ref = (dense.sub(M, sites) @ psi.reshape(-1)).reshape(S, 4, 3)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_even_odd_determinant_identity(small):
    """det D_X = det A_oo det A_ee det(1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe) on a 2^4 box."""
    L, U = small
    kappa, csw = 0.12, 1.3
    box = ((1, 0, 0, 2), (2, 2, 2, 2))
    S = 16
    M = np.empty((12 * S, 12 * S), dtype=complex)
    e = np.zeros((S, 4, 3), dtype=complex)
    ef = e.reshape(-1)
    A = clover.clover_matrix(L, U, kappa, csw)
    for j in range(12 * S):
        ef[j] = 1.0
        M[:, j] = clover.dirac_clover_box(L, -1, kappa, csw, U, *box, e, A=A).reshape(-1)
        ef[j] = 0.0
    par = wilson.box_parity(L, *box)
    ev, od = dense.dof(np.nonzero(par == 0)[0]), dense.dof(np.nonzero(par == 1)[0])
    Aee, Aoo = M[np.ix_(ev, ev)], M[np.ix_(od, od)]
    Heo, Hoe = -M[np.ix_(ev, od)] / kappa, -M[np.ix_(od, ev)] / kappa
    Dp = np.eye(len(ev)) - kappa**2 * np.linalg.solve(Aee, Heo @ np.linalg.solve(Aoo, Hoe))
    lhs = dense.logdet(M)
    rhs = dense.logdet(Aoo) + dense.logdet(Aee) + dense.logdet(Dp)
    assert abs(lhs.real - rhs.real) < 1e-11
    assert abs(np.exp(1j * (lhs.imag - rhs.imag)) - 1) < 1e-11
    # the even-even and odd-odd blocks are the clover term alone (site-diagonal)
    sites = geometry.box_sites(L, *box)
    for i in np.nonzero(par == 0)[0][:3]:
        blk = M[12 * i:12 * i + 12, 12 * i:12 * i + 12]
        assert np.max(np.abs(blk - A[sites[i]])) < 1e-14
