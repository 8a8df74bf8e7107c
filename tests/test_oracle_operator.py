"""Pins of the oracle's Wilson-Dirac operator against mathematics.

Each test checks the oracle against something other than itself: Clifford
algebra, the free-field plane-wave closed form and momentum-space determinant,
gamma_5-hermiticity, gauge covariance, and the Dirichlet restriction as a
principal sub-matrix of the full operator.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import dense, geometry, wilson


def test_gamma_clifford_and_gamma5():
    g = [wilson.gamma(mu) for mu in range(4)]
    eye = np.eye(4)
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)  # hermitian
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2 * eye * (mu == nu), atol=0)
    g5 = wilson.gamma(4)
    assert np.allclose(g5, g[0] @ g[1] @ g[2] @ g[3], atol=0)
    assert np.allclose(g5, np.diag([1, 1, -1, -1]), atol=0)
    for mu in range(4):
        assert np.allclose(g5 @ g[mu] + g[mu] @ g5, 0, atol=0)


def _plane_wave(L, n, u):
    """psi(x) = exp(i p.x) u, p_k = 2 pi n_k / L_k (space), p_0 = (2 n_0 + 1) pi / L_0."""
    p = np.array([(2 * n[0] + 1) * np.pi / L[0]] + [2 * np.pi * n[k] / L[k] for k in (1, 2, 3)])
    x = geometry.coords(L).astype(np.float64)
    ph = np.exp(1j * (x @ p))
    return p, ph[:, None, None] * u[None, :, :]


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 2, 0, 3), (2, 1, 3, 1), (3, 3, 1, 0)])
def test_free_field_plane_wave_closed_form(n):
    """D e^{ipx}u = [1 - 2 kappa sum cos p + 2 i kappa sum gamma_mu sin p] e^{ipx}u (U = 1)."""
    L = (6, 4, 4, 4)
    kappa = 0.137
    U = synth.unit_gauge(L)
    rng = np.random.default_rng(7)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    p, psi = _plane_wave(L, n, u)
    out = wilson.dirac_full(L, -1, kappa, U, psi)
    M = (1 - 2 * kappa * np.sum(np.cos(p))) * np.eye(4, dtype=complex)
    for mu in range(4):
        M = M + 2j * kappa * np.sin(p[mu]) * wilson.gamma(mu)
    expect = np.einsum("st,vtc->vsc", M, psi)
    assert np.max(np.abs(out - expect)) < 1e-13


def test_free_field_determinant_momentum_space():
    """det D(U=1) = prod_p [(1 - 2k sum cos p)^2 + 4k^2 sum sin^2 p]^6 on a 2x2x2x4 lattice."""
    L = (4, 2, 2, 2)
    kappa = 0.11
    U = synth.unit_gauge(L)
    M = dense.dense_dirac_full(L, -1, kappa, U)
    ld = dense.logdet(M)
    expect = 0.0
    for n in itertools.product(range(L[0]), range(L[1]), range(L[2]), range(L[3])):
        p = np.array([(2 * n[0] + 1) * np.pi / L[0]] + [2 * np.pi * n[k] / L[k] for k in (1, 2, 3)])
        A = 1 - 2 * kappa * np.sum(np.cos(p))
        B2 = 4 * kappa**2 * np.sum(np.sin(p) ** 2)
        expect += 6 * np.log(A * A + B2)
    assert abs(ld.real - expect) < 1e-10
    assert abs(np.sin(ld.imag)) < 1e-10  # det real and positive here


def test_periodic_time_changes_momenta():
    """With tbc=+1 the zero mode p=0 gives D u = (1 - 8 kappa) u."""
    L = (4, 4, 4, 4)
    kappa = 0.1
    U = synth.unit_gauge(L)
    u = np.ones((4, 3), dtype=complex)
    psi = np.broadcast_to(u, (256, 4, 3)).copy()
    out = wilson.dirac_full(L, +1, kappa, U, psi)
    assert np.max(np.abs(out - (1 - 8 * kappa) * psi)) < 1e-14
    out_ap = wilson.dirac_full(L, -1, kappa, U, psi)
    assert np.max(np.abs(out_ap - (1 - 8 * kappa) * psi)) > 0.1


BOXES = [
    ((0, 0, 0, 0), (2, 2, 2, 2)),
    ((3, 1, 0, 1), (2, 2, 2, 2)),   # wraps across the time edge: carries the sign
    ((1, 0, 0, 0), (4, 2, 1, 2)),   # spans the full time extent: keeps the wrap link
    ((2, 3, 1, 0), (3, 2, 2, 2)),   # odd extent, wraps in direction 1
    ((0, 0, 0, 0), (4, 4, 2, 2)),   # the whole lattice
]


@pytest.fixture(scope="module")
def small_lattice():
    L = (4, 4, 2, 2)
    U = synth.gauge_field(L, 0.5, 11)
    return L, U


@pytest.mark.parametrize("box", BOXES)
def test_box_is_principal_submatrix(small_lattice, box):
    L, U = small_lattice
    kappa = 0.12
    M = dense.dense_dirac_full(L, -1, kappa, U)
    sites = geometry.box_sites(L, *box)
    Mb = dense.dense_dirac_box(L, -1, kappa, U, *box)
    assert np.max(np.abs(Mb - dense.sub(M, sites))) < 1e-15


@pytest.mark.parametrize("box", BOXES)
def test_gamma5_hermiticity(small_lattice, box):
    L, U = small_lattice
    kappa = 0.13
    S = int(np.prod(box[1]))
    phi = synth.gaussian_complex((S, 4, 3), 1)
    psi = synth.gaussian_complex((S, 4, 3), 2)
    g5 = np.diag([1.0, 1.0, -1.0, -1.0])
    lhs = np.vdot(phi, np.einsum("st,vtc->vsc", g5, wilson.dirac_box(L, -1, kappa, U, *box, psi)))
    rhs = np.vdot(np.einsum("st,vtc->vsc", g5, wilson.dirac_box(L, -1, kappa, U, *box, phi)), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("box", BOXES)
def test_gauge_covariance(small_lattice, box):
    """D_Lambda[U^Omega](Omega psi) = Omega D_Lambda[U] psi."""
    L, U = small_lattice
    kappa = 0.125
    V = int(np.prod(L))
    Om = synth.random_su3(V, 99)
    nbr = geometry.neighbours(L)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[:, mu] = Om @ U[:, mu] @ np.conj(np.swapaxes(Om[nbr[:, 2 * mu]], 1, 2))
    sites = geometry.box_sites(L, *box)
    S = sites.size
    psi = synth.gaussian_complex((S, 4, 3), 5)
    Ob = Om[sites]
    psi_g = np.einsum("vab,vsb->vsa", Ob, psi)
    lhs = wilson.dirac_box(L, -1, kappa, Ug, *box, psi_g)
    rhs = np.einsum("vab,vsb->vsa", Ob, wilson.dirac_box(L, -1, kappa, U, *box, psi))
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_kappa_zero_is_identity(small_lattice):
    L, U = small_lattice
    psi = synth.gaussian_complex((64, 4, 3), 3)
    assert np.array_equal(wilson.dirac_full(L, -1, 0.0, U, psi), psi)


def test_hop_connects_opposite_parity(small_lattice):
    L, U = small_lattice
    box = ((1, 1, 0, 0), (2, 4, 2, 2))
    par = wilson.box_parity(L, *box)
    assert np.array_equal(par, geometry.box_parity(L, *box))
    psi = synth.gaussian_complex((par.size, 4, 3), 4)
    psi[par == 1] = 0
    h = wilson.hop_box(L, -1, U, *box, psi)
    assert np.max(np.abs(h[par == 0])) == 0.0
    assert np.max(np.abs(h[par == 1])) > 0.0


@pytest.mark.parametrize("frame", [
    ((0, 0, 0, 0), (3, 3, 3, 2), (1, 1, 1, 0), (1, 1, 1, 2)),  # hole spans the box in direction 3
    ((3, 2, 1, 1), (4, 3, 2, 2), (1, 0, 0, 0), (2, 2, 1, 1)),  # spans the time extent, wraps in 1
])
def test_frame_is_principal_submatrix(frame):
    """D_Phi on a frame (box minus hole) is the full operator restricted to the frame's sites."""
    L, kappa = (4, 4, 4, 2), 0.13
    U = synth.gauge_field(L, 0.5, 17)
    origin, extent, ho, he = frame
    M = dense.dense_dirac_full(L, -1, kappa, U)
    sites = geometry.box_sites(L, origin, extent)
    m = wilson.frame_mask(extent, ho, he)
    assert 0 < m.sum() < len(m)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((len(m), 4, 3)) + 1j * rng.standard_normal((len(m), 4, 3))
    psi[~m] = 0
    got = wilson.dirac_frame(L, -1, kappa, U, origin, extent, ho, he, psi)
    ref = (dense.sub(M, sites[m]) @ psi[m].reshape(-1)).reshape(-1, 4, 3)
    assert np.max(np.abs(got[m] - ref)) < 1e-13
    assert np.all(got[~m] == 0)
