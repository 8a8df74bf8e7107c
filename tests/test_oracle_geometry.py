"""Pins of the oracle's domain geometry and of the block factorisation of det D.

Set properties the derivation of Section 3 relies on are checked directly,
and the determinant identities of Section 3 are checked by dense LU on tiny
lattices:
  * det D = det D_{Lambda0bar} det D_{Lambda1} det Dtilde_{dLambda0}   (first Schur step)
  * Dhat_{dLambda0^a} is the Schur complement of D_{Omega0^a}, so
    (D_{Omega0^a}^{-1}) restricted to dLambda0^a equals Dhat_{dLambda0^a}^{-1}
  * det D = det W1 det D_{Lambda1} prod_a det D_{Omega0^a} / prod_a det D_{Phi1^a}
    (eq. detD), with det W1 = det Dtilde / prod_a det Dhat_{dLambda0^a}
  * the one-dimensional special case with thick time slices.
"""
import numpy as np
import pytest

import synth
from oracle import dense, geometry


def test_tiling_partitions_lattice():
    L = (8, 4, 6, 4)
    boxes = geometry.tile_boxes(L, [[4, 4], [2, 2], [2, 4], [4]], shift=(1, 0, 3, 2))
    seen = np.zeros(int(np.prod(L)), dtype=int)
    for bx in boxes:
        seen[geometry.box_sites(L, bx[:4], bx[4:])] += 1
    assert np.all(seen == 1)
    # direction 3 fastest in the block order
    assert boxes.shape == (2 * 2 * 2 * 1, 8)
    assert list(boxes[0]) == [1, 0, 3, 2, 4, 2, 2, 4]
    assert list(boxes[1]) == [1, 0, 5, 2, 4, 2, 4, 4]


def test_eo_order():
    L = (4, 4, 4, 4)
    box = ((1, 2, 0, 3), (2, 2, 2, 2))
    perm, pos = geometry.box_eo_order(L, *box)
    par = geometry.box_parity(L, *box)
    assert np.all(par[perm[:8]] == 0) and np.all(par[perm[8:]] == 1)
    assert np.all(np.diff(perm[:8]) > 0) and np.all(np.diff(perm[8:]) > 0)
    assert np.array_equal(perm[pos], np.arange(16))


def test_inner_boundary_of_8x4_tile():
    """An 8^4 block with an inner 6^4 box: |dLambda0| = 6^4 - 4^4 = 1040."""
    L = (16, 16, 16, 16)
    box = np.array([8, 0, 8, 0, 8, 8, 8, 8])
    bl = geometry.inner_boundary_local(L, box, [1, 1, 1, 1], [6, 6, 6, 6])
    assert bl.size == 6**4 - 4**4
    y = np.indices((8, 8, 8, 8)).reshape(4, -1).T[bl]
    assert np.all((y >= 1) & (y <= 6))
    assert np.all(np.any((y == 1) | (y == 6), axis=1))


# The four tiny geometries: (lattice, per-direction (b, d) or None)
T1 = ((4, 4, 4, 4), [(1, 1)] * 4)
T2 = ((8, 2, 2, 2), [(3, 1), None, None, None])
T3 = ((8, 8, 2, 2), [(3, 1), (3, 1), None, None])
T4 = ((8, 4, 4, 4), [(3, 1), (1, 1), (1, 1), (1, 1)])


@pytest.mark.parametrize("geom", [T1, T2, T3, T4], ids=["T1", "T2", "T3", "T4"])
def test_domain_set_properties(geom):
    L, spec = geom
    P = geometry.PaperDomains(L, spec)
    nbr = P.nbr
    # dPi n Lambda0 = dLambda0
    assert np.array_equal(P.dPi & P.lam0, P.dlam0)
    # Lambda0bar has no neighbour in Lambda1
    assert not np.any(P.lam1[nbr[P.lam0bar]])
    for a in range(len(P.blocks)):
        # blocks are disjoint and not adjacent (Lambda0 disconnected)
        for b2 in range(a + 1, len(P.blocks)):
            assert not np.any(P.lam0_a[a] & P.lam0_a[b2])
            assert not np.any(P.lam0_a[b2][nbr[P.lam0_a[a]]])
        # frames lie in Lambda1; block bulk does not touch its frame
        assert not np.any(P.phi_a[a] & P.lam0)
        assert not np.any(P.phi_a[a][nbr[P.lam0bar_a[a]]])
        # exterior boundary of Omega0^a lies in dLambda0 u dPi1
        assert np.all((P.dlam0 | P.dPi1)[P.ext_omega_a[a]])


def test_T1_counts():
    """4^4 with b = d = 1: 16 single-site blocks at even coordinates, 3^4 framed boxes."""
    P = geometry.PaperDomains(*T1)
    assert len(P.blocks) == 16
    assert P.lam0.sum() == 16 and P.dlam0.sum() == 16 and P.lam0bar.sum() == 0
    # dPi: some coordinate even -> 256 - 2^4 sites; dPi1 removes the 16 blocks
    assert P.dPi.sum() == 240 and P.dPi1.sum() == 224
    assert all(o.sum() == 81 for o in P.omega_a) and all(f.sum() == 80 for f in P.phi_a)


def test_T4_counts():
    """8 x 4^3 with b = 3, d = 1 in time and b = d = 1 in space: 2 x 2^3 = 16 blocks of 3 x 1^3 sites
    (all on dLambda_0), 5 x 3^3 framed boxes; the inactive region is the rest of the 512 sites."""
    P = geometry.PaperDomains(*T4)
    assert len(P.blocks) == 16
    assert P.lam0.sum() == 48 and P.dlam0.sum() == 48 and P.lam0bar.sum() == 0
    assert P.lam1.sum() == 464 and P.dPi1.sum() == 432 and (P.lam1 & ~P.dPi1).sum() == 32
    assert all(o.sum() == 135 for o in P.omega_a) and all(f.sum() == 132 for f in P.phi_a)


def test_1d_frames_cover_lambda1_twice():
    """Thick time slices: dPi1 is empty and every Lambda1 site is in exactly two frames."""
    P = geometry.PaperDomains(*T2)
    assert P.dPi1.sum() == 0
    cover = np.sum(P.phi_a, axis=0)
    assert np.all(cover[P.lam1] == 2) and np.all(cover[P.lam0] == 0)
    # each frame is all of Lambda1 here
    assert all(np.array_equal(f, P.lam1) for f in P.phi_a)


def test_active_fraction_about_half():
    """Blocks 2.5 units with 0.5-unit frames (b:d = 5:1): about half the lattice is active."""
    P = geometry.PaperDomains((6, 6, 6, 6), [(5, 1)] * 4)
    frac = P.lam0.sum() / P.V
    assert abs(frac - (5 / 6) ** 4) < 1e-15 and 0.45 < frac < 0.55


def _logdet_identities(L, spec, kappa, eps, seed):
    P = geometry.PaperDomains(L, spec)
    U = synth.gauge_field(L, eps, seed)
    M = dense.dense_dirac_full(L, -1, kappa, U)
    s = P.sites
    dl0, l0b, l1 = s(P.dlam0), s(P.lam0bar), s(P.lam1)
    # Lambda0bar and Lambda1 do not couple
    assert np.max(np.abs(dense.sub(M, l0b, l1)), initial=0) == 0
    Dt = dense.sub(M, dl0)
    Dt = Dt - (dense.sub(M, dl0, l0b) @ np.linalg.solve(dense.sub(M, l0b), dense.sub(M, l0b, dl0))
               if l0b.size else 0)
    Dt = Dt - dense.sub(M, dl0, l1) @ np.linalg.solve(dense.sub(M, l1), dense.sub(M, l1, dl0))
    ld_D = dense.logdet(M)
    ld_l0b = dense.logdet(dense.sub(M, l0b))
    ld_l1 = dense.logdet(dense.sub(M, l1))
    ld_Dt = dense.logdet(Dt)
    rel = abs(np.exp(ld_l0b + ld_l1 + ld_Dt - ld_D) - 1)
    assert rel < 1e-9, "first Schur step"
    ld_hat = 0
    ld_om = 0
    ld_phi = 0
    for a in range(len(P.blocks)):
        d, bb, f, om = s(P.dlam0_a[a]), s(P.lam0bar_a[a]), s(P.phi_a[a]), s(P.omega_a[a])
        assert np.max(np.abs(dense.sub(M, bb, f)), initial=0) == 0
        Dh = dense.sub(M, d)
        if bb.size:
            Dh = Dh - dense.sub(M, d, bb) @ np.linalg.solve(dense.sub(M, bb), dense.sub(M, bb, d))
        Dh = Dh - dense.sub(M, d, f) @ np.linalg.solve(dense.sub(M, f), dense.sub(M, f, d))
        Mom = dense.sub(M, om)
        # the dLambda0^a block of D_Omega^{-1} is Dhat^{-1}
        pos = np.searchsorted(om, d)
        idx = dense.dof(pos)
        Minv = np.linalg.inv(Mom)
        assert np.max(np.abs(Minv[np.ix_(idx, idx)] - np.linalg.inv(Dh))) < 1e-10
        ld_hat += dense.logdet(Dh)
        ld_om += dense.logdet(Mom)
        ld_phi += dense.logdet(dense.sub(M, f))
        assert abs(np.exp(dense.logdet(dense.sub(M, bb)) + dense.logdet(dense.sub(M, f)) + dense.logdet(Dh)
                          - dense.logdet(Mom)) - 1) < 1e-9
    ld_W1 = ld_Dt - ld_hat
    # eq. (detD): det D = det W1 det D_Lambda1 prod det D_Omega / prod det D_Phi
    rel = abs(np.exp(ld_W1 + ld_l1 + ld_om - ld_phi - ld_D) - 1)
    assert rel < 1e-9, "block factorisation"
    return P, M, ld_D, ld_W1, ld_l1


@pytest.mark.slow
def test_factorisation_T1():
    _logdet_identities(*T1, kappa=0.12, eps=0.5, seed=1101)


@pytest.mark.slow
def test_factorisation_T4():
    _logdet_identities(*T4, kappa=0.12, eps=0.5, seed=41)


def test_factorisation_T3_corners():
    _logdet_identities(*T3, kappa=0.12, eps=0.5, seed=31)


def test_factorisation_1d_special_case():
    """Two thick time slices: det D = det W1 det D_Omega0 det D_Omega2 / det D_Lambda1."""
    P, M, ld_D, ld_W1, ld_l1 = _logdet_identities(*T2, kappa=0.12, eps=0.5, seed=21)
    om = [dense.logdet(dense.sub(M, P.sites(o))) for o in P.omega_a]
    assert abs(np.exp(ld_W1 + om[0] + om[1] - ld_l1 - ld_D) - 1) < 1e-9
