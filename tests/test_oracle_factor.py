"""Pins of the Section 3 decomposition pieces (oracle/factor.py) and of the exterior source of
eq. (localMB) (oracle/mb.py) by dense linear algebra on tiny lattices.

* the second decomposition Dtilde = Dhat^d + Dhat^h - Dhat_{dL0,dPi1} Dhat_{dPi1}^{-1} Dhat_{dPi1,dL0}
  holds exactly with the reading of Dhat^h and Dhat_{dPi1,dL0} (T2: 1D slices, T3: 2D corners,
  T1: all four directions decomposed);
* det W_1 (eq. Wz at z = 1, assembled from the pieces) = det Dtilde / det Dhat^d, and eq. (detD);
* in one dimension the reading equals the printed bracket term for term; in two it does not, and
  the printed bracket read with zero-extended inverses misses det W_1;
* the sets of geometry.BoxDomains (explicit boxes) are those of geometry.PaperDomains;
* S^a of eq. (localMB) from the dense W_z equals |u chi + D_Omega^{-1} xi| on dLambda_0^a with
  xi the exterior source (hops from dPi into Omega_0^a), and the parts of xi add up;
* S^r of eq. (globalMB) from one solve on Lambda_1 (mb.mb_global_action) equals the dPi_1 rows of the
  dense W_z chi, which with the block terms make up |W_z chi|^2 (eq. MBaction).
"""
import numpy as np
import pytest

import synth
from oracle import dense, factor, geometry, mb

T1 = ((4, 4, 4, 4), [(1, 1)] * 4, 1101)
T2 = ((8, 2, 2, 2), [(3, 1), None, None, None], 21)
T3 = ((8, 8, 2, 2), [(3, 1), (3, 1), None, None], 31)


def _setup(L, spec, seed, kappa=0.12, eps=0.5):
    P = geometry.PaperDomains(L, spec)
    U = synth.gauge_field(L, eps, seed)
    M = dense.dense_dirac_full(L, -1, kappa, U)
    return P, U, M, factor.pieces(M, P)


def _second(pc):
    out = pc["Dd"] + pc["Dh"]
    if pc["Dp"].shape[0]:
        out = out - pc["Bl"] @ np.linalg.solve(pc["Dp"], pc["Kp"])
    return out


@pytest.mark.parametrize("geom", [T2, T3, pytest.param(T1, marks=pytest.mark.slow)], ids=["T2", "T3", "T1"])
def test_second_decomposition_is_exact(geom):
    P, U, M, pc = _setup(*geom)
    Dt = pc["Dtilde"]
    assert np.abs(_second(pc) - Dt).max() <= 1e-12 * np.abs(Dt).max()
    # Dhat^h only couples different blocks, and only neighbouring ones
    for a, ra in enumerate(pc["blk"]):
        assert np.abs(pc["Dh"][np.ix_(ra, ra)]).max(initial=0) == 0


@pytest.mark.parametrize("geom", [T2, T3], ids=["T2", "T3"])
def test_det_w1_and_block_factorisation(geom):
    P, U, M, pc = _setup(*geom)
    W1 = factor.w_z(pc, 1.0)
    ld_W1 = dense.logdet(W1)
    assert abs(np.exp(ld_W1 - dense.logdet(pc["Dtilde"]) + dense.logdet(pc["Dd"])) - 1) < 1e-9
    s = P.sites
    ld = dense.logdet(M)
    ld_l1 = dense.logdet(dense.sub(M, s(P.lam1)))
    ld_om = sum(dense.logdet(dense.sub(M, s(o))) for o in P.omega_a)
    ld_phi = sum(dense.logdet(dense.sub(M, s(f))) for f in P.phi_a)
    # eq. (detD): det D = det W1 det D_Lambda1 prod det D_Omega / prod det D_Phi
    assert abs(np.exp(ld_W1 + ld_l1 + ld_om - ld_phi - ld) - 1) < 1e-9


def test_hopping_term_equals_printed_bracket_in_1d():
    P, U, M, pc = _setup(*T2)
    assert pc["Dp"].shape[0] == 0  # dPi_1 is empty for slices
    pr = factor.printed_dhat_h(M, P)
    assert np.abs(pr - pc["Dh"]).max() <= 1e-14 * np.abs(pc["Dh"]).max()


def test_printed_bracket_with_zero_extension_is_not_exact_with_corners():
    """Why the reading is needed: with dPi_1 present, the printed bracket (inverses zero-extended)
    differs from the exact hopping term and det W_1 built from it misses det Dtilde / det Dhat^d."""
    P, U, M, pc = _setup(*T3)
    pr = factor.printed_dhat_h(M, P)
    assert np.abs(pr - pc["Dh"]).max() > 1e-3 * np.abs(pc["Dh"]).max()
    bad = dict(pc, Dh=pr)
    miss = abs(np.exp(dense.logdet(factor.w_z(bad, 1.0)) - dense.logdet(pc["Dtilde"]) + dense.logdet(pc["Dd"])) - 1)
    assert miss > 1e-3


def _box_lists(P):
    boxes, inner = [], []
    for blk in P.blocks:
        (lo, le), (oo, oe) = blk["lambda0"], blk["omega"]
        boxes.append(list(oo) + list(oe))
        inner.append([(lo[m] - oo[m]) % P.L[m] for m in range(4)] + list(le))
    return np.asarray(boxes), np.asarray(inner)


@pytest.mark.parametrize("geom", [T1, T3], ids=["T1", "T3"])
def test_box_domains_match_paper_domains(geom):
    L, spec, _ = geom
    P = geometry.PaperDomains(L, spec)
    boxes, inner = _box_lists(P)
    B = geometry.BoxDomains(L, boxes, inner)
    assert np.array_equal(B.dPi, P.dPi) and np.array_equal(B.dPi1, P.dPi1)
    assert np.array_equal(B.lam0, P.lam0) and np.array_equal(B.dlam0, P.dlam0)
    for a in range(len(P.blocks)):
        assert np.array_equal(B.phi_a[a], P.phi_a[a]) and np.array_equal(B.ext_a[a], P.ext_omega_a[a])
        # the exterior boundary of a framed block lies on the hyperplanes
        assert not np.any(B.ext_a[a] & ~B.dPi)


@pytest.mark.parametrize("geom", [T3, pytest.param(T1, marks=pytest.mark.slow)], ids=["T3", "T1"])
def test_exterior_source_reproduces_local_mb_action(geom):
    L, spec, seed = geom
    kappa = 0.12
    P, U, M, pc = _setup(L, spec, seed, kappa)
    boxes, inner = _box_lists(P)
    z = complex(np.cos(2 * np.pi / 7), 0.8 * np.sin(2 * np.pi / 7))
    chi = synth.gaussian_complex((1, P.V, 4, 3), seed + 7)
    chi[0][~P.dPi] = 0.0
    # dense eq. (localMB): rows of W_z chi on each dLambda_0^a
    c = np.concatenate([chi[0][pc["dl0"]].reshape(-1), chi[0][pc["dp1"]].reshape(-1)])
    Wc = factor.w_z(pc, z) @ c
    n0 = pc["Dd"].shape[0]
    S_dense = np.array([np.sum(np.abs(Wc[ra]) ** 2) for ra in pc["blk"]])
    S_rest = np.sum(np.abs(Wc[n0:]) ** 2)
    # the library form: u chi + D_Omega^{-1} xi on dLambda_0^a, xi = hops from dPi into Omega_0^a
    xi = mb.exterior_source(L, -1, kappa, U, boxes, inner, chi, "all")
    parts = mb.exterior_source(L, -1, kappa, U, boxes, inner, chi, "dPi1") + \
        mb.exterior_source(L, -1, kappa, U, boxes, inner, chi, "dLam0")
    assert np.abs(parts - xi).max() <= 1e-15 * np.abs(xi).max()
    bl = mb.boundary_lists(L, boxes, inner)
    off = 0
    S_lib = []
    for a, bx in enumerate(boxes):
        sites = geometry.box_sites(L, bx[:4], bx[4:8])
        Mo = dense.sub(M, sites)
        S = sites.size
        y = np.linalg.solve(Mo, xi[0, off:off + S].reshape(-1)).reshape(S, 4, 3)
        v = z * chi[0][sites[bl[a]]] + y[bl[a]]
        S_lib.append(np.sum(np.abs(v) ** 2))
        off += S
    S_lib = np.asarray(S_lib)
    assert np.max(np.abs(S_lib - S_dense) / S_dense) <= 1e-12
    # eq. (MBaction): the block terms and the global rest make up |W_z chi|^2
    assert abs(S_dense.sum() + S_rest - np.sum(np.abs(Wc) ** 2)) <= 1e-12 * np.sum(np.abs(Wc) ** 2)
    # eq. (globalMB) from one solve on Lambda_1 equals the dense dPi_1 rows of W_z chi
    S_r = mb.mb_global_action(L, -1, kappa, U, boxes, inner, [z], chi)
    assert S_rest > 0 and abs(S_r[0] - S_rest) <= 1e-10 * S_rest


def test_exterior_source_dpi1_part_is_the_offdiagonal_term():
    """xi restricted to the dPi_1 part is D_{Phi_1^a, dOmega^{a*}} chi_{dPi_1} (eq. offdiagW1's source)."""
    L, spec, seed = T3
    kappa = 0.12
    P, U, M, pc = _setup(L, spec, seed, kappa)
    boxes, inner = _box_lists(P)
    chi = synth.gaussian_complex((2, P.V, 4, 3), 77)
    xi = mb.exterior_source(L, -1, kappa, U, boxes, inner, chi, "dPi1")
    off = 0
    for a, bx in enumerate(boxes):
        sites = geometry.box_sites(L, bx[:4], bx[4:8])
        est = P.sites(P.ext_omega_a[a] & P.dPi1)
        for f in range(2):
            ref = dense.sub(M, sites, est) @ chi[f][est].reshape(-1)
            got = xi[f, off:off + sites.size].reshape(-1)
            assert np.abs(got - ref).max() <= 1e-15 * max(np.abs(ref).max(), 1e-300)
            # only frame sites receive it
            lam = np.isin(sites, P.sites(P.lam0_a[a]))
            assert np.all(xi[f, off:off + sites.size][lam] == 0)
        off += sites.size
