"""Pins of the global pieces of Section 4 in the oracle (oracle/mb.py) by dense linear algebra on tiny
lattices (the dense W_z of oracle.factor, itself pinned by the exact second decomposition and
det W_1 = det Dtilde / det Dhat^d in test_oracle_factor.py):

* apply_w (W_z chi from block solves and one solve on Lambda_1) equals the dense W_z chi row for row,
  on dLambda_0 and on dPi_1, for several z (z = 0: the off-diagonal part W_1 - 1);
* generate (chi = W_u^{-1} eta by BiCGStab over apply_w) equals the dense solve;
* apply_remainder (Chebyshev recurrence in -W_0/c) equals R_{N+1}(W_1) = 1 - W_1 P_N(W_1) with P_N in
  its product form c_N prod_k (W_1 - z_k) over the printed roots (a different route to the same
  polynomial), and both agree with the eigenvalue form;
* the reweighting estimator summed over the unit vectors of dPi is the exact truncated series
  -sum_m Tr(R^m)/m, which tends to ln det(1 - R) = ln W_N (eq. rw) from the dense slogdet.
"""
import numpy as np
import pytest

import synth
from oracle import dense, factor, geometry, mb, roots

KAPPA = 0.12
T2 = ((8, 2, 2, 2), [(3, 1), None, None, None], 21)
T3 = ((8, 8, 2, 2), [(3, 1), (3, 1), None, None], 31)


def _setup(L, spec, seed, kappa=KAPPA, eps=0.5):
    P = geometry.PaperDomains(L, spec)
    U = synth.gauge_field(L, eps, seed)
    M = dense.dense_dirac_full(L, -1, kappa, U)
    return P, U, M, factor.pieces(M, P)


def _box_lists(P):
    """The paper-mode blocks as explicit boxes (Omega_0^a, and Lambda_0^a relative to it)."""
    boxes, inner = [], []
    for blk in P.blocks:
        (lo, le), (oo, oe) = blk["lambda0"], blk["omega"]
        boxes.append(list(oo) + list(oe))
        inner.append([(lo[m] - oo[m]) % P.L[m] for m in range(4)] + list(le))
    return np.asarray(boxes), np.asarray(inner)


def _vec(pc, f):
    """A field [V, 4, 3] as the dense vector of W_z (dLambda_0 sites first, then dPi_1)."""
    return np.concatenate([f[pc["dl0"]].reshape(-1), f[pc["dp1"]].reshape(-1)])


@pytest.mark.parametrize("geom", [T2, T3], ids=["T2", "T3"])
def test_apply_w_matches_dense(geom):
    L, spec, seed = geom
    P, U, M, pc = _setup(L, spec, seed, KAPPA)
    boxes, inner = _box_lists(P)
    z = [complex(np.cos(2 * np.pi / 7), 0.8 * np.sin(2 * np.pi / 7)), 0.0, -0.4 + 0.9j]
    chi = synth.gaussian_complex((3, P.V, 4, 3), seed + 11)
    chi[1] = chi[0]
    out = mb.apply_w(L, -1, KAPPA, U, boxes, inner, z, chi)
    for k in range(3):
        ref = factor.w_z(pc, z[k]) @ _vec(pc, chi[k])
        got = _vec(pc, out[k])
        assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref), k
        # nothing off dPi
        assert np.all(out[k][~P.dPi] == 0)
    # z enters as z chi on dPi and nowhere else
    assert np.abs((out[0] - out[1]) - z[0] * np.where(P.dPi[:, None, None], chi[0], 0)).max() <= 1e-13


@pytest.mark.parametrize("geom", [T2, T3], ids=["T2", "T3"])
def test_generate_matches_dense_solve(geom):
    L, spec, seed = geom
    P, U, M, pc = _setup(L, spec, seed, KAPPA)
    boxes, inner = _box_lists(P)
    u = roots.mb_roots(6, 0.5)[:3]
    eta = synth.gaussian_complex((3, P.V, 4, 3), seed + 12) / np.sqrt(2)
    chi, its = mb.generate(L, -1, KAPPA, U, boxes, inner, u, eta, tol=1e-12)
    assert np.all(its > 0)
    for k in range(3):
        ref = np.linalg.solve(factor.w_z(pc, u[k]), _vec(pc, eta[k]))
        assert np.linalg.norm(_vec(pc, chi[k]) - ref) <= 1e-10 * np.linalg.norm(ref), k
        assert np.all(chi[k][~P.dPi] == 0)


def _dense_remainder(W1, N, c):
    """1 - W_1 P_N(W_1), P_N = c_N prod_{k=1}^N (W_1 - z_k), z_k = 1 - u_k (the printed roots)."""
    n = W1.shape[0]
    P = roots.leading_coeff(N, c) * np.eye(n, dtype=complex)
    for uk in roots.mb_roots(N, c):
        P = P @ (W1 - (1 - uk) * np.eye(n))
    return np.eye(n) - W1 @ P


@pytest.mark.parametrize("N,c", [(2, 0.9), (4, 0.8)])
def test_remainder_matches_product_form(N, c):
    L, spec, seed = T3
    P, U, M, pc = _setup(L, spec, seed, KAPPA)
    boxes, inner = _box_lists(P)
    W1 = factor.w_z(pc, 1.0)
    R = _dense_remainder(W1, N, c)
    # the eigenvalue form: R(W_1) has the eigenvalues R(lambda_i)
    lam = np.linalg.eigvals(W1)
    ev = np.sort_complex(np.linalg.eigvals(R))
    assert np.abs(ev - np.sort_complex(roots.remainder(N, c, lam))).max() <= 1e-10
    y = synth.gaussian_complex((2, P.V, 4, 3), seed + 13)
    out = mb.apply_remainder(L, -1, KAPPA, U, boxes, inner, N, c, y)
    for j in range(2):
        ref = R @ _vec(pc, y[j])
        assert np.linalg.norm(_vec(pc, out[j]) - ref) <= 1e-10 * np.linalg.norm(ref), j


def test_reweight_estimator_over_the_basis_is_exact():
    L, spec, seed = T2
    N, c, order = 2, 0.9, 3
    P, U, M, pc = _setup(L, spec, seed, KAPPA)
    boxes, inner = _box_lists(P)
    R = _dense_remainder(factor.w_z(pc, 1.0), N, c)
    sites = np.flatnonzero(P.dPi)
    n = 12 * sites.size
    eta = np.zeros((n, P.V, 4, 3), dtype=complex)
    for j in range(n):
        eta[j].reshape(P.V, 12)[sites[j // 12], j % 12] = 1.0
    e = mb.log_reweight_estimate(L, -1, KAPPA, U, boxes, inner, N, c, eta, order)
    # the basis order of eta is the dense vector order up to a permutation of sites: traces agree
    Rm = np.eye(R.shape[0], dtype=complex)
    series = 0j
    for m in range(1, order + 1):
        Rm = Rm @ R
        series -= np.trace(Rm) / m
    assert abs(e.sum() - series) <= 1e-10 * abs(series)
    # the truncated series approaches ln W_N = ln det(1 - R)
    sign, ld = np.linalg.slogdet(np.eye(R.shape[0]) - R)
    lnW = ld + 1j * np.angle(sign)
    # |ln(1 - r) + sum_{m <= order} r^m / m| <= |r|^(order+1) / ((order + 1)(1 - |r|)) per eigenvalue
    ar = np.abs(np.linalg.eigvals(R))
    assert ar.max() < 1
    bound = float(np.sum(ar ** (order + 1) / ((order + 1) * (1 - ar))))
    assert abs(series.real - lnW.real) <= bound
    assert abs(e.sum().real - lnW.real) <= bound and abs(lnW.real) > 10 * bound


def test_reweight_estimator_is_unbiased_in_the_mean():
    """Gaussian noise with E[eta eta^+] = 1: the mean over many vectors is within a few standard
    errors of the exact truncated series (a statistical check, fixed seed)."""
    L, spec, seed = T2
    N, c, order = 2, 0.9, 2
    P, U, M, pc = _setup(L, spec, seed, KAPPA)
    boxes, inner = _box_lists(P)
    R = _dense_remainder(factor.w_z(pc, 1.0), N, c)
    exact = -np.trace(R) - np.trace(R @ R) / 2
    eta = synth.gaussian_complex((200, P.V, 4, 3), 2024) / np.sqrt(2)
    e = mb.log_reweight_estimate(L, -1, KAPPA, U, boxes, inner, N, c, eta, order)
    se = e.real.std(ddof=1) / np.sqrt(e.size)
    assert abs(e.real.mean() - exact.real) <= 4 * se


def _clover_setup(kappa, csw):
    """T3 with the Sheikholeslami-Wohlert operator: domains, links, and the pieces of its dense matrix."""
    from oracle import clover

    L, spec, seed = T3
    P = geometry.PaperDomains(L, spec)
    U = synth.gauge_field(L, 0.5, seed)
    A = clover.clover_matrix(L, U, kappa, csw)
    n = 12 * P.V
    M = np.empty((n, n), dtype=complex)
    e = np.zeros((P.V, 4, 3), dtype=complex)
    ef = e.reshape(-1)
    for j in range(n):
        ef[j] = 1.0
        M[:, j] = clover.dirac_clover_full(L, -1, kappa, csw, U, e, A=A).reshape(-1)
        ef[j] = 0.0
    return L, seed, P, U, factor.pieces(M, P)


def test_global_action_with_clover_matches_dense():
    """S^r_MB with the Sheikholeslami-Wohlert operator (one masked solve on Lambda_1 with the clover
    term) equals the dPi_1 rows of the dense W_z built from the dense clover matrix (T3)."""
    kappa, csw = 0.12, 1.4
    L, seed, P, U, pc = _clover_setup(kappa, csw)
    boxes, inner = _box_lists(P)
    z = complex(0.3, 0.7)
    chi = synth.gaussian_complex((1, P.V, 4, 3), seed + 21)
    Wc = factor.w_z(pc, z) @ _vec(pc, chi[0])
    n0 = pc["Dd"].shape[0]
    S_rest = float(np.sum(np.abs(Wc[n0:]) ** 2))
    S_r = mb.mb_global_action(L, -1, kappa, U, boxes, inner, [z], chi, csw=csw)
    assert S_rest > 0 and abs(S_r[0] - S_rest) <= 1e-10 * S_rest
    # and the term matters
    S_w = mb.mb_global_action(L, -1, kappa, U, boxes, inner, [z], chi)
    assert abs(S_w[0] - S_r[0]) > 1e-3 * S_rest


def test_apply_w_and_generate_with_clover_match_dense():
    """W_z chi and chi = W_u^{-1} eta with the Sheikholeslami-Wohlert operator against the dense W_z
    built from the dense clover matrix (T3), row for row; and the term matters."""
    kappa, csw = 0.12, 1.4
    L, seed, P, U, pc = _clover_setup(kappa, csw)
    boxes, inner = _box_lists(P)
    z = [0.3 + 0.7j, 0.0]
    chi = synth.gaussian_complex((2, P.V, 4, 3), seed + 31)
    out = mb.apply_w(L, -1, kappa, U, boxes, inner, z, chi, csw=csw)
    for k in range(2):
        ref = factor.w_z(pc, z[k]) @ _vec(pc, chi[k])
        assert np.linalg.norm(_vec(pc, out[k]) - ref) <= 1e-11 * np.linalg.norm(ref), k
    wil = mb.apply_w(L, -1, kappa, U, boxes, inner, z, chi)
    assert np.linalg.norm(wil[0] - out[0]) > 1e-3 * np.linalg.norm(out[0])
    u = roots.mb_roots(4, 0.5)[:1]
    eta = synth.gaussian_complex((1, P.V, 4, 3), seed + 32) / np.sqrt(2)
    x, its = mb.generate(L, -1, kappa, U, boxes, inner, u, eta, tol=1e-12, csw=csw)
    ref = np.linalg.solve(factor.w_z(pc, u[0]), _vec(pc, eta[0]))
    assert np.linalg.norm(_vec(pc, x[0]) - ref) <= 1e-10 * np.linalg.norm(ref)


def test_exterior_source_of_one_block_alone():
    """The hops of chi from dPi into one block are the same whether dPi is built from that block alone
    or from all blocks (8^4 tiles with 4^4 active boxes on 16^4: every tile's active-box faces lie on
    the same hyperplanes, and the exterior shell's own perpendicular coordinate is on none of them),
    for every block.  This is what lets a full-size test compare sampled blocks with the oracle."""
    L, kappa = (16, 16, 16, 16), 0.12
    boxes = np.asarray(geometry.tile_boxes(L, [[8, 8]] * 4))
    inner = np.tile(np.array([2, 2, 2, 2, 4, 4, 4, 4]), (len(boxes), 1))
    U = synth.gauge_field(L, 0.2, 41)
    P = geometry.BoxDomains(L, boxes, inner)
    chi = synth.gaussian_complex((1, P.V, 4, 3), 42)
    chi[:, ~P.dPi] = 0
    xa = mb.exterior_source(L, -1, kappa, U, boxes, inner, chi, "all")
    S = 8**4
    for a in range(len(boxes)):
        box, inn = boxes[a:a + 1], inner[a:a + 1]
        Pa = geometry.BoxDomains(L, box, inn)
        assert np.array_equal(Pa.ext_a[0] & Pa.dPi, P.ext_a[a] & P.dPi), a
        assert np.array_equal(mb.exterior_source(L, -1, kappa, U, box, inn, chi, "all"), xa[:, a * S:(a + 1) * S]), a
