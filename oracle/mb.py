"""Block-local multi-boson action (oracle).  Test infrastructure only.

Section 4 writes the multi-boson action |W_z chi|^2 as a sum of block-local
terms S_MB^a plus a global rest.  The block-local term is the squared norm, on
the internal boundary dLambda_0^a, of
    z chi + [Dhat_{dLambda_0^a}]^{-1} Dhat^h chi + D_{Omega_0^a}^{-1} D_{Phi_1^a, dOmega^{a*}} chi.
Reading used here:
  * field k is taken at z = u_k (because z_k - W_1 = -W_{u_k});
  * [Dhat_{dLambda_0^a}]^{-1} equals the dLambda_0^a block of D_{Omega_0^a}^{-1}
    (Dhat_{dLambda_0^a} is the Schur complement of D_{Omega_0^a} onto
    dLambda_0^a, since the block bulk and the frame do not touch), so both
    operator terms are one solve with D_{Omega_0^a} restricted to dLambda_0^a;
  * the source xi_k^a on Omega_0^a collects both hop-in terms.  With the
    exact hopping term of oracle.factor, the dLambda_0^a rows of
    D_{Omega_0^a}^{-1} applied to the frame part of the Dhat^h term equal
    those of [Dhat_{dLambda_0^a}]^{-1} Dhat^h chi, so xi_k^a is the hop of
    chi_k from the exterior boundary of Omega_0^a (which lies in dPi) into
    Omega_0^a: exterior_source.  mb_local_action takes any xi.
Hence  S^a = sum_k sum_{x in dLambda_0^a} |u_k chi_k(x) + (D_{Omega_0^a}^{-1} xi_k^a)(x)|^2.
"""
from __future__ import annotations

import numpy as np

from . import clover, geometry, roots, wilson

__all__ = ["boundary_lists", "mb_local_action", "exterior_source", "mb_local_action_from_chi", "mb_global_action",
           "solve_masked", "apply_w", "generate", "apply_remainder", "log_reweight_estimate"]


def boundary_lists(L, boxes, inner):
    """dLambda_0^a as box-local canonical indices for every block.

    inner[b] = (offset[4], extent[4]) of the active box inside block b.
    """
    out = []
    for b in range(len(boxes)):
        out.append(geometry.inner_boundary_local(L, boxes[b], inner[b][:4], inner[b][4:8]))
    return out


def mb_local_action(L, tbc, kappa, U, boxes, inner, u, chi, xi, tol=1e-12, nthreads=0):
    """Per-block actions S^a and their sum.

    boxes [nb, 8]; inner [nb, 8]; u [n_fields] complex;
    chi [n_fields, sum_b |dLambda_0^b|, 4, 3]; xi [n_fields, sum_b S_b, 4, 3].
    """
    boxes = np.asarray(boxes, dtype=np.int32).reshape(-1, 8)
    nb = boxes.shape[0]
    u = np.asarray(u, dtype=np.complex128).reshape(-1)
    nf = u.size
    chi = np.asarray(chi, dtype=np.complex128)
    xi = np.asarray(xi, dtype=np.complex128)
    y, _, rel, fails = wilson.solve_many(L, tbc, kappa, U, boxes, xi, tol=tol, nthreads=nthreads)
    if fails:
        raise RuntimeError("oracle block solve did not converge")
    bl = boundary_lists(L, boxes, inner)
    S = np.zeros(nb, dtype=np.float64)
    soff = 0
    boff = 0
    for b in range(nb):
        Sb = int(np.prod(boxes[b, 4:8]))
        nbd = bl[b].size
        for k in range(nf):
            v = u[k] * chi[k, boff:boff + nbd] + y[k, soff + bl[b]]
            S[b] += float(np.sum(np.abs(v) ** 2))
        soff += Sb
        boff += nbd
    return S, float(np.sum(S))


def exterior_source(L, tbc, kappa, U, boxes, inner, chi, part="all"):
    """The source xi^a = D_{Omega_0^a, E^a} chi of every block, on its box.

    chi [n_fields, V, 4, 3] is a field on the whole lattice of which only the
    sites of dPi are used; E^a is the exterior boundary of Omega_0^a (sites
    outside it with a neighbour inside) restricted to
      part = "dPi1": dPi_1, the D_{Phi_1^a, dOmega^{a*}} chi_{dPi_1} term of eq. (localMB);
      part = "dLam0": dLambda_0 (the active boundaries of the other blocks);
      part = "all":  both, i.e. dPi.
    The "dLam0" part replaces [Dhat_{dLambda_0^a}]^{-1} Dhat^h chi of eq.
    (localMB): with Dhat^h_{aa'} = -D_{dLambda_0^a, Phi_1^a} D_{Phi_1^a}^{-1}
    P_{Phi_1^a} D_{Phi_1^{a'}, dLambda_0^{a'}} (the exact reading; see
    oracle.factor) the dLambda_0^a rows of D_{Omega_0^a}^{-1} applied to
    P_{Phi_1^a} sum_{a' != a} D_{Phi_1^a, dLambda_0^{a'}} chi equal those of
    [Dhat_{dLambda_0^a}]^{-1} Dhat^h chi, since Lambda_0^a meets Phi_1^a
    only through dLambda_0^a.
    Computed as the restriction to Omega_0^a of D applied to chi masked to
    E^a (the diagonal term vanishes there).  Returns [n_fields, sum_a S_a, 4, 3]
    in box-local canonical order, blocks concatenated.
    """
    P = geometry.BoxDomains(L, boxes, inner)
    sel = {"dPi1": P.dPi1, "dLam0": P.dlam0, "all": P.dPi}[part]
    chi = np.asarray(chi, dtype=np.complex128)
    out = []
    for b in range(len(P.omega_a)):
        E = P.ext_a[b] & sel
        sites = geometry.box_sites(L, P.boxes[b][:4], P.boxes[b][4:8])
        per_f = []
        for f in range(chi.shape[0]):
            psi = np.zeros_like(chi[f])
            psi[E] = chi[f][E]
            per_f.append(wilson.dirac_full(L, tbc, kappa, U, psi)[sites])
        out.append(np.stack(per_f))
    return np.concatenate(out, axis=1)


def mb_local_action_from_chi(L, tbc, kappa, U, boxes, inner, u, chi, tol=1e-12, nthreads=0):
    """S^a of eq. (localMB) from the multi-boson fields alone: chi [n_fields, V, 4, 3] on dPi (the
    values elsewhere are not used); the boundary values u_k chi_k on dLambda_0^a and the source
    xi^a = exterior_source(..., part="all")."""
    chi = np.asarray(chi, dtype=np.complex128)
    bl = boundary_lists(L, boxes, inner)
    chib = []
    for b, bx in enumerate(np.asarray(boxes).reshape(-1, 8)):
        sites = geometry.box_sites(L, bx[:4], bx[4:8])
        chib.append(chi[:, sites[bl[b]]])
    chib = np.concatenate(chib, axis=1)
    xi = exterior_source(L, tbc, kappa, U, boxes, inner, chi, "all")
    return mb_local_action(L, tbc, kappa, U, boxes, inner, u, chib, xi, tol=tol, nthreads=nthreads)


def solve_masked(L, tbc, kappa, U, mask, f, tol=1e-13, maxit=20000, csw=0.0, A=None):
    """y = D_X^{-1} f for the site set X = mask (Dirichlet: D_X is the principal sub-matrix of D on
    X), by plain BiCGStab on the vectors supported on X; f [V, 4, 3] (its values outside X are not
    used); y is zero outside X.  With csw != 0, D is the Sheikholeslami-Wohlert operator
    (oracle.clover; A its clover matrices, computed when not given)."""
    if csw != 0.0 and A is None:
        A = clover.clover_matrix(L, U, kappa, csw)

    def op(y):
        if csw != 0.0:
            out = clover.dirac_clover_full(L, tbc, kappa, csw, U, y, A=A)
        else:
            out = wilson.dirac_full(L, tbc, kappa, U, y)
        out[~mask] = 0.0
        return out

    b = np.zeros_like(np.asarray(f, dtype=np.complex128))
    b[mask] = np.asarray(f)[mask]
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bn == 0.0:
        return x
    r = b.copy()
    rh = r.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    for _ in range(maxit):
        rho_new = np.vdot(rh, r)
        beta = (rho_new / rho) * (alpha / omega)
        rho = rho_new
        p = r + beta * (p - omega * v)
        v = op(p)
        alpha = rho / np.vdot(rh, v)
        s = r - alpha * v
        t = op(s)
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        if np.linalg.norm(r) <= tol * bn:
            break
    else:
        raise RuntimeError("oracle masked solve did not converge")
    true = np.linalg.norm(b - op(x)) / bn
    if true > 100 * tol:
        raise RuntimeError("oracle masked solve: true residual %.3g" % true)
    return x


def mb_global_action(L, tbc, kappa, U, boxes, inner, u, chi, tol=1e-13, csw=0.0):
    """S^r_MB of eq. (globalMB) per field k: |u_k chi_k + W_{dPi1,dL0} chi_k|^2 summed over dPi_1 (the
    dPi_1 rows of W_{u_k} chi_k; field k at z = u_k as for the local term).  Reading: eliminating
    Lambda1bar from D_{Lambda_1} (Lambda_1 = Lambda1bar u dPi_1) gives
      W_{dPi1,dL0} chi = Dhat_{dPi1}^{-1} Dhat_{dPi1,dL0} chi = [D_{Lambda_1}^{-1} D_{Lambda_1,dL0} chi]_{dPi_1},
    one solve on the inactive region Lambda_1 per field.  chi [n_fields, V, 4, 3] on dPi (values
    elsewhere not used).  With csw != 0 the operator is the Sheikholeslami-Wohlert one (its clover
    term is site-diagonal, so the hops D_{Lambda_1, dLambda_0} are those of the Wilson operator).
    Returns the per-field values [n_fields]."""
    B = geometry.BoxDomains(L, boxes, inner)
    u = np.asarray(u, dtype=np.complex128).reshape(-1)
    chi = np.asarray(chi, dtype=np.complex128)
    out = np.zeros(u.size)
    A = clover.clover_matrix(L, U, kappa, csw) if csw != 0.0 else None
    for k in range(u.size):
        c = np.zeros_like(chi[k])
        c[B.dlam0] = chi[k][B.dlam0]
        f = wilson.dirac_full(L, tbc, kappa, U, c)  # D_{Lambda_1, dLambda_0} chi on Lambda_1
        v = solve_masked(L, tbc, kappa, U, B.lam1, f, tol=tol, csw=csw, A=A)
        w = u[k] * chi[k][B.dPi1] + v[B.dPi1]
        out[k] = float(np.sum(np.abs(w) ** 2))
    return out


def apply_w(L, tbc, kappa, U, boxes, inner, z, chi, tol=1e-13, csw=0.0):
    """W_z chi of eq. (MBaction) as a vector on dPi, one z per field: z [n_fields] complex, chi
    [n_fields, V, 4, 3] (only its dPi values are used).  Rows on dLambda_0^a are the vector whose norm
    is S_MB^a (eq. localMB): z chi + (D_{Omega_0^a}^{-1} xi^a) with xi^a the hops of chi from dPi
    into Omega_0^a (exterior_source); rows on dPi_1 are those whose norm is S^r_MB (eq. globalMB):
    z chi + [D_{Lambda_1}^{-1} D_{Lambda_1, dLambda_0} chi] (as in mb_global_action).  Zero off dPi.
    At z = 0 it is the off-diagonal part W_1 - 1 of W_1.  With csw != 0 the operator is the
    Sheikholeslami-Wohlert one: its clover term is site-diagonal, so the hops (the sources) are
    unchanged and the block and inactive-region solves take it (masked solves on each box's sites;
    the boxes must not wrap onto themselves)."""
    boxes = np.asarray(boxes, dtype=np.int32).reshape(-1, 8)
    B = geometry.BoxDomains(L, boxes, inner)
    z = np.asarray(z, dtype=np.complex128).reshape(-1)
    c = np.zeros_like(np.asarray(chi, dtype=np.complex128))
    c[:, B.dPi] = np.asarray(chi)[:, B.dPi]
    out = np.zeros_like(c)
    A = clover.clover_matrix(L, U, kappa, csw) if csw != 0.0 else None
    xi = exterior_source(L, tbc, kappa, U, boxes, inner, c, "all")
    if A is None:
        y, _, _, fails = wilson.solve_many(L, tbc, kappa, U, boxes, xi, tol=tol)
        if fails:
            raise RuntimeError("oracle block solve did not converge")
    bl = boundary_lists(L, boxes, inner)
    off = 0
    for b, bx in enumerate(boxes):
        sites = geometry.box_sites(L, bx[:4], bx[4:8])
        g = sites[bl[b]]
        for k in range(z.size):
            if A is None:
                yb = y[k, off + bl[b]]
            else:
                mask = np.zeros(c.shape[1], dtype=bool)
                mask[sites] = True
                f = np.zeros_like(c[k])
                f[sites] = xi[k, off:off + sites.size]
                yb = solve_masked(L, tbc, kappa, U, mask, f, tol=tol, csw=csw, A=A)[g]
            out[k][g] = z[k] * c[k][g] + yb
        off += sites.size
    for k in range(z.size):
        d = np.zeros_like(c[k])
        d[B.dlam0] = c[k][B.dlam0]
        v = solve_masked(L, tbc, kappa, U, B.lam1, wilson.dirac_full(L, tbc, kappa, U, d), tol=tol, csw=csw, A=A)
        out[k][B.dPi1] = z[k] * c[k][B.dPi1] + v[B.dPi1]
    return out


def generate(L, tbc, kappa, U, boxes, inner, u, eta, tol=1e-11, inner_tol=1e-13, maxit=200, csw=0.0):
    """The multi-boson fields of Section 4 from Gaussian noise: chi_k = W_{u_k}^{-1} eta_k on dPi
    (then chi_k has the density exp(-|W_{u_k} chi_k|^2) when eta_k has exp(-|eta_k|^2)).  This is
    the one global inversion of the method, on a vector of dPi (Conclusions).  u [n_fields] complex;
    eta [n_fields, V, 4, 3] (values off dPi are not used).  Plain BiCGStab per field on the vectors
    supported on dPi with apply_w as the operator, stopped at |eta - W chi| <= tol |eta|.  Returns
    (chi [n_fields, V, 4, 3], zero off dPi; iterations per field)."""
    B = geometry.BoxDomains(L, boxes, inner)
    u = np.asarray(u, dtype=np.complex128).reshape(-1)
    eta = np.asarray(eta, dtype=np.complex128)
    chi = np.zeros_like(eta)
    its = np.zeros(u.size, dtype=np.int64)

    def op(k, y):
        return apply_w(L, tbc, kappa, U, boxes, inner, [u[k]], y[None], tol=inner_tol, csw=csw)[0]

    for k in range(u.size):
        b = np.zeros_like(eta[k])
        b[B.dPi] = eta[k][B.dPi]
        bn = np.linalg.norm(b)
        if bn == 0.0:
            continue
        x = np.zeros_like(b)
        r = b.copy()
        rh = r.copy()
        rho = alpha = omega = 1.0 + 0j
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        for it in range(1, maxit + 1):
            rho_new = np.vdot(rh, r)
            beta = (rho_new / rho) * (alpha / omega)
            rho = rho_new
            p = r + beta * (p - omega * v)
            v = op(k, p)
            alpha = rho / np.vdot(rh, v)
            s = r - alpha * v
            t = op(k, s)
            omega = np.vdot(t, s) / np.vdot(t, t)
            x = x + alpha * p + omega * s
            r = s - omega * t
            if np.linalg.norm(r) <= tol * bn:
                break
        else:
            raise RuntimeError("oracle field generation did not converge")
        chi[k] = x
        its[k] = it
    return chi, its


def apply_remainder(L, tbc, kappa, U, boxes, inner, N, c, y, tol=1e-13, csw=0.0):
    """R_{N+1}(W_1) y on dPi for y [n_vec, V, 4, 3], with the remainder in its Chebyshev form
    R_{N+1}(z) = T_{N+1}((1 - z)/c) / T_{N+1}(1/c) (oracle.roots; it has the printed roots).  Its
    argument (1 - W_1)/c is -(W_1 - 1)/c = -W_0/c, so the three-term recurrence
    T_0 y = y, T_1 y = X y, T_{j+1} y = 2 X T_j y - T_{j-1} y applies X = -apply_w(z = 0)/c alone and
    never forms 1 - W_1 P_N(W_1), whose entries cancel to the size of R."""
    B = geometry.BoxDomains(L, boxes, inner)
    y = np.asarray(y, dtype=np.complex128)
    t0 = np.zeros_like(y)
    t0[:, B.dPi] = y[:, B.dPi]
    zero = np.zeros(y.shape[0])

    def X(v):
        return -apply_w(L, tbc, kappa, U, boxes, inner, zero, v, tol=tol, csw=csw) / c

    t1 = X(t0)
    for _ in range(N):
        t0, t1 = t1, 2 * X(t1) - t0
    return t1 / float(np.real(roots.chebyshev_T(N + 1, np.asarray(1.0 / c))))


def log_reweight_estimate(L, tbc, kappa, U, boxes, inner, N, c, eta, order, tol=1e-13, csw=0.0):
    """Stochastic estimate of ln W_N, W_N = det{1 - R_{N+1}(W_1)} of eq. (rw), by
    ln det(1 - R) = Tr ln(1 - R) = -sum_{m >= 1} Tr(R^m)/m truncated after `order` terms, each trace
    by the noise vectors eta [n_vec, V, 4, 3] (values on dPi; any noise with E[eta eta^+] = 1, or the
    unit vectors of dPi, for which the sum is the exact trace): per vector
    e_j = -sum_{m=1}^{order} eta_j^+ R^m eta_j / m.  Returns the per-vector terms e [n_vec] complex;
    their mean estimates ln W_N.  The paper defines W_N only; this estimator is a reading."""
    B = geometry.BoxDomains(L, boxes, inner)
    eta = np.asarray(eta, dtype=np.complex128)
    e0 = np.zeros_like(eta)
    e0[:, B.dPi] = eta[:, B.dPi]
    out = np.zeros(eta.shape[0], dtype=np.complex128)
    w = e0
    for m in range(1, order + 1):
        w = apply_remainder(L, tbc, kappa, U, boxes, inner, N, c, w, tol=tol, csw=csw)
        for j in range(eta.shape[0]):
            out[j] -= np.vdot(e0[j], w[j]) / m
    return out
