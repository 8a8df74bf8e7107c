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

from . import geometry, wilson

__all__ = ["boundary_lists", "mb_local_action", "exterior_source", "mb_local_action_from_chi", "mb_global_action",
           "solve_masked"]


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


def solve_masked(L, tbc, kappa, U, mask, f, tol=1e-13, maxit=20000):
    """y = D_X^{-1} f for the site set X = mask (Dirichlet: D_X is the principal sub-matrix of D on
    X), by plain BiCGStab on the vectors supported on X; f [V, 4, 3] (its values outside X are not
    used); y is zero outside X."""
    def op(y):
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


def mb_global_action(L, tbc, kappa, U, boxes, inner, u, chi, tol=1e-13):
    """S^r_MB of eq. (globalMB) per field k: |u_k chi_k + W_{dPi1,dL0} chi_k|^2 summed over dPi_1 (the
    dPi_1 rows of W_{u_k} chi_k; field k at z = u_k as for the local term).  Reading: eliminating
    Lambda1bar from D_{Lambda_1} (Lambda_1 = Lambda1bar u dPi_1) gives
      W_{dPi1,dL0} chi = Dhat_{dPi1}^{-1} Dhat_{dPi1,dL0} chi = [D_{Lambda_1}^{-1} D_{Lambda_1,dL0} chi]_{dPi_1},
    one solve on the inactive region Lambda_1 per field.  chi [n_fields, V, 4, 3] on dPi (values
    elsewhere not used).  Returns the per-field values [n_fields]."""
    B = geometry.BoxDomains(L, boxes, inner)
    u = np.asarray(u, dtype=np.complex128).reshape(-1)
    chi = np.asarray(chi, dtype=np.complex128)
    out = np.zeros(u.size)
    for k in range(u.size):
        c = np.zeros_like(chi[k])
        c[B.dlam0] = chi[k][B.dlam0]
        f = wilson.dirac_full(L, tbc, kappa, U, c)  # D_{Lambda_1, dLambda_0} chi on Lambda_1
        v = solve_masked(L, tbc, kappa, U, B.lam1, f, tol=tol)
        w = u[k] * chi[k][B.dPi1] + v[B.dPi1]
        out[k] = float(np.sum(np.abs(w) ** 2))
    return out
