/*
 * dd_oracle.c -- plain FP64 CPU oracle for the block-restricted Wilson-Dirac
 * operator D_Lambda and the block solves D_Lambda^{-1} b.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP path.
 *
 * What it computes (paper: Section 1 for fields on sites and links, Section 3
 * for the local lattice Dirac operator D and its restrictions D_X to subsets X
 * of the lattice):
 *
 *   (D psi)(x) = psi(x) - kappa * sum_{mu=0..3} [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                               + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *
 * i.e. the Wilson-Dirac operator in hopping normalisation without clover term.
 * Space is periodic; time (mu = 0) is antiperiodic for the fermion when
 * tbc = -1: a hop across x0 = L0-1 <-> 0 picks up a factor -1.
 * The restriction D_X keeps only hops whose source site lies in X (Dirichlet
 * boundary), which is the principal submatrix of D on X.
 *
 * Gamma matrices: chiral basis, gamma_0 = [[0,-1],[-1,0]],
 * gamma_k = [[0,-i sigma_k],[i sigma_k,0]], gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3.
 *
 * Storage: complex numbers are interleaved (re, im) doubles.
 *   links    U[n][mu][row][col]   (global canonical site n, x3 fastest)
 *   spinors  psi[site][spin][col] (global canonical order for the full lattice,
 *                                  box-local canonical order for a box)
 *
 * A box is (origin o[4], extent e[4]); local coordinate y maps to global
 * x = (o + y) mod L.  A box may wrap across the lattice edge; when e_mu == L_mu
 * the box spans the full direction and keeps its wrap-around links.
 *
 * Everything here is deliberately plain: explicit 4x4 gamma matrices, explicit
 * 3x3 products, textbook BiCGStab.  No blocking, no fusion.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* gamma matrices                                                           */
/* ------------------------------------------------------------------------ */

static void gamma_matrix(int mu, cplx g[4][4])
{
    memset(g, 0, sizeof(cplx) * 16);
    if (mu == 0) {
        /* [[0, -1], [-1, 0]] in 2x2 spin blocks */
        g[0][2] = -1; g[1][3] = -1;
        g[2][0] = -1; g[3][1] = -1;
        return;
    }
    if (mu >= 1 && mu <= 3) {
        /* Pauli matrix sigma_mu */
        cplx s[2][2] = {{0, 0}, {0, 0}};
        if (mu == 1) { s[0][1] = 1; s[1][0] = 1; }
        if (mu == 2) { s[0][1] = -I; s[1][0] = I; }
        if (mu == 3) { s[0][0] = 1; s[1][1] = -1; }
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                g[a][2 + b] = -I * s[a][b];   /* upper-right: -i sigma */
                g[2 + a][b] = I * s[a][b];    /* lower-left:  +i sigma */
            }
        return;
    }
    /* mu == 4: gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3 */
    cplx acc[4][4], t[4][4], gm[4][4];
    gamma_matrix(0, acc);
    for (int m = 1; m <= 3; m++) {
        gamma_matrix(m, gm);
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
                cplx s = 0;
                for (int k = 0; k < 4; k++) s += acc[i][k] * gm[k][j];
                t[i][j] = s;
            }
        memcpy(acc, t, sizeof(t));
    }
    memcpy(g, acc, sizeof(acc));
}

/* Export gamma_mu (mu = 0..3, 4 = gamma_5) as 16 interleaved complex numbers. */
void or_gamma(int mu, double *out)
{
    cplx g[4][4];
    gamma_matrix(mu, g);
    memcpy(out, g, sizeof(g));
}

/* ------------------------------------------------------------------------ */
/* one hop term: out += sgn * (1 + pm*gamma_mu) * W * psi                   */
/* where W = U (forward) or U^+ (backward)                                  */
/* ------------------------------------------------------------------------ */

static void add_hop_term(cplx out[4][3], const cplx G[4][4], double pm, const cplx *U,
                         int dagger, const cplx psi[4][3], double sgn)
{
    /* chi = W psi (colour multiply per spin) */
    cplx chi[4][3];
    for (int s = 0; s < 4; s++)
        for (int a = 0; a < 3; a++) {
            cplx v = 0;
            for (int b = 0; b < 3; b++) {
                cplx w = dagger ? conj(U[b * 3 + a]) : U[a * 3 + b];
                v += w * psi[s][b];
            }
            chi[s][a] = v;
        }
    /* out += sgn * (1 + pm*gamma) chi */
    for (int s = 0; s < 4; s++)
        for (int a = 0; a < 3; a++) {
            cplx v = chi[s][a];
            for (int t = 0; t < 4; t++) v += pm * G[s][t] * chi[t][a];
            out[s][a] += sgn * v;
        }
}

static int site_of(const int L[4], const int x[4])
{
    return ((x[0] * L[1] + x[1]) * L[2] + x[2]) * L[3] + x[3];
}

/* ------------------------------------------------------------------------ */
/* full-lattice hopping term H and D = 1 - kappa H                          */
/* ------------------------------------------------------------------------ */

/* (H psi)(x) = sum_mu [ (1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu) ] */
void or_hop_full(const int *L, int tbc, const double *Ud, const double *ind, double *outd)
{
    const cplx *U = (const cplx *)Ud;
    const cplx (*in)[4][3] = (const cplx (*)[4][3])ind;
    cplx (*out)[4][3] = (cplx (*)[4][3])outd;
    cplx G[4][4][4];
    for (int mu = 0; mu < 4; mu++) gamma_matrix(mu, G[mu]);
    const int V = L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
    for (int n = 0; n < V; n++) {
        int x[4];
        int r = n;
        x[3] = r % L[3]; r /= L[3];
        x[2] = r % L[2]; r /= L[2];
        x[1] = r % L[1]; r /= L[1];
        x[0] = r;
        cplx acc[4][3];
        memset(acc, 0, sizeof(acc));
        for (int mu = 0; mu < 4; mu++) {
            int xf[4], xb[4];
            memcpy(xf, x, sizeof(xf));
            memcpy(xb, x, sizeof(xb));
            xf[mu] = (x[mu] + 1) % L[mu];
            xb[mu] = (x[mu] - 1 + L[mu]) % L[mu];
            double sf = 1.0, sb = 1.0;
            if (mu == 0 && tbc < 0) {
                if (x[0] == L[0] - 1) sf = -1.0; /* hop from x0 = 0 into x0 = L0-1 */
                if (x[0] == 0) sb = -1.0;        /* hop from x0 = L0-1 into x0 = 0 */
            }
            int nf = site_of(L, xf), nb = site_of(L, xb);
            add_hop_term(acc, G[mu], -1.0, &U[((size_t)n * 4 + mu) * 9], 0, in[nf], sf);
            add_hop_term(acc, G[mu], +1.0, &U[((size_t)nb * 4 + mu) * 9], 1, in[nb], sb);
        }
        memcpy(out[n], acc, sizeof(acc));
    }
}

void or_dirac_full(const int *L, int tbc, double kappa, const double *U, const double *in,
                   double *out)
{
    const size_t n = (size_t)L[0] * L[1] * L[2] * L[3] * 12;
    or_hop_full(L, tbc, U, in, out);
    for (size_t i = 0; i < 2 * n; i++) out[i] = in[i] - kappa * out[i];
}

/* ------------------------------------------------------------------------ */
/* box-restricted hopping term (Dirichlet): hops from outside the box dropped */
/* ------------------------------------------------------------------------ */

typedef struct {
    int L[4];
    int tbc;
    int o[4], e[4];
    int S; /* sites in the box */
} box_t;

static void box_init(box_t *b, const int *L, int tbc, const int *o, const int *e)
{
    for (int m = 0; m < 4; m++) {
        b->L[m] = L[m];
        b->o[m] = ((o[m] % L[m]) + L[m]) % L[m];
        b->e[m] = e[m];
    }
    b->tbc = tbc;
    b->S = e[0] * e[1] * e[2] * e[3];
}

static void box_local_coords(const box_t *b, int s, int y[4])
{
    y[3] = s % b->e[3]; s /= b->e[3];
    y[2] = s % b->e[2]; s /= b->e[2];
    y[1] = s % b->e[1]; s /= b->e[1];
    y[0] = s;
}

static int box_local_index(const box_t *b, const int y[4])
{
    return ((y[0] * b->e[1] + y[1]) * b->e[2] + y[2]) * b->e[3] + y[3];
}

static void box_global_coords(const box_t *b, const int y[4], int x[4])
{
    for (int m = 0; m < 4; m++) x[m] = (b->o[m] + y[m]) % b->L[m];
}

/* parity of a box site in global coordinates */
static int box_parity(const box_t *b, int s)
{
    int y[4], x[4];
    box_local_coords(b, s, y);
    box_global_coords(b, y, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

static void box_hop(const box_t *b, const cplx *U, const cplx (*in)[4][3], cplx (*out)[4][3])
{
    cplx G[4][4][4];
    for (int mu = 0; mu < 4; mu++) gamma_matrix(mu, G[mu]);
    for (int s = 0; s < b->S; s++) {
        int y[4], x[4];
        box_local_coords(b, s, y);
        box_global_coords(b, y, x);
        cplx acc[4][3];
        memset(acc, 0, sizeof(acc));
        for (int mu = 0; mu < 4; mu++) {
            const int full = (b->e[mu] == b->L[mu]);
            /* forward neighbour y + mu */
            int yf[4];
            memcpy(yf, y, sizeof(yf));
            yf[mu] = y[mu] + 1;
            int f_in = 1;
            if (yf[mu] == b->e[mu]) {
                if (full) yf[mu] = 0; else f_in = 0;
            }
            if (f_in) {
                double sg = (mu == 0 && b->tbc < 0 && x[0] == b->L[0] - 1) ? -1.0 : 1.0;
                const int n = site_of(b->L, x);
                add_hop_term(acc, G[mu], -1.0, &U[((size_t)n * 4 + mu) * 9], 0,
                             in[box_local_index(b, yf)], sg);
            }
            /* backward neighbour y - mu */
            int yb[4];
            memcpy(yb, y, sizeof(yb));
            yb[mu] = y[mu] - 1;
            int b_in = 1;
            if (yb[mu] < 0) {
                if (full) yb[mu] = b->e[mu] - 1; else b_in = 0;
            }
            if (b_in) {
                double sg = (mu == 0 && b->tbc < 0 && x[0] == 0) ? -1.0 : 1.0;
                int xb[4];
                memcpy(xb, x, sizeof(xb));
                xb[mu] = (x[mu] - 1 + b->L[mu]) % b->L[mu];
                const int nb = site_of(b->L, xb);
                add_hop_term(acc, G[mu], +1.0, &U[((size_t)nb * 4 + mu) * 9], 1,
                             in[box_local_index(b, yb)], sg);
            }
        }
        memcpy(out[s], acc, sizeof(acc));
    }
}

void or_hop_box(const int *L, int tbc, const double *U, const int *o, const int *e,
                const double *in, double *out)
{
    box_t b;
    box_init(&b, L, tbc, o, e);
    box_hop(&b, (const cplx *)U, (const cplx (*)[4][3])in, (cplx (*)[4][3])out);
}

void or_dirac_box(const int *L, int tbc, double kappa, const double *U, const int *o,
                  const int *e, const double *in, double *out)
{
    box_t b;
    box_init(&b, L, tbc, o, e);
    box_hop(&b, (const cplx *)U, (const cplx (*)[4][3])in, (cplx (*)[4][3])out);
    for (size_t i = 0; i < (size_t)b.S * 24; i++) out[i] = in[i] - kappa * out[i];
}

/* Global parity of every site of a box, in box-local canonical order. */
void or_box_parity(const int *L, const int *o, const int *e, int *par)
{
    box_t b;
    box_init(&b, L, -1, o, e);
    for (int s = 0; s < b.S; s++) par[s] = box_parity(&b, s);
}

/* ------------------------------------------------------------------------ */
/* vector helpers on box-sized spinor fields (n = 12*S complex numbers)      */
/* ------------------------------------------------------------------------ */

static cplx vdot(const cplx *a, const cplx *b, size_t n)
{
    cplx s = 0;
    for (size_t i = 0; i < n; i++) s += conj(a[i]) * b[i];
    return s;
}

static double vnorm2(const cplx *a, size_t n)
{
    double s = 0;
    for (size_t i = 0; i < n; i++) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

/* zero the sites of parity p */
static void zero_parity(const box_t *b, const int *par, cplx *v, int p)
{
    for (int s = 0; s < b->S; s++)
        if (par[s] == p) memset(&v[(size_t)s * 12], 0, sizeof(cplx) * 12);
}

/* Even-odd reduced operator on even sites:
 *   Dhat v_e = v_e - kappa^2 H_eo H_oe v_e
 * With no clover term the diagonal blocks of D_Lambda are the identity, so the
 * Schur complement of the odd-odd block is exactly this.  Vectors are stored
 * box-sized with zeros on odd sites. */
static void apply_dhat(const box_t *b, const int *par, double kappa, const cplx *U,
                       const cplx *v, cplx *out, cplx *tmp)
{
    const size_t n = (size_t)b->S * 12;
    box_hop(b, U, (const cplx (*)[4][3])v, (cplx (*)[4][3])tmp); /* H v_e: lands on odd */
    zero_parity(b, par, tmp, 0);
    box_hop(b, U, (const cplx (*)[4][3])tmp, (cplx (*)[4][3])out); /* H_eo (H_oe v_e) */
    zero_parity(b, par, out, 1);
    for (size_t i = 0; i < n; i++) out[i] = v[i] - kappa * kappa * out[i];
}

/* Textbook BiCGStab (van der Vorst 1992) for Dhat x = rhs on the even sites.
 * x enters as the initial guess.  Stops when the recursive residual satisfies
 * |r| <= tol |rhs|, or after maxit iterations.  Returns the iteration count. */
static int bicgstab_dhat(const box_t *b, const int *par, double kappa, const cplx *U,
                         const cplx *rhs, cplx *x, double tol, int maxit, cplx *work)
{
    const size_t n = (size_t)b->S * 12;
    cplx *r = work, *rh = r + n, *p = rh + n, *v = p + n, *s = v + n, *t = s + n, *tmp = t + n;
    apply_dhat(b, par, kappa, U, x, t, tmp);
    for (size_t i = 0; i < n; i++) r[i] = rhs[i] - t[i];
    memcpy(rh, r, sizeof(cplx) * n);
    memset(p, 0, sizeof(cplx) * n);
    memset(v, 0, sizeof(cplx) * n);
    const double bn2 = vnorm2(rhs, n);
    if (bn2 == 0.0) {
        memset(x, 0, sizeof(cplx) * n);
        return 0;
    }
    cplx rho = 1, alpha = 1, omega = 1;
    int it = 0;
    double rn2 = vnorm2(r, n);
    while (rn2 > tol * tol * bn2 && it < maxit) {
        cplx rho_new = vdot(rh, r, n);
        cplx beta = (rho_new / rho) * (alpha / omega);
        for (size_t i = 0; i < n; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        apply_dhat(b, par, kappa, U, p, v, tmp);
        alpha = rho_new / vdot(rh, v, n);
        for (size_t i = 0; i < n; i++) s[i] = r[i] - alpha * v[i];
        apply_dhat(b, par, kappa, U, s, t, tmp);
        omega = vdot(t, s, n) / vdot(t, t, n);
        for (size_t i = 0; i < n; i++) {
            x[i] += alpha * p[i] + omega * s[i];
            r[i] = s[i] - omega * t[i];
        }
        rho = rho_new;
        rn2 = vnorm2(r, n);
        it++;
        if (!isfinite(rn2)) break;
    }
    return it;
}

/* Solve D_Lambda x = b on one box by the even-odd Schur complement:
 *   Dhat x_e = b_e + kappa H_eo b_o,   x_o = b_o + kappa H_oe x_e,
 * iterated as FP64 defect correction on the true residual b - D_Lambda x until
 * |b - D_Lambda x| <= tol |b|.  Returns total inner iterations, or -1 on
 * failure; *relres receives the final true relative residual. */
static int solve_box(const box_t *b, double kappa, const cplx *U, const cplx *bvec, cplx *x,
                     double tol, int maxit, double *relres)
{
    const size_t n = (size_t)b->S * 12;
    int *par = (int *)malloc(sizeof(int) * b->S);
    cplx *mem = (cplx *)calloc(n * 12, sizeof(cplx));
    if (!par || !mem) {
        free(par);
        free(mem);
        return -1;
    }
    for (int s = 0; s < b->S; s++) par[s] = box_parity(b, s);
    cplx *res = mem, *rhs = res + n, *e = rhs + n, *tmp = e + n, *work = tmp + n;
    memset(x, 0, sizeof(cplx) * n);
    memcpy(res, bvec, sizeof(cplx) * n);
    const double bn2 = vnorm2(bvec, n);
    int total = 0, status = 0;
    double rr = bn2;
    for (int outer = 0; outer < 20 && rr > tol * tol * bn2; outer++) {
        /* rhs_e = res_e + kappa (H res_o)_e */
        memcpy(tmp, res, sizeof(cplx) * n);
        zero_parity(b, par, tmp, 0);
        box_hop(b, U, (const cplx (*)[4][3])tmp, (cplx (*)[4][3])rhs);
        zero_parity(b, par, rhs, 1);
        for (size_t i = 0; i < n; i++) rhs[i] = kappa * rhs[i];
        for (int s = 0; s < b->S; s++)
            if (par[s] == 0)
                for (int k = 0; k < 12; k++) rhs[(size_t)s * 12 + k] += res[(size_t)s * 12 + k];
        memset(e, 0, sizeof(cplx) * n);
        /* the inner tolerance is set below the outer one; the defect
         * correction loop removes the drift of the recursive residual */
        int it = bicgstab_dhat(b, par, kappa, U, rhs, e, tol * 0.1, maxit, work);
        total += it;
        /* e_o = res_o + kappa (H e_e)_o */
        box_hop(b, U, (const cplx (*)[4][3])e, (cplx (*)[4][3])tmp);
        for (int s = 0; s < b->S; s++)
            if (par[s] == 1)
                for (int k = 0; k < 12; k++) {
                    size_t i = (size_t)s * 12 + k;
                    e[i] = res[i] + kappa * tmp[i];
                }
        for (size_t i = 0; i < n; i++) x[i] += e[i];
        /* true residual */
        box_hop(b, U, (const cplx (*)[4][3])x, (cplx (*)[4][3])tmp);
        for (size_t i = 0; i < n; i++) res[i] = bvec[i] - (x[i] - kappa * tmp[i]);
        rr = vnorm2(res, n);
        if (!isfinite(rr)) {
            status = -1;
            break;
        }
    }
    *relres = bn2 > 0 ? sqrt(rr / bn2) : 0.0;
    free(par);
    free(mem);
    return status < 0 ? -1 : total;
}

int or_solve_box(const int *L, int tbc, double kappa, const double *U, const int *o,
                 const int *e, const double *bvec, double *x, double tol, int maxit,
                 double *relres)
{
    box_t b;
    box_init(&b, L, tbc, o, e);
    return solve_box(&b, kappa, (const cplx *)U, (const cplx *)bvec, (cplx *)x, tol, maxit,
                     relres);
}

/* Many independent block solves, in parallel over (block, rhs) pairs.
 *   boxes   [nblk][8]: origin[4], extent[4]
 *   b, x    [nrhs][sum_b S_b][4][3] complex (blocks concatenated in list order,
 *           each block in box-local canonical order)
 *   iters, relres [nrhs*nblk] (rhs-major)
 * nthreads <= 0 uses the OpenMP default.  Returns the number of pairs that
 * missed tol (or failed). */
int or_solve_many(const int *L, int tbc, double kappa, const double *U, int nblk,
                  const int *boxes, int nrhs, const double *bvec, double *x, double tol,
                  int maxit, int *iters, double *relres, int nthreads)
{
    size_t *off = (size_t *)malloc(sizeof(size_t) * (nblk + 1));
    off[0] = 0;
    for (int k = 0; k < nblk; k++) {
        const int *bx = &boxes[8 * k];
        off[k + 1] = off[k] + (size_t)bx[4] * bx[5] * bx[6] * bx[7];
    }
    const size_t per_rhs = off[nblk] * 12; /* complex numbers per rhs */
    int fails = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : fails)
    for (int pair = 0; pair < nrhs * nblk; pair++) {
        const int r = pair / nblk, k = pair % nblk;
        box_t b;
        box_init(&b, L, tbc, &boxes[8 * k], &boxes[8 * k + 4]);
        const cplx *bb = (const cplx *)bvec + (size_t)r * per_rhs + off[k] * 12;
        cplx *xx = (cplx *)x + (size_t)r * per_rhs + off[k] * 12;
        double rr = 0;
        int it = solve_box(&b, kappa, (const cplx *)U, bb, xx, tol, maxit, &rr);
        iters[pair] = it;
        relres[pair] = rr;
        if (it < 0 || !(rr <= tol)) fails++;
    }
    free(off);
    return fails;
}

/* Number of OpenMP threads a parallel region would use. */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
