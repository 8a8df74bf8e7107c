// The clover (Sheikholeslami-Wohlert) term of the Dirac operator (Section 3
// takes D to be the Wilson or Sheikholeslami-Wohlert operator; the term is
// the textbook one, in the hopping normalisation D = 1 - kappa H + (A - 1)):
//
//   A(x) = 1 + i kappa c_sw sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}(x),
//   sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu],
//   Fhat_{mu nu}(x) = (Q_{mu nu}(x) - Q_{mu nu}(x)^+) / 8,
//
// Q_{mu nu}(x) the sum of the four plaquettes of the (mu, nu) plane that start
// and end at x, each traversed mu-then-nu.  The gauge field is periodic in
// every direction.  A(x) is block diagonal in the chirality (it commutes with
// gamma_5), each block a hermitian 6x6 over (spin within the block, colour).
// A block restriction D_Lambda keeps A(x) of the whole lattice at its sites,
// so the build reads the global gauge field around every block site.
//
// Storage per block site (kCloverReals, the layout of clover_mul in
// dd_stencil.h), structure of arrays per block like the links: real k of
// block slot s at soff[b] * kCloverReals + k * S_b + s.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <string>

#include "dd_geometry.h"
#include "dd_host.h"
#include "dd_internal.h"
#include "dd_stencil.h"

using namespace dd;

namespace {

// The chirality blocks of sigma_{mu nu} for the six planes (0,1), (0,2),
// (0,3), (1,2), (1,3), (2,3): s[c][p][2a + b] (re, im).
struct Sigmas {
    double re[2][6][4], im[2][6][4];
};

constexpr int kPlaneMu[6] = {0, 0, 0, 1, 1, 2};
constexpr int kPlaneNu[6] = {1, 2, 3, 2, 3, 3};

// sigma_{mu nu} = i gamma_mu gamma_nu (mu != nu).  In the chiral basis of the
// hop kernels gamma_mu = [[0, e_mu], [e_mu^+, 0]] (the projector table of
// dd_stencil.h), so gamma_mu gamma_nu = diag(e_mu e_nu^+, e_mu^+ e_nu):
// e_0 = -1, e_1 = [[0, -i], [-i, 0]], e_2 = [[0, -1], [1, 0]], e_3 = [[-i, 0], [0, i]].
Sigmas make_sigmas()
{
    using cd = std::complex<double>;
    const cd I(0, 1);
    const cd e[4][2][2] = {
        {{-1.0, 0.0}, {0.0, -1.0}},
        {{0.0, -I}, {-I, 0.0}},
        {{0.0, -1.0}, {1.0, 0.0}},
        {{-I, 0.0}, {0.0, I}},
    };
    Sigmas s{};
    for (int p = 0; p < 6; p++) {
        const int mu = kPlaneMu[p], nu = kPlaneNu[p];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                cd up = 0, dn = 0;
                for (int k = 0; k < 2; k++) {
                    up += e[mu][a][k] * std::conj(e[nu][b][k]);  // (e_mu e_nu^+)_{ab}
                    dn += std::conj(e[mu][k][a]) * e[nu][k][b];  // (e_mu^+ e_nu)_{ab}
                }
                up *= I;
                dn *= I;
                s.re[0][p][2 * a + b] = up.real();
                s.im[0][p][2 * a + b] = up.imag();
                s.re[1][p][2 * a + b] = dn.real();
                s.im[1][p][2 * a + b] = dn.imag();
            }
    }
    return s;
}

// 3x3 complex matrix
struct M3 {
    double r[9], i[9];
};

__device__ __forceinline__ void load_u(const double *U, int64_t n, int mu, M3 &m)
{
    const double *u = U + (n * 4 + mu) * 18;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        m.r[k] = u[2 * k];
        m.i[k] = u[2 * k + 1];
    }
}

// C = op(A) op(B), op = identity or conjugate transpose
template <bool DA, bool DB>
__device__ __forceinline__ void mul3(const M3 &A, const M3 &B, M3 &C)
{
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) {
            double cr = 0, ci = 0;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const int ia = DA ? 3 * k + a : 3 * a + k, ib = DB ? 3 * b + k : 3 * k + b;
                const double ar = A.r[ia], ai = DA ? -A.i[ia] : A.i[ia];
                const double br = B.r[ib], bi = DB ? -B.i[ib] : B.i[ib];
                cr = fma(ar, br, fma(-ai, bi, cr));
                ci = fma(ar, bi, fma(ai, br, ci));
            }
            C.r[3 * a + b] = cr;
            C.i[3 * a + b] = ci;
        }
}

struct Lat {
    int L[4];
    __device__ __forceinline__ int64_t idx(const int x[4]) const
    {
        return (((int64_t)x[0] * L[1] + x[1]) * L[2] + x[2]) * L[3] + x[3];
    }
    // the site x + dmu mu-hat + dnu nu-hat (periodic)
    __device__ __forceinline__ int64_t at(const int x[4], int mu, int dmu, int nu, int dnu) const
    {
        int y[4] = {x[0], x[1], x[2], x[3]};
        y[mu] = (y[mu] + dmu + L[mu]) % L[mu];
        y[nu] = (y[nu] + dnu + L[nu]) % L[nu];
        return idx(y);
    }
};

// Fhat_{mu nu}(x) from the four leaves
__device__ void field_strength(const double *U, const Lat &lat, const int x[4], int mu, int nu, M3 &F)
{
    const int64_t n = lat.idx(x);
    M3 Q, a, b, t, u;
#pragma unroll
    for (int k = 0; k < 9; k++) Q.r[k] = Q.i[k] = 0;
    // leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    load_u(U, n, mu, a);
    load_u(U, lat.at(x, mu, 1, nu, 0), nu, b);
    mul3<false, false>(a, b, t);
    load_u(U, lat.at(x, mu, 0, nu, 1), mu, a);
    mul3<false, true>(t, a, u);
    load_u(U, n, nu, a);
    mul3<false, true>(u, a, t);
#pragma unroll
    for (int k = 0; k < 9; k++) { Q.r[k] += t.r[k]; Q.i[k] += t.i[k]; }
    // leaf 2: U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu)
    load_u(U, n, nu, a);
    load_u(U, lat.at(x, mu, -1, nu, 1), mu, b);
    mul3<false, true>(a, b, t);
    load_u(U, lat.at(x, mu, -1, nu, 0), nu, a);
    mul3<false, true>(t, a, u);
    load_u(U, lat.at(x, mu, -1, nu, 0), mu, a);
    mul3<false, false>(u, a, t);
#pragma unroll
    for (int k = 0; k < 9; k++) { Q.r[k] += t.r[k]; Q.i[k] += t.i[k]; }
    // leaf 3: U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
    load_u(U, lat.at(x, mu, -1, nu, 0), mu, a);
    load_u(U, lat.at(x, mu, -1, nu, -1), nu, b);
    mul3<true, true>(a, b, t);
    load_u(U, lat.at(x, mu, -1, nu, -1), mu, a);
    mul3<false, false>(t, a, u);
    load_u(U, lat.at(x, mu, 0, nu, -1), nu, a);
    mul3<false, false>(u, a, t);
#pragma unroll
    for (int k = 0; k < 9; k++) { Q.r[k] += t.r[k]; Q.i[k] += t.i[k]; }
    // leaf 4: U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+
    load_u(U, lat.at(x, mu, 0, nu, -1), nu, a);
    load_u(U, lat.at(x, mu, 0, nu, -1), mu, b);
    mul3<true, false>(a, b, t);
    load_u(U, lat.at(x, mu, 1, nu, -1), nu, a);
    mul3<false, false>(t, a, u);
    load_u(U, n, mu, a);
    mul3<false, true>(u, a, t);
#pragma unroll
    for (int k = 0; k < 9; k++) { Q.r[k] += t.r[k]; Q.i[k] += t.i[k]; }
#pragma unroll
    for (int a3 = 0; a3 < 3; a3++)
#pragma unroll
        for (int b3 = 0; b3 < 3; b3++) {
            F.r[3 * a3 + b3] = (Q.r[3 * a3 + b3] - Q.r[3 * b3 + a3]) * 0.125;
            F.i[3 * a3 + b3] = (Q.i[3 * a3 + b3] + Q.i[3 * b3 + a3]) * 0.125;
        }
}

// Packed hermitian store of a 6x6 (diagonal real parts, then the entries
// above the diagonal row by row) at real offset k0 of the site.
template <typename T>
__device__ __forceinline__ void store_packed(T *blk, int64_t S, int s, int k0, const double (&mr)[6][6],
                                             const double (&mi)[6][6])
{
#pragma unroll
    for (int i = 0; i < 6; i++) blk[(int64_t)(k0 + i) * S + s] = (T)mr[i][i];
    int t = 0;
#pragma unroll
    for (int i = 0; i < 6; i++)
#pragma unroll
        for (int j = i + 1; j < 6; j++, t++) {
            blk[(int64_t)(k0 + 6 + 2 * t) * S + s] = (T)mr[i][j];
            blk[(int64_t)(k0 + 7 + 2 * t) * S + s] = (T)mi[i][j];
        }
}

// One thread per block site: A and A^-1 (Gauss-Jordan with partial pivoting,
// FP64, the row exchanges as selects so that every register index is static).
// Sites in a block's hole (hole[q] != 0; hole may be null) get A = 1, so the
// operator stays the identity there as it is for the Wilson operator.
__global__ void __launch_bounds__(64) k_clover_build(PackGeom g, const double *U, Sigmas sg, double kc, double *a64,
                                                     double *i64, float *a32, float *i32, int64_t total,
                                                     const uint8_t *hole)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const bool in_hole = hole && hole[q] != 0;
    const int b = find_block(g.soff, g.nb, q);
    const int s = (int)(q - g.soff[b]);
    const int64_t S = 2 * (int64_t)g.h[b];
    int c[4];
    local_coords(g.perm[g.perm_off[b] + s], g.ext + 4 * b, c);
    int x[4];
    Lat lat;
    for (int m = 0; m < 4; m++) {
        lat.L[m] = g.L[m];
        x[m] = (g.origin[4 * b + m] + c[m]) % g.L[m];
    }
    const int64_t base = g.soff[b] * kCloverReals;
    for (int ch = 0; ch < 2; ch++) {
        double ar[6][6], ai[6][6];
#pragma unroll
        for (int i = 0; i < 6; i++)
#pragma unroll
            for (int j = 0; j < 6; j++) {
                ar[i][j] = i == j ? 1.0 : 0.0;
                ai[i][j] = 0.0;
            }
#pragma unroll 1
        for (int p = 0; p < (in_hole ? 0 : 6); p++) {
            M3 F;
            field_strength(U, lat, x, kPlaneMu[p], kPlaneNu[p], F);
            // A += i kc (s_p (x) F): entry (3a + ci, 3b + di) += i kc s[a][b] F[ci][di]
#pragma unroll
            for (int a2 = 0; a2 < 2; a2++)
#pragma unroll
                for (int b2 = 0; b2 < 2; b2++) {
                    const double sr = sg.re[ch][p][2 * a2 + b2], si = sg.im[ch][p][2 * a2 + b2];
#pragma unroll
                    for (int ci = 0; ci < 3; ci++)
#pragma unroll
                        for (int di = 0; di < 3; di++) {
                            const double fr = F.r[3 * ci + di], fi = F.i[3 * ci + di];
                            // i (s F) = -(s_r f_i + s_i f_r) + i (s_r f_r - s_i f_i)
                            ar[3 * a2 + ci][3 * b2 + di] -= kc * (sr * fi + si * fr);
                            ai[3 * a2 + ci][3 * b2 + di] += kc * (sr * fr - si * fi);
                        }
                }
        }
        const int k0 = ch * kCloverHalf;
        store_packed(a64 + base, S, s, k0, ar, ai);
        if (a32) store_packed(a32 + base, S, s, k0, ar, ai);
        // [A | 1] -> [1 | A^-1]
        double er[6][12], ei[6][12];
#pragma unroll
        for (int i = 0; i < 6; i++)
#pragma unroll
            for (int j = 0; j < 12; j++) {
                er[i][j] = j < 6 ? ar[i][j] : (j - 6 == i ? 1.0 : 0.0);
                ei[i][j] = j < 6 ? ai[i][j] : 0.0;
            }
#pragma unroll
        for (int k = 0; k < 6; k++) {
            int piv = k;
            double best = er[k][k] * er[k][k] + ei[k][k] * ei[k][k];
#pragma unroll
            for (int r = k + 1; r < 6; r++) {
                const double m = er[r][k] * er[r][k] + ei[r][k] * ei[r][k];
                if (m > best) {
                    best = m;
                    piv = r;
                }
            }
#pragma unroll
            for (int r = k + 1; r < 6; r++) {
                const bool sw = piv == r;
#pragma unroll
                for (int j = 0; j < 12; j++) {
                    const double tr = er[k][j], ti = ei[k][j];
                    er[k][j] = sw ? er[r][j] : tr;
                    ei[k][j] = sw ? ei[r][j] : ti;
                    er[r][j] = sw ? tr : er[r][j];
                    ei[r][j] = sw ? ti : ei[r][j];
                }
            }
            const double den = er[k][k] * er[k][k] + ei[k][k] * ei[k][k];
            const double pr = er[k][k] / den, pi = -ei[k][k] / den;  // 1 / pivot
#pragma unroll
            for (int j = 0; j < 12; j++) {
                const double vr = er[k][j], vi = ei[k][j];
                er[k][j] = vr * pr - vi * pi;
                ei[k][j] = vr * pi + vi * pr;
            }
#pragma unroll
            for (int r = 0; r < 6; r++) {
                if (r == k) continue;
                const double fr = er[r][k], fi = ei[r][k];
#pragma unroll
                for (int j = 0; j < 12; j++) {
                    er[r][j] -= fr * er[k][j] - fi * ei[k][j];
                    ei[r][j] -= fr * ei[k][j] + fi * er[k][j];
                }
            }
        }
        double vr[6][6], vi[6][6];
#pragma unroll
        for (int i = 0; i < 6; i++)
#pragma unroll
            for (int j = 0; j < 6; j++) {
                vr[i][j] = er[i][6 + j];
                vi[i][j] = ei[i][6 + j];
            }
        store_packed(i64 + base, S, s, k0, vr, vi);
        if (i32) store_packed(i32 + base, S, s, k0, vr, vi);
    }
}

// y = C x on half field `parity`: one thread per (rhs, half-field site).
template <typename SP>
__global__ void __launch_bounds__(256) k_clover_apply(const int64_t *soff, const int32_t *hh, int nb, const SP *C,
                                                      const SP *x, SP *y, int parity, int nr, int64_t half_total,
                                                      const int32_t *mask)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= half_total * nr) return;
    const int r = (int)(t / half_total);
    const int64_t q = t - (int64_t)r * half_total;
    const int b = find_block(soff, nb, 2 * q);  // soff[b] / 2 <= q < soff[b + 1] / 2
    if (mask && !mask[r * nb + b]) return;
    const int hb = hh[b];
    const int h = (int)(q - soff[b] / 2);
    const int64_t base = (soff[b] >> 1) * 24 * nr + (int64_t)r * 24 * hb + h;
    SP v[24];
#pragma unroll
    for (int c = 0; c < 24; c++) v[c] = x[base + (int64_t)c * hb];
    const Buf cb = make_buf(C + soff[b] * kCloverReals, (uint32_t)(kCloverReals * 2 * hb) * (uint32_t)sizeof(SP));
    clover_mul<SP, SP>(v, cb, (uint32_t)(parity * hb + h) * (uint32_t)sizeof(SP), (uint32_t)(2 * hb) * (uint32_t)sizeof(SP));
#pragma unroll
    for (int c = 0; c < 24; c++) y[base + (int64_t)c * hb] = v[c];
}

// ln det A(x) of every block site from the stored FP64 packed hermitian
// chirality blocks: LU with partial pivoting per block (row exchanges as
// selects, so that every register index is static); out[2 q] = sum of
// ln |U_ii| over both blocks, out[2 q + 1] = the sum of their phases plus pi
// per exchange (A is hermitian, so the phase is a multiple of pi up to
// rounding).
__global__ void __launch_bounds__(64) k_clover_logdet(const int64_t *soff, int nb, const double *a64, double *out,
                                                      int64_t total)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int b = find_block(soff, nb, q);
    const int64_t S = soff[b + 1] - soff[b], s = q - soff[b];
    const double *blk = a64 + soff[b] * kCloverReals;
    double lr = 0, ph = 0;
    for (int ch = 0; ch < 2; ch++) {
        const int k0 = ch * kCloverHalf;
        double mr[6][6], mi[6][6];
#pragma unroll
        for (int i = 0; i < 6; i++) {
            mr[i][i] = blk[(int64_t)(k0 + i) * S + s];
            mi[i][i] = 0.0;
        }
        int t = 0;
#pragma unroll
        for (int i = 0; i < 6; i++)
#pragma unroll
            for (int j = i + 1; j < 6; j++, t++) {
                const double hr = blk[(int64_t)(k0 + 6 + 2 * t) * S + s], hi = blk[(int64_t)(k0 + 7 + 2 * t) * S + s];
                mr[i][j] = hr;
                mi[i][j] = hi;
                mr[j][i] = hr;
                mi[j][i] = -hi;
            }
#pragma unroll
        for (int p = 0; p < 6; p++) {
            int piv = p;
            double best = mr[p][p] * mr[p][p] + mi[p][p] * mi[p][p];
#pragma unroll
            for (int r = p + 1; r < 6; r++) {
                const double m2 = mr[r][p] * mr[r][p] + mi[r][p] * mi[r][p];
                if (m2 > best) {
                    best = m2;
                    piv = r;
                }
            }
#pragma unroll
            for (int r = p + 1; r < 6; r++) {
                const bool sw = r == piv;
#pragma unroll
                for (int j = 0; j < 6; j++) {
                    const double xr = mr[p][j], xi = mi[p][j], yr = mr[r][j], yi = mi[r][j];
                    mr[p][j] = sw ? yr : xr;
                    mi[p][j] = sw ? yi : xi;
                    mr[r][j] = sw ? xr : yr;
                    mi[r][j] = sw ? xi : yi;
                }
            }
            if (piv != p) ph += M_PI;
            const double dr = mr[p][p], di = mi[p][p], d2 = dr * dr + di * di;
            lr += 0.5 * log(d2);
            ph += atan2(di, dr);
#pragma unroll
            for (int r = p + 1; r < 6; r++) {
                // f = m[r][p] / d
                const double fr = (mr[r][p] * dr + mi[r][p] * di) / d2, fi = (mi[r][p] * dr - mr[r][p] * di) / d2;
#pragma unroll
                for (int j = p + 1; j < 6; j++) {
                    mr[r][j] -= fr * mr[p][j] - fi * mi[p][j];
                    mi[r][j] -= fr * mi[p][j] + fi * mr[p][j];
                }
            }
        }
    }
    out[2 * q] = lr;
    out[2 * q + 1] = ph;
}

// ld[2 b] += sum of the block's site values, ld[2 b + 1] += their phases
// (wrapped into (-pi, pi]); fixed-order sums, one workgroup per block.
__global__ void __launch_bounds__(256) k_clover_logdet_add(const double *site, const int64_t *soff, double *ld)
{
    __shared__ double sre[256], sim[256];
    const int b = blockIdx.x;
    double re = 0, im = 0;
    for (int64_t q = soff[b] + threadIdx.x; q < soff[b + 1]; q += 256) {
        re += site[2 * q];
        im += site[2 * q + 1];
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sre[threadIdx.x] += sre[threadIdx.x + w];
            sim[threadIdx.x] += sim[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ld[2 * b] += sre[0];
        double p = fmod(ld[2 * b + 1] + sim[0], 2 * M_PI);
        if (p > M_PI) p -= 2 * M_PI;
        if (p <= -M_PI) p += 2 * M_PI;
        ld[2 * b + 1] = p;
    }
}

}  // namespace

namespace dd {

hipError_t launch_clover_build(const dd_blocks *B, const double *U, double kappa, double csw, double *a64,
                               double *i64, float *a32, float *i32, const uint8_t *hole, hipStream_t s)
{
    const int64_t total = B->soff[B->nb];
    if (total == 0) return hipSuccess;
    const PackGeom g = pack_geom(B);
    hipLaunchKernelGGL(k_clover_build, dim3((unsigned)((total + 63) / 64)), dim3(64), 0, s, g, U, make_sigmas(),
                       kappa * csw, a64, i64, a32, i32, total, hole);
    return hipGetLastError();
}

hipError_t launch_clover_apply(const dd_blocks *B, const void *C, const void *x, void *y, int parity, int n_rhs,
                               dd_prec sp, const int32_t *mask, hipStream_t s)
{
    const int64_t half = B->soff[B->nb] / 2, n = half * n_rhs;
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256)), t(256);
    if (sp == DD_F64)
        hipLaunchKernelGGL(k_clover_apply<double>, grid, t, 0, s, B->d_soff, B->d_h, B->nb, (const double *)C,
                           (const double *)x, (double *)y, parity, n_rhs, half, mask);
    else if (sp == DD_F32)
        hipLaunchKernelGGL(k_clover_apply<float>, grid, t, 0, s, B->d_soff, B->d_h, B->nb, (const float *)C,
                           (const float *)x, (float *)y, parity, n_rhs, half, mask);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_clover_logdet_add(const dd_blocks *B, const double *a64, double *site, double *ld, hipStream_t s)
{
    const int64_t total = B->soff[B->nb];
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_clover_logdet, dim3((unsigned)((total + 63) / 64)), dim3(64), 0, s, B->d_soff, B->nb, a64,
                       site, total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_clover_logdet_add, dim3(B->nb), dim3(256), 0, s, site, B->d_soff, ld);
    return hipGetLastError();
}

void clover_release(dd_gauge *G)
{
    hipFree(G->d_cla64);
    hipFree(G->d_cli64);
    hipFree(G->d_cla32);
    hipFree(G->d_cli32);
    G->d_cla64 = G->d_cli64 = nullptr;
    G->d_cla32 = G->d_cli32 = nullptr;
    G->cl_kappa = G->cl_csw = 0.0;
}

}  // namespace dd

extern "C" dd_status dd_gauge_set_clover(dd_ctx *ctx, dd_gauge *G, const void *U_dev, double kappa, double csw)
{
    if (!ctx || !G) return fail(ctx, DD_EINVAL, "null argument");
    if (!std::isfinite(kappa) || !std::isfinite(csw)) return fail(ctx, DD_EINVAL, "kappa and c_sw must be finite");
    HIPCHECK(ctx, enter(ctx));
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    clover_release(G);
    if (csw == 0.0) return DD_OK;
    if (!U_dev) return fail(ctx, DD_EINVAL, "null gauge field");
    const dd_blocks *B = G->blocks;
    if ((int64_t)2 * B->max_h * kCloverReals * 8 >= ((int64_t)1 << 32))
        return fail(ctx, DD_EUNSUPPORTED, "block too large for the clover term's 32-bit offsets");
    const size_t n = (size_t)B->soff[B->nb] * kCloverReals;
    hipError_t e = hipMalloc(&G->d_cla64, std::max<size_t>(n, 1) * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&G->d_cli64, std::max<size_t>(n, 1) * sizeof(double));
    if (e == hipSuccess && G->low != DD_F64) e = hipMalloc(&G->d_cla32, std::max<size_t>(n, 1) * sizeof(float));
    if (e == hipSuccess && G->low != DD_F64) e = hipMalloc(&G->d_cli32, std::max<size_t>(n, 1) * sizeof(float));
    if (e != hipSuccess) {
        clover_release(G);
        return fail(ctx, DD_ENOMEM, std::string("clover term: ") + hipGetErrorString(e));
    }
    // hole sites (frames, inactive regions) keep the identity
    const std::vector<uint8_t> hs = hole_slots(B);
    uint8_t *hole = nullptr;
    if (e == hipSuccess && !hs.empty()) {
        hole = (uint8_t *)workspace(ctx, "cl_hole", hs.size(), &e);
        if (hole) e = hipMemcpyAsync(hole, hs.data(), hs.size(), hipMemcpyHostToDevice, ctx->stream);
    }
    if (e == hipSuccess)
        e = launch_clover_build(B, (const double *)U_dev, kappa, csw, G->d_cla64, G->d_cli64, G->d_cla32,
                                G->d_cli32, hole, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        clover_release(G);
        return fail(ctx, DD_EDEVICE, std::string("clover build: ") + hipGetErrorString(e));
    }
    G->cl_kappa = kappa;
    G->cl_csw = csw;
    return DD_OK;
}
