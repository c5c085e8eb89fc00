/*
 * Plain CPU FP64 oracle for the MRT lattice Boltzmann model of Chai, Shi & Guo.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Shares no code
 * with the GPU library.  Build: gcc -O2 -ffp-contract=off -fopenmp (see
 * oracle/build.py).
 *
 * What each part follows:
 *   lattices           Eq. 5 (D2Q9), Eq. 6 (D3Q19); cs^2 = c^2/3, c = 1
 *   transform M        Eq. 15 (D2Q9); D3Q19: the orthogonal polynomial basis of
 *                      d'Humieres et al. (2002), which the paper cites for the
 *                      3-D extension it leaves to the reader (end of Sec. 2.3)
 *   M^-1               Gaussian elimination (not the transpose formula)
 *   C(phi)             Eq. 7, integral from 0, Gauss-Legendre quadrature
 *   equilibrium        Eq. 3, in velocity space
 *   relaxation         Eq. 2 / Eq. 17: S diagonal, A block (Eq. 21) on the
 *                      flux rows, A from K by Eq. 26
 *   source             Eq. 9 with Btilde of Eq. 28; Scheme A and B of Remark II
 *   initialisation     Eq. 40
 *   walls              anti-bounce-back with the wall half a link beyond the
 *                      last node (Sec. 3.6, the channel problem)
 *   adjoint            complex-step differentiation (Squire & Trapp 1998) of
 *                      the per-node collision map, transposed streaming
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#include "lbm_oracle.h"

#define ORC_CS2 (1.0 / 3.0)
#define ORC_NGL 8
#define ORC_H 1e-30

typedef struct orc_tabs {
    int q, dim;
    int c[19][3];
    double w[19];
    int opp[19];
    int jrow[3];
    double M[19 * 19];
    double Minv[19 * 19];
    double glx[ORC_NGL], glw[ORC_NGL];
} orc_tabs;

/* ---- lattices (Eq. 5, Eq. 6) ------------------------------------------- */

static const int C9[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                             {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};

static const int C19[19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {-1, 0, 1},
    {1, 0, -1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

/* Eq. 15, rows rho, e, eps, jx, qx, jy, qy, pxx, pxy */
static const int M9[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

/* D3Q19 polynomial basis rows evaluated at one velocity (d'Humieres et al.). */
static void d3q19_basis_row(const int *cv, double *row)
{
    double cx = cv[0], cy = cv[1], cz = cv[2];
    double c2 = cx * cx + cy * cy + cz * cz;
    row[0] = 1.0;
    row[1] = 19.0 * c2 - 30.0;
    row[2] = (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    row[3] = cx;
    row[4] = (5.0 * c2 - 9.0) * cx;
    row[5] = cy;
    row[6] = (5.0 * c2 - 9.0) * cy;
    row[7] = cz;
    row[8] = (5.0 * c2 - 9.0) * cz;
    row[9] = 3.0 * cx * cx - c2;
    row[10] = (3.0 * c2 - 5.0) * (3.0 * cx * cx - c2);
    row[11] = cy * cy - cz * cz;
    row[12] = (3.0 * c2 - 5.0) * (cy * cy - cz * cz);
    row[13] = cx * cy;
    row[14] = cy * cz;
    row[15] = cx * cz;
    row[16] = (cy * cy - cz * cz) * cx;
    row[17] = (cz * cz - cx * cx) * cy;
    row[18] = (cx * cx - cy * cy) * cz;
}

/* Alternative orthogonal D3Q19 basis: same density and flux rows, the other
 * fifteen rows from Gram-Schmidt on fixed pseudo-random integer vectors.
 * Only used to show that results with equal non-flux rates do not depend on
 * the choice of basis. */
static void d3q19_alt_basis(double *M)
{
    const int q = 19;
    int fixed[4] = {0, 3, 5, 7};
    int have[19] = {0};
    for (int k = 0; k < q; ++k) {
        M[0 * q + k] = 1.0;
        M[3 * q + k] = C19[k][0];
        M[5 * q + k] = C19[k][1];
        M[7 * q + k] = C19[k][2];
    }
    for (int i = 0; i < 4; ++i) have[fixed[i]] = 1;
    unsigned long long state = 0x9E3779B97F4A7C15ULL;
    for (int r = 0; r < q; ++r) {
        if (have[r]) continue;
        for (;;) {
            double v[19];
            for (int k = 0; k < q; ++k) {
                state = state * 6364136223846793005ULL + 1442695040888963407ULL;
                v[k] = (double)((int)((state >> 33) % 7ULL) - 3);
            }
            for (int r2 = 0; r2 < q; ++r2) {
                if (!have[r2]) continue;
                double num = 0.0, den = 0.0;
                for (int k = 0; k < q; ++k) { num += v[k] * M[r2 * q + k]; den += M[r2 * q + k] * M[r2 * q + k]; }
                for (int k = 0; k < q; ++k) v[k] -= num / den * M[r2 * q + k];
            }
            double nrm = 0.0;
            for (int k = 0; k < q; ++k) nrm += v[k] * v[k];
            if (nrm > 1e-6) {
                for (int k = 0; k < q; ++k) M[r * q + k] = v[k] / sqrt(nrm);
                have[r] = 1;
                break;
            }
        }
    }
}

/* Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n. */
static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1; p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

static void build_tabs(const orc_params *p, orc_tabs *tb)
{
    memset(tb, 0, sizeof(*tb));
    tb->q = p->q;
    tb->dim = (p->q == 9) ? 2 : 3;
    if (p->q == 9) {
        for (int k = 0; k < 9; ++k) {
            tb->c[k][0] = C9[k][0]; tb->c[k][1] = C9[k][1]; tb->c[k][2] = 0;
            tb->w[k] = (k == 0) ? 4.0 / 9.0 : (k < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        }
        for (int i = 0; i < 9; ++i) for (int k = 0; k < 9; ++k) tb->M[i * 9 + k] = M9[i][k];
        tb->jrow[0] = 3; tb->jrow[1] = 5; tb->jrow[2] = -1;
    } else {
        for (int k = 0; k < 19; ++k) {
            for (int a = 0; a < 3; ++a) tb->c[k][a] = C19[k][a];
            tb->w[k] = (k == 0) ? 1.0 / 3.0 : (k < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
        }
        if (p->basis == 0) {
            for (int k = 0; k < 19; ++k) {
                double row[19];
                d3q19_basis_row(C19[k], row);
                for (int i = 0; i < 19; ++i) tb->M[i * 19 + k] = row[i];
            }
        } else {
            d3q19_alt_basis(tb->M);
        }
        tb->jrow[0] = 3; tb->jrow[1] = 5; tb->jrow[2] = 7;
    }
    for (int k = 0; k < tb->q; ++k) {
        for (int j = 0; j < tb->q; ++j)
            if (tb->c[j][0] == -tb->c[k][0] && tb->c[j][1] == -tb->c[k][1] && tb->c[j][2] == -tb->c[k][2])
                tb->opp[k] = j;
    }
    /* M^-1 by Gaussian elimination against the identity */
    {
        const int q = tb->q;
        double a[19 * 19];
        memcpy(a, tb->M, sizeof(double) * q * q);
        for (int i = 0; i < q; ++i) for (int j = 0; j < q; ++j) tb->Minv[i * q + j] = (i == j) ? 1.0 : 0.0;
        for (int col = 0; col < q; ++col) {
            int piv = col;
            for (int r = col + 1; r < q; ++r) if (fabs(a[r * q + col]) > fabs(a[piv * q + col])) piv = r;
            for (int j = 0; j < q; ++j) {
                double t = a[col * q + j]; a[col * q + j] = a[piv * q + j]; a[piv * q + j] = t;
                t = tb->Minv[col * q + j]; tb->Minv[col * q + j] = tb->Minv[piv * q + j]; tb->Minv[piv * q + j] = t;
            }
            double inv = 1.0 / a[col * q + col];
            for (int j = 0; j < q; ++j) { a[col * q + j] *= inv; tb->Minv[col * q + j] *= inv; }
            for (int r = 0; r < q; ++r) {
                if (r == col) continue;
                double fct = a[r * q + col];
                if (fct == 0.0) continue;
                for (int j = 0; j < q; ++j) { a[r * q + j] -= fct * a[col * q + j]; tb->Minv[r * q + j] -= fct * tb->Minv[col * q + j]; }
            }
        }
    }
    gauss_legendre(ORC_NGL, tb->glx, tb->glw);
}

/* ---- per-node arithmetic, real and complex instantiations --------------- */

#define T double
#define SFX(x) x##_r
#define REPART(x) (x)
#include "orc_node.inc"
#undef T
#undef SFX
#undef REPART

#define T double complex
#define SFX(x) x##_c
#define REPART(x) creal(x)
#include "orc_node.inc"
#undef T
#undef SFX
#undef REPART

/* ---- public entry points ------------------------------------------------- */

int orc_check(const orc_params *p)
{
    if (p->q != 9 && p->q != 19) return -1;
    if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0) return -1;
    if (p->q == 9 && p->nz != 1) return -1;
    if (!(p->d > 0.0)) return -1;
    int nwall = 0;
    for (int a = 0; a < 3; ++a) {
        if (p->bc[a] != 0 && p->bc[a] != 1) return -1;
        nwall += p->bc[a];
    }
    if (nwall > 1) return -1;
    if (p->q == 9 && p->bc[2] != 0) return -1;
    if (p->scheme != 0 && p->scheme != 1) return -1;
    if (p->variant != 0 && p->variant != 1) return -1;
    {
        int rational = p->bden[0] != 0.0 && p->bden[0] != 1.0;
        for (int i = 1; i < ORC_MAXP; ++i) if (p->bden[i] != 0.0) rational = 1;
        if (rational && p->variant != 1) return -2;   /* C of Eq. 7 for a rational B: Remark III */
    }
    return 0;
}

void orc_tables(const orc_params *p, int *c, double *w, double *M, double *Minv)
{
    orc_tabs tb;
    build_tabs(p, &tb);
    const int q = tb.q;
    for (int k = 0; k < q; ++k) {
        for (int a = 0; a < 3; ++a) c[k * 3 + a] = tb.c[k][a];
        w[k] = tb.w[k];
    }
    memcpy(M, tb.M, sizeof(double) * q * q);
    memcpy(Minv, tb.Minv, sizeof(double) * q * q);
}

static void k0_real(const orc_params *p, const double *kloc, double K[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) K[a][b] = kloc ? kloc[a * 3 + b] : p->k0[a][b];
}

void orc_ctensor(const orc_params *p, double phi, double *out)
{
    orc_tabs tb;
    build_tabs(p, &tb);
    double C[3][3];
    ctensor_r(&tb, p, phi, C);
    for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) out[a * 3 + b] = C[a][b];
}

void orc_feq(const orc_params *p, double phi, double *out)
{
    orc_tabs tb;
    build_tabs(p, &tb);
    double K[3][3];
    k0_real(p, NULL, K);
    coef_r o;
    coefficients_r(&tb, p, phi, (const double (*)[3])K, 0.0, &o);
    equilibrium_r(&tb, p, phi, &o, out);
}

void orc_ablock(const orc_params *p, double phi, const double *kloc, double *out)
{
    orc_tabs tb;
    build_tabs(p, &tb);
    double K[3][3];
    k0_real(p, kloc, K);
    coef_r o;
    coefficients_r(&tb, p, phi, (const double (*)[3])K, 0.0, &o);
    for (int a = 0; a < tb.dim; ++a)
        for (int b = 0; b < tb.dim; ++b) out[a * tb.dim + b] = o.A[a][b];
}

void orc_collide(const orc_params *p, const double *f, double pprev,
                 double rext, double rext_prev, const double *kloc,
                 double *out, double *phi_out)
{
    orc_tabs tb;
    build_tabs(p, &tb);
    double K[3][3];
    k0_real(p, kloc, K);
    collide_r(&tb, p, f, pprev, (const double (*)[3])K, rext, rext_prev, out, phi_out);
}

void orc_init(const orc_params *p, const double *phi0, const double *rext0,
              double *f, double *pprev)
{
    orc_tabs tb;
    build_tabs(p, &tb);
    const long N = (long)p->nx * p->ny * p->nz;
    const int q = tb.q;
    double K[3][3];
    k0_real(p, NULL, K);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double fl[19];
        init_node_r(&tb, p, phi0[n], (const double (*)[3])K, rext0 ? rext0[n] : 0.0, fl);
        for (int k = 0; k < q; ++k) f[(long)k * N + n] = fl[k];
        pprev[n] = phi0[n];
    }
}

/* Even part of Eq. 3 at the wall value: the anti-bounce-back wall term. */
static double wall_even(const orc_tabs *tb, const orc_params *p, int k, double phiw)
{
    double K[3][3];
    k0_real(p, NULL, K);
    coef_r o;
    coefficients_r(tb, p, phiw, (const double (*)[3])K, 0.0, &o);
    double contr = 0.0;
    for (int a = 0; a < tb->dim; ++a)
        for (int b = 0; b < tb->dim; ++b) {
            double tens = o.C[a][b] + p->d * ORC_CS2 * o.D[a][b] - (a == b ? ORC_CS2 * phiw : 0.0);
            double ccm = (double)(tb->c[k][a] * tb->c[k][b]) - (a == b ? ORC_CS2 : 0.0);
            contr += tens * ccm;
        }
    return tb->w[k] * (phiw + contr / (2.0 * ORC_CS2 * ORC_CS2));
}

/* Where population k leaving node (ix,iy,iz) lands.  Returns the target node
 * index, or -1 when it crosses a wall; then *axis and *side name the wall. */
static long target_node(const orc_params *p, const orc_tabs *tb, int ix, int iy, int iz, int k,
                        int *axis, int *side)
{
    int t[3] = {ix + tb->c[k][0], iy + tb->c[k][1], iz + tb->c[k][2]};
    int n[3] = {p->nx, p->ny, p->nz};
    for (int a = 0; a < 3; ++a) {
        if (t[a] >= 0 && t[a] < n[a]) continue;
        if (p->bc[a] == 0) {
            t[a] = (t[a] + n[a]) % n[a];
        } else {
            *axis = a;
            *side = (t[a] < 0) ? 0 : 1;
            return -1;
        }
    }
    return ((long)t[2] * p->ny + t[1]) * p->nx + t[0];
}

int orc_step(const orc_params *p, double *f, double *pprev,
             const double *rext, const double *rext_prev, const double *kfield,
             int nthreads)
{
    if (orc_check(p) != 0) return -1;
    orc_tabs tb;
    build_tabs(p, &tb);
    const long N = (long)p->nx * p->ny * p->nz;
    const int q = tb.q;
    double ewall[3][2][19];
    for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s)
            for (int k = 0; k < q; ++k) ewall[a][s][k] = wall_even(&tb, p, k, p->phi_wall[a][s]);
    double *fn = (double *)malloc(sizeof(double) * q * N);
    double *pn = (double *)malloc(sizeof(double) * N);
    if (!fn || !pn) { free(fn); free(pn); return -3; }
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (long n = 0; n < N; ++n) {
        int ix = (int)(n % p->nx), iy = (int)((n / p->nx) % p->ny), iz = (int)(n / ((long)p->nx * p->ny));
        double fl[19], out[19], phi, K[3][3];
        k0_real(p, kfield ? kfield + 9 * n : NULL, K);
        for (int k = 0; k < q; ++k) fl[k] = f[(long)k * N + n];
        collide_r(&tb, p, fl, pprev[n], (const double (*)[3])K, rext ? rext[n] : 0.0,
                  rext_prev ? rext_prev[n] : 0.0, out, &phi);
        pn[n] = phi;
        for (int k = 0; k < q; ++k) {
            int axis = -1, side = 0;
            long t = target_node(p, &tb, ix, iy, iz, k, &axis, &side);
            if (t >= 0) fn[(long)k * N + t] = out[k];
            else fn[(long)tb.opp[k] * N + n] = -out[k] + 2.0 * ewall[axis][side][k];
        }
    }
    memcpy(f, fn, sizeof(double) * q * N);
    memcpy(pprev, pn, sizeof(double) * N);
    free(fn);
    free(pn);
    return 0;
}

void orc_phi(const orc_params *p, const double *f, const double *rext, double *phi)
{
    const long N = (long)p->nx * p->ny * p->nz;
    for (long n = 0; n < N; ++n) {
        double s = 0.0;
        for (int k = 0; k < p->q; ++k) s += f[(long)k * N + n];
        if (p->scheme == 1) s = phi_scheme_b_r(p, s, rext ? rext[n] : 0.0);   /* Eq. 35 */
        phi[n] = s;
    }
}

/* complex copy of the (possibly local) K matrix */
static void k0_complex(const orc_params *p, const double *kloc, double complex K[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) K[a][b] = kloc ? kloc[a * 3 + b] : p->k0[a][b];
}

/* Columns of the node map's Jacobian by complex step.  Inputs 0..q-1: f,
 * q: pprev, q+1..q+6: K0 upper triangle (xx, xy, xz, yy, yz, zz), perturbed
 * symmetrically.  jac[(q+1) x (q+7)]: rows out[0..q-1], phi. */
static void node_jacobian(const orc_tabs *tb, const orc_params *p, const double *f, double pprev,
                          const double *kloc, double rext, double rext_prev, double *jac)
{
    const int q = tb->q, nin = q + 7;
    static const int tri[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int j = 0; j < nin; ++j) {
        double complex fc[19], out[19], phi, pc = pprev, K[3][3];
        k0_complex(p, kloc, K);
        for (int k = 0; k < q; ++k) fc[k] = f[k];
        if (j < q) fc[j] += I * ORC_H;
        else if (j == q) pc += I * ORC_H;
        else {
            int a = tri[j - q - 1][0], b = tri[j - q - 1][1];
            if (a >= tb->dim || b >= tb->dim) {
                for (int r = 0; r <= q; ++r) jac[r * nin + j] = 0.0;
                continue;
            }
            K[a][b] += I * ORC_H;
            if (a != b) K[b][a] += I * ORC_H;
        }
        collide_c(tb, p, fc, pc, (const double complex (*)[3])K, rext, rext_prev, out, &phi);
        for (int r = 0; r < q; ++r) jac[r * nin + j] = cimag(out[r]) / ORC_H;
        jac[q * nin + j] = cimag(phi) / ORC_H;
    }
}

void orc_node_jacobian(const orc_params *p, const double *f, double pprev, double *jac)
{
    orc_tabs tb;
    build_tabs(p, &tb);
    node_jacobian(&tb, p, f, pprev, NULL, 0.0, 0.0, jac);
}

void orc_adjoint_step(const orc_params *p, const double *f, const double *pprev,
                      const double *lam_next, const double *mu_next,
                      const double *rext, const double *rext_prev,
                      double *lam, double *mu, double *gk, int nthreads)
{
    orc_tabs tb;
    build_tabs(p, &tb);
    const long N = (long)p->nx * p->ny * p->nz;
    const int q = tb.q, nin = q + 7;
    static const int tri[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    double gsum[6] = {0, 0, 0, 0, 0, 0};
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads) reduction(+ : gsum[0:6])
    for (long n = 0; n < N; ++n) {
        int ix = (int)(n % p->nx), iy = (int)((n / p->nx) % p->ny), iz = (int)(n / ((long)p->nx * p->ny));
        double fl[19], lt[19], jac[20 * 26];
        for (int k = 0; k < q; ++k) fl[k] = f[(long)k * N + n];
        /* transposed streaming: where did out[k] of this node go? */
        for (int k = 0; k < q; ++k) {
            int axis = -1, side = 0;
            long t = target_node(p, &tb, ix, iy, iz, k, &axis, &side);
            lt[k] = (t >= 0) ? lam_next[(long)k * N + t] : -lam_next[(long)tb.opp[k] * N + n];
        }
        node_jacobian(&tb, p, fl, pprev[n], NULL, rext ? rext[n] : 0.0, rext_prev ? rext_prev[n] : 0.0, jac);
        for (int j = 0; j < nin; ++j) {
            double acc = 0.0;
            for (int r = 0; r < q; ++r) acc += jac[r * nin + j] * lt[r];
            acc += jac[q * nin + j] * mu_next[n];
            if (j < q) lam[(long)j * N + n] = acc;
            else if (j == q) mu[n] = acc;
            else gsum[j - q - 1] += acc;
        }
    }
    for (int i = 0; i < 6; ++i) gk[tri[i][0] * 3 + tri[i][1]] += gsum[i];
}

void orc_adjoint_init(const orc_params *p, const double *phi0, const double *rext0,
                      const double *lam0, const double *mu0, double *gphi0)
{
    orc_tabs tb;
    build_tabs(p, &tb);
    const long N = (long)p->nx * p->ny * p->nz;
    const int q = tb.q;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double complex K[3][3], fl[19];
        k0_complex(p, NULL, K);
        init_node_c(&tb, p, phi0[n] + I * ORC_H, (const double complex (*)[3])K, rext0 ? rext0[n] : 0.0, fl);
        double acc = mu0[n];   /* pprev(0) = phi0 */
        for (int k = 0; k < q; ++k) acc += cimag(fl[k]) / ORC_H * lam0[(long)k * N + n];
        gphi0[n] = acc;
    }
}
