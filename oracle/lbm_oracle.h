/*
 * Plain CPU FP64 oracle for the MRT lattice Boltzmann model of Chai, Shi & Guo
 * (general MRT model for nonlinear anisotropic convection-diffusion equations).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library: it works in velocity space
 * (Eq. 2, 3, 9, 34 applied literally), inverts M by Gaussian elimination,
 * integrates Eq. 7 by Gauss-Legendre quadrature, and obtains adjoint
 * Jacobians by complex-step differentiation.
 *
 * Units: lattice units, c = dx = dt = 1, cs^2 = 1/3 (Sec. 2.2, below Eq. 6).
 * Field layout: distributions f[k][z][y][x] (k slowest), scalars [z][y][x].
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXP 9          /* polynomial coefficients per function (degree 8) */

typedef struct orc_params {
    int q;                  /* 9 (D2Q9, Eq. 5) or 19 (D3Q19, Eq. 6)           */
    int nx, ny, nz;         /* nz = 1 for D2Q9                                 */
    int bc[3];              /* per axis: 0 periodic, 1 anti-bounce-back walls  */
    double phi_wall[3][2];  /* Dirichlet value at the low / high wall of axis  */
    int scheme;             /* 0: Scheme A (gamma = 0), 1: Scheme B (gamma = 1) */
    double d;               /* positive parameter of Eq. 3                     */
    double s[19];           /* diagonal relaxation rates, moment-row order;
                               the rows of the flux moments come from K (Eq. 26) */
    int basis;              /* D3Q19 only: 0 polynomial basis, 1 alternative
                               Gram-Schmidt basis (both orthogonal)            */
    double bpoly[3][ORC_MAXP]; /* B_a(phi) = sum_p bpoly[a][p] phi^p            */
    double dpoly[ORC_MAXP];    /* D(phi) = dpoly(phi) * dten                    */
    double dten[3][3];
    double k0[3][3];           /* K(phi, x) = K0 * kpoly(phi)                   */
    double kpoly[ORC_MAXP];
    double rpoly[ORC_MAXP];    /* R(phi) = rpoly(phi)  (+ optional field R(x,t)) */
    int variant;               /* 0: equilibrium of Eq. 3; 1: Remark III (Eq. 36-38):
                                  C = 0 in the equilibrium and the source G_k of
                                  Eq. 37 with an explicit time difference of B    */
    double bden[ORC_MAXP];     /* B_a = bpoly_a(phi) / bden(phi), a rational flux
                                  such as the Buckley-Leverett one (Sec. 3.3, Eq.
                                  54); all zero: bden = 1.  A non-constant bden
                                  needs variant 1 (C of Eq. 7 is not integrated) */
} orc_params;

/* 0 on success, negative on an invalid parameter set. */
int orc_check(const orc_params *p);

/* Lattice and transform tables: c[q][3], w[q], M[q][q], Minv[q][q] (row major). */
void orc_tables(const orc_params *p, int *c, double *w, double *M, double *Minv);

/* C(phi) of Eq. 7 with C(0) = 0, by Gauss-Legendre quadrature: out[3][3]. */
void orc_ctensor(const orc_params *p, double phi, double *out);

/* Equilibrium distribution of Eq. 3 at one phi value: out[q]. */
void orc_feq(const orc_params *p, double phi, double *out);

/* Diffusion matrix block A of Eq. 26 at phi (kfield may be NULL): out[dim][dim]. */
void orc_ablock(const orc_params *p, double phi, const double *kloc, double *out);

/* One node's collision (Eq. 2 with Scheme A source, or Eq. 34), before streaming.
 * f[q]: pre-collision distributions, pprev: phi at the previous step (Scheme A),
 * rext/rext_prev: external source R(x,t), R(x,t-1) added to rpoly(phi),
 * kloc: 3x3 local K replacing K0 (or NULL).  out[q], *phi_out. */
void orc_collide(const orc_params *p, const double *f, double pprev,
                 double rext, double rext_prev, const double *kloc,
                 double *out, double *phi_out);

/* Eq. 40 initialisation.  Scheme B stores fbar = feq - R_k/2 (Eq. 33).
 * rext0 may be NULL.  f: q*N, pprev: N (set to phi0). */
void orc_init(const orc_params *p, const double *phi0, const double *rext0,
              double *f, double *pprev);

/* One full time step in place: collision at every node, then push streaming
 * with periodic wrap or anti-bounce-back at walls; pprev <- phi(t).
 * rext, rext_prev, kfield (9 doubles per node) may be NULL. */
int orc_step(const orc_params *p, double *f, double *pprev,
             const double *rext, const double *rext_prev, const double *kfield,
             int nthreads);

/* Macroscopic phi (Eq. 10a; Scheme B: Eq. 35, solved by Newton's method
 * when R depends on phi). */
void orc_phi(const orc_params *p, const double *f, const double *rext, double *phi);

/* Reverse step of the discrete adjoint, from complex-step local Jacobians.
 * Given the state at step t (f: q*N pre-collision, pprev: N) and the adjoint
 * of the state at t+1 (lam_next: q*N, mu_next: N), returns lam (q*N), mu (N)
 * and adds dL/dK0 (gk[3][3], symmetric entries each counted once into the
 * upper triangle: gk[a][b] for a <= b).  rext/rext_prev/kfield as orc_step. */
void orc_adjoint_step(const orc_params *p, const double *f, const double *pprev,
                      const double *lam_next, const double *mu_next,
                      const double *rext, const double *rext_prev,
                      double *lam, double *mu, double *gk, int nthreads);

/* Adjoint of the initialisation: dL/dphi0 from lam(0), mu(0). */
void orc_adjoint_init(const orc_params *p, const double *phi0, const double *rext0,
                      const double *lam0, const double *mu0, double *gphi0);

/* Local Jacobian of one node's collision map (complex step), for pins:
 * inputs (f[q], pprev, k0 upper-triangle entries[6]) -> outputs (out[q], phi).
 * jac is (q+1) x (q+1+6), row major. */
void orc_node_jacobian(const orc_params *p, const double *f, double pprev,
                       double *jac);

#ifdef __cplusplus
}
#endif
#endif
