/* CPU oracle for the electromagnetic PIC macro-particle operators.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, scalar, serial implementation
 * that the tests, the smoke check and the benchmark's CPU-baseline leg use to
 * check the HIP library.  Nothing in the library calls it, and it shares no
 * code with it.
 *
 * All arithmetic is in `real` (double by default; the same source is also
 * built with long double for finite-difference references).  Built with
 * -O2 -ffp-contract=off, no fast-math, so every a*b+c below is two roundings.
 *
 * Conventions (the paper gives the operator sequence and the spline order;
 * the formulas come from the published methods it relies on):
 *   - normalised units, c = 1; u = p/(m c); grid cell sizes d[a];
 *   - Yee grid, periodic; every component array has prod(n) entries, x
 *     fastest; entry (i,j,k) of a component with stagger bits (sx,sy,sz)
 *     sits at ((i+sx/2) d_x, (j+sy/2) d_y, (k+sz/2) d_z);
 *     Ex(1,0,0) Ey(0,1,0) Ez(0,0,1) Bx(0,1,1) By(1,0,1) Bz(1,1,0); J as E;
 *     in 2D the z bit is dropped;
 *   - order-2 (quadratic B-spline, three-point) shape functions;
 *   - relativistic Boris push; Esirkepov charge-conserving deposit.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_ERR_CFL = 1, ORC_ERR_POS = 2, ORC_ERR_ARG = 3 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_REFLECT = 1, ORC_BC_REMOVE = 2 };

typedef struct {
  int32_t dim;      /* 2 (2D3V) or 3 (3D3V) */
  int32_t n[3];     /* cells per axis; n[2] = 1 in 2D */
  double d[3];      /* cell sizes */
  double dt;        /* time step */
  int32_t patch[3]; /* patch size in cells per axis; patch[2] = 1 in 2D */
  int32_t bc[3];    /* particle boundary per axis: ORC_BC_PERIODIC,
                       ORC_BC_REFLECT (walls at 0 and L mirror particles:
                       the paper's reflective particle condition of its
                       radiation-pressure case, section "Basic performance
                       benchmarks") or ORC_BC_REMOVE (particles that leave
                       [0, L) are deleted: the paper's "delete" condition,
                       section "Parallelization without tasks"); fields
                       stay periodic */
} orc_grid;

typedef struct {
  double q, m;      /* charge (units of e) and mass (units of m_e) */
  int64_t n;        /* number of particles */
  double *x[3];     /* positions, x[2] unused in 2D */
  double *u[3];     /* momenta u = p/(m c) */
  double *w;        /* weights */
  int64_t *id;      /* particle ids */
  int64_t *off;     /* [n_patches + 1] patch offsets after orc_bin */
} orc_species;

/* Shape: node index and three weights of a position xi (in cell units) on an
 * axis with stagger bit s. */
void orc_shape(double xi, int32_t s, int64_t *i, double S[3]);

/* Interpolate the six field components at n positions (x[a][p]); out[c][p],
 * c = Ex,Ey,Ez,Bx,By,Bz. */
void orc_interp(const orc_grid *g, const double *const E[3], const double *const B[3],
                int64_t n, const double *const x[3], double *const out[6]);

/* nsteps Boris pushes of one particle in uniform fields E, B.  Trajectory
 * (positions before each step and after the last; momenta after each
 * step, starting with the input) into xs[(nsteps+1)*3], us[(nsteps+1)*3]. */
void orc_boris_traj(double q, double m, double dt, int32_t dim, const double E[3],
                    const double B[3], const double x0[3], const double u0[3],
                    int64_t nsteps, double *xs, double *us);

/* Esirkepov deposit of one particle moving from x0 (wrapped) to x1
 * (unwrapped), out-of-plane velocity vz (2D only).  J[c] += contribution;
 * if A != NULL, A[c] += the sum of the absolute values of the products that
 * make up the contribution (the scale of its rounding error).  Returns ORC_ERR_CFL if the particle
 * moves more than one node along an axis. */
int orc_deposit(const orc_grid *g, double q, double w, const double x0[3],
                const double x1[3], double vz, double *const J[3], double *const A[3]);

/* Periodic wrap, patch key and stable counting sort by patch (in place);
 * writes s->off.  On a reflecting axis a position outside [0, L) is an
 * error (ORC_ERR_POS), not wrapped; on a removing axis the particle is
 * deleted (s->n shrinks). */
int orc_bin(const orc_grid *g, orc_species *s);

/* One PIC step of the macro-particle operators for nsp species already
 * sorted by patch (s->off valid): J <- 0, then per patch, per species,
 * Interpolation, Push, pre-BC, Projection; then the periodic boundary
 * condition and the sort.  A particle that leaves through a removing wall
 * deposits no current and is deleted by the sort (sp[s].n shrinks).  A
 * (optional) receives, per node, the sum of the absolute values of all
 * products that entered J there. */
int orc_step(const orc_grid *g, orc_species *sp, int32_t nsp, const double *const E[3],
             const double *const B[3], double *const J[3], double *const A[3]);

/* Charge density rho = sum q w prod_a S_a on primal nodes (accumulated). */
void orc_rho(const orc_grid *g, double q, int64_t n, const double *const x[3],
             const double *w, double *rho);

/* Forward-mode derivative of nsteps particle steps of one species, for the
 * loss L = sum W . J_final.  Particles are advanced one by one (fields are
 * static, so particles do not interact).  Inputs: start state (x wrapped, u),
 * fields, tangent directions du (3 x n or NULL), dE, dB (3 x cells or NULL).
 * Outputs: J (deposit of the last step) and dJ, its directional derivative. */
int orc_jvp(const orc_grid *g, double q, double m, int64_t n, const double *const x[3],
            const double *const u[3], const double *w, const double *const E[3],
            const double *const B[3], const double *const du[3], const double *const dE[3],
            const double *const dB[3], int64_t nsteps, double *const J[3], double *const dJ[3]);

/* Central finite difference of L = sum W . J_final along (du, dE, dB) with
 * step h, everything in `real`.  Returns the difference quotient through *fd
 * and L at the unperturbed point through *L0. */
int orc_fd(const orc_grid *g, double q, double m, int64_t n, const double *const x[3],
           const double *const u[3], const double *w, const double *const E[3],
           const double *const B[3], const double *const W[3], const double *const du[3],
           const double *const dE[3], const double *const dB[3], int64_t nsteps, double h,
           double *fd, double *L0);

/* Field solver of the PIC loop (the paper's loop solves Maxwell's equations
 * on the grid with the projected current as source, section "Parallelization
 * without tasks"; the scheme is Yee's finite-difference time-domain method,
 * normalised units c = 1): nsteps times, with the same J,
 *   E <- E + dt (curl B - J)    (Ampere; B at the half step),
 *   B <- B - dt curl E          (Faraday; with the new E),
 * the curls as differences of neighbouring staggered values over the cell
 * size, periodic.  With c_a = dt / d_a, per component and in this order:
 *   Ex <- ((Ex + c_y dy Bz) - c_z dz By) - dt Jx     dy Bz = Bz(j) - Bz(j-1) ...
 *   Ey <- ((Ey + c_z dz Bx) - c_x dx Bz) - dt Jy
 *   Ez <- ((Ez + c_x dx By) - c_y dy Bx) - dt Jz
 *   Bx <- (Bx - c_y dy Ez) + c_z dz Ey               dy Ez = Ez(j+1) - Ez(j) ...
 *   By <- (By - c_z dz Ex) + c_x dx Ez
 *   Bz <- (Bz - c_x dx Ey) + c_y dy Ex
 * (backward differences of B, forward differences of E, as the staggering
 * puts them); in 2D the z differences are absent and their terms dropped.
 * Arrays are updated in place. */
void orc_maxwell(const orc_grid *g, double *const E[3], double *const B[3],
                 const double *const J[3], int64_t nsteps);

/* Reverse mode of orc_maxwell: given the cotangents Eb, Bb of the fields
 * after nsteps steps, overwrite them with the cotangents of the fields
 * before, and accumulate into Jb the cotangent of the current (used in
 * every step).  The transpose of one step taken in reverse order: the
 * transpose of Faraday (B' = B - C_f E', C_f the forward-difference curl)
 * then of Ampere (E' = E + C_b B - dt J, C_b the backward-difference curl),
 * with C_f^T = C_b and C_b^T = C_f on the periodic staggered grid:
 *   Ebx <- (Ebx - c_y dyBbz) + c_z dzBby   (backward differences of Bb)
 *   Eby <- (Eby - c_z dzBbx) + c_x dxBbz
 *   Ebz <- (Ebz - c_x dxBby) + c_y dyBbx
 *   Jb  <- Jb - dt Eb
 *   Bbx <- (Bbx + c_y dyEbz) - c_z dzEby   (forward differences of Eb)
 *   Bby <- (Bby + c_z dzEbx) - c_x dxEbz
 *   Bbz <- (Bbz + c_x dxEby) - c_y dyEbx
 * (no z terms in 2D). */
void orc_maxwell_adjoint(const orc_grid *g, double *const Eb[3], double *const Bb[3],
                         double *const Jb[3], int64_t nsteps);

/* sizeof(real) of this compiled variant of the oracle (double, or long double
 * for the finite-difference references) */
int32_t orc_real_size(void);

#ifdef __cplusplus
}
#endif
#endif
