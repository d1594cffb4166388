/* CPU oracle for the electromagnetic PIC macro-particle operators.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the
 * benchmark's CPU-baseline leg to check the HIP library; shares no code with
 * it.  Plain scalar C, serial, in `real` (double unless ORC_REAL is defined,
 * or binary128 with ORC_QUAD), built with -O2 -ffp-contract=off and no
 * fast-math.
 *
 * What it follows:
 *   - the PIC iteration's macro-particle operators, per patch and species, in
 *     the order Interpolation, Push, pre-boundary-condition operations,
 *     Projection (paper, section "Parallelization without tasks",
 *     Algorithm 1), with the boundary conditions themselves and the particle
 *     sort done afterwards in the synchronisation phase (same section);
 *   - periodic, reflecting or removing particle boundaries per axis (the
 *     paper's radiation-pressure case reflects particles at its x borders,
 *     section "Basic performance benchmarks"; the pre-BC operation flags
 *     particles to delete, section "Parallelization without tasks"); the
 *     pre-BC operation mirrors a particle that crossed a reflecting wall
 *     before its current is projected, and a particle that crossed a
 *     removing wall deposits nothing and is deleted at the sort;
 *   - order-2 interpolation / projection shapes on a three-point stencil
 *     (paper, section "Basic performance benchmarks" and the plasma-expansion
 *     set-up);
 *   - the formulas of the published methods the paper relies on for these
 *     operators (it does not print them): the quadratic B-spline shape, Yee's
 *     staggered grid, Boris's relativistic push and Esirkepov's
 *     charge-conserving current deposit (Comput. Phys. Commun. 135, 144).
 *
 * Floating-point evaluation order is fixed and stated at each function so
 * that a second implementation can reproduce particle results bit for bit.
 */
#include "pic_oracle.h"

#include <stdlib.h>
#include <string.h>

#ifdef ORC_QUAD
/* binary128 (finite-difference references whose rounding must stay far
 * below the derivative's seventh digit): the math functions of that type */
#define __STDC_WANT_IEC_60559_TYPES_EXT__ 1
#include <math.h>
typedef _Float128 real;
#define sqrt sqrtf128
#define floor floorf128
#define fabs fabsf128
#define nextafter nextafterf128
#else
#include <tgmath.h>
#ifndef ORC_REAL
#define ORC_REAL double
#endif
typedef ORC_REAL real;
#endif

int32_t orc_real_size(void) { return (int32_t)sizeof(real); }

/* stagger bits (x, y, z) of Ex, Ey, Ez and Bx, By, Bz on the Yee grid */
static const int STAG_E[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
static const int STAG_B[3][3] = {{0, 1, 1}, {1, 0, 1}, {1, 1, 0}};

typedef struct {
  int dim;
  int64_t n[3], patch[3], np[3], npatch, ncell;
  real d[3], inv_d[3], L[3], dt;
  int bc[3];
} G;

static void mk_grid(const orc_grid *g, G *G_) {
  memset(G_, 0, sizeof(*G_));
  G_->dim = g->dim;
  G_->npatch = 1;
  G_->ncell = 1;
  for (int a = 0; a < 3; a++) {
    G_->n[a] = a < g->dim ? g->n[a] : 1;
    G_->patch[a] = a < g->dim ? g->patch[a] : 1;
    G_->np[a] = G_->n[a] / G_->patch[a];
    G_->npatch *= G_->np[a];
    G_->ncell *= G_->n[a];
    G_->d[a] = (real)g->d[a];
    G_->inv_d[a] = (real)1 / (real)g->d[a];
    G_->L[a] = (real)G_->n[a] * (real)g->d[a];
    G_->bc[a] = a < g->dim ? g->bc[a] : ORC_BC_PERIODIC;
  }
  G_->dt = (real)g->dt;
}

static int64_t wrapi(int64_t k, int64_t n) {
  int64_t r = k % n;
  return r < 0 ? r + n : r;
}

static int64_t node(const G *g, int64_t i, int64_t j, int64_t k) {
  return (wrapi(k, g->n[2]) * g->n[1] + wrapi(j, g->n[1])) * g->n[0] + wrapi(i, g->n[0]);
}

/* ---------------------------------------------------------------------- */
/* Quadratic B-spline shape.  For a particle at xi (cell units) on an axis
 * with stagger bit s the nearest node is i = floor(xi - s/2 + 1/2) and
 * delta = (xi - s/2) - i lies in [-1/2, 1/2).  The weights on nodes i-1, i,
 * i+1 are the order-2 B-spline evaluated at distances 1+delta, delta, 1-delta:
 *   S- = (1/2 - delta)^2 / 2,  S0 = 3/4 - delta^2,  S+ = (1/2 + delta)^2 / 2,
 * evaluated as 0.5*((0.5-d)*(0.5-d)), 0.75 - d*d, 0.5*((0.5+d)*(0.5+d)). */
static void shape_weights(real delta, real S[3]) {
  real a = (real)0.5 - delta;
  real b = (real)0.5 + delta;
  S[0] = (real)0.5 * (a * a);
  S[1] = (real)0.75 - delta * delta;
  S[2] = (real)0.5 * (b * b);
}

/* dS/d(delta) of the three weights */
static void shape_slopes(real delta, real dS[3]) {
  dS[0] = -((real)0.5 - delta);
  dS[1] = (real)-2 * delta;
  dS[2] = (real)0.5 + delta;
}

static int64_t locate(real xi, int s, real *delta) {
  real xs = xi - (real)0.5 * (real)s;
  real f = floor(xs + (real)0.5);
  *delta = xs - f;
  return (int64_t)f;
}

void orc_shape(double xi, int32_t s, int64_t *i, double S[3]) {
  real delta, w[3];
  *i = locate((real)xi, s, &delta);
  shape_weights(delta, w);
  for (int k = 0; k < 3; k++) S[k] = (double)w[k];
}

/* ---------------------------------------------------------------------- */
/* Interpolation of one component: F_p = sum_c Sz_c sum_b Sy_b sum_a Sx_a F.
 * Order: x innermost (r = Sx0*F0; r = r + Sx1*F1; r = r + Sx2*F2), then the
 * same over y of the row results, then over z of the plane results.
 * If grad != NULL it receives dF_p/dxi_a (any order; used for derivatives). */
static real interp_comp(const G *g, const real *F, const int st[3], const real xi[3],
                        real grad[3]) {
  int64_t i[3] = {0, 0, 0};
  real S[3][3], dS[3][3];
  for (int a = 0; a < g->dim; a++) {
    real delta;
    i[a] = locate(xi[a], st[a], &delta);
    shape_weights(delta, S[a]);
    shape_slopes(delta, dS[a]);
  }
  if (g->dim == 2) {
    real r[3], rx[3];
    for (int b = 0; b < 3; b++) {
      const real f0 = F[node(g, i[0] - 1, i[1] - 1 + b, 0)];
      const real f1 = F[node(g, i[0], i[1] - 1 + b, 0)];
      const real f2 = F[node(g, i[0] + 1, i[1] - 1 + b, 0)];
      real v = S[0][0] * f0;
      v = v + S[0][1] * f1;
      v = v + S[0][2] * f2;
      r[b] = v;
      rx[b] = dS[0][0] * f0 + dS[0][1] * f1 + dS[0][2] * f2;
    }
    real val = S[1][0] * r[0];
    val = val + S[1][1] * r[1];
    val = val + S[1][2] * r[2];
    if (grad) {
      grad[0] = S[1][0] * rx[0] + S[1][1] * rx[1] + S[1][2] * rx[2];
      grad[1] = dS[1][0] * r[0] + dS[1][1] * r[1] + dS[1][2] * r[2];
      grad[2] = 0;
    }
    return val;
  }
  real p[3];
  for (int c = 0; c < 3; c++) {
    real r[3];
    for (int b = 0; b < 3; b++) {
      real v = S[0][0] * F[node(g, i[0] - 1, i[1] - 1 + b, i[2] - 1 + c)];
      v = v + S[0][1] * F[node(g, i[0], i[1] - 1 + b, i[2] - 1 + c)];
      v = v + S[0][2] * F[node(g, i[0] + 1, i[1] - 1 + b, i[2] - 1 + c)];
      r[b] = v;
    }
    real v = S[1][0] * r[0];
    v = v + S[1][1] * r[1];
    v = v + S[1][2] * r[2];
    p[c] = v;
  }
  real val = S[2][0] * p[0];
  val = val + S[2][1] * p[1];
  val = val + S[2][2] * p[2];
  if (grad) {
    grad[0] = grad[1] = grad[2] = 0;
    for (int c = 0; c < 3; c++)
      for (int b = 0; b < 3; b++)
        for (int a = 0; a < 3; a++) {
          real f = F[node(g, i[0] - 1 + a, i[1] - 1 + b, i[2] - 1 + c)];
          grad[0] += dS[0][a] * S[1][b] * S[2][c] * f;
          grad[1] += S[0][a] * dS[1][b] * S[2][c] * f;
          grad[2] += S[0][a] * S[1][b] * dS[2][c] * f;
        }
  }
  return val;
}

/* Interpolate the six components at position x (physical units). */
static void interp6(const G *g, real *const E[3], real *const B[3], const real x[3],
                    real out[6], real grad[6][3]) {
  real xi[3] = {0, 0, 0};
  for (int a = 0; a < g->dim; a++) xi[a] = x[a] * g->inv_d[a];
  for (int c = 0; c < 3; c++) {
    out[c] = interp_comp(g, E[c], STAG_E[c], xi, grad ? grad[c] : NULL);
    out[3 + c] = interp_comp(g, B[c], STAG_B[c], xi, grad ? grad[3 + c] : NULL);
  }
}

/* ---------------------------------------------------------------------- */
/* Relativistic Boris push (Boris 1970, rotation form).  alpha = (q/m)*(dt/2).
 *   u-  = u + alpha E
 *   g-  = sqrt(1 + ((u-x^2 + u-y^2) + u-z^2))
 *   t   = (alpha / g-) B
 *   s   = (2 / (1 + ((tx^2 + ty^2) + tz^2))) t
 *   u'  = u- + u- x t          ((a x b)_x = a_y b_z - a_z b_y, cyclic)
 *   u+  = u- + u' x s
 *   u   = u+ + alpha E
 *   g   = sqrt(1 + ((ux^2 + uy^2) + uz^2)),  v = u * (1/g)
 * The half-acceleration alpha*E is computed once per component. */
static void boris(real alpha, const real F[6], real u[3], real v[3]) {
  const real ae[3] = {alpha * F[0], alpha * F[1], alpha * F[2]};
  real um[3] = {u[0] + ae[0], u[1] + ae[1], u[2] + ae[2]};
  real gm = sqrt((real)1 + ((um[0] * um[0] + um[1] * um[1]) + um[2] * um[2]));
  real tau = alpha / gm;
  real t[3] = {tau * F[3], tau * F[4], tau * F[5]};
  real sig = (real)2 / ((real)1 + ((t[0] * t[0] + t[1] * t[1]) + t[2] * t[2]));
  real s[3] = {sig * t[0], sig * t[1], sig * t[2]};
  real up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]), um[1] + (um[2] * t[0] - um[0] * t[2]),
                um[2] + (um[0] * t[1] - um[1] * t[0])};
  real upl[3] = {um[0] + (up[1] * s[2] - up[2] * s[1]), um[1] + (up[2] * s[0] - up[0] * s[2]),
                 um[2] + (up[0] * s[1] - up[1] * s[0])};
  u[0] = upl[0] + ae[0];
  u[1] = upl[1] + ae[1];
  u[2] = upl[2] + ae[2];
  real gam = sqrt((real)1 + ((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]));
  real ig = (real)1 / gam;
  v[0] = u[0] * ig;
  v[1] = u[1] * ig;
  v[2] = u[2] * ig;
}

static real species_alpha(const G *g, real q, real m) { return (q / m) * ((real)0.5 * g->dt); }

void orc_boris_traj(double q, double m, double dt, int32_t dim, const double E[3],
                    const double B[3], const double x0[3], const double u0[3],
                    int64_t nsteps, double *xs, double *us) {
  real alpha = ((real)q / (real)m) * ((real)0.5 * (real)dt);
  real F[6], x[3], u[3], v[3];
  for (int c = 0; c < 3; c++) {
    F[c] = E[c];
    F[3 + c] = B[c];
    x[c] = x0[c];
    u[c] = u0[c];
  }
  for (int c = 0; c < 3; c++) {
    xs[c] = (double)x[c];
    us[c] = (double)u[c];
  }
  for (int64_t k = 1; k <= nsteps; k++) {
    boris(alpha, F, u, v);
    for (int a = 0; a < dim; a++) x[a] = x[a] + (real)dt * v[a];
    for (int c = 0; c < 3; c++) {
      xs[3 * k + c] = (double)x[c];
      us[3 * k + c] = (double)u[c];
    }
  }
}

/* ---------------------------------------------------------------------- */
/* Esirkepov deposit with the quadratic shape on a five-point stencil.
 * Per axis a: xi0 = x0*inv_d, xi1 = x1*inv_d (x1 unwrapped); primal nodes
 * i0 = floor(xi0+1/2), i1 likewise; shift m = i1 - i0 must be -1, 0 or 1.
 * Slot r = 0..4 is node i0-2+r; S0 = (0, S(d0), 0); S1 = S(d1) in slots
 * 1+m..3+m; DS = S1 - S0.
 * 2D:  Wx = DSx[r] (S0y[t] + DSy[t]/2),  Wy = DSy[t] (S0x[r] + DSx[r]/2),
 *      Wz = S0x S0y + (DSx S0y + S0x DSy)/2 + DSx DSy / 3;
 *      Jx[i0-2+r, j0-2+t] += -(q w) (dx/dt) sum_{r'<=r} Wx[r'][t]  (r = 0..3)
 *      Jy likewise along y; Jz[...] += q w vz Wz.
 * 3D:  Wx = DSx (S0y S0z + DSy S0z/2 + S0y DSz/2 + DSy DSz/3), y, z cyclic,
 *      each J component the running sum along its own axis.
 * Jx entry i sits at (i + 1/2) dx, as Ex.  A[c] collects, per node, the
 * absolute values of all products entering the node's contributions. */
typedef struct {
  int64_t i0[3];
  real S0[3][5], DS[3][5];
} stencil;

static int build_stencil(const G *g, const real x0[3], const real x1[3], stencil *st) {
  for (int a = 0; a < 3; a++)
    for (int r = 0; r < 5; r++) st->S0[a][r] = st->DS[a][r] = 0;
  for (int a = 0; a < g->dim; a++) {
    real d0, d1, s0[3], s1[3], S1[5] = {0, 0, 0, 0, 0};
    int64_t k0 = locate(x0[a] * g->inv_d[a], 0, &d0);
    int64_t k1 = locate(x1[a] * g->inv_d[a], 0, &d1);
    int64_t m = k1 - k0;
    if (m < -1 || m > 1) return ORC_ERR_CFL;
    shape_weights(d0, s0);
    shape_weights(d1, s1);
    for (int r = 0; r < 3; r++) {
      st->S0[a][1 + r] = s0[r];
      S1[1 + m + r] = s1[r];
    }
    for (int r = 0; r < 5; r++) st->DS[a][r] = S1[r] - st->S0[a][r];
    st->i0[a] = k0;
  }
  return ORC_OK;
}

/* J[c] += v at node (i,j,k); A[c] += a, where a is the sum of the absolute
 * values of every product that entered v (the scale of v's rounding error,
 * which stays meaningful where the exact value of v is zero). */
static void add_node(const G *g, real *const J[3], real *const A[3], int c, int64_t i, int64_t j,
                     int64_t k, real v, real a) {
  int64_t at = node(g, i, j, k);
  J[c][at] += v;
  if (A) A[c][at] += a;
}

static int deposit(const G *g, real q, real w, const real x0[3], const real x1[3], real vz,
                   real *const J[3], real *const A[3]) {
  stencil st;
  int err = build_stencil(g, x0, x1, &st);
  if (err) return err;
  const real half = (real)0.5, third = (real)1 / (real)3;
  const real (*S0)[5] = st.S0, (*DS)[5] = st.DS;
  const int64_t *i0 = st.i0;
  if (g->dim == 2) {
    const real cx = -(q * w) * (g->d[0] / g->dt);
    const real cy = -(q * w) * (g->d[1] / g->dt);
    const real cz = (q * w) * vz;
    for (int t = 0; t < 5; t++) {
      real acc = 0, sc = 0;
      for (int r = 0; r < 4; r++) {
        acc = acc + DS[0][r] * (S0[1][t] + half * DS[1][t]);
        sc += fabs(DS[0][r]) * (fabs(S0[1][t]) + half * fabs(DS[1][t]));
        add_node(g, J, A, 0, i0[0] - 2 + r, i0[1] - 2 + t, 0, cx * acc, fabs(cx) * sc);
      }
    }
    for (int r = 0; r < 5; r++) {
      real acc = 0, sc = 0;
      for (int t = 0; t < 4; t++) {
        acc = acc + DS[1][t] * (S0[0][r] + half * DS[0][r]);
        sc += fabs(DS[1][t]) * (fabs(S0[0][r]) + half * fabs(DS[0][r]));
        add_node(g, J, A, 1, i0[0] - 2 + r, i0[1] - 2 + t, 0, cy * acc, fabs(cy) * sc);
      }
    }
    for (int t = 0; t < 5; t++)
      for (int r = 0; r < 5; r++) {
        real wz = S0[0][r] * S0[1][t] + half * DS[0][r] * S0[1][t] + half * S0[0][r] * DS[1][t] +
                  third * DS[0][r] * DS[1][t];
        real sc = fabs(S0[0][r] * S0[1][t]) + half * fabs(DS[0][r] * S0[1][t]) +
                  half * fabs(S0[0][r] * DS[1][t]) + third * fabs(DS[0][r] * DS[1][t]);
        add_node(g, J, A, 2, i0[0] - 2 + r, i0[1] - 2 + t, 0, cz * wz, fabs(cz) * sc);
      }
    return ORC_OK;
  }
  real c3[3];
  for (int a = 0; a < 3; a++) c3[a] = -(q * w) * (g->d[a] / g->dt);
  /* component a accumulates along axis a; the other two axes are b, c */
  for (int a = 0; a < 3; a++) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    for (int tb = 0; tb < 5; tb++)
      for (int tc = 0; tc < 5; tc++) {
        real acc = 0, sc = 0;
        const real fsc = fabs(S0[b][tb] * S0[c][tc]) + half * fabs(DS[b][tb] * S0[c][tc]) +
                         half * fabs(S0[b][tb] * DS[c][tc]) + third * fabs(DS[b][tb] * DS[c][tc]);
        for (int ta = 0; ta < 4; ta++) {
          real wa = DS[a][ta] * (S0[b][tb] * S0[c][tc] + half * DS[b][tb] * S0[c][tc] +
                                 half * S0[b][tb] * DS[c][tc] + third * DS[b][tb] * DS[c][tc]);
          acc = acc + wa;
          sc += fabs(DS[a][ta]) * fsc;
          int64_t o[3];
          o[a] = ta;
          o[b] = tb;
          o[c] = tc;
          add_node(g, J, A, a, i0[0] - 2 + o[0], i0[1] - 2 + o[1], i0[2] - 2 + o[2], c3[a] * acc,
                   fabs(c3[a]) * sc);
        }
      }
  }
  return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* pre-boundary-condition operation at walls.  A pushed position outside
 * [0, L) on an axis with removing walls marks the particle for deletion: it
 * deposits no current in this step (its weight is spent) and the sort of
 * the synchronisation phase drops it; the function then returns -1 and
 * changes nothing.  Otherwise, on an axis with reflecting walls, a position
 * that left [0, L) is mirrored back inside about the wall it crossed
 * (x -> -x, or x -> 2L - x) and its momentum component along the axis
 * changes sign.  Both mirror images are exact in floating point (Sterbenz's
 * lemma: x and 2L lie within a factor two of each other); the one position
 * that lands on L itself, x = L, is moved to the largest value below L so
 * that it stays in the last cell.  The paper flags such particles in the
 * pre-BC operation, which writes positions and momenta (section
 * "Parallelization with OpenMP task"); here the mirror is applied there too,
 * before the Projection, so the current is deposited along the mirrored move
 * (readings in the design notes).  Returns the mirrored axes as bits. */
static int outside_removing(const G *g, const real x[3]) {
  for (int a = 0; a < g->dim; a++)
    if (g->bc[a] == ORC_BC_REMOVE && !(x[a] >= 0 && x[a] < g->L[a])) return 1;
  return 0;
}

static int walls(const G *g, real x1[3], real u[3]) {
  if (outside_removing(g, x1)) return -1;
  int hit = 0;
  for (int a = 0; a < g->dim; a++) {
    if (g->bc[a] != ORC_BC_REFLECT) continue;
    if (x1[a] < 0) {
      x1[a] = -x1[a];
    } else if (x1[a] >= g->L[a]) {
      x1[a] = (real)2 * g->L[a] - x1[a];
      if (x1[a] >= g->L[a]) x1[a] = nextafter(g->L[a], (real)0);
    } else {
      continue;
    }
    u[a] = -u[a];
    hit |= 1 << a;
  }
  return hit;
}

/* pre-boundary-condition operation: the patch the particle will belong to,
 * from a periodically wrapped copy of its position:
 *   if (x < 0) x += L;  if (x >= L) x -= L;   (the second test also catches
 *   x + L rounding to L), cell c = floor(x * inv_d) clamped to n-1,
 *   patch P_a = c_a / patch_a, key = Px + NPx (Py + NPy Pz).
 * An axis with walls is not wrapped (its positions were mirrored inside).
 * Returns -1 if the position is more than one period outside the box, or
 * outside [0, L) on an axis with walls. */
static int64_t patch_key(const G *g, const real x1[3], real xw[3]) {
  int64_t P[3] = {0, 0, 0};
  for (int a = 0; a < g->dim; a++) {
    real v = x1[a];
    if (g->bc[a] == ORC_BC_PERIODIC) {
      if (v < 0) v += g->L[a];
      if (v >= g->L[a]) v -= g->L[a];
    }
    if (!(v >= 0 && v < g->L[a])) return -1;
    xw[a] = v;
    int64_t c = (int64_t)floor(v * g->inv_d[a]);
    if (c >= g->n[a]) c = g->n[a] - 1;
    P[a] = c / g->patch[a];
  }
  return P[0] + g->np[0] * (P[1] + g->np[1] * P[2]);
}

/* key of a particle deleted at a removing wall */
#define REMOVED (-2)

/* Stable counting sort of one species by key (keys in [0, npatch), or
 * REMOVED: the particle is dropped and s->n shrinks). */
static void sort_by_key(const G *g, orc_species *s, const int64_t *key) {
  const int64_t n = s->n, np = g->npatch;
  int64_t *cnt = calloc((size_t)np + 1, sizeof(int64_t));
  for (int64_t p = 0; p < n; p++)
    if (key[p] != REMOVED) cnt[key[p] + 1]++;
  for (int64_t P = 0; P < np; P++) cnt[P + 1] += cnt[P];
  for (int64_t P = 0; P <= np; P++) s->off[P] = cnt[P];
  const int64_t kept = cnt[np];
  int64_t *dest = malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  for (int64_t p = 0; p < n; p++) dest[p] = key[p] == REMOVED ? -1 : cnt[key[p]]++;
  double *tmp = malloc((size_t)(n ? n : 1) * sizeof(double));
  int64_t *itmp = malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  double *arrs[7] = {s->x[0], s->x[1], g->dim == 3 ? s->x[2] : NULL, s->u[0], s->u[1], s->u[2],
                     s->w};
  for (int k = 0; k < 7; k++) {
    if (!arrs[k]) continue;
    for (int64_t p = 0; p < n; p++)
      if (dest[p] >= 0) tmp[dest[p]] = arrs[k][p];
    memcpy(arrs[k], tmp, (size_t)kept * sizeof(double));
  }
  for (int64_t p = 0; p < n; p++)
    if (dest[p] >= 0) itmp[dest[p]] = s->id[p];
  memcpy(s->id, itmp, (size_t)kept * sizeof(int64_t));
  s->n = kept;
  free(cnt);
  free(dest);
  free(tmp);
  free(itmp);
}

/* Boundary conditions (periodic wrap, deletion outside a removing axis) and
 * sort: the synchronisation phase.  A position outside a reflecting axis is
 * an error here: only the pre-BC operation mirrors (pushed positions). */
int orc_bin(const orc_grid *gi, orc_species *s) {
  G g;
  mk_grid(gi, &g);
  int64_t *key = malloc((size_t)(s->n ? s->n : 1) * sizeof(int64_t));
  for (int64_t p = 0; p < s->n; p++) {
    real x[3] = {0, 0, 0}, xw[3] = {0, 0, 0};
    for (int a = 0; a < g.dim; a++) x[a] = s->x[a][p];
    if (outside_removing(&g, x)) {  /* deleted */
      key[p] = REMOVED;
      continue;
    }
    key[p] = patch_key(&g, x, xw);
    if (key[p] < 0) {
      free(key);
      return ORC_ERR_POS;
    }
    for (int a = 0; a < g.dim; a++) s->x[a][p] = (double)xw[a];
  }
  sort_by_key(&g, s, key);
  free(key);
  return ORC_OK;
}

static real *to_real(const double *a, int64_t n) {
  real *r = malloc((size_t)n * sizeof(real));
  for (int64_t i = 0; i < n; i++) r[i] = a ? (real)a[i] : 0;
  return r;
}

int orc_step(const orc_grid *gi, orc_species *sp, int32_t nsp, const double *const E[3],
             const double *const B[3], double *const J[3], double *const A[3]) {
  G g;
  mk_grid(gi, &g);
  const int dim = g.dim;
  /* the particles must be sorted by patch: offsets cover [0, n) in order */
  for (int s = 0; s < nsp; s++) {
    if (sp[s].off[0] != 0 || sp[s].off[g.npatch] != sp[s].n) return ORC_ERR_ARG;
    for (int64_t P = 0; P < g.npatch; P++)
      if (sp[s].off[P + 1] < sp[s].off[P]) return ORC_ERR_ARG;
  }
  real *Er[3], *Br[3], *Jr[3], *Ar[3];
  for (int c = 0; c < 3; c++) {
    Er[c] = to_real(E[c], g.ncell);
    Br[c] = to_real(B[c], g.ncell);
    Jr[c] = to_real(NULL, g.ncell);
    Ar[c] = to_real(NULL, g.ncell);
  }
  int64_t nmax = 1;
  for (int s = 0; s < nsp; s++)
    for (int64_t P = 0; P < g.npatch; P++)
      if (sp[s].off[P + 1] - sp[s].off[P] > nmax) nmax = sp[s].off[P + 1] - sp[s].off[P];
  /* per-particle buffers of one [patch, species]: interpolated fields, the
   * start-of-step position, the velocity and the pre-BC destination */
  real(*Fp)[6] = malloc((size_t)nmax * sizeof(*Fp));
  real(*x0)[3] = malloc((size_t)nmax * sizeof(*x0));
  real(*vel)[3] = malloc((size_t)nmax * sizeof(*vel));
  int64_t **keys = malloc((size_t)nsp * sizeof(int64_t *));
  for (int s = 0; s < nsp; s++) keys[s] = malloc((size_t)(sp[s].n ? sp[s].n : 1) * sizeof(int64_t));
  int err = ORC_OK;
  for (int64_t P = 0; P < g.npatch && !err; P++) {
    for (int s = 0; s < nsp && !err; s++) {
      orc_species *S = &sp[s];
      const int64_t b = S->off[P], e = S->off[P + 1];
      const real q = (real)S->q, alpha = species_alpha(&g, q, (real)S->m);
      /* Interpolation */
      for (int64_t p = b; p < e; p++) {
        real x[3] = {0, 0, 0};
        for (int a = 0; a < dim; a++) x[a] = x0[p - b][a] = S->x[a][p];
        interp6(&g, Er, Br, x, Fp[p - b], NULL);
      }
      /* Push */
      for (int64_t p = b; p < e; p++) {
        real u[3] = {S->u[0][p], S->u[1][p], S->u[2][p]};
        boris(alpha, Fp[p - b], u, vel[p - b]);
        for (int c = 0; c < 3; c++) S->u[c][p] = (double)u[c];
        for (int a = 0; a < dim; a++) S->x[a][p] = (double)(x0[p - b][a] + g.dt * vel[p - b][a]);
      }
      /* pre-BC: flag particles leaving through a removing wall, mirror at
       * reflecting walls, flag the destination patch (the periodic wrap
       * itself is applied in the synchronisation phase below) */
      for (int64_t p = b; p < e; p++) {
        real x1[3] = {0, 0, 0}, xw[3];
        for (int a = 0; a < dim; a++) x1[a] = S->x[a][p];
        real u[3] = {S->u[0][p], S->u[1][p], S->u[2][p]};
        const int hit = walls(&g, x1, u);
        if (hit < 0) {
          keys[s][p] = REMOVED;
          continue;
        }
        if (hit) {
          for (int a = 0; a < dim; a++) S->x[a][p] = (double)x1[a];
          for (int c = 0; c < 3; c++) S->u[c][p] = (double)u[c];
        }
        keys[s][p] = patch_key(&g, x1, xw);
        if (keys[s][p] < 0) err = ORC_ERR_POS;
      }
      /* Projection */
      for (int64_t p = b; p < e && !err; p++) {
        if (keys[s][p] == REMOVED) continue;
        real x1[3] = {0, 0, 0};
        for (int a = 0; a < dim; a++) x1[a] = S->x[a][p];
        err = deposit(&g, q, (real)S->w[p], x0[p - b], x1, vel[p - b][2], Jr, A ? Ar : NULL);
      }
    }
  }
  /* synchronisation: boundary conditions (periodic wrap; the sort drops the
   * particles flagged for deletion), then the sort by patch */
  for (int s = 0; s < nsp && !err; s++) {
    orc_species *S = &sp[s];
    for (int64_t p = 0; p < S->n; p++) {
      if (keys[s][p] == REMOVED) continue;
      real x1[3] = {0, 0, 0}, xw[3] = {0, 0, 0};
      for (int a = 0; a < dim; a++) x1[a] = S->x[a][p];
      patch_key(&g, x1, xw);
      for (int a = 0; a < dim; a++) S->x[a][p] = (double)xw[a];
    }
    sort_by_key(&g, S, keys[s]);
  }
  for (int c = 0; c < 3; c++) {
    for (int64_t i = 0; i < g.ncell; i++) {
      J[c][i] = (double)Jr[c][i];
      if (A) A[c][i] = (double)Ar[c][i];
    }
    free(Er[c]);
    free(Br[c]);
    free(Jr[c]);
    free(Ar[c]);
  }
  for (int s = 0; s < nsp; s++) free(keys[s]);
  free(keys);
  free(Fp);
  free(x0);
  free(vel);
  return err;
}

void orc_interp(const orc_grid *gi, const double *const E[3], const double *const B[3],
                int64_t n, const double *const x[3], double *const out[6]) {
  G g;
  mk_grid(gi, &g);
  real *Er[3], *Br[3];
  for (int c = 0; c < 3; c++) {
    Er[c] = to_real(E[c], g.ncell);
    Br[c] = to_real(B[c], g.ncell);
  }
  for (int64_t p = 0; p < n; p++) {
    real xp[3] = {0, 0, 0}, F[6];
    for (int a = 0; a < g.dim; a++) xp[a] = x[a][p];
    interp6(&g, Er, Br, xp, F, NULL);
    for (int c = 0; c < 6; c++) out[c][p] = (double)F[c];
  }
  for (int c = 0; c < 3; c++) {
    free(Er[c]);
    free(Br[c]);
  }
}

int orc_deposit(const orc_grid *gi, double q, double w, const double x0[3], const double x1[3],
                double vz, double *const J[3], double *const A[3]) {
  G g;
  mk_grid(gi, &g);
  real *Jr[3], *Ar[3];
  for (int c = 0; c < 3; c++) {
    Jr[c] = to_real(J[c], g.ncell);
    Ar[c] = to_real(A ? A[c] : NULL, g.ncell);
  }
  real a0[3] = {x0[0], x0[1], x0[2]}, a1[3] = {x1[0], x1[1], x1[2]};
  int err = deposit(&g, (real)q, (real)w, a0, a1, (real)vz, Jr, Ar);
  for (int c = 0; c < 3; c++) {
    for (int64_t i = 0; i < g.ncell; i++) {
      J[c][i] = (double)Jr[c][i];
      if (A) A[c][i] = (double)Ar[c][i];
    }
    free(Jr[c]);
    free(Ar[c]);
  }
  return err;
}

void orc_rho(const orc_grid *gi, double q, int64_t n, const double *const x[3], const double *w,
             double *rho) {
  G g;
  mk_grid(gi, &g);
  for (int64_t p = 0; p < n; p++) {
    int64_t i[3] = {0, 0, 0};
    real S[3][3] = {{0, 1, 0}, {0, 1, 0}, {0, 1, 0}};
    for (int a = 0; a < g.dim; a++) {
      real delta;
      i[a] = locate((real)x[a][p] * g.inv_d[a], 0, &delta);
      shape_weights(delta, S[a]);
    }
    const int nc = g.dim == 3 ? 3 : 1;
    for (int c = 0; c < nc; c++)
      for (int b = 0; b < 3; b++)
        for (int a = 0; a < 3; a++) {
          real s = S[0][a] * S[1][b] * (g.dim == 3 ? S[2][c] : (real)1);
          rho[node(&g, i[0] - 1 + a, i[1] - 1 + b, g.dim == 3 ? i[2] - 1 + c : 0)] +=
              (double)((real)q * (real)w[p] * s);
        }
  }
}

/* ---------------------------------------------------------------------- */
/* Yee field solver: Ampere for every node, then Faraday with the new E. */
void orc_maxwell(const orc_grid *gi, double *const E[3], double *const B[3],
                 const double *const J[3], int64_t nsteps) {
  G g;
  mk_grid(gi, &g);
  const int three = g.dim == 3;
  const real dt = g.dt;
  const real cx = dt / g.d[0], cy = dt / g.d[1], cz = three ? dt / g.d[2] : (real)0;
  for (int64_t s = 0; s < nsteps; s++) {
    for (int64_t k = 0; k < g.n[2]; k++)
      for (int64_t j = 0; j < g.n[1]; j++)
        for (int64_t i = 0; i < g.n[0]; i++) {
          const int64_t o = node(&g, i, j, k);
          const int64_t xm = node(&g, i - 1, j, k), ym = node(&g, i, j - 1, k);
          const real dyBz = (real)B[2][o] - (real)B[2][ym];
          const real dxBz = (real)B[2][o] - (real)B[2][xm];
          const real dxBy = (real)B[1][o] - (real)B[1][xm];
          const real dyBx = (real)B[0][o] - (real)B[0][ym];
          real ex = (real)E[0][o] + cy * dyBz;
          real ey = (real)E[1][o];
          if (three) {
            const int64_t zm = node(&g, i, j, k - 1);
            const real dzBy = (real)B[1][o] - (real)B[1][zm];
            const real dzBx = (real)B[0][o] - (real)B[0][zm];
            ex = ex - cz * dzBy;
            ey = ey + cz * dzBx;
          }
          ey = ey - cx * dxBz;
          real ez = ((real)E[2][o] + cx * dxBy) - cy * dyBx;
          E[0][o] = (double)(ex - dt * (real)J[0][o]);
          E[1][o] = (double)(ey - dt * (real)J[1][o]);
          E[2][o] = (double)(ez - dt * (real)J[2][o]);
        }
    for (int64_t k = 0; k < g.n[2]; k++)
      for (int64_t j = 0; j < g.n[1]; j++)
        for (int64_t i = 0; i < g.n[0]; i++) {
          const int64_t o = node(&g, i, j, k);
          const int64_t xp = node(&g, i + 1, j, k), yp = node(&g, i, j + 1, k);
          const real dyEz = (real)E[2][yp] - (real)E[2][o];
          const real dxEz = (real)E[2][xp] - (real)E[2][o];
          const real dxEy = (real)E[1][xp] - (real)E[1][o];
          const real dyEx = (real)E[0][yp] - (real)E[0][o];
          real bx = (real)B[0][o] - cy * dyEz;
          real by = (real)B[1][o];
          if (three) {
            const int64_t zp = node(&g, i, j, k + 1);
            const real dzEy = (real)E[1][zp] - (real)E[1][o];
            const real dzEx = (real)E[0][zp] - (real)E[0][o];
            bx = bx + cz * dzEy;
            by = by - cz * dzEx;
          }
          by = by + cx * dxEz;
          const real bz = ((real)B[2][o] - cx * dxEy) + cy * dyEx;
          B[0][o] = (double)bx;
          B[1][o] = (double)by;
          B[2][o] = (double)bz;
        }
  }
}

/* Reverse mode of the Yee solver: per step, the transposed Faraday update
 * of Eb, the current's cotangent, then the transposed Ampere update of Bb. */
void orc_maxwell_adjoint(const orc_grid *gi, double *const Eb[3], double *const Bb[3],
                         double *const Jb[3], int64_t nsteps) {
  G g;
  mk_grid(gi, &g);
  const int three = g.dim == 3;
  const real dt = g.dt;
  const real cx = dt / g.d[0], cy = dt / g.d[1], cz = three ? dt / g.d[2] : (real)0;
  for (int64_t s = 0; s < nsteps; s++) {
    for (int64_t k = 0; k < g.n[2]; k++)
      for (int64_t j = 0; j < g.n[1]; j++)
        for (int64_t i = 0; i < g.n[0]; i++) {
          const int64_t o = node(&g, i, j, k);
          const int64_t xm = node(&g, i - 1, j, k), ym = node(&g, i, j - 1, k);
          const real dyBz = (real)Bb[2][o] - (real)Bb[2][ym];
          const real dxBz = (real)Bb[2][o] - (real)Bb[2][xm];
          const real dxBy = (real)Bb[1][o] - (real)Bb[1][xm];
          const real dyBx = (real)Bb[0][o] - (real)Bb[0][ym];
          real ex = (real)Eb[0][o] - cy * dyBz;
          real ey = (real)Eb[1][o];
          if (three) {
            const int64_t zm = node(&g, i, j, k - 1);
            const real dzBy = (real)Bb[1][o] - (real)Bb[1][zm];
            const real dzBx = (real)Bb[0][o] - (real)Bb[0][zm];
            ex = ex + cz * dzBy;
            ey = ey - cz * dzBx;
          }
          ey = ey + cx * dxBz;
          const real ez = ((real)Eb[2][o] - cx * dxBy) + cy * dyBx;
          Eb[0][o] = (double)ex;
          Eb[1][o] = (double)ey;
          Eb[2][o] = (double)ez;
          Jb[0][o] = (double)((real)Jb[0][o] - dt * ex);
          Jb[1][o] = (double)((real)Jb[1][o] - dt * ey);
          Jb[2][o] = (double)((real)Jb[2][o] - dt * ez);
        }
    for (int64_t k = 0; k < g.n[2]; k++)
      for (int64_t j = 0; j < g.n[1]; j++)
        for (int64_t i = 0; i < g.n[0]; i++) {
          const int64_t o = node(&g, i, j, k);
          const int64_t xp = node(&g, i + 1, j, k), yp = node(&g, i, j + 1, k);
          const real dyEz = (real)Eb[2][yp] - (real)Eb[2][o];
          const real dxEz = (real)Eb[2][xp] - (real)Eb[2][o];
          const real dxEy = (real)Eb[1][xp] - (real)Eb[1][o];
          const real dyEx = (real)Eb[0][yp] - (real)Eb[0][o];
          real bx = (real)Bb[0][o] + cy * dyEz;
          real by = (real)Bb[1][o];
          if (three) {
            const int64_t zp = node(&g, i, j, k + 1);
            const real dzEy = (real)Eb[1][zp] - (real)Eb[1][o];
            const real dzEx = (real)Eb[0][zp] - (real)Eb[0][o];
            bx = bx - cz * dzEy;
            by = by + cz * dzEx;
          }
          by = by - cx * dxEz;
          const real bz = ((real)Bb[2][o] + cx * dxEy) - cy * dyEx;
          Bb[0][o] = (double)bx;
          Bb[1][o] = (double)by;
          Bb[2][o] = (double)bz;
        }
  }
}

/* ---------------------------------------------------------------------- */
/* Derivatives of L = sum W . J_final (2D3V).  Fields are static and J is
 * rebuilt from zero at every step, so only the last step's deposit reaches
 * L, and every particle can be advanced on its own; the sort is a
 * permutation and does not enter.  The forward-mode code below follows the
 * chain rule through the same operators. */

/* Boris push with its tangent: (u, F) -> u_new, v and du_new, dv for input
 * tangents du, dF. */
static void boris_tangent(real alpha, const real F[6], const real dF[6], real u[3], real du[3],
                          real v[3], real dv[3]) {
  real ae[3], dae[3], um[3], dum[3];
  for (int c = 0; c < 3; c++) {
    ae[c] = alpha * F[c];
    dae[c] = alpha * dF[c];
    um[c] = u[c] + ae[c];
    dum[c] = du[c] + dae[c];
  }
  real gm = sqrt((real)1 + ((um[0] * um[0] + um[1] * um[1]) + um[2] * um[2]));
  real dgm = (um[0] * dum[0] + um[1] * dum[1] + um[2] * dum[2]) / gm;
  real tau = alpha / gm;
  real dtau = -tau * dgm / gm;
  real t[3], dtt[3];
  for (int c = 0; c < 3; c++) {
    t[c] = tau * F[3 + c];
    dtt[c] = dtau * F[3 + c] + tau * dF[3 + c];
  }
  real den = (real)1 + ((t[0] * t[0] + t[1] * t[1]) + t[2] * t[2]);
  real dden = (real)2 * (t[0] * dtt[0] + t[1] * dtt[1] + t[2] * dtt[2]);
  real sig = (real)2 / den;
  real dsig = -sig * dden / den;
  real s[3], ds[3];
  for (int c = 0; c < 3; c++) {
    s[c] = sig * t[c];
    ds[c] = dsig * t[c] + sig * dtt[c];
  }
  real up[3], dup[3], upl[3], dupl[3];
  for (int c = 0; c < 3; c++) {
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    up[c] = um[c] + (um[a] * t[b] - um[b] * t[a]);
    dup[c] = dum[c] + (dum[a] * t[b] + um[a] * dtt[b] - dum[b] * t[a] - um[b] * dtt[a]);
  }
  for (int c = 0; c < 3; c++) {
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    upl[c] = um[c] + (up[a] * s[b] - up[b] * s[a]);
    dupl[c] = dum[c] + (dup[a] * s[b] + up[a] * ds[b] - dup[b] * s[a] - up[b] * ds[a]);
  }
  for (int c = 0; c < 3; c++) {
    u[c] = upl[c] + ae[c];
    du[c] = dupl[c] + dae[c];
  }
  real gam = sqrt((real)1 + ((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]));
  real dgam = (u[0] * du[0] + u[1] * du[1] + u[2] * du[2]) / gam;
  real ig = (real)1 / gam;
  real dig = -ig * ig * dgam;
  for (int c = 0; c < 3; c++) {
    v[c] = u[c] * ig;
    dv[c] = du[c] * ig + u[c] * dig;
  }
}

/* 2D Esirkepov deposit with its tangent for position tangents dx0, dx1 and
 * velocity tangent dvz. */
static int deposit_tangent2(const G *g, real q, real w, const real x0[3], const real x1[3],
                            real vz, const real dx0[3], const real dx1[3], real dvz,
                            real *const J[3], real *const dJ[3]) {
  stencil st;
  int err = build_stencil(g, x0, x1, &st);
  if (err) return err;
  real dS0[2][5], dDS[2][5];
  for (int a = 0; a < 2; a++) {
    real d0, d1, sl0[3], sl1[3], dS1[5] = {0, 0, 0, 0, 0};
    int64_t k0 = locate(x0[a] * g->inv_d[a], 0, &d0);
    int64_t k1 = locate(x1[a] * g->inv_d[a], 0, &d1);
    int64_t m = k1 - k0;
    shape_slopes(d0, sl0);
    shape_slopes(d1, sl1);
    for (int r = 0; r < 5; r++) dS0[a][r] = 0;
    for (int r = 0; r < 3; r++) {
      dS0[a][1 + r] = sl0[r] * (dx0[a] * g->inv_d[a]);
      dS1[1 + m + r] = sl1[r] * (dx1[a] * g->inv_d[a]);
    }
    for (int r = 0; r < 5; r++) dDS[a][r] = dS1[r] - dS0[a][r];
  }
  const real half = (real)0.5, third = (real)1 / (real)3;
  const real (*S0)[5] = st.S0, (*DS)[5] = st.DS;
  const int64_t *i0 = st.i0;
  const real cx = -(q * w) * (g->d[0] / g->dt), cy = -(q * w) * (g->d[1] / g->dt);
  for (int t = 0; t < 5; t++) {
    real acc = 0, dacc = 0;
    for (int r = 0; r < 4; r++) {
      acc += DS[0][r] * (S0[1][t] + half * DS[1][t]);
      dacc += dDS[0][r] * (S0[1][t] + half * DS[1][t]) + DS[0][r] * (dS0[1][t] + half * dDS[1][t]);
      int64_t at = node(g, i0[0] - 2 + r, i0[1] - 2 + t, 0);
      J[0][at] += cx * acc;
      dJ[0][at] += cx * dacc;
    }
  }
  for (int r = 0; r < 5; r++) {
    real acc = 0, dacc = 0;
    for (int t = 0; t < 4; t++) {
      acc += DS[1][t] * (S0[0][r] + half * DS[0][r]);
      dacc += dDS[1][t] * (S0[0][r] + half * DS[0][r]) + DS[1][t] * (dS0[0][r] + half * dDS[0][r]);
      int64_t at = node(g, i0[0] - 2 + r, i0[1] - 2 + t, 0);
      J[1][at] += cy * acc;
      dJ[1][at] += cy * dacc;
    }
  }
  for (int t = 0; t < 5; t++)
    for (int r = 0; r < 5; r++) {
      real wz = S0[0][r] * S0[1][t] + half * DS[0][r] * S0[1][t] + half * S0[0][r] * DS[1][t] +
                third * DS[0][r] * DS[1][t];
      real dwz = dS0[0][r] * S0[1][t] + S0[0][r] * dS0[1][t] +
                 half * (dDS[0][r] * S0[1][t] + DS[0][r] * dS0[1][t]) +
                 half * (dS0[0][r] * DS[1][t] + S0[0][r] * dDS[1][t]) +
                 third * (dDS[0][r] * DS[1][t] + DS[0][r] * dDS[1][t]);
      int64_t at = node(g, i0[0] - 2 + r, i0[1] - 2 + t, 0);
      J[2][at] += (q * w) * vz * wz;
      dJ[2][at] += (q * w) * (dvz * wz + vz * dwz);
    }
  return ORC_OK;
}

int orc_jvp(const orc_grid *gi, double q, double m, int64_t n, const double *const x[3],
            const double *const u[3], const double *w, const double *const E[3],
            const double *const B[3], const double *const du[3], const double *const dE[3],
            const double *const dB[3], int64_t nsteps, double *const J[3], double *const dJ[3]) {
  G g;
  mk_grid(gi, &g);
  if (g.dim != 2 || nsteps < 1) return ORC_ERR_ARG;
  real *Er[3], *Br[3], *dEr[3], *dBr[3], *Jr[3], *dJr[3];
  for (int c = 0; c < 3; c++) {
    Er[c] = to_real(E[c], g.ncell);
    Br[c] = to_real(B[c], g.ncell);
    dEr[c] = to_real(dE ? dE[c] : NULL, g.ncell);
    dBr[c] = to_real(dB ? dB[c] : NULL, g.ncell);
    Jr[c] = to_real(NULL, g.ncell);
    dJr[c] = to_real(NULL, g.ncell);
  }
  const real alpha = species_alpha(&g, (real)q, (real)m);
  int err = ORC_OK;
  for (int64_t p = 0; p < n && !err; p++) {
    real xp[3] = {x[0][p], x[1][p], 0}, dxp[3] = {0, 0, 0};
    real up[3] = {u[0][p], u[1][p], u[2][p]};
    real dup[3] = {du ? du[0][p] : 0, du ? du[1][p] : 0, du ? du[2][p] : 0};
    for (int64_t k = 1; k <= nsteps && !err; k++) {
      real F[6], grad[6][3], Fd[6], dF[6], v[3], dv[3];
      interp6(&g, Er, Br, xp, F, grad);
      interp6(&g, dEr, dBr, xp, Fd, NULL);
      for (int c = 0; c < 6; c++)
        dF[c] = Fd[c] + grad[c][0] * dxp[0] * g.inv_d[0] + grad[c][1] * dxp[1] * g.inv_d[1];
      boris_tangent(alpha, F, dF, up, dup, v, dv);
      real x1[3] = {0, 0, 0}, dx1[3] = {0, 0, 0};
      for (int a = 0; a < 2; a++) {
        x1[a] = xp[a] + g.dt * v[a];
        dx1[a] = dxp[a] + g.dt * dv[a];
      }
      /* a removed particle contributes nothing more; a mirror at a wall
       * negates the tangents it negates the values of */
      const int hit = walls(&g, x1, up);
      if (hit < 0) break;
      for (int a = 0; a < 2; a++)
        if (hit >> a & 1) {
          dx1[a] = -dx1[a];
          dup[a] = -dup[a];
        }
      if (k == nsteps) {
        err = deposit_tangent2(&g, (real)q, (real)w[p], xp, x1, v[2], dxp, dx1, dv[2], Jr, dJr);
      } else {
        real xw[3];
        if (patch_key(&g, x1, xw) < 0) err = ORC_ERR_POS;
        xp[0] = xw[0];
        xp[1] = xw[1];
        dxp[0] = dx1[0];
        dxp[1] = dx1[1];
      }
    }
  }
  for (int c = 0; c < 3; c++) {
    for (int64_t i = 0; i < g.ncell; i++) {
      J[c][i] = (double)Jr[c][i];
      dJ[c][i] = (double)dJr[c][i];
    }
    free(Er[c]);
    free(Br[c]);
    free(dEr[c]);
    free(dBr[c]);
    free(Jr[c]);
    free(dJr[c]);
  }
  return err;
}

/* L = sum W . J_final at the start state (x, u + s du) and fields
 * (E + s dE, B + s dB), everything in `real`. */
static int loss_at(const G *g, real q, real m, int64_t n, const double *const x[3],
                   const double *const u[3], const double *w, const double *const E[3],
                   const double *const B[3], const double *const W[3], const double *const du[3],
                   const double *const dE[3], const double *const dB[3], int64_t nsteps, real s,
                   real *L) {
  real *Er[3], *Br[3], *Jr[3];
  for (int c = 0; c < 3; c++) {
    Er[c] = malloc((size_t)g->ncell * sizeof(real));
    Br[c] = malloc((size_t)g->ncell * sizeof(real));
    Jr[c] = to_real(NULL, g->ncell);
    for (int64_t i = 0; i < g->ncell; i++) {
      Er[c][i] = (real)E[c][i] + (dE ? s * (real)dE[c][i] : 0);
      Br[c][i] = (real)B[c][i] + (dB ? s * (real)dB[c][i] : 0);
    }
  }
  const real alpha = species_alpha(g, q, m);
  int err = ORC_OK;
  for (int64_t p = 0; p < n && !err; p++) {
    real xp[3] = {x[0][p], x[1][p], 0};
    real up[3];
    for (int c = 0; c < 3; c++) up[c] = (real)u[c][p] + (du ? s * (real)du[c][p] : 0);
    for (int64_t k = 1; k <= nsteps && !err; k++) {
      real F[6], v[3], x1[3] = {0, 0, 0};
      interp6(g, Er, Br, xp, F, NULL);
      boris(alpha, F, up, v);
      for (int a = 0; a < 2; a++) x1[a] = xp[a] + g->dt * v[a];
      if (walls(g, x1, up) < 0) break;  /* removed: contributes nothing more */
      if (k == nsteps) {
        err = deposit(g, q, (real)w[p], xp, x1, v[2], Jr, NULL);
      } else {
        real xw[3];
        if (patch_key(g, x1, xw) < 0) err = ORC_ERR_POS;
        xp[0] = xw[0];
        xp[1] = xw[1];
      }
    }
  }
  /* Neumaier's compensated summation: the central difference divides the
   * change of L by 2h, so the rounding of a plain sum over every node would
   * reach the derivative's leading digits */
  real acc = 0, comp = 0;
  for (int c = 0; c < 3; c++)
    for (int64_t i = 0; i < g->ncell; i++) {
      const real t = (real)W[c][i] * Jr[c][i];
      const real y = acc + t;
      const real aa = acc < 0 ? -acc : acc, at = t < 0 ? -t : t;
      comp += aa >= at ? (acc - y) + t : (t - y) + acc;
      acc = y;
    }
  *L = acc + comp;
  for (int c = 0; c < 3; c++) {
    free(Er[c]);
    free(Br[c]);
    free(Jr[c]);
  }
  return err;
}

int orc_fd(const orc_grid *gi, double q, double m, int64_t n, const double *const x[3],
           const double *const u[3], const double *w, const double *const E[3],
           const double *const B[3], const double *const W[3], const double *const du[3],
           const double *const dE[3], const double *const dB[3], int64_t nsteps, double h,
           double *fd, double *L0) {
  G g;
  mk_grid(gi, &g);
  if (g.dim != 2 || nsteps < 1) return ORC_ERR_ARG;
  real Lp, Lm, Lz;
  int err = loss_at(&g, (real)q, (real)m, n, x, u, w, E, B, W, du, dE, dB, nsteps, (real)h, &Lp);
  if (!err) err = loss_at(&g, (real)q, (real)m, n, x, u, w, E, B, W, du, dE, dB, nsteps, -(real)h, &Lm);
  if (!err) err = loss_at(&g, (real)q, (real)m, n, x, u, w, E, B, W, du, dE, dB, nsteps, 0, &Lz);
  *fd = (double)((Lp - Lm) / ((real)2 * (real)h));
  *L0 = (double)Lz;
  return err;
}
