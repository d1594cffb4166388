// Reverse-mode derivative (adjoint) of the 2D3V particle steps, for a loss
// that depends on the current J deposited by the last step: L = <Jbar, J_N>.
// Fields are static and J is rebuilt every step, so only the last step's
// deposit reaches L and particles do not interact: every particle's
// trajectory is differentiated on its own (one thread per particle), and the
// field cotangents are the sum over particles and steps of the interpolation
// weights times the interpolated fields' cotangents.
//
// A segment of K <= kAdjMaxSteps steps is recomputed from its checkpoint in
// registers (same operation sequence as the forward kernels, so the
// trajectory is the forward one bit for bit), then reversed:
//   deposit (last step only) -> position update -> Boris -> interpolation.
// Cotangents of the particle state are stored by particle id, so segments
// whose checkpoints were sorted differently connect.
#include <hip/hip_runtime.h>

#include "pic_common.h"

namespace pic {

namespace {

__device__ __forceinline__ int wrap_near_a(int k, int n) {
  return k < 0 ? k + n : (k >= n ? k - n : k);
}

__device__ __forceinline__ void glb_add_a(double *p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Quadratic B-spline weights and their slopes d/d(delta).
__device__ __forceinline__ void shape3(double delta, double S[3]) {
  const double a = 0.5 - delta;
  const double b = 0.5 + delta;
  S[0] = 0.5 * (a * a);
  S[1] = 0.75 - delta * delta;
  S[2] = 0.5 * (b * b);
}

__device__ __forceinline__ void slope3(double delta, double D[3]) {
  D[0] = -(0.5 - delta);
  D[1] = -2.0 * delta;
  D[2] = 0.5 + delta;
}

// Node index of the first stencil node and offset, for stagger bit s.
__device__ __forceinline__ int locate_s(double xi, int s, double &delta) {
  const double xs = s ? xi - 0.5 : xi;
  const double f = floor(xs + 0.5);
  delta = xs - f;
  return (int)f - 1;
}

struct Ax {
  double S[3], D[3];
  int i0;  // first stencil node (unwrapped)
};

__device__ __forceinline__ Ax axis_at(double xi, int s) {
  Ax a;
  double delta;
  a.i0 = locate_s(xi, s, delta);
  shape3(delta, a.S);
  slope3(delta, a.D);
  return a;
}

// One interpolated component from global memory, with the forward kernels'
// operation order (x innermost, then y).
__device__ __forceinline__ double gather_g(const GridDev &g, const double *F, const Ax &ax,
                                           const Ax &ay) {
  double r[3];
#pragma unroll
  for (int b = 0; b < 3; b++) {
    const int row = wrap_near_a(ay.i0 + b, g.n[1]) * g.n[0];
    const double f0 = F[row + wrap_near_a(ax.i0, g.n[0])];
    const double f1 = F[row + wrap_near_a(ax.i0 + 1, g.n[0])];
    const double f2 = F[row + wrap_near_a(ax.i0 + 2, g.n[0])];
    double v = ax.S[0] * f0;
    v = v + ax.S[1] * f1;
    v = v + ax.S[2] * f2;
    r[b] = v;
  }
  double v = ay.S[0] * r[0];
  v = v + ay.S[1] * r[1];
  v = v + ay.S[2] * r[2];
  return v;
}

// Stagger bits (x, y) in 2D: Ex(1,0) Ey(0,1) Ez(0,0) Bx(0,1) By(1,0) Bz(1,1).
__constant__ int kStagX[6] = {1, 0, 0, 0, 1, 1};
__constant__ int kStagY[6] = {0, 1, 0, 1, 0, 1};

struct AdjFields {
  const double *f[6];  // Ex Ey Ez Bx By Bz
  const double *jb[3]; // cotangent of J (the loss weights)
  double *fb[6];       // cotangents of the six field components (accumulated)
};

__device__ __forceinline__ void interp_g(const GridDev &g, const AdjFields &f, const double x[2],
                                         double F[6]) {
  const double xi = x[0] * g.inv_d[0], yi = x[1] * g.inv_d[1];
  const Ax x0 = axis_at(xi, 0), x1 = axis_at(xi, 1), y0 = axis_at(yi, 0), y1 = axis_at(yi, 1);
#pragma unroll
  for (int c = 0; c < 6; c++)
    F[c] = gather_g(g, f.f[c], kStagX[c] ? x1 : x0, kStagY[c] ? y1 : y0);
}

// Adjoint of the interpolation at x: given Fb (cotangents of the six
// interpolated values) add d<Fb,F>/dx to xb and scatter Fb times the weights
// into the field cotangents.
__device__ __forceinline__ void interp_adj(const GridDev &g, const AdjFields &f, const double x[2],
                                           const double Fb[6], double xb[2]) {
  const double xi = x[0] * g.inv_d[0], yi = x[1] * g.inv_d[1];
  const Ax x0 = axis_at(xi, 0), x1 = axis_at(xi, 1), y0 = axis_at(yi, 0), y1 = axis_at(yi, 1);
  double gx = 0.0, gy = 0.0;
#pragma unroll
  for (int c = 0; c < 6; c++) {
    const Ax &ax = kStagX[c] ? x1 : x0;
    const Ax &ay = kStagY[c] ? y1 : y0;
    const double *F = f.f[c];
    double *Fbg = f.fb[c];
    const double fb = Fb[c];
#pragma unroll
    for (int b = 0; b < 3; b++) {
      const int row = wrap_near_a(ay.i0 + b, g.n[1]) * g.n[0];
#pragma unroll
      for (int a = 0; a < 3; a++) {
        const int at = row + wrap_near_a(ax.i0 + a, g.n[0]);
        const double v = F[at];
        gx += fb * ax.D[a] * ay.S[b] * v;
        gy += fb * ax.S[a] * ay.D[b] * v;
        if (fb != 0.0) glb_add_a(Fbg + at, fb * ax.S[a] * ay.S[b]);
      }
    }
  }
  xb[0] += gx * g.inv_d[0];
  xb[1] += gy * g.inv_d[1];
}

// Boris push (same sequence as the forward kernels).
__device__ __forceinline__ void boris_f(double alpha, const double F[6], double u[3], double v[3]) {
  const double ae0 = alpha * F[0], ae1 = alpha * F[1], ae2 = alpha * F[2];
  const double um0 = u[0] + ae0, um1 = u[1] + ae1, um2 = u[2] + ae2;
  const double gm = sqrt(1.0 + ((um0 * um0 + um1 * um1) + um2 * um2));
  const double tau = alpha / gm;
  const double t0 = tau * F[3], t1 = tau * F[4], t2 = tau * F[5];
  const double sig = 2.0 / (1.0 + ((t0 * t0 + t1 * t1) + t2 * t2));
  const double s0 = sig * t0, s1 = sig * t1, s2 = sig * t2;
  const double up0 = um0 + (um1 * t2 - um2 * t1);
  const double up1 = um1 + (um2 * t0 - um0 * t2);
  const double up2 = um2 + (um0 * t1 - um1 * t0);
  const double upl0 = um0 + (up1 * s2 - up2 * s1);
  const double upl1 = um1 + (up2 * s0 - up0 * s2);
  const double upl2 = um2 + (up0 * s1 - up1 * s0);
  u[0] = upl0 + ae0;
  u[1] = upl1 + ae1;
  u[2] = upl2 + ae2;
  const double gam = sqrt(1.0 + ((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]));
  const double ig = 1.0 / gam;
  v[0] = u[0] * ig;
  v[1] = u[1] * ig;
  v[2] = u[2] * ig;
}

__device__ __forceinline__ void cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Adjoint of one Boris push from (u, F).  In: ub (cotangent of the new u),
// vb (cotangent of v).  Out: ub replaced by the cotangent of the old u, Fb
// set to the cotangents of the six interpolated fields.  For c = a x b the
// cotangents are abar = b x cbar, bbar = cbar x a.
__device__ __forceinline__ void boris_adj(double alpha, const double F[6], const double u[3],
                                          double ub[3], const double vb[3], double Fb[6]) {
  double ae[3], um[3], t[3], s[3], up[3], un[3];
  for (int k = 0; k < 3; k++) {
    ae[k] = alpha * F[k];
    um[k] = u[k] + ae[k];
  }
  const double g1 = sqrt(1.0 + ((um[0] * um[0] + um[1] * um[1]) + um[2] * um[2]));
  const double tau = alpha / g1;
  for (int k = 0; k < 3; k++) t[k] = tau * F[3 + k];
  const double D = 1.0 + ((t[0] * t[0] + t[1] * t[1]) + t[2] * t[2]);
  const double sig = 2.0 / D;
  for (int k = 0; k < 3; k++) s[k] = sig * t[k];
  double c1[3], c2[3];
  cross(um, t, c1);
  for (int k = 0; k < 3; k++) up[k] = um[k] + c1[k];
  cross(up, s, c2);
  for (int k = 0; k < 3; k++) un[k] = (um[k] + c2[k]) + ae[k];
  const double g2 = sqrt(1.0 + ((un[0] * un[0] + un[1] * un[1]) + un[2] * un[2]));
  const double ig = 1.0 / g2;
  // v = un * ig
  double unb[3];
  double igb = 0.0;
  for (int k = 0; k < 3; k++) {
    unb[k] = ub[k] + vb[k] * ig;
    igb += vb[k] * un[k];
  }
  const double g2b = -ig * ig * igb;
  for (int k = 0; k < 3; k++) unb[k] += g2b * un[k] / g2;
  // un = upl + ae, upl = um + up x s
  double aeb[3], umb[3], upb[3], sb[3], tb[3];
  for (int k = 0; k < 3; k++) {
    aeb[k] = unb[k];
    umb[k] = unb[k];
  }
  cross(s, unb, upb);  // up_bar = s x upl_bar
  cross(unb, up, sb);  // s_bar = upl_bar x up
  // up = um + um x t
  double tmp[3];
  cross(t, upb, tmp);  // um_bar += t x up_bar
  for (int k = 0; k < 3; k++) umb[k] += upb[k] + tmp[k];
  cross(upb, um, tb);  // t_bar = up_bar x um
  // s = sig t
  const double sigb = sb[0] * t[0] + sb[1] * t[1] + sb[2] * t[2];
  for (int k = 0; k < 3; k++) tb[k] += sig * sb[k];
  // sig = 2 / D, D = 1 + t.t
  const double Db = -sig / D * sigb;
  for (int k = 0; k < 3; k++) tb[k] += 2.0 * Db * t[k];
  // t = tau B
  const double taub = tb[0] * F[3] + tb[1] * F[4] + tb[2] * F[5];
  for (int k = 0; k < 3; k++) Fb[3 + k] = tau * tb[k];
  // tau = alpha / g1, g1 = sqrt(1 + um.um)
  const double g1b = -tau / g1 * taub;
  for (int k = 0; k < 3; k++) umb[k] += g1b * um[k] / g1;
  // um = u + ae, ae = alpha E
  for (int k = 0; k < 3; k++) {
    ub[k] = umb[k];
    aeb[k] += umb[k];
    Fb[k] = alpha * aeb[k];
  }
}

// Esirkepov window along one axis (as the forward kernels) plus what the
// adjoint needs: the start/end offsets and shifts.
struct WinA {
  double S0[4], DS[4], A[4];
  double d0, d1;
  int lo, hi;
  int b;  // first window node (unwrapped)
};

__device__ __forceinline__ bool win_a(double xi0, double xi1, WinA &w) {
  double d0, d1;
  const int k0 = (int)floor(xi0 + 0.5);
  d0 = xi0 - (double)k0;
  const int k1 = (int)floor(xi1 + 0.5);
  d1 = xi1 - (double)k1;
  const int m = k1 - k0;
  if (m < -1 || m > 1) return false;
  double a[3], c[3];
  shape3(d0, a);
  shape3(d1, c);
  w.lo = m < 0;
  w.hi = m > 0;
  for (int r = 0; r < 4; r++) {
    const int j0 = r - w.lo, j1 = r - w.hi;
    w.S0[r] = (j0 >= 0 && j0 < 3) ? a[j0] : 0.0;
    const double s1 = (j1 >= 0 && j1 < 3) ? c[j1] : 0.0;
    w.DS[r] = s1 - w.S0[r];
    w.A[r] = w.S0[r] + 0.5 * w.DS[r];
  }
  w.d0 = d0;
  w.d1 = d1;
  w.b = k0 - 1 - w.lo;
  return true;
}

// Cotangents of the window vectors -> cotangents of xi0, xi1 along the axis.
__device__ __forceinline__ void win_back(const WinA &w, const double Ab[4], double DSb[4],
                                         double &xi0b, double &xi1b) {
  double S0b[4], S1b[4];
  for (int r = 0; r < 4; r++) {
    const double dsb = DSb[r] + 0.5 * Ab[r];  // A = S0 + DS/2
    S0b[r] = Ab[r] - dsb;                     // DS = S1 - S0
    S1b[r] = dsb;
  }
  double D0[3], D1[3];
  slope3(w.d0, D0);
  slope3(w.d1, D1);
  double g0 = 0.0, g1 = 0.0;
  for (int j = 0; j < 3; j++) {
    g0 += S0b[j + w.lo] * D0[j];
    g1 += S1b[j + w.hi] * D1[j];
  }
  xi0b = g0;
  xi1b = g1;
}

// Adjoint of the 2D Esirkepov deposit contracted with Jbar: cotangents of
// the start position x0, the end position x1 and the out-of-plane velocity.
__device__ __forceinline__ bool deposit_adj(const GridDev &g, const AdjFields &f, double qw,
                                            const double x0[2], const double x1[2], double vz,
                                            double x0b[2], double x1b[2], double &vzb) {
  WinA wx, wy;
  if (!win_a(x0[0] * g.inv_d[0], x1[0] * g.inv_d[0], wx)) return false;
  if (!win_a(x0[1] * g.inv_d[1], x1[1] * g.inv_d[1], wy)) return false;
  const double cx = -qw * g.d_over_dt[0], cy = -qw * g.d_over_dt[1], cz = qw * vz;
  double Cx[3], Cy[3];
  Cx[0] = wx.DS[0];
  Cx[1] = Cx[0] + wx.DS[1];
  Cx[2] = Cx[1] + wx.DS[2];
  Cy[0] = wy.DS[0];
  Cy[1] = Cy[0] + wy.DS[1];
  Cy[2] = Cy[1] + wy.DS[2];
  double Axb[4] = {0, 0, 0, 0}, Ayb[4] = {0, 0, 0, 0}, DSxb[4] = {0, 0, 0, 0},
         DSyb[4] = {0, 0, 0, 0}, Cxb[3] = {0, 0, 0}, Cyb[3] = {0, 0, 0};
  double czb = 0.0;
  for (int t = 0; t < 4; t++) {
    const int row = wrap_near_a(wy.b + t, g.n[1]) * g.n[0];
    for (int r = 0; r < 4; r++) {
      const int at = row + wrap_near_a(wx.b + r, g.n[0]);
      const double Wx = f.jb[0][at], Wy = f.jb[1][at], Wz = f.jb[2][at];
      if (r < 3) {  // Jx = cx Cx[r] Ay[t]
        Cxb[r] += cx * Wx * wy.A[t];
        Ayb[t] += cx * Wx * Cx[r];
      }
      if (t < 3) {  // Jy = cy Ax[r] Cy[t]
        Axb[r] += cy * Wy * Cy[t];
        Cyb[t] += cy * Wy * wx.A[r];
      }
      // Jz = cz (Ax Ay + DSx DSy / 12)
      Axb[r] += cz * Wz * wy.A[t];
      Ayb[t] += cz * Wz * wx.A[r];
      DSxb[r] += cz * Wz * wy.DS[t] * (1.0 / 12.0);
      DSyb[t] += cz * Wz * wx.DS[r] * (1.0 / 12.0);
      czb += Wz * (wx.A[r] * wy.A[t] + wx.DS[r] * wy.DS[t] * (1.0 / 12.0));
    }
  }
  // C[r] = sum_{r' <= r} DS[r']
  for (int r = 2; r >= 0; r--)
    for (int k = 0; k <= r; k++) {
      DSxb[k] += Cxb[r];
      DSyb[k] += Cyb[r];
    }
  double a0, a1, b0, b1;
  win_back(wx, Axb, DSxb, a0, a1);
  win_back(wy, Ayb, DSyb, b0, b1);
  x0b[0] += a0 * g.inv_d[0];
  x1b[0] += a1 * g.inv_d[0];
  x0b[1] += b0 * g.inv_d[1];
  x1b[1] += b1 * g.inv_d[1];
  vzb += qw * czb;
  return true;
}

// Transpose of the mirror at reflecting walls (bit a of h: axis a was
// mirrored): the cotangents of the position and momentum components along a
// mirrored axis change sign.
__device__ __forceinline__ void unmirror(uint32_t h, double xb[2], double ub[3]) {
  if (h & 1) {
    xb[0] = -xb[0];
    ub[0] = -ub[0];
  }
  if (h & 2) {
    xb[1] = -xb[1];
    ub[1] = -ub[1];
  }
}

__device__ __forceinline__ void wrap2(const GridDev &g, double x[2]) {
  for (int a = 0; a < 2; a++) {
    double v = x[a];
    if (v < 0.0) v += g.L[a];
    if (v >= g.L[a]) v -= g.L[a];
    x[a] = v;
  }
}

// One particle per thread: recompute `nsteps` steps from the checkpoint in
// registers, then reverse them.  with_dep 1: the last step's deposit is
// contracted with Jbar (the seed); 0: the cotangents of the state after the
// segment are read from xb/ub (by particle id); 2: both are added.  On exit
// xb/ub hold the cotangents of the checkpoint state.
__global__ void __launch_bounds__(128) k_adjoint(GridDev g, AdjArgs aa, AdjFields f, int nsteps,
                                                 int with_dep, int *err) {
  const AdjSp &S = aa.s[blockIdx.y];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= S.n) return;
  const int64_t id = S.id[p];
  if (id < 0 || id >= S.nid) {
    atomicOr(err, kErrPos);
    return;
  }
  double xs[kAdjMaxSteps][2], us[kAdjMaxSteps][3];
  double x[2] = {S.x[0][p], S.x[1][p]};
  double u[3] = {S.u[0][p], S.u[1][p], S.u[2][p]};
  double xlast[2] = {0, 0}, xend[2] = {0, 0}, vend[3] = {0, 0, 0};
  uint32_t hits = 0;  // axes mirrored at a wall, two bits per step
  bool gone = false;  // deleted at a removing wall inside the segment
#pragma unroll
  for (int k = 0; k < kAdjMaxSteps; k++) {
    if (k < nsteps && !gone) {
      xs[k][0] = x[0];
      xs[k][1] = x[1];
      us[k][0] = u[0];
      us[k][1] = u[1];
      us[k][2] = u[2];
      double F[6], v[3];
      interp_g(g, f, x, F);
      boris_f(S.alpha, F, u, v);
      double x1[3] = {x[0] + g.dt * v[0], x[1] + g.dt * v[1], 0.0};
      if (g.reflect | g.remove) {
        const int h = wall_bc<2>(g, x1, u);
        gone = h < 0;
        if (!gone) hits |= (uint32_t)h << (2 * k);
      }
      if (k == nsteps - 1) {
        xlast[0] = x[0];
        xlast[1] = x[1];
        xend[0] = x1[0];
        xend[1] = x1[1];
        vend[0] = v[0];
        vend[1] = v[1];
        vend[2] = v[2];
      }
      wrap2(g, x1);
      x[0] = x1[0];
      x[1] = x1[1];
    }
  }
  if (gone) {  // no later state and no deposit: nothing depends on its start
    S.xb[0][id] = S.xb[1][id] = 0.0;
    S.ub[0][id] = S.ub[1][id] = S.ub[2][id] = 0.0;
    return;
  }
  double xb[2], ub[3], vzb = 0.0;
  if (with_dep) {
    double x0b[2] = {0, 0}, x1b[2] = {0, 0};
    if (!deposit_adj(g, f, S.q * S.w[p], xlast, xend, vend[2], x0b, x1b, vzb)) {
      atomicOr(err, kErrCFL);
      return;
    }
    // x_end = x_{N-1} + dt v: the cotangent of x_end enters the position update
    xb[0] = x1b[0];
    xb[1] = x1b[1];
    ub[0] = ub[1] = ub[2] = 0.0;
    // the start-position part joins after the position update is reversed
    x[0] = x0b[0];
    x[1] = x0b[1];
    if (with_dep == 2) {  // and the cotangents of the state after the segment
      xb[0] += S.xb[0][id];
      xb[1] += S.xb[1][id];
      ub[0] = S.ub[0][id];
      ub[1] = S.ub[1][id];
      ub[2] = S.ub[2][id];
    }
  } else {
    xb[0] = S.xb[0][id];
    xb[1] = S.xb[1][id];
    ub[0] = S.ub[0][id];
    ub[1] = S.ub[1][id];
    ub[2] = S.ub[2][id];
    x[0] = x[1] = 0.0;
  }
#pragma unroll
  for (int k = kAdjMaxSteps - 1; k >= 0; k--) {
    if (k < nsteps) {
      // step k: state (xs[k], us[k]) -> x_{k+1} = x + dt v(u'), u', each
      // then mirrored at a wall it crossed: the mirror negates the
      // cotangents of the components it negates
      unmirror(hits >> (2 * k), xb, ub);
      double F[6];
      interp_g(g, f, xs[k], F);
      double vb[3] = {g.dt * xb[0], g.dt * xb[1], 0.0};
      if (with_dep && k == nsteps - 1) vb[2] += vzb;
      double Fb[6];
      boris_adj(S.alpha, F, us[k], ub, vb, Fb);
      double xprev[2] = {xb[0], xb[1]};  // x_{k+1} = x_k + ...: identity part
      if (with_dep && k == nsteps - 1) {
        xprev[0] += x[0];  // deposit's dependence on the step's start position
        xprev[1] += x[1];
      }
      interp_adj(g, f, xs[k], Fb, xprev);
      xb[0] = xprev[0];
      xb[1] = xprev[1];
    }
  }
  S.xb[0][id] = xb[0];
  S.xb[1][id] = xb[1];
  S.ub[0][id] = ub[0];
  S.ub[1][id] = ub[1];
  S.ub[2][id] = ub[2];
}

// ---------------------------------------------------------------------------
// Tiled variant: one workgroup per (patch, species) of a checkpoint sorted
// by patch.  The fields and their cotangents live in LDS tiles covering the
// patch plus everything a particle starting in it can reach in the segment
// (nsteps cells, the Courant limit, plus the stencil), so the interpolation,
// its adjoint and the scatter of the field cotangents stay on chip; the
// cotangent tile is added to the grid once at the end.  A stencil that does
// not lie inside the tile (a particle outside its patch) falls back to the
// global arrays, so the result never depends on the sort.
struct ATile {
  int org[2];   // first tile node (unwrapped grid index)
  int T;        // tile extent per axis
  const double *F;  // 6 component tiles
  double *Fb;       // 6 cotangent tiles
};

// Tile offset of grid node i along axis a (periodic), or -1 if outside.
__device__ __forceinline__ int tile_off(const GridDev &g, const ATile &t, int a, int i) {
  int d = i - t.org[a];
  if (d < 0) d += g.n[a];
  if (d >= g.n[a]) d -= g.n[a];
  return d < t.T ? d : -1;
}

__device__ __forceinline__ double gather_t(const GridDev &g, const ATile &t, int c,
                                           const double *Fg, const Ax &ax, const Ax &ay) {
  const int dx = tile_off(g, t, 0, ax.i0), dy = tile_off(g, t, 1, ay.i0);
  if (dx < 0 || dy < 0 || dx + 2 >= t.T || dy + 2 >= t.T) return gather_g(g, Fg, ax, ay);
  const double *r = t.F + c * t.T * t.T + dy * t.T + dx;
  double rr[3];
#pragma unroll
  for (int b = 0; b < 3; b++) {
    double v = ax.S[0] * r[0];
    v = v + ax.S[1] * r[1];
    v = v + ax.S[2] * r[2];
    rr[b] = v;
    r += t.T;
  }
  double v = ay.S[0] * rr[0];
  v = v + ay.S[1] * rr[1];
  v = v + ay.S[2] * rr[2];
  return v;
}

__device__ __forceinline__ void interp_t(const GridDev &g, const ATile &t, const AdjFields &f,
                                         const double x[2], double F[6]) {
  const double xi = x[0] * g.inv_d[0], yi = x[1] * g.inv_d[1];
  const Ax x0 = axis_at(xi, 0), x1 = axis_at(xi, 1), y0 = axis_at(yi, 0), y1 = axis_at(yi, 1);
#pragma unroll
  for (int c = 0; c < 6; c++)
    F[c] = gather_t(g, t, c, f.f[c], kStagX[c] ? x1 : x0, kStagY[c] ? y1 : y0);
}

__device__ __forceinline__ void interp_adj_t(const GridDev &g, const ATile &t, const AdjFields &f,
                                             const double x[2], const double Fb[6],
                                             double xb[2]) {
  const double xi = x[0] * g.inv_d[0], yi = x[1] * g.inv_d[1];
  const Ax x0 = axis_at(xi, 0), x1 = axis_at(xi, 1), y0 = axis_at(yi, 0), y1 = axis_at(yi, 1);
  double gx = 0.0, gy = 0.0;
#pragma unroll
  for (int c = 0; c < 6; c++) {
    const Ax &ax = kStagX[c] ? x1 : x0;
    const Ax &ay = kStagY[c] ? y1 : y0;
    const double fb = Fb[c];
    const int dx = tile_off(g, t, 0, ax.i0), dy = tile_off(g, t, 1, ay.i0);
    if (dx < 0 || dy < 0 || dx + 2 >= t.T || dy + 2 >= t.T) {
      // outside the tile: global reads and atomics (one component)
      const double *F = f.f[c];
      double *Fbg = f.fb[c];
#pragma unroll
      for (int b = 0; b < 3; b++) {
        const int row = wrap_near_a(ay.i0 + b, g.n[1]) * g.n[0];
#pragma unroll
        for (int a = 0; a < 3; a++) {
          const int at = row + wrap_near_a(ax.i0 + a, g.n[0]);
          const double v = F[at];
          gx += fb * ax.D[a] * ay.S[b] * v;
          gy += fb * ax.S[a] * ay.D[b] * v;
          if (fb != 0.0) glb_add_a(Fbg + at, fb * ax.S[a] * ay.S[b]);
        }
      }
      continue;
    }
    const int base = c * t.T * t.T + dy * t.T + dx;
#pragma unroll
    for (int b = 0; b < 3; b++) {
#pragma unroll
      for (int a = 0; a < 3; a++) {
        const int at = base + b * t.T + a;
        const double v = t.F[at];
        gx += fb * ax.D[a] * ay.S[b] * v;
        gy += fb * ax.S[a] * ay.D[b] * v;
        if (fb != 0.0)
          __hip_atomic_fetch_add(t.Fb + at, fb * ax.S[a] * ay.S[b], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
  xb[0] += gx * g.inv_d[0];
  xb[1] += gy * g.inv_d[1];
}

// Tile extent for a segment of nsteps steps: the patch, nsteps cells each
// side (Courant limit), the stencil's reach (one node below, two above).
__host__ __device__ constexpr int adj_tile_extent(int p, int nsteps) { return p + 2 * nsteps + 5; }

template <int NS>
__global__ void __launch_bounds__(256) k_adjoint_tiled(GridDev g, AdjArgs aa, AdjFields f,
                                                       int with_dep, int *err) {
  extern __shared__ __align__(16) double lds[];
  const AdjSp &S = aa.s[blockIdx.y];
  const int P = blockIdx.x;
  const int px = P % g.np[0], py = P / g.np[0];
  ATile t;
  t.T = adj_tile_extent(g.patch[0], NS);  // square patches checked on the host
  t.org[0] = px * g.patch[0] - NS - 2;
  t.org[1] = py * g.patch[1] - NS - 2;
  const int TT = t.T * t.T;
  double *tf = lds, *tb = lds + 6 * TT;
  t.F = tf;
  t.Fb = tb;
  for (int r = threadIdx.x; r < TT; r += blockDim.x) {
    const int j = r / t.T, i = r - j * t.T;
    int gx = t.org[0] + i, gy = t.org[1] + j;
    gx = ((gx % g.n[0]) + g.n[0]) % g.n[0];
    gy = ((gy % g.n[1]) + g.n[1]) % g.n[1];
    const int64_t at = (int64_t)gy * g.n[0] + gx;
#pragma unroll
    for (int c = 0; c < 6; c++) {
      tf[c * TT + r] = f.f[c][at];
      tb[c * TT + r] = 0.0;
    }
  }
  __syncthreads();
  const int64_t beg = S.off[P], end = S.off[P + 1];
  int bad = 0;
  for (int64_t p = beg + threadIdx.x; p < end; p += blockDim.x) {
    const int64_t id = S.id[p];
    if (id < 0 || id >= S.nid) {
      bad |= kErrPos;
      continue;
    }
    double xs[NS][2], us[NS][3];
    double x[2] = {S.x[0][p], S.x[1][p]};
    double u[3] = {S.u[0][p], S.u[1][p], S.u[2][p]};
    double xlast[2] = {0, 0}, xend[2] = {0, 0}, vend[3] = {0, 0, 0};
    uint32_t hits = 0;  // axes mirrored at a wall, two bits per step
    bool gone = false;  // deleted at a removing wall inside the segment
#pragma unroll
    for (int k = 0; k < NS; k++) {
      if (gone) break;
      xs[k][0] = x[0];
      xs[k][1] = x[1];
      us[k][0] = u[0];
      us[k][1] = u[1];
      us[k][2] = u[2];
      double F[6], v[3];
      interp_t(g, t, f, x, F);
      boris_f(S.alpha, F, u, v);
      double x1[3] = {x[0] + g.dt * v[0], x[1] + g.dt * v[1], 0.0};
      if (g.reflect | g.remove) {
        const int h = wall_bc<2>(g, x1, u);
        gone = h < 0;
        if (!gone) hits |= (uint32_t)h << (2 * k);
      }
      if (k == NS - 1) {
        xlast[0] = x[0];
        xlast[1] = x[1];
        xend[0] = x1[0];
        xend[1] = x1[1];
        vend[0] = v[0];
        vend[1] = v[1];
        vend[2] = v[2];
      }
      wrap2(g, x1);
      x[0] = x1[0];
      x[1] = x1[1];
    }
    if (gone) {  // no later state and no deposit: nothing depends on its start
      S.xb[0][id] = S.xb[1][id] = 0.0;
      S.ub[0][id] = S.ub[1][id] = S.ub[2][id] = 0.0;
      continue;
    }
    double xb[2], ub[3], vzb = 0.0;
    if (with_dep) {
      double x0b[2] = {0, 0}, x1b[2] = {0, 0};
      if (!deposit_adj(g, f, S.q * S.w[p], xlast, xend, vend[2], x0b, x1b, vzb)) {
        bad |= kErrCFL;
        continue;
      }
      xb[0] = x1b[0];
      xb[1] = x1b[1];
      ub[0] = ub[1] = ub[2] = 0.0;
      x[0] = x0b[0];
      x[1] = x0b[1];
      if (with_dep == 2) {  // and the cotangents of the state after the segment
        xb[0] += S.xb[0][id];
        xb[1] += S.xb[1][id];
        ub[0] = S.ub[0][id];
        ub[1] = S.ub[1][id];
        ub[2] = S.ub[2][id];
      }
    } else {
      xb[0] = S.xb[0][id];
      xb[1] = S.xb[1][id];
      ub[0] = S.ub[0][id];
      ub[1] = S.ub[1][id];
      ub[2] = S.ub[2][id];
      x[0] = x[1] = 0.0;
    }
#pragma unroll
    for (int k = NS - 1; k >= 0; k--) {
      unmirror(hits >> (2 * k), xb, ub);
      double F[6];
      interp_t(g, t, f, xs[k], F);
      double vb[3] = {g.dt * xb[0], g.dt * xb[1], 0.0};
      if (with_dep && k == NS - 1) vb[2] += vzb;
      double Fb[6];
      boris_adj(S.alpha, F, us[k], ub, vb, Fb);
      double xprev[2] = {xb[0], xb[1]};
      if (with_dep && k == NS - 1) {
        xprev[0] += x[0];
        xprev[1] += x[1];
      }
      interp_adj_t(g, t, f, xs[k], Fb, xprev);
      xb[0] = xprev[0];
      xb[1] = xprev[1];
    }
    S.xb[0][id] = xb[0];
    S.xb[1][id] = xb[1];
    S.ub[0][id] = ub[0];
    S.ub[1][id] = ub[1];
    S.ub[2][id] = ub[2];
  }
  if (bad) atomicOr(err, bad);
  __syncthreads();
  for (int r = threadIdx.x; r < TT; r += blockDim.x) {
    const int j = r / t.T, i = r - j * t.T;
    int gx = t.org[0] + i, gy = t.org[1] + j;
    gx = ((gx % g.n[0]) + g.n[0]) % g.n[0];
    gy = ((gy % g.n[1]) + g.n[1]) % g.n[1];
    const int64_t at = (int64_t)gy * g.n[0] + gx;
#pragma unroll
    for (int c = 0; c < 6; c++) {
      const double v = tb[c * TT + r];
      if (v != 0.0) glb_add_a(f.fb[c] + at, v);
    }
  }
}

template <int NS>
void launch_tiled(const GridDev &g, const AdjArgs &aa, const AdjFields &f, int with_dep, int *err,
                  hipStream_t st) {
  const int T = adj_tile_extent(g.patch[0], NS);
  const size_t lds = (size_t)12 * T * T * sizeof(double);
  (void)hipFuncSetAttribute((const void *)k_adjoint_tiled<NS>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_adjoint_tiled<NS>, dim3(g.npatch, aa.nsp), dim3(256), lds, st, g, aa, f,
                     with_dep, err);
}

}  // namespace

hipError_t launch_adjoint(const GridDev &g, const AdjArgs &aa, const double *const e[3],
                          const double *const b[3], const double *const jb[3],
                          double *const eb[3], double *const bb[3], int nsteps, int with_dep,
                          int *err, hipStream_t st) {
  AdjFields f;
  for (int c = 0; c < 3; c++) {
    f.f[c] = e[c];
    f.f[3 + c] = b[c];
    f.jb[c] = jb ? jb[c] : nullptr;
    f.fb[c] = eb[c];
    f.fb[3 + c] = bb[c];
  }
  // tiled when every species brings its patch offsets, patches are square
  // and the two tiles fit in LDS with the grid at least a tile wide
  bool tiled = g.dim == 2 && g.patch[0] == g.patch[1];
  for (int s = 0; s < aa.nsp; s++) tiled = tiled && aa.s[s].off != nullptr;
  const int T = adj_tile_extent(g.patch[0], nsteps);
  tiled = tiled && (size_t)12 * T * T * sizeof(double) <= 150 * 1024 && g.n[0] >= T &&
          g.n[1] >= T;
  if (tiled) {
    switch (nsteps) {
      case 1: launch_tiled<1>(g, aa, f, with_dep, err, st); break;
      case 2: launch_tiled<2>(g, aa, f, with_dep, err, st); break;
      case 3: launch_tiled<3>(g, aa, f, with_dep, err, st); break;
      case 4: launch_tiled<4>(g, aa, f, with_dep, err, st); break;
      case 5: launch_tiled<5>(g, aa, f, with_dep, err, st); break;
      case 6: launch_tiled<6>(g, aa, f, with_dep, err, st); break;
      case 7: launch_tiled<7>(g, aa, f, with_dep, err, st); break;
      default: launch_tiled<8>(g, aa, f, with_dep, err, st); break;
    }
    return hipGetLastError();
  }
  int64_t nmax = 1;
  for (int s = 0; s < aa.nsp; s++) nmax = std::max<int64_t>(nmax, aa.s[s].n);
  const dim3 grid((unsigned)((nmax + 127) / 128), aa.nsp);
  hipLaunchKernelGGL(k_adjoint, grid, dim3(128), 0, st, g, aa, f, nsteps, with_dep, err);
  return hipGetLastError();
}

}  // namespace pic
