// Device-side building blocks shared by the kernel files of the library:
// shape functions, LDS tile gathers, the Boris push, the Esirkepov window and
// deposit, pre-BC codes, tile staging and flushing, and the per-particle
// step.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "pic_common.h"

namespace pic {

namespace {


// Largest workgroup per dimension: 3D tiles (and 2D x-bins of tall
// patches) take most of a CU's LDS, so such a workgroup runs alone on its CU
// and needs more waves to hide latency.  The slab-layout kernels fit 128
// registers and take 1024 threads (four waves per SIMD on one tile); the
// dense-layout ones stop at 256 in 2D and 512 in 3D.
template <int DIM>
constexpr int kMaxWg = DIM == 2 ? 256 : 512;
template <int DIM>
constexpr int kMaxWgSlab = 1024;
// Waves per SIMD the register allocation must allow: four in 2D (a 2D
// workgroup's tiles take ~28 KB, so LDS admits several per CU), two in 3D.
template <int DIM>
constexpr int kMinWaves = DIM == 2 ? 4 : 2;

__device__ __forceinline__ int wrap_near(int k, int n) {
  // k is within one period of [0, n)
  return k < 0 ? k + n : (k >= n ? k - n : k);
}

__device__ __forceinline__ void lds_add(double *p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void glb_add(double *p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Quadratic B-spline weights on nodes i-1, i, i+1 for offset delta from i.
__device__ __forceinline__ void shape_w(double delta, double &s0, double &s1, double &s2) {
  const double a = 0.5 - delta;
  const double b = 0.5 + delta;
  s0 = 0.5 * (a * a);
  s1 = 0.75 - delta * delta;
  s2 = 0.5 * (b * b);
}

// Nearest primal node of xi (cell units) and the offset from it.
__device__ __forceinline__ int locate0(double xi, double &delta) {
  const double f = floor(xi + 0.5);
  delta = xi - f;
  return (int)f;
}

// Nearest dual node (position i + 1/2) of xi and the offset from it.
__device__ __forceinline__ int locate1(double xi, double &delta) {
  const double xs = xi - 0.5;
  const double f = floor(xs + 0.5);
  delta = xs - f;
  return (int)f;
}

struct Sh {
  double s[3];
  int i;  // tile index of the first stencil node (node i-1)
};

// Shape of one axis for stagger bit s; org = tile origin node (patch origin - 1).
template <int S>
__device__ __forceinline__ Sh axis_shape(double xi, int org) {
  Sh r;
  double delta;
  const int i = S ? locate1(xi, delta) : locate0(xi, delta);
  shape_w(delta, r.s[0], r.s[1], r.s[2]);
  r.i = i - 1 - org;
  return r;
}

// Sum of three nodes with the x weights, in the oracle's order.
__device__ __forceinline__ double xrow(const Sh &sx, double a, double b, double c) {
  double r = sx.s[0] * a;
  r = r + sx.s[1] * b;
  r = r + sx.s[2] * c;
  return r;
}

// One component from an LDS tile: x innermost, then y, then z.  All nodes
// of a 2D stencil are read before any is used, so the wave has the nine
// reads in flight together.
template <int DIM>
__device__ __forceinline__ double gather(const double *t, int Tx, int Txy, const Sh &sx,
                                         const Sh &sy, const Sh &sz) {
  if constexpr (DIM == 2) {
    const double *r = t + sy.i * Tx + sx.i;
    double n[3][3];
#pragma unroll
    for (int b = 0; b < 3; b++)
#pragma unroll
      for (int a = 0; a < 3; a++) n[b][a] = r[b * Tx + a];
    const double r0 = xrow(sx, n[0][0], n[0][1], n[0][2]);
    const double r1 = xrow(sx, n[1][0], n[1][1], n[1][2]);
    const double r2 = xrow(sx, n[2][0], n[2][1], n[2][2]);
    double v = sy.s[0] * r0;
    v = v + sy.s[1] * r1;
    v = v + sy.s[2] * r2;
    return v;
  } else {
    double pl[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const double *r = t + (sz.i + c) * Txy + sy.i * Tx + sx.i;
      double rr[3];
#pragma unroll
      for (int b = 0; b < 3; b++) {
        rr[b] = xrow(sx, r[0], r[1], r[2]);
        r += Tx;
      }
      double v = sy.s[0] * rr[0];
      v = v + sy.s[1] * rr[1];
      v = v + sy.s[2] * rr[2];
      pl[c] = v;
    }
    double v = sz.s[0] * pl[0];
    v = v + sz.s[1] * pl[1];
    v = v + sz.s[2] * pl[2];
    return v;
  }
}

// Gather a pair of components stored interleaved (a, b) per node (2D: the
// pairs (Ex, By) and (Ey, Bx) share their staggering), with the same
// operation order as gather<2> for each of them; the nine node pairs are
// read before any is used.
__device__ __forceinline__ void gather_pair(const double2 *t, int Tx, const Sh &sx, const Sh &sy,
                                            double &fa, double &fb) {
  const double2 *r = t + sy.i * Tx + sx.i;
  double2 q[3][3];
#pragma unroll
  for (int b = 0; b < 3; b++)
#pragma unroll
    for (int a = 0; a < 3; a++) q[b][a] = r[b * Tx + a];
  double ra[3], rb[3];
#pragma unroll
  for (int b = 0; b < 3; b++) {
    ra[b] = xrow(sx, q[b][0].x, q[b][1].x, q[b][2].x);
    rb[b] = xrow(sx, q[b][0].y, q[b][1].y, q[b][2].y);
  }
  double a = sy.s[0] * ra[0];
  a = a + sy.s[1] * ra[1];
  a = a + sy.s[2] * ra[2];
  double bb = sy.s[0] * rb[0];
  bb = bb + sy.s[1] * rb[1];
  bb = bb + sy.s[2] * rb[2];
  fa = a;
  fb = bb;
}

// Shapes of a position on every axis: primal (p) and dual (d) stagger.
struct Shapes {
  Sh p[3], d[3];
};

template <int DIM>
__device__ __forceinline__ Shapes shapes_at(const double xi[3], const int org[3]) {
  Shapes s;
#pragma unroll
  for (int a = 0; a < DIM; a++) {
    s.p[a] = axis_shape<0>(xi[a], org[a]);
    s.d[a] = axis_shape<1>(xi[a], org[a]);
  }
  if constexpr (DIM == 2) s.p[2] = s.d[2] = Sh{{0.0, 1.0, 0.0}, 0};
  return s;
}

// E/B tile layout.  2D: [(Ex,By) pairs | (Ey,Bx) pairs | Ez | Bz], each block
// TE nodes; 3D: Ex, Ey, Ez, Bx, By, Bz, TE doubles each.
// Stagger bits: Ex(1,0,0) Ey(0,1,0) Ez(0,0,1) Bx(0,1,1) By(1,0,1) Bz(1,1,0).
template <int DIM>
__device__ __forceinline__ void interp6(const double *tile, int TE, int Tx, int Txy,
                                        const Shapes &s, double F[6]) {
  if constexpr (DIM == 2) {
    const double2 *pr = reinterpret_cast<const double2 *>(tile);
    gather_pair(pr, Tx, s.d[0], s.p[1], F[0], F[4]);       // Ex, By
    gather_pair(pr + TE, Tx, s.p[0], s.d[1], F[1], F[3]);  // Ey, Bx
    F[2] = gather<2>(tile + 4 * TE, Tx, Txy, s.p[0], s.p[1], s.p[2]);  // Ez
    F[5] = gather<2>(tile + 5 * TE, Tx, Txy, s.d[0], s.d[1], s.p[2]);  // Bz
  } else {
    F[0] = gather<3>(tile + 0 * TE, Tx, Txy, s.d[0], s.p[1], s.p[2]);
    F[1] = gather<3>(tile + 1 * TE, Tx, Txy, s.p[0], s.d[1], s.p[2]);
    F[2] = gather<3>(tile + 2 * TE, Tx, Txy, s.p[0], s.p[1], s.d[2]);
    F[3] = gather<3>(tile + 3 * TE, Tx, Txy, s.p[0], s.d[1], s.d[2]);
    F[4] = gather<3>(tile + 4 * TE, Tx, Txy, s.d[0], s.p[1], s.d[2]);
    F[5] = gather<3>(tile + 5 * TE, Tx, Txy, s.d[0], s.d[1], s.p[2]);
  }
}

// Relativistic Boris push, same operation sequence as the CPU oracle.
__device__ __forceinline__ void boris(double alpha, const double F[6], double u[3], double v[3]) {
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

// Esirkepov quantities along one axis on the four nodes that the start and
// end stencils can cover.  p0 is the start position's primal shape (nearest
// node i0, weights on i0-1..i0+1, p0.i = E/B-tile index of node i0-1); i1 is
// the end position's nearest node, m = i1 - i0 in {-1, 0, 1}.  The window
// starts at node i0 - 1 + min(m, 0) and holds S0 (start weights), DS = S1 - S0
// and A = S0 + DS/2 (the path-averaged weight); for m = 0 its fourth node
// carries zeros.  it = J-tile index of the window's first node (the J tile
// starts one node before the E/B tile).  False on a larger shift.
struct Win {
  double S0[4], DS[4], A[4];
  int it;
  bool moved;  // m != 0: the fourth window node is live
};

__device__ __forceinline__ bool esk_win(const Sh &p0, double xi1, int i0, Win &w) {
  double d1;
  const int k1 = locate0(xi1, d1);
  const int m = k1 - i0;
  if (m < -1 || m > 1) return false;
  double b0, b1, b2;
  shape_w(d1, b0, b1, b2);
  const bool lo = m < 0, hi = m > 0;
  const double a0 = p0.s[0], a1 = p0.s[1], a2 = p0.s[2];
  w.S0[0] = lo ? 0.0 : a0;
  w.S0[1] = lo ? a0 : a1;
  w.S0[2] = lo ? a1 : a2;
  w.S0[3] = lo ? a2 : 0.0;
  const double S1[4] = {hi ? 0.0 : b0, hi ? b0 : b1, hi ? b1 : b2, hi ? b2 : 0.0};
#pragma unroll
  for (int r = 0; r < 4; r++) {
    w.DS[r] = S1[r] - w.S0[r];
    w.A[r] = __builtin_fma(0.5, w.DS[r], w.S0[r]);
  }
  w.it = p0.i + (lo ? 0 : 1);
  w.moved = m != 0;
  return true;
}

// Esirkepov deposit of one particle into the LDS J tile, in factored form:
// with A = S0 + DS/2 on each axis,
//   2D  Wx = DSx (x) Ay, Wy = Ax (x) DSy, Wz = Ax (x) Ay + DSx (x) DSy / 12,
//   3D  Wx = DSx (x) (Ay (x) Az + DSy (x) DSz / 12), y and z cyclic,
// which equals Esirkepov's weights (expand A); J along a component's own axis
// is the running sum of its W times -q w d/dt, so 3 of the 4 window nodes are
// nonzero.  Adds per particle: 2D at most 12 + 12 + 16, 3D 3 x 48; 6 + 6 + 9
// and 3 x 18 when the particle stays nearest to the same node.
template <int DIM>
__device__ __forceinline__ void deposit(const GridDev &g, double *tJ, int TJn, int TJx, int TJxy,
                                        double qw, const Win *w, double vz) {
  if constexpr (DIM == 2) {
    double *Jx = tJ + w[1].it * TJx + w[0].it;
    double *Jy = Jx + TJn, *Jz = Jx + 2 * TJn;
    const double cx = -qw * g.d_over_dt[0];
    const double cy = -qw * g.d_over_dt[1];
    const double cz = qw * vz;
    const double cz12 = cz * (1.0 / 12.0);
    double Cx[3], Cy[3];
    Cx[0] = w[0].DS[0];
    Cx[1] = Cx[0] + w[0].DS[1];
    Cx[2] = Cx[1] + w[0].DS[2];
    Cy[0] = w[1].DS[0];
    Cy[1] = Cy[0] + w[1].DS[1];
    Cy[2] = Cy[1] + w[1].DS[2];
#pragma unroll
    for (int k = 0; k < 3; k++) {
      Cx[k] *= cx;
      Cy[k] *= cy;
    }
    // Without a node change along an axis (the common case) the window's
    // last node carries zero weight and the running sum is exactly zero
    // from the third node on; those adds are masked off per lane.
    const bool mx = w[0].moved, my = w[1].moved;
    double az[4], dz[4];
#pragma unroll
    for (int r = 0; r < 4; r++) {
      az[r] = cz * w[0].A[r];
      dz[r] = cz12 * w[0].DS[r];
    }
    // The three components' adds alternate, so consecutive LDS atomics never
    // hit the same word (a read-modify-write of an address still in flight
    // stalls the LDS pipeline).
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        if ((t < 3 || my) && (r < 3 || mx))
          lds_add(Jz + t * TJx + r, __builtin_fma(az[r], w[1].A[t], dz[r] * w[1].DS[t]));
        if (r < 3 && (t < 3 || my) && (r < 2 || mx)) lds_add(Jx + t * TJx + r, Cx[r] * w[1].A[t]);
        if (t < 3 && (r < 3 || mx) && (t < 2 || my)) lds_add(Jy + t * TJx + r, w[0].A[r] * Cy[t]);
      }
  } else {
    const int stride[3] = {1, TJx, TJxy};
    double *J0 = tJ + w[2].it * TJxy + w[1].it * TJx + w[0].it;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      const double ca = -qw * g.d_over_dt[a];
      double C[3];
      C[0] = w[a].DS[0];
      C[1] = C[0] + w[a].DS[1];
      C[2] = C[1] + w[a].DS[2];
#pragma unroll
      for (int k = 0; k < 3; k++) C[k] *= ca;
      double *Ja = J0 + a * TJn;
      const bool ma = w[a].moved, mb = w[b].moved, mc = w[c].moved;
#pragma unroll
      for (int tb = 0; tb < 4; tb++) {
        const double db12 = w[b].DS[tb] * (1.0 / 12.0);
#pragma unroll
        for (int tc = 0; tc < 4; tc++) {
          const double f = __builtin_fma(w[b].A[tb], w[c].A[tc], db12 * w[c].DS[tc]);
          double *line = Ja + tb * stride[b] + tc * stride[c];
#pragma unroll
          for (int ta = 0; ta < 3; ta++)
            if ((tb < 3 || mb) && (tc < 3 || mc) && (ta < 2 || ma))
              lds_add(line + ta * stride[a], C[ta] * f);
        }
      }
    }
  }
}

// Patch coordinates of patch P.
__device__ __forceinline__ void patch_coords(const GridDev &g, int P, int pc[3]) {
  pc[0] = P % g.np[0];
  const int r = P / g.np[0];
  pc[1] = r % g.np[1];
  pc[2] = r / g.np[1];
}

// pre-BC: wrap x1 into the box (in place) and return the neighbour code of
// the destination patch of a particle of the patch whose first cell is lo
// (-1 on a bad position).  The destination is the patch of the wrapped
// position's cell c = min(floor(x inv_d), n-1); with the particle at most
// one cell from its patch, d = (c - lo) mod n picks it without a division:
// d < p stays, p <= d < 2p is the next patch, d >= n - p the previous one.
template <int DIM>
__device__ __forceinline__ int dest_code(const GridDev &g, const int lo[3], double x[3]) {
  int code = 0, mul = 1;
#pragma unroll
  for (int a = 0; a < DIM; a++) {
    double v = x[a];
    if (v < 0.0) v += g.L[a];
    if (v >= g.L[a]) v -= g.L[a];
    if (!(v >= 0.0 && v < g.L[a])) return -1;
    x[a] = v;
    int c = (int)floor(v * g.inv_d[a]);
    if (c >= g.n[a]) c = g.n[a] - 1;
    int d = c - lo[a];
    if (d < 0) d += g.n[a];
    const int p = g.patch[a];
    int delta;
    if (d < p)
      delta = 0;
    else if (d < 2 * p)
      delta = 1;
    else if (d >= g.n[a] - p)
      delta = -1;
    else
      return -1;
    code += (delta + 1) * mul;
    mul *= 3;
  }
  return code;
}

// Destination patch of code c from patch coordinates pc (-1 for kGone: the
// particle is deleted).
__device__ __forceinline__ int dest_patch(const GridDev &g, const int pc[3], int c) {
  if (c == kGone) return -1;
  int D = 0, mul = 1;
  for (int a = 0; a < 3; a++) {
    int delta = 0;
    if (a < g.dim) {
      delta = c % 3 - 1;
      c /= 3;
    }
    int q = pc[a] + delta;
    if (q < 0) q += g.np[a];
    if (q >= g.np[a]) q -= g.np[a];
    D += q * mul;
    mul *= g.np[a];
  }
  return D;
}

// Stable rank of each lane's particle among the wave's earlier particles with
// the same code, plus the ranking unit's running count per code (lane c of
// `run` holds code c's count).  One ballot per distinct code in the wave.
__device__ __forceinline__ uint32_t wave_rank(bool valid, int code, int lane, int &run) {
  uint64_t todo = __ballot(valid);
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  uint32_t r = 0;
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const int lc = __builtin_amdgcn_readlane(code, leader);
    const uint64_t m = __ballot(valid && code == lc);
    const int base = __builtin_amdgcn_readlane(run, lc);
    if (valid && code == lc) r = (uint32_t)(base + __popcll(m & lt));
    if (lane == lc) run += __popcll(m);
    todo &= ~m;
  }
  return r;
}

struct Fields {
  const double *e[3];
  const double *b[3];
  double *j[3];
};

struct TileGeom {
  int org[3];   // E/B tile origin node (patch origin - 1)
  int org2[3];  // J tile origin node (patch origin - 2)
  int pc[3];
  int lo[3], hi[3];  // patch cell range [lo, hi] (as doubles: xi in [lo, hi])
  int Tx, Txy, TE;   // E/B tile extents
  int Jx, Jxy, TJ;   // J tile extents
};

template <int DIM>
__device__ __forceinline__ TileGeom tile_geom(const GridDev &g, int P) {
  TileGeom t;
  patch_coords(g, P, t.pc);
  for (int a = 0; a < 3; a++) {
    const int o = a < DIM ? t.pc[a] * g.patch[a] : 0;
    t.lo[a] = o;
    t.hi[a] = o + g.patch[a];
    t.org[a] = o - 1;
    t.org2[a] = o - 2;
  }
  const int ex = g.patch[0] + 3, ey = g.patch[1] + 3, ez = DIM == 3 ? g.patch[2] + 3 : 1;
  t.Tx = ex;
  t.Txy = ex * ey;
  t.TE = ex * ey * ez;
  const int jx = g.patch[0] + 5, jy = g.patch[1] + 5, jz = DIM == 3 ? g.patch[2] + 5 : 1;
  t.Jx = jx;
  t.Jxy = jx * jy;
  t.TJ = jx * jy * jz;
  return t;
}

// Global index of node r of a tile of extents tx, ty (x fastest) whose first
// node sits at org (periodic wrap into the grid).
template <int DIM>
__device__ __forceinline__ int64_t tile_node(const GridDev &g, const int org[3], int r, int tx,
                                             int ty) {
  const int txy = tx * ty;
  const int k = DIM == 3 ? r / txy : 0;
  const int rr = r - k * txy;
  const int j = rr / tx;
  const int i = rr - j * tx;
  const int gx = wrap_near(org[0] + i, g.n[0]);
  const int gy = wrap_near(org[1] + j, g.n[1]);
  const int gz = DIM == 3 ? wrap_near(org[2] + k, g.n[2]) : 0;
  return ((int64_t)gz * g.n[1] + gy) * g.n[0] + gx;
}

// Stage the E/B tile: each thread takes up to kStageNodes nodes at a time
// and issues the loads of all six components before any LDS store, so the
// staging costs one memory round trip per batch (the component loop is
// uniform: the field pointers stay in scalar registers).
constexpr int kStageNodes = 4;

template <int DIM>
__device__ void stage_eb(const GridDev &g, const TileGeom &t, const Fields &f, double *tile) {
  const int Ty = t.Txy / t.Tx;
  const int nt = blockDim.x;
  for (int b0 = 0; b0 < t.TE; b0 += kStageNodes * nt) {
    int64_t gi[kStageNodes];
    int rr[kStageNodes];
#pragma unroll
    for (int k = 0; k < kStageNodes; k++) {
      rr[k] = b0 + (int)threadIdx.x + k * nt;
      gi[k] = rr[k] < t.TE ? tile_node<DIM>(g, t.org, rr[k], t.Tx, Ty) : 0;
    }
    double v[6][kStageNodes];
#pragma unroll
    for (int c = 0; c < 6; c++) {
      const double *F = c < 3 ? f.e[c] : f.b[c - 3];
      // unconditional loads (a node past the tile reads grid node 0), so
      // the memory-counter waits need not assume a skipped load
#pragma unroll
      for (int k = 0; k < kStageNodes; k++) v[c][k] = F[gi[k]];
    }
#pragma unroll
    for (int k = 0; k < kStageNodes; k++) {
      const int r = rr[k];
      if (r >= t.TE) continue;
      if constexpr (DIM == 2) {
        // (Ex, By) pairs, (Ey, Bx) pairs, Ez, Bz
        tile[2 * r] = v[0][k];
        tile[2 * r + 1] = v[4][k];
        tile[2 * t.TE + 2 * r] = v[1][k];
        tile[2 * t.TE + 2 * r + 1] = v[3][k];
        tile[4 * t.TE + r] = v[2][k];
        tile[5 * t.TE + r] = v[5][k];
      } else {
#pragma unroll
        for (int c = 0; c < 6; c++) tile[c * t.TE + r] = v[c][k];
      }
    }
  }
}

template <int DIM>
__device__ void zero_tile(double *tJ, int n) {
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) tJ[idx] = 0.0;
}

// Add the J tile into the grid with one global atomic per nonzero entry;
// the component loop is uniform, so the grid pointers stay in scalar
// registers and no global load precedes the atomics.
template <int DIM>
__device__ void flush_j(const GridDev &g, const TileGeom &t, const double *tJ, double *const j[3]) {
  const int Jy = t.Jxy / t.Jx;
  const int nt = blockDim.x;
#pragma unroll
  for (int c = 0; c < 3; c++) {
    double *J = j[c];
    const double *T = tJ + c * t.TJ;
    for (int r = threadIdx.x; r < t.TJ; r += nt) {
      const double v = T[r];
      if (v == 0.0) continue;
      glb_add(J + tile_node<DIM>(g, t.org2, r, t.Jx, Jy), v);
    }
  }
}

// True if the particle at xi lies in the patch (as the sort placed it).
template <int DIM>
__device__ __forceinline__ bool in_patch(const TileGeom &t, const double xi[3]) {
  bool ok = true;
#pragma unroll
  for (int a = 0; a < DIM; a++) ok = ok && xi[a] >= (double)t.lo[a] && xi[a] <= (double)t.hi[a];
  return ok;
}

// Element k of a particle array through a 32-bit byte offset (k < 2^29):
// loads and stores then take the array's base from scalar registers and one
// vector register for the offset, shared by every array.
template <typename T>
__device__ __forceinline__ T &at(T *p, uint32_t k) {
  return *reinterpret_cast<T *>(reinterpret_cast<char *>(p) + (k * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ const T &at(const T *p, uint32_t k) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) + (k * (uint32_t)sizeof(T)));
}

// State of one particle as read at the start of a step (with its id when
// the particle moves to another slot).
template <int DIM, bool ID>
struct Part {
  double x[DIM], u[3], w;
  int64_t id;
};

template <int DIM, bool ID>
__device__ __forceinline__ void load_part(const SpDev &S, uint32_t src, Part<DIM, ID> &p) {
#pragma unroll
  for (int a = 0; a < DIM; a++) p.x[a] = at(S.x[a], src);
  p.u[0] = at(S.u[0], src);
  p.u[1] = at(S.u[1], src);
  p.u[2] = at(S.u[2], src);
  p.w = at(S.w, src);
  if (ID) p.id = at(S.id, src);
}

// The 64-particle blocks one wave processes: sub-blocks of ranking segments
// k = k0 + wv, k0 + wv + nw, ... below k1 (segments hold kSeg consecutive
// particles of the patch; only the patch's last one can be short, so only
// the wave's last block can be partial).  All fields are wave-uniform.  A
// step past the wave's last block leaves the block where it is, marked dead.
struct Blk {
  int k;          // ranking segment inside the patch
  uint32_t base;  // first particle of the block
  uint32_t se;    // end of the segment
  bool dead;
  __device__ void start(int k_, uint32_t beg, uint32_t end) {
    k = k_;
    base = beg + (uint32_t)k * kSeg;
    se = base + kSeg < end ? base + kSeg : end;
    dead = false;
  }
  __device__ void next(int nw, int k1, uint32_t beg, uint32_t end) {
    if (dead) return;
    if (base + 64 < se) {
      base += 64;
    } else if (k + nw < k1) {
      start(k + nw, beg, end);
    } else {
      dead = true;
    }
  }
  __device__ bool full() const { return base + 64 <= se; }
  // lane's slot, clamped into the block (always a valid particle)
  __device__ uint32_t slot(int lane) const {
    const uint32_t i = base + (uint32_t)lane;
    return i < se ? i : se - 1;
  }
};

// Interpolation, Push, Projection and pre-BC of one particle: advances x
// (wrapped, or mirrored at reflecting walls before the Projection) and u in
// place and returns its neighbour code (CENTER when the particle is
// rejected, with the error bit set; kGone, with no deposit, when it left
// through a removing wall).  WALLS = false compiles the walls out (a kernel
// instance for periodic grids only).
template <int DIM, bool WALLS>
__device__ __forceinline__ int step_particle(const GridDev &g, const TileGeom &t, const double *tEB,
                                             double *tJ, double q, double alpha, double w,
                                             double x[3], double u[3], int &bad) {
  constexpr int CENTER = DIM == 2 ? 4 : 13;
  double xi[3], v[3], F[6];
#pragma unroll
  for (int a = 0; a < DIM; a++) xi[a] = x[a] * g.inv_d[a];
  if (!in_patch<DIM>(t, xi)) {
    bad |= kErrUnsorted;
    return CENTER;
  }
  const Shapes sh = shapes_at<DIM>(xi, t.org);
  interp6<DIM>(tEB, t.TE, t.Tx, t.Txy, sh, F);
  boris(alpha, F, u, v);
  double x1[3];
  Win win[DIM];
  bool ok = true;
  if constexpr (WALLS) {
#pragma unroll
    for (int a = 0; a < DIM; a++) x1[a] = x[a] + g.dt * v[a];
    if ((g.reflect | g.remove) && wall_bc<DIM>(g, x1, u) < 0) {
#pragma unroll
      for (int a = 0; a < DIM; a++) x[a] = x1[a];
      return kGone;  // deleted at a removing wall: no deposit
    }
#pragma unroll
    for (int a = 0; a < DIM; a++)
      ok = ok && esk_win(sh.p[a], x1[a] * g.inv_d[a], sh.p[a].i + 1 + t.org[a], win[a]);
  } else {
#pragma unroll
    for (int a = 0; a < DIM; a++) {
      x1[a] = x[a] + g.dt * v[a];
      ok = ok && esk_win(sh.p[a], x1[a] * g.inv_d[a], sh.p[a].i + 1 + t.org[a], win[a]);
    }
  }
  if (ok)
    deposit<DIM>(g, tJ, t.TJ, t.Jx, t.Jxy, q * w, win, v[2]);
  else
    bad |= kErrCFL;
  const int c = dest_code<DIM>(g, t.lo, x1);
#pragma unroll
  for (int a = 0; a < DIM; a++) x[a] = x1[a];
  if (c < 0) {
    bad |= kErrPos;
    return CENTER;
  }
  return c;
}

// Exclusive scan of n int64 values from `in` into out[0..n] (out[n] = total),
// by one workgroup of 1024 threads.
__device__ void block_scan_1024(const int64_t *in, int64_t *out, int n, int64_t *part) {
  const int per = (n + blockDim.x - 1) / blockDim.x;
  const int b = threadIdx.x * per;
  const int e = min(n, b + per);
  int64_t sum = 0;
  for (int k = b; k < e; k++) sum += in[k];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const int64_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t run = part[threadIdx.x] - sum;
  for (int k = b; k < e; k++) {
    const int64_t v = in[k];
    out[k] = run;
    run += v;
  }
  if (threadIdx.x == blockDim.x - 1) out[n] = part[threadIdx.x];
  __syncthreads();
}


inline Fields mkfields(const double *const e[3], const double *const b[3], double *const j[3]) {
  Fields f;
  for (int c = 0; c < 3; c++) {
    f.e[c] = e ? e[c] : nullptr;
    f.b[c] = b ? b[c] : nullptr;
    f.j[c] = j ? j[c] : nullptr;
  }
  return f;
}

inline size_t tile_eb_bytes(const GridDev &g) {
  size_t t = 1;
  for (int a = 0; a < g.dim; a++) t *= (size_t)(g.patch[a] + 3);
  return 6 * t * sizeof(double);
}

inline size_t tile_j_bytes(const GridDev &g) {
  size_t t = 1;
  for (int a = 0; a < g.dim; a++) t *= (size_t)(g.patch[a] + 5);
  return 3 * t * sizeof(double);
}

}  // namespace

}  // namespace pic
