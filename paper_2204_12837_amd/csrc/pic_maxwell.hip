// Field solver of the PIC loop (gfx950): Yee's finite-difference
// time-domain update of E and B on the staggered periodic grid, normalised
// units (c = 1), with the projected current as source (the paper's loop
// solves Maxwell's equations with the current densities of the projection,
// section "Parallelization without tasks").
//
// One step is two kernels over every node, each a streaming stencil bound
// by HBM bandwidth:
//   Ampere   E <- E + dt (curl B - J): backward differences of B, read
//            B (3 arrays, with the x-1, y-1, z-1 neighbours), E, J (6),
//            write E (3) = 96 B per node;
//   Faraday  B <- B - dt curl E: forward differences of the new E, read
//            E (3, with the x+1, y+1, z+1 neighbours), B (3), write B (3)
//            = 72 B per node.
// Ampere reads no E but its own and writes only its own, Faraday likewise
// for B, so both update in place.  A workgroup takes 256 consecutive nodes
// of one x-row (grid: x-chunks, rows, planes), so neighbours along x come
// from the same or the adjacent chunk and the y-1 / z-1 rows were just
// streamed by neighbouring workgroups (cache hits).  Every sum is evaluated
// in a fixed order without contraction:
//   Ex <- ((Ex + c_y dyBz) - c_z dzBy) - dt Jx
//   Ey <- ((Ey + c_z dzBx) - c_x dxBz) - dt Jy
//   Ez <- ((Ez + c_x dxBy) - c_y dyBx) - dt Jz
//   Bx <- (Bx - c_y dyEz) + c_z dzEy
//   By <- (By - c_z dzEx) + c_x dxEz
//   Bz <- (Bz - c_x dxEy) + c_y dyEx
// (in 2D the z terms are absent).
#include <hip/hip_runtime.h>

#include "pic_fields.h"

namespace pic {

namespace {

constexpr int kYeeWg = 256;

__device__ __forceinline__ int prev(int i, int n) { return i == 0 ? n - 1 : i - 1; }
__device__ __forceinline__ int next(int i, int n) { return i == n - 1 ? 0 : i + 1; }

// ADJ: the reverse-mode form (the transposed Faraday update of the E
// cotangent; the host passes the coefficients negated): no current term,
// and the current's cotangent j (writable) accumulates -dt times the new
// value.
template <int DIM, bool ADJ>
__global__ void __launch_bounds__(kYeeWg) k_ampere(YeeArgs a) {
  const int i = blockIdx.x * kYeeWg + threadIdx.x;
  const int nx = a.n[0], ny = a.n[1];
  if (i >= nx) return;
  const int j = blockIdx.y, k = blockIdx.z;
  const int64_t row = ((int64_t)k * ny + j) * nx;
  const int64_t o = row + i;
  const int64_t xm = row + prev(i, nx);
  const int64_t ym = ((int64_t)k * ny + prev(j, ny)) * nx + i;
  const double dyBz = a.b[2][o] - a.b[2][ym];
  const double dxBz = a.b[2][o] - a.b[2][xm];
  const double dxBy = a.b[1][o] - a.b[1][xm];
  const double dyBx = a.b[0][o] - a.b[0][ym];
  double ex = a.e[0][o] + a.c[1] * dyBz;
  double ey = a.e[1][o];
  if constexpr (DIM == 3) {
    const int64_t zm = ((int64_t)prev(k, a.n[2]) * ny + j) * nx + i;
    const double dzBy = a.b[1][o] - a.b[1][zm];
    const double dzBx = a.b[0][o] - a.b[0][zm];
    ex = ex - a.c[2] * dzBy;
    ey = ey + a.c[2] * dzBx;
  }
  ey = ey - a.c[0] * dxBz;
  const double ez = (a.e[2][o] + a.c[0] * dxBy) - a.c[1] * dyBx;
  if constexpr (ADJ) {
    a.e[0][o] = ex;
    a.e[1][o] = ey;
    a.e[2][o] = ez;
    a.j[0][o] = a.j[0][o] - a.dt * ex;
    a.j[1][o] = a.j[1][o] - a.dt * ey;
    a.j[2][o] = a.j[2][o] - a.dt * ez;
  } else {
    a.e[0][o] = ex - a.dt * a.j[0][o];
    a.e[1][o] = ey - a.dt * a.j[1][o];
    a.e[2][o] = ez - a.dt * a.j[2][o];
  }
}

template <int DIM>
__global__ void __launch_bounds__(kYeeWg) k_faraday(YeeArgs a) {
  const int i = blockIdx.x * kYeeWg + threadIdx.x;
  const int nx = a.n[0], ny = a.n[1];
  if (i >= nx) return;
  const int j = blockIdx.y, k = blockIdx.z;
  const int64_t row = ((int64_t)k * ny + j) * nx;
  const int64_t o = row + i;
  const int64_t xp = row + next(i, nx);
  const int64_t yp = ((int64_t)k * ny + next(j, ny)) * nx + i;
  const double dyEz = a.e[2][yp] - a.e[2][o];
  const double dxEz = a.e[2][xp] - a.e[2][o];
  const double dxEy = a.e[1][xp] - a.e[1][o];
  const double dyEx = a.e[0][yp] - a.e[0][o];
  double bx = a.b[0][o] - a.c[1] * dyEz;
  double by = a.b[1][o];
  if constexpr (DIM == 3) {
    const int64_t zp = ((int64_t)next(k, a.n[2]) * ny + j) * nx + i;
    const double dzEy = a.e[1][zp] - a.e[1][o];
    const double dzEx = a.e[0][zp] - a.e[0][o];
    bx = bx + a.c[2] * dzEy;
    by = by - a.c[2] * dzEx;
  }
  by = by + a.c[0] * dxEz;
  const double bz = (a.b[2][o] - a.c[0] * dxEy) + a.c[1] * dyEx;
  a.b[0][o] = bx;
  a.b[1][o] = by;
  a.b[2][o] = bz;
}

}  // namespace

hipError_t launch_yee_step(const YeeArgs &a, hipStream_t st) {
  const dim3 grid((unsigned)((a.n[0] + kYeeWg - 1) / kYeeWg), (unsigned)a.n[1],
                  (unsigned)a.n[2]);
  if (a.dim == 2) {
    hipLaunchKernelGGL((k_ampere<2, false>), grid, dim3(kYeeWg), 0, st, a);
    hipLaunchKernelGGL(k_faraday<2>, grid, dim3(kYeeWg), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_ampere<3, false>), grid, dim3(kYeeWg), 0, st, a);
    hipLaunchKernelGGL(k_faraday<3>, grid, dim3(kYeeWg), 0, st, a);
  }
  return hipGetLastError();
}

// Reverse mode: with e, b the cotangents and j the current's cotangent, the
// transposed Faraday step (the Ampere kernel with negated coefficients and
// the cotangent of the current) then the transposed Ampere step (the
// Faraday kernel with negated coefficients): -c d = -(c d) and x + (-y) =
// x - y exactly, so the values are those of the transposed formulas.
hipError_t launch_yee_adjoint_step(const YeeArgs &a, hipStream_t st) {
  YeeArgs r = a;
  for (int k = 0; k < 3; k++) r.c[k] = -a.c[k];
  const dim3 grid((unsigned)((a.n[0] + kYeeWg - 1) / kYeeWg), (unsigned)a.n[1],
                  (unsigned)a.n[2]);
  if (a.dim == 2) {
    hipLaunchKernelGGL((k_ampere<2, true>), grid, dim3(kYeeWg), 0, st, r);
    hipLaunchKernelGGL(k_faraday<2>, grid, dim3(kYeeWg), 0, st, r);
  } else {
    hipLaunchKernelGGL((k_ampere<3, true>), grid, dim3(kYeeWg), 0, st, r);
    hipLaunchKernelGGL(k_faraday<3>, grid, dim3(kYeeWg), 0, st, r);
  }
  return hipGetLastError();
}

}  // namespace pic
