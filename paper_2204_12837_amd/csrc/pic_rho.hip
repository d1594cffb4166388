// Charge density on the grid (gfx950): rho = sum q w S(x - node) over the
// particles, with the quadratic B-spline S of the Interpolation and
// Projection operators, on the primal nodes (the charge-density projection
// of the paper's Projection operator, section "Parallelization with OpenMP
// task": current and charge densities are projected on per-patch local
// grids and reduced into the grid).
//
// One workgroup per (patch, species): every particle of the patch adds its
// 3^dim terms into an LDS tile of the patch's nodes and their one-node
// ghosts ((p+3)^dim values), which is then added to the grid with float64
// atomics (neighbouring patches share the ghost nodes).  Each term is
// (q w) (Sx Sy [Sz]), the oracle's product order; only the order of the
// additions at a node differs.
#include <hip/hip_runtime.h>

#include "pic_common.h"
#include "pic_device.h"
#include "pic_fields.h"

namespace pic {

namespace {

constexpr int kRhoWg = 256;

template <int DIM, bool TILE>
__global__ void __launch_bounds__(kRhoWg) k_rho(RhoArgs a, int *err) {
  extern __shared__ __align__(16) double lds[];
  const int P = blockIdx.x;
  const RhoArgs::Sp &S = a.s[blockIdx.y];
  int pc[3], org[3], T[3];
  {
    int r = P;
    pc[0] = r % a.np[0];
    r /= a.np[0];
    pc[1] = r % a.np[1];
    pc[2] = r / a.np[1];
  }
  for (int d = 0; d < 3; d++) {
    const bool on = d < DIM;
    org[d] = on ? pc[d] * a.patch[d] - 1 : 0;
    T[d] = on ? a.patch[d] + 3 : 1;
  }
  const int tn = T[0] * T[1] * T[2];
  if constexpr (TILE) {
    for (int k = threadIdx.x; k < tn; k += blockDim.x) lds[k] = 0.0;
    __syncthreads();
  }
  const int64_t b = S.off[P], e = S.off[P + 1];
  int bad = 0;
  for (int64_t p = b + threadIdx.x; p < e; p += blockDim.x) {
    double sw[3][3];
    int i0[3] = {0, 0, 0};
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; d++) {
      double delta;
      const int i = locate0(S.x[d][p] * a.inv_d[d], delta);
      shape_w(delta, sw[d][0], sw[d][1], sw[d][2]);
      i0[d] = i - 1 - org[d];  // tile index of the first stencil node
      ok = ok && i0[d] >= 0 && i0[d] + 2 < T[d];
    }
    if (!ok) {
      bad = 1;
      continue;
    }
    const double qw = S.q * S.w[p];
    const int nz = DIM == 3 ? 3 : 1;
    for (int c = 0; c < nz; c++)
      for (int bb = 0; bb < 3; bb++)
#pragma unroll
        for (int aa = 0; aa < 3; aa++) {
          const double s = DIM == 3 ? (sw[0][aa] * sw[1][bb]) * sw[2][c] : sw[0][aa] * sw[1][bb];
          const double v = qw * s;
          const int tz = DIM == 3 ? i0[2] + c : 0;
          if constexpr (TILE) {
            lds_add(lds + ((tz * T[1] + i0[1] + bb) * T[0] + i0[0] + aa), v);
          } else {
            const int gx = wrap_near(org[0] + i0[0] + aa, a.n[0]);
            const int gy = wrap_near(org[1] + i0[1] + bb, a.n[1]);
            const int gz = DIM == 3 ? wrap_near(org[2] + tz, a.n[2]) : 0;
            glb_add(a.rho + ((int64_t)gz * a.n[1] + gy) * a.n[0] + gx, v);
          }
        }
  }
  if (bad) atomicOr(err, kErrUnsorted);
  if constexpr (TILE) {
    __syncthreads();
    for (int k = threadIdx.x; k < tn; k += blockDim.x) {
      const double v = lds[k];
      if (v == 0.0) continue;
      const int tx = k % T[0], ty = (k / T[0]) % T[1], tz = k / (T[0] * T[1]);
      const int gx = wrap_near(org[0] + tx, a.n[0]);
      const int gy = wrap_near(org[1] + ty, a.n[1]);
      const int gz = DIM == 3 ? wrap_near(org[2] + tz, a.n[2]) : 0;
      glb_add(a.rho + ((int64_t)gz * a.n[1] + gy) * a.n[0] + gx, v);
    }
  }
}

}  // namespace

hipError_t launch_rho(const RhoArgs &a, int *err, size_t tile_bytes, hipStream_t st) {
  int np = 1;
  for (int d = 0; d < a.dim; d++) np *= a.np[d];
  const dim3 grid((unsigned)np, (unsigned)a.nsp);
  const bool tile = tile_bytes <= 96 * 1024;
  if (a.dim == 2) {
    if (tile)
      hipLaunchKernelGGL((k_rho<2, true>), grid, dim3(kRhoWg), tile_bytes, st, a, err);
    else
      hipLaunchKernelGGL((k_rho<2, false>), grid, dim3(kRhoWg), 0, st, a, err);
  } else {
    if (tile) {
      (void)hipFuncSetAttribute((const void *)k_rho<3, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)tile_bytes);
      hipLaunchKernelGGL((k_rho<3, true>), grid, dim3(kRhoWg), tile_bytes, st, a, err);
    } else {
      hipLaunchKernelGGL((k_rho<3, false>), grid, dim3(kRhoWg), 0, st, a, err);
    }
  }
  return hipGetLastError();
}

}  // namespace pic
