// Internal declarations of the field solver (pic_maxwell.hip).  Not part of
// the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// One Yee step's arguments: cells per axis (1 for an absent axis), the
// coefficients c_a = dt / d_a (computed once on the host, 0 for an absent
// axis) and dt.  j is read by the forward step and accumulated into by the
// reverse mode.
struct YeeArgs {
  int dim;
  int n[3];
  double c[3];
  double dt;
  double *e[3], *b[3], *j[3];
};

// One Yee step: Ampere (E from B and J), then Faraday (B from the new E).
hipError_t launch_yee_step(const YeeArgs &a, hipStream_t st);
// Reverse mode of one step: e, b hold the cotangents (updated in place), j
// the current's cotangent (accumulated).
hipError_t launch_yee_adjoint_step(const YeeArgs &a, hipStream_t st);

// Charge density: per species the particles sorted by patch (offsets of
// the configuration's patches).
constexpr int kRhoMaxSpecies = 8;
struct RhoArgs {
  int dim;
  int n[3], patch[3], np[3];
  double inv_d[3];
  int nsp;
  struct Sp {
    double q;
    const double *x[3];
    const double *w;
    const int64_t *off;
  } s[kRhoMaxSpecies];
  double *rho;
};

// rho += sum over species and particles of q w S(x - node) on the primal
// nodes; one workgroup per (patch, species), LDS tile of the patch's nodes
// when it fits (tile_bytes), global atomics otherwise.
hipError_t launch_rho(const RhoArgs &a, int *err, size_t tile_bytes, hipStream_t st);

}  // namespace pic
