// Internal declarations of the field solver (pic_maxwell.hip).  Not part of
// the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// One Yee step's arguments: cells per axis (1 for an absent axis), the
// coefficients c_a = dt / d_a (computed once on the host, 0 for an absent
// axis) and dt.
struct YeeArgs {
  int dim;
  int n[3];
  double c[3];
  double dt;
  double *e[3], *b[3];
  const double *j[3];
};

// One Yee step: Ampere (E from B and J), then Faraday (B from the new E).
hipError_t launch_yee_step(const YeeArgs &a, hipStream_t st);
// Reverse mode of one step: e, b hold the cotangents (updated in place), j
// the current's cotangent (accumulated; written through the const pointer).
hipError_t launch_yee_adjoint_step(const YeeArgs &a, hipStream_t st);

}  // namespace pic
