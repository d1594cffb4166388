/* A C program that drives the library through its C ABI alone (no Python,
 * no torch): host-only configuration checks, and with "gpu" a short run of
 * free-streaming particles on the device whose total current and final
 * positions have closed forms -- once as one pic_step call, once as
 * one-step calls with PIC_FLAG_RESIDENT and a closing pic_sync.  Prints
 * "ok" and exits 0 on success. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pic.h"

#define NX 32
#define NY 32
#define PPC 4
#define NP (NX * NY * PPC)
#define STEPS 5

static int fail(const char *what) {
  printf("FAIL: %s\n", what);
  return 1;
}

static pic_config config(void) {
  pic_config c;
  memset(&c, 0, sizeof c);
  c.dim = 2;
  c.n[0] = NX;
  c.n[1] = NY;
  c.n[2] = 1;
  c.d[0] = c.d[1] = c.d[2] = 0.1;
  c.dt = 0.95 / sqrt(2.0 / (0.1 * 0.1));
  c.patch[0] = c.patch[1] = 8;
  c.patch[2] = 1;
  c.shape_order = 2;
  c.mode = PIC_MODE_PER_PATCH;
  return c;
}

static int host_checks(void) {
  pic_config c = config();
  char msg[256];
  if (pic_validate_config(&c, msg, sizeof msg) != PIC_OK) return fail(msg);
  if (pic_num_patches(&c) != (NX / 8) * (NY / 8)) return fail("pic_num_patches");
  if (pic_bin_width(&c) != 8) return fail("pic_bin_width");
  c.patch[0] = 5;
  if (pic_validate_config(&c, msg, sizeof msg) != PIC_ERR_ARG || !strstr(msg, "below 6"))
    return fail("a patch of 5 cells must be rejected");
  return 0;
}

#define CHECK(call)                                  \
  do {                                               \
    if ((call) != hipSuccess) return fail(#call);    \
  } while (0)

static int gpu_run(int resident) {
  pic_config c = config();
  if (resident) c.flags |= PIC_FLAG_RESIDENT;
  /* resident calls need the slab layout's room: n + n/8 + 80 per patch */
  const int64_t cap = resident ? NP + NP / 8 + 80 * (int64_t)pic_num_patches(&c) + 64 : NP;
  const size_t cells = (size_t)NX * NY;
  const double q = -1.0, w = 1.0 / PPC, u[3] = {0.3, -0.2, 0.1};
  double *hx = malloc(2 * NP * sizeof(double)), *hw = malloc(NP * sizeof(double));
  int64_t *hid = malloc(NP * sizeof(int64_t));
  /* four particles per cell at fixed offsets inside it */
  for (int p = 0; p < NP; p++) {
    const int cell = p / PPC, k = p % PPC;
    hx[p] = ((cell % NX) + 0.2 + 0.2 * k) * c.d[0];
    hx[NP + p] = ((cell / NX) + 0.7 - 0.15 * k) * c.d[1];
    hw[p] = w;
    hid[p] = p;
  }
  pic_species s;
  memset(&s, 0, sizeof s);
  s.q = q;
  s.m = 1.0;
  s.n = NP;
  s.capacity = cap;
  double *fld;
  CHECK(hipMalloc((void **)&fld, 9 * cells * sizeof(double)));
  CHECK(hipMemset(fld, 0, 9 * cells * sizeof(double)));
  for (int a = 0; a < 2; a++) {
    CHECK(hipMalloc((void **)&s.x[a], cap * sizeof(double)));
    CHECK(hipMalloc((void **)&s.x_alt[a], cap * sizeof(double)));
    CHECK(hipMemcpy(s.x[a], hx + a * NP, NP * sizeof(double), hipMemcpyHostToDevice));
  }
  double *hu = malloc(NP * sizeof(double));
  for (int a = 0; a < 3; a++) {
    for (int p = 0; p < NP; p++) hu[p] = u[a];
    CHECK(hipMalloc((void **)&s.u[a], cap * sizeof(double)));
    CHECK(hipMalloc((void **)&s.u_alt[a], cap * sizeof(double)));
    CHECK(hipMemcpy(s.u[a], hu, NP * sizeof(double), hipMemcpyHostToDevice));
  }
  CHECK(hipMalloc((void **)&s.w, cap * sizeof(double)));
  CHECK(hipMalloc((void **)&s.w_alt, cap * sizeof(double)));
  CHECK(hipMalloc((void **)&s.id, cap * sizeof(int64_t)));
  CHECK(hipMalloc((void **)&s.id_alt, cap * sizeof(int64_t)));
  CHECK(hipMalloc((void **)&s.offset, (pic_num_patches(&c) + 1) * sizeof(int64_t)));
  CHECK(hipMemcpy(s.w, hw, NP * sizeof(double), hipMemcpyHostToDevice));
  CHECK(hipMemcpy(s.id, hid, NP * sizeof(int64_t), hipMemcpyHostToDevice));
  pic_fields f;
  for (int k = 0; k < 3; k++) {
    f.e[k] = fld + k * cells;
    f.b[k] = fld + (3 + k) * cells;
    f.j[k] = fld + (6 + k) * cells;
  }
  pic_ctx *ctx = NULL;
  if (pic_init(&c, 0, &ctx) != PIC_OK) return fail("pic_init");
  if (pic_bin(ctx, &s, 1, NULL) != PIC_OK) return fail(pic_last_error(ctx));
  if (resident) {
    for (int k = 0; k < STEPS; k++)
      if (pic_step(ctx, &s, 1, &f, 1, NULL) != PIC_OK) return fail(pic_last_error(ctx));
    if (pic_sync(ctx, NULL) != PIC_OK) return fail(pic_last_error(ctx));
  } else if (pic_step(ctx, &s, 1, &f, STEPS, NULL) != PIC_OK) {
    return fail(pic_last_error(ctx));
  }
  if (pic_check(ctx, NULL) != PIC_OK) return fail(pic_last_error(ctx));
  /* closed forms: without fields every particle moves at v = u / gamma */
  const double gam = sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
  const double L[2] = {NX * c.d[0], NY * c.d[1]};
  double *hj = malloc(3 * cells * sizeof(double));
  CHECK(hipMemcpy(hj, fld + 6 * cells, 3 * cells * sizeof(double), hipMemcpyDeviceToHost));
  for (int a = 0; a < 3; a++) {
    double sum = 0.0;
    for (size_t i = 0; i < cells; i++) sum += hj[a * cells + i];
    const double want = NP * q * w * u[a] / gam; /* total current of the last step */
    if (fabs(sum - want) > 1e-11 * fabs(want)) return fail("total current");
  }
  for (int a = 0; a < 2; a++)
    CHECK(hipMemcpy(hx + a * NP, s.x[a], NP * sizeof(double), hipMemcpyDeviceToHost));
  CHECK(hipMemcpy(hid, s.id, NP * sizeof(int64_t), hipMemcpyDeviceToHost));
  for (int p = 0; p < NP; p++) {
    const int64_t i = hid[p];
    const int cell = (int)(i / PPC), k = (int)(i % PPC);
    const double x0[2] = {((cell % NX) + 0.2 + 0.2 * k) * c.d[0],
                          ((cell / NX) + 0.7 - 0.15 * k) * c.d[1]};
    for (int a = 0; a < 2; a++) {
      double want = fmod(x0[a] + STEPS * c.dt * u[a] / gam, L[a]);
      if (want < 0) want += L[a];
      double err = fabs(hx[a * NP + p] - want);
      if (err > L[a] / 2) err = L[a] - err; /* across the periodic seam */
      if (err > 1e-12 * L[a]) return fail("position");
    }
  }
  pic_free(ctx);
  for (int a = 0; a < 2; a++) {
    CHECK(hipFree(s.x[a]));
    CHECK(hipFree(s.x_alt[a]));
  }
  for (int a = 0; a < 3; a++) {
    CHECK(hipFree(s.u[a]));
    CHECK(hipFree(s.u_alt[a]));
  }
  CHECK(hipFree(s.w));
  CHECK(hipFree(s.w_alt));
  CHECK(hipFree(s.id));
  CHECK(hipFree(s.id_alt));
  CHECK(hipFree(s.offset));
  CHECK(hipFree(fld));
  free(hx);
  free(hw);
  free(hid);
  free(hu);
  free(hj);
  return 0;
}

int main(int argc, char **argv) {
  int rc = host_checks();
  if (rc) return rc;
  if (argc > 1 && strcmp(argv[1], "gpu") == 0) {
    if ((rc = gpu_run(0)) != 0 || (rc = gpu_run(1)) != 0) return rc;
    printf("ok: %d particles, %d steps, one call and resident one-step calls\n", NP, STEPS);
    return 0;
  }
  printf("ok: host checks\n");
  return 0;
}
