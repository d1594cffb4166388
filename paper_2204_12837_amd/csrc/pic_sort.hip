// General sort of particles by patch, for input in any order (e.g. freshly
// loaded particles): periodic wrap (a position outside the box on an axis
// with reflecting walls is an error; one outside an axis with removing walls
// is deleted: its key sorts past the last patch, so the patch offsets end
// before it), patch key, stable radix sort of
// (key, index) pairs, gather into the second buffer set, patch offsets.
// The per-step sort after a push uses the neighbour-code counting sort in
// pic_kernels.hip instead; both give the same stable order.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "pic_common.h"

namespace pic {

namespace {

__global__ void k_keys(GridDev g, SpDev s, int32_t *keys, int64_t *idx, int *err) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    idx[i] = i;
    if (g.remove) {  // outside a removing wall: deleted (sorts past the last patch)
      double x[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < g.dim; a++) x[a] = s.x[a][i];
      const bool out = g.dim == 2 ? outside_removing<2>(g, x) : outside_removing<3>(g, x);
      if (out) {
        keys[i] = g.npatch;
        continue;
      }
    }
    int key = 0, mul = 1;
    for (int a = 0; a < g.dim; a++) {
      double v = s.x[a][i];
      if (!(((g.reflect | g.remove) >> a) & 1)) {  // a walled axis is not wrapped
        if (v < 0.0) v += g.L[a];
        if (v >= g.L[a]) v -= g.L[a];
      }
      if (!(v >= 0.0 && v < g.L[a])) {
        bad |= kErrPos;
        v = 0.0;
      }
      s.x[a][i] = v;
      int c = (int)floor(v * g.inv_d[a]);
      if (c >= g.n[a]) c = g.n[a] - 1;
      key += (c / g.patch[a]) * mul;
      mul *= g.np[a];
    }
    keys[i] = key;
  }
  if (bad) atomicOr(err, bad);
}

__global__ void k_gather(SpDev s, const int64_t *idx, int dim) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = idx[i];
    for (int a = 0; a < dim; a++) s.xa[a][i] = s.x[a][k];
    s.ua[0][i] = s.u[0][k];
    s.ua[1][i] = s.u[1][k];
    s.ua[2][i] = s.u[2][k];
    s.wa[i] = s.w[k];
    s.ida[i] = s.id[k];
  }
}

__global__ void k_offsets_sorted(GridDev g, SpDev s, const int32_t *keys) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= s.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int prev = i == 0 ? -1 : keys[i - 1];
    const int cur = i == s.n ? g.npatch : keys[i];
    for (int P = prev + 1; P <= cur; P++) s.off[P] = i;
  }
}

template <typename T>
hipError_t grow(T *&p, int64_t n) {
  if (p) {
    hipError_t e = hipFree(p);
    if (e != hipSuccess) return e;
    p = nullptr;
  }
  return hipMalloc(&p, (size_t)(n > 0 ? n : 1) * sizeof(T));
}

}  // namespace

void free_sort_scratch(SortScratch &scr) {
  (void)hipFree(scr.temp);
  (void)hipFree(scr.keys);
  (void)hipFree(scr.keys_out);
  (void)hipFree(scr.idx);
  (void)hipFree(scr.idx_out);
  scr = SortScratch{};
}

hipError_t general_sort(const GridDev &g, SpDev &s, SortScratch &scr, int *err, hipStream_t st) {
  hipError_t e;
  if (s.n > scr.cap) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if ((e = grow(scr.keys, s.n)) != hipSuccess) return e;
    if ((e = grow(scr.keys_out, s.n)) != hipSuccess) return e;
    if ((e = grow(scr.idx, s.n)) != hipSuccess) return e;
    if ((e = grow(scr.idx_out, s.n)) != hipSuccess) return e;
    scr.cap = s.n;
  }
  // keys lie in [0, npatch), and at npatch for particles deleted at a
  // removing wall
  const long long nkeys = (long long)g.npatch + (g.remove ? 1 : 0);
  int bits = 1;
  while ((1ll << bits) < nkeys) bits++;
  size_t need = 0;
  e = hipcub::DeviceRadixSort::SortPairs(nullptr, need, scr.keys, scr.keys_out, scr.idx,
                                         scr.idx_out, (int)s.n, 0, bits, st);
  if (e != hipSuccess) return e;
  if (need > scr.temp_bytes) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if (scr.temp) (void)hipFree(scr.temp);
    scr.temp = nullptr;
    if ((e = hipMalloc(&scr.temp, need)) != hipSuccess) return e;
    scr.temp_bytes = need;
  }
  const int blocks = (int)std::min<int64_t>((s.n + 255) / 256 + 1, 8192);
  hipLaunchKernelGGL(k_keys, dim3(blocks), dim3(256), 0, st, g, s, scr.keys, scr.idx, err);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  size_t tb = scr.temp_bytes;
  e = hipcub::DeviceRadixSort::SortPairs(scr.temp, tb, scr.keys, scr.keys_out, scr.idx,
                                         scr.idx_out, (int)s.n, 0, bits, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(256), 0, st, s, scr.idx_out, g.dim);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_offsets_sorted, dim3(blocks), dim3(256), 0, st, g, s, scr.keys_out);
  return hipGetLastError();
}

}  // namespace pic
