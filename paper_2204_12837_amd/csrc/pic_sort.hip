// Sorts of the synchronisation phase that the neighbour-code counting sort
// of pic_kernels.hip does not cover (paper, section "Parallelization
// without tasks": after the operators the particle boundary conditions are
// applied and the particles sorted by patch).
//
// General sort, for particles in any order (e.g. freshly loaded): periodic
// wrap (a position outside the box on an axis with reflecting walls is an
// error; one outside an axis with removing walls is deleted: its key sorts
// past the last patch, so the patch offsets end before it), patch key, then
// a stable least-significant-digit radix sort of (key, index) pairs with
// 8-bit digits, then a gather of the particles into the second buffer set and
// the patch offsets.  Each radix pass is a counting sort written out by hand:
// per-tile digit histograms, a scan over the tiles of each digit, and a
// scatter whose ranks inside a tile come from wave ballots (the lanes holding
// the same digit are found with eight ballots, one per digit bit).
//
// Bin order, for particles already sorted by patch whose patches are cut
// into x-bins (paper, section "Parallelization with OpenMP task": bins of
// bin_x_size cells inside a patch): a stable counting sort into the nb bins
// of each patch.  Each patch's range is cut into units of 4096 particles
// (one workgroup each): bin counts per unit, running sums over a patch's
// units, a scan into the bin offsets, then every particle copied to its
// bin's next slot in order (ranks from the same ballot match).  It moves
// each particle once, as one copy does.
#include <hip/hip_runtime.h>

#include "pic_common.h"
#include "pic_device.h"

namespace pic {

namespace {

constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 16;  // elements per thread and tile
constexpr int kRadixTile = kRadixThreads * kRadixItems;

__device__ __forceinline__ uint64_t lanes_below(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Lanes of the wave whose `valid` flag is set and whose value v agrees with
// this lane's in its low NBITS bits (this lane included when valid).
template <int NBITS>
__device__ __forceinline__ uint64_t match_peers(bool valid, uint32_t v) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < NBITS; b++) {
    const bool bit = (v >> b) & 1u;
    const uint64_t m = __ballot(valid && bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

__global__ void k_keys(GridDev g, SpDev s, uint32_t *keys, int *err) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (g.remove) {  // outside a removing wall: deleted (sorts past the last patch)
      double x[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < g.dim; a++) x[a] = s.x[a][i];
      const bool out = g.dim == 2 ? outside_removing<2>(g, x) : outside_removing<3>(g, x);
      if (out) {
        keys[i] = (uint32_t)g.npatch;
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
    keys[i] = (uint32_t)key;
  }
  if (bad) atomicOr(err, bad);
}

// Radix pass, step 1: digit histogram of each tile of kRadixTile keys;
// hist[digit * ntile + tile].
__global__ void __launch_bounds__(kRadixThreads) k_radix_hist(const uint32_t *keys, int64_t n,
                                                              int shift, uint32_t *hist,
                                                              int ntile) {
  __shared__ uint32_t h[kRadixBins];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kRadixTile;
  const int64_t t1 = t0 + kRadixTile < n ? t0 + kRadixTile : n;
  for (int64_t i = t0 + threadIdx.x; i < t1; i += kRadixThreads)
    atomicAdd(&h[(keys[i] >> shift) & (kRadixBins - 1)], 1u);
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntile + blockIdx.x] = h[threadIdx.x];
}

// Radix pass, step 2: for each digit (one workgroup each), the exclusive
// scan of its tiles' counts in place, and the digit's total in dtot.
__global__ void __launch_bounds__(kRadixThreads) k_radix_scan(uint32_t *hist, int ntile,
                                                              uint32_t *dtot) {
  constexpr int kWaves = kRadixThreads / 64;
  constexpr int kPer = 4;  // consecutive entries per thread and chunk
  __shared__ uint32_t ws[kWaves];
  uint32_t *h = hist + (int64_t)blockIdx.x * ntile;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (int c0 = 0; c0 < ntile; c0 += kRadixThreads * kPer) {
    const int b = c0 + (int)threadIdx.x * kPer;
    uint32_t v[kPer], sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; k++) {
      v[k] = b + k < ntile ? h[b + k] : 0u;
      sum += v[k];
    }
    uint32_t x = sum;  // inclusive scan of the threads' sums inside the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) ws[wv] = x;
    __syncthreads();
    uint32_t run = carry + x - sum, all = 0;
    for (int w = 0; w < kWaves; w++) {
      if (w < wv) run += ws[w];
      all += ws[w];
    }
#pragma unroll
    for (int k = 0; k < kPer; k++) {
      if (b + k < ntile) h[b + k] = run;
      run += v[k];
    }
    carry += all;
    __syncthreads();  // ws is read before the next chunk writes it
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

// Radix pass, step 3: stable scatter of each tile.  The tile is taken in
// chunks of kRadixThreads keys in order; inside a chunk an element's rank
// is the number of earlier elements with its digit (earlier lanes of its
// wave, then every lane of the earlier waves); run[] carries each digit's
// count over the earlier chunks.  idx_in = nullptr: the indices are the
// positions (first pass).
__global__ void __launch_bounds__(kRadixThreads) k_radix_scatter(
    const uint32_t *keys_in, const uint32_t *idx_in, uint32_t *keys_out, uint32_t *idx_out,
    int64_t n, int shift, const uint32_t *hist, const uint32_t *dtot, int ntile) {
  constexpr int kWaves = kRadixThreads / 64;
  __shared__ uint32_t run[kRadixBins];
  __shared__ uint32_t wc[kWaves][kRadixBins];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  {
    // this tile's first slot of each digit: the earlier digits' totals (an
    // exclusive scan over the 256 digits) plus the earlier tiles' counts
    const uint32_t t = dtot[threadIdx.x];
    uint32_t x = t;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wc[0][wv] = x;
    __syncthreads();
    uint32_t base = x - t;
    for (int w = 0; w < wv; w++) base += wc[0][w];
    run[threadIdx.x] = base + hist[(int64_t)threadIdx.x * ntile + blockIdx.x];
    __syncthreads();  // wc is cleared by the first chunk below
  }
  const int64_t t0 = (int64_t)blockIdx.x * kRadixTile;
  const int64_t t1 = t0 + kRadixTile < n ? t0 + kRadixTile : n;
  for (int64_t base = t0; base < t1; base += kRadixThreads) {
#pragma unroll
    for (int w = 0; w < kWaves; w++) wc[w][threadIdx.x] = 0u;
    __syncthreads();
    const int64_t i = base + threadIdx.x;
    const bool valid = i < t1;
    const uint32_t key = valid ? keys_in[i] : 0u;
    const uint32_t d = (key >> shift) & (kRadixBins - 1);
    const uint64_t peers = match_peers<kRadixBits>(valid, d);
    const uint32_t r = (uint32_t)__popcll(peers & lanes_below(lane));
    if (valid && r == 0) wc[wv][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t dst = run[d] + r;
      for (int w = 0; w < wv; w++) dst += wc[w][d];
      keys_out[dst] = key;
      idx_out[dst] = idx_in ? idx_in[i] : (uint32_t)i;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) add += wc[w][threadIdx.x];
    run[threadIdx.x] += add;
  }
}

__global__ void k_gather(SpDev s, const uint32_t *idx, int dim) {
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

__global__ void k_offsets_sorted(GridDev g, SpDev s, const uint32_t *keys) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= s.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int prev = i == 0 ? -1 : (int)keys[i - 1];
    const int cur = i == s.n ? g.npatch : (int)keys[i];
    for (int P = prev + 1; P <= cur; P++) s.off[P] = i;
  }
}

// Bin of the particle at x inside API patch P (coordinates pc), for bins of
// g.patch[0] cells: its cell's bin along x minus the patch's first bin; -1
// if the particle lies outside the patch.
template <int DIM>
__device__ __forceinline__ int bin_in_patch(const GridDev &g, int nb, const int pc[3],
                                            const double x[3]) {
  int b = 0;
#pragma unroll
  for (int a = 0; a < DIM; a++) {
    int c = (int)floor(x[a] * g.inv_d[a]);
    if (c >= g.n[a]) c = g.n[a] - 1;
    const int w = a == 0 ? g.patch[0] * nb : g.patch[a];  // API patch width
    const int lo = pc[a] * w;
    if (c < lo || c >= lo + w) return -1;
    if (a == 0) b = (c - lo) / g.patch[0];
  }
  return b;
}

__device__ __forceinline__ void api_patch_coords(const GridDev &g, int nb, int P, int pc[3]) {
  const int npx = g.np[0] / nb;
  pc[0] = P % npx;
  const int r = P / npx;
  pc[1] = r % g.np[1];
  pc[2] = r / g.np[1];
}

constexpr int kBinThreads = 256;
constexpr int kMaxBinsPerPatch = 256;  // bins of one patch the ballot match can tell apart
constexpr int kBinUnit = 4096;         // particles per work unit of the bin order

// Bin order, step 0: each API patch's particle range is cut into units of
// kBinUnit particles; ustart[P] = first unit of patch P (scan of the unit
// counts; in and tmp are scan scratch).
__global__ void __launch_bounds__(1024) k_bin_units(const int64_t *off, int npatch, int64_t *in,
                                                    int64_t *tmp, int32_t *ustart) {
  __shared__ int64_t part[1024];
  for (int P = threadIdx.x; P < npatch; P += blockDim.x)
    in[P] = (off[P + 1] - off[P] + kBinUnit - 1) / kBinUnit;
  __syncthreads();
  block_scan_1024(in, tmp, npatch, part);
  for (int P = threadIdx.x; P <= npatch; P += blockDim.x) ustart[P] = (int32_t)tmp[P];
}

// The API patch of unit u (largest P with ustart[P] <= u) and the unit's
// particle range; false past the last unit.
__device__ __forceinline__ bool unit_range(const int32_t *ustart, int npatch, const int64_t *off,
                                           int u, int &P, int64_t &b, int64_t &e) {
  if (u >= ustart[npatch]) return false;
  int lo = 0, hi = npatch;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ustart[mid] <= u)
      lo = mid;
    else
      hi = mid;
  }
  P = lo;
  b = off[P] + (int64_t)(u - ustart[P]) * kBinUnit;
  e = b + kBinUnit < off[P + 1] ? b + kBinUnit : off[P + 1];
  return true;
}

// Bin order, step 1: particles per bin of each unit into uh[u * nb + b];
// a particle outside its patch is reported (and counted in bin 0).
template <int DIM>
__global__ void __launch_bounds__(kBinThreads) k_bin_hist(GridDev g, SpDev s, const int64_t *off,
                                                          int npatch, int nb,
                                                          const int32_t *ustart, int32_t *uh,
                                                          int *err) {
  __shared__ int h[kMaxBinsPerPatch];
  int P;
  int64_t b0, b1;
  if (!unit_range(ustart, npatch, off, blockIdx.x, P, b0, b1)) return;
  for (int b = threadIdx.x; b < nb; b += kBinThreads) h[b] = 0;
  __syncthreads();
  int pc[3];
  api_patch_coords(g, nb, P, pc);
  int bad = 0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kBinThreads) {
    double x[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < DIM; a++) x[a] = s.x[a][i];
    int b = bin_in_patch<DIM>(g, nb, pc, x);
    if (b < 0) {
      bad |= kErrUnsorted;
      b = 0;
    }
    atomicAdd(&h[b], 1);
  }
  if (bad) atomicOr(err, bad);
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += kBinThreads) uh[(int64_t)blockIdx.x * nb + b] = h[b];
}

// Bin order, step 2: per (API patch, bin), the running count over the
// patch's units (upre) and the bin's total (cnt[P * nb + b]).
__global__ void k_bin_prefix(int npatch, int nb, const int32_t *ustart, const int32_t *uh,
                             int32_t *upre, int64_t *cnt) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)npatch * nb) return;
  const int P = (int)(id / nb), b = (int)(id - (int64_t)P * nb);
  int32_t run = 0;
  for (int u = ustart[P]; u < ustart[P + 1]; u++) {
    upre[(int64_t)u * nb + b] = run;
    run += uh[(int64_t)u * nb + b];
  }
  cnt[id] = run;
}

// Bin order, step 3: bin offsets (exclusive scan of the bin counts).
__global__ void __launch_bounds__(1024) k_bin_scan(GridDev g, const int64_t *cnt, int64_t *boff) {
  __shared__ int64_t part[1024];
  block_scan_1024(cnt, boff, g.npatch, part);
}

// Bin order, step 4: each particle of a unit to the next slot of its bin in
// the second buffer set, in order (stable): the bin's offset, the bin's
// count in the patch's earlier units, the earlier chunks of this unit, the
// earlier waves of the chunk and the earlier lanes of the wave.
// dst[bin] is the first slot of each bin: the bin offsets (dense layout) or
// the slab starts of pic_step's slab layout, whose plan is then checked
// first (ctl[1] == 2: the slabs do not fit and nothing is written).
template <int DIM>
__global__ void __launch_bounds__(kBinThreads) k_bin_place(GridDev g, SpDev s, const int64_t *off,
                                                           int npatch, int nb,
                                                           const int32_t *ustart,
                                                           const int32_t *upre,
                                                           const int64_t *dst0,
                                                           const int32_t *ctl) {
  constexpr int kWaves = kBinThreads / 64;
  __shared__ int64_t run[kMaxBinsPerPatch];
  __shared__ int wc[kWaves][kMaxBinsPerPatch];
  if (ctl && ctl[1] == 2) return;
  int P;
  int64_t beg, end;
  if (!unit_range(ustart, npatch, off, blockIdx.x, P, beg, end)) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int b = threadIdx.x; b < nb; b += kBinThreads)
    run[b] = dst0[(int64_t)P * nb + b] + upre[(int64_t)blockIdx.x * nb + b];
  int pc[3];
  api_patch_coords(g, nb, P, pc);
  for (int64_t base = beg; base < end; base += kBinThreads) {
    for (int b = threadIdx.x; b < nb; b += kBinThreads)
#pragma unroll
      for (int w = 0; w < kWaves; w++) wc[w][b] = 0;
    __syncthreads();
    const int64_t i = base + threadIdx.x;
    const bool valid = i < end;
    double x[3] = {0.0, 0.0, 0.0};
    int b = 0;
    if (valid) {
#pragma unroll
      for (int a = 0; a < DIM; a++) x[a] = s.x[a][i];
      b = bin_in_patch<DIM>(g, nb, pc, x);
      if (b < 0) b = 0;  // reported by k_bin_hist
    }
    const uint64_t peers = match_peers<8>(valid, (uint32_t)b);
    const int r = __popcll(peers & lanes_below(lane));
    if (valid && r == 0) wc[wv][b] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int64_t dst = run[b] + r;
      for (int w = 0; w < wv; w++) dst += wc[w][b];
#pragma unroll
      for (int a = 0; a < DIM; a++) s.xa[a][dst] = x[a];
      s.ua[0][dst] = s.u[0][i];
      s.ua[1][dst] = s.u[1][i];
      s.ua[2][dst] = s.u[2][i];
      s.wa[dst] = s.w[i];
      s.ida[dst] = s.id[i];
    }
    __syncthreads();
    for (int bb = threadIdx.x; bb < nb; bb += kBinThreads) {
      int add = 0;
#pragma unroll
      for (int w = 0; w < kWaves; w++) add += wc[w][bb];
      run[bb] += add;
    }
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
  (void)hipFree(scr.keys);
  (void)hipFree(scr.keys_out);
  (void)hipFree(scr.idx);
  (void)hipFree(scr.idx_out);
  (void)hipFree(scr.hist);
  scr = SortScratch{};
}

hipError_t general_sort(const GridDev &g, SpDev &s, SortScratch &scr, int *err, hipStream_t st) {
  hipError_t e;
  const int64_t n = s.n;
  const int ntile = (int)((n + kRadixTile - 1) / kRadixTile);
  if (n > scr.cap) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if ((e = grow(scr.keys, n)) != hipSuccess) return e;
    if ((e = grow(scr.keys_out, n)) != hipSuccess) return e;
    if ((e = grow(scr.idx, n)) != hipSuccess) return e;
    if ((e = grow(scr.idx_out, n)) != hipSuccess) return e;
    if ((e = grow(scr.hist, (int64_t)kRadixBins * ((n + kRadixTile - 1) / kRadixTile) +
                                kRadixBins)) != hipSuccess)
      return e;
    scr.cap = n;
  }
  const int blocks = (int)std::min<int64_t>((n + 255) / 256 + 1, 8192);
  if (n > 0) {
    hipLaunchKernelGGL(k_keys, dim3(blocks), dim3(256), 0, st, g, s, scr.keys, err);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // keys lie in [0, npatch), and at npatch for particles deleted at a
  // removing wall; digits of 8 bits from the least significant up
  const int64_t nkeys = (int64_t)g.npatch + (g.remove ? 1 : 0);
  int bits = 0;
  while (((int64_t)1 << bits) < nkeys) bits++;
  uint32_t *kin = scr.keys, *kout = scr.keys_out, *iin = nullptr, *iout = scr.idx;
  if (n > 0)
    for (int shift = 0; shift < bits || shift == 0; shift += kRadixBits) {
      hipLaunchKernelGGL(k_radix_hist, dim3(ntile), dim3(kRadixThreads), 0, st, kin, n, shift,
                         scr.hist, ntile);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      uint32_t *dtot = scr.hist + (int64_t)kRadixBins * ntile;  // per-digit totals
      hipLaunchKernelGGL(k_radix_scan, dim3(kRadixBins), dim3(kRadixThreads), 0, st, scr.hist,
                         ntile, dtot);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_radix_scatter, dim3(ntile), dim3(kRadixThreads), 0, st, kin, iin, kout,
                         iout, n, shift, scr.hist, dtot, ntile);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      std::swap(kin, kout);
      iin = iout;
      iout = iout == scr.idx ? scr.idx_out : scr.idx;
    }
  // the sorted keys and indices are in kin and iin
  if (n > 0) {
    hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(256), 0, st, s, iin, g.dim);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_offsets_sorted, dim3(blocks), dim3(256), 0, st, g, s, kin);
  return hipGetLastError();
}

bool bin_order_supported(int nb) { return nb >= 1 && nb <= kMaxBinsPerPatch; }

hipError_t bin_count(const GridDev &g, SpDev &s, const int64_t *off_api, int64_t npatch_api, int nb,
                     int64_t n, int *err, hipStream_t st) {
  if (npatch_api < 1) return hipSuccess;
  const int np = (int)npatch_api;
  // scratch: unit starts in sstart, the units' bin counts and their running
  // sums in cnt (units * nb each), bin counts in tmp, scan scratch in and noff
  const int64_t umax = npatch_api + n / kBinUnit + 1;
  int32_t *ustart = s.sstart, *uh = s.cnt, *upre = s.cnt + umax * nb;
  hipLaunchKernelGGL(k_bin_units, dim3(1), dim3(1024), 0, st, off_api, np, s.in, s.noff, ustart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)umax);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_bin_hist<2>, grid, dim3(kBinThreads), 0, st, g, s, off_api, np, nb,
                       ustart, uh, err);
  else
    hipLaunchKernelGGL(k_bin_hist<3>, grid, dim3(kBinThreads), 0, st, g, s, off_api, np, nb,
                       ustart, uh, err);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t pb = npatch_api * nb;
  hipLaunchKernelGGL(k_bin_prefix, dim3((unsigned)((pb + 255) / 256)), dim3(256), 0, st, np, nb,
                     ustart, uh, upre, s.tmp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, st, g, s.tmp, s.off);
  return hipGetLastError();
}

hipError_t bin_place(const GridDev &g, SpDev &s, const int64_t *off_api, int64_t npatch_api, int nb,
                     int64_t n, const int64_t *dst0, const int32_t *ctl, hipStream_t st) {
  if (npatch_api < 1) return hipSuccess;
  const int np = (int)npatch_api;
  const int64_t umax = npatch_api + n / kBinUnit + 1;
  const int32_t *ustart = s.sstart, *upre = s.cnt + umax * nb;
  const dim3 grid((unsigned)umax);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_bin_place<2>, grid, dim3(kBinThreads), 0, st, g, s, off_api, np, nb,
                       ustart, upre, dst0, ctl);
  else
    hipLaunchKernelGGL(k_bin_place<3>, grid, dim3(kBinThreads), 0, st, g, s, off_api, np, nb,
                       ustart, upre, dst0, ctl);
  return hipGetLastError();
}

hipError_t bin_order(const GridDev &g, SpDev &s, const int64_t *off_api, int64_t npatch_api, int nb,
                     int64_t n, int *err, hipStream_t st) {
  hipError_t e = bin_count(g, s, off_api, npatch_api, nb, n, err, st);
  if (e != hipSuccess) return e;
  return bin_place(g, s, off_api, npatch_api, nb, n, s.off, nullptr, st);
}

}  // namespace pic
