// Slab layout of the particles inside a pic_step call (gfx950).
//
// Between calls the particles of a species are dense and sorted by patch (the
// layout the C ABI documents).  Inside a call of several steps they live in
// the species' second buffer set in per-patch slabs: patch P owns slots
// [sb[P], sb[P] + cap[P]), of which the first cnt[P] hold its particles and
// the rest is room for arrivals.  A step then
//   * updates every particle in place (Interpolation, Push, pre-BC,
//     Projection: the fused kernel reads and writes each particle once and
//     records its neighbour code in one byte);
//   * moves only the particles that changed patch (the paper's exchange of
//     particles between patches in the synchronisation phase): departures
//     are copied to an outbox and their slots refilled from the slab's tail,
//     then arrivals are appended to their destination slab.
// After this the particles of each patch are again contiguous, as after the
// paper's per-patch sort; their order inside a patch is arbitrary.  A slab
// that runs out of room triggers, on the device, a new slab plan and a copy
// through the first buffer set.  The last step of a call copies the slabs
// back into the dense sorted layout.
#include <hip/hip_runtime.h>

#include "pic_common.h"
#include "pic_device.h"

namespace pic {

namespace {

constexpr int32_t kUnplaced = 1 << 30;  // outbox entry waiting for a new slab plan

// Room of a slab holding c particles: c + c/8 + 64, rounded up to 16 slots
// (128 bytes), so every slab starts on a cache-line boundary.
__device__ __forceinline__ int64_t slab_room(int64_t c) {
  return (c + (c >> 3) + 64 + 15) & ~(int64_t)15;
}

template <int DIM>
__device__ __forceinline__ void copy_particle(double *const dx[3], double *const du[3], double *dw,
                                              int64_t *did, int64_t d, const double *const sx[3],
                                              const double *const su[3], const double *sw,
                                              const int64_t *sid, int64_t s) {
#pragma unroll
  for (int a = 0; a < DIM; a++) dx[a][d] = sx[a][s];
  du[0][d] = su[0][s];
  du[1][d] = su[1][s];
  du[2][d] = su[2][s];
  dw[d] = sw[s];
  did[d] = sid[s];
}

// Copies particles src + j -> dst + j for j in [0, c), four per thread at a
// time (all loads of a batch before its stores).
template <int DIM>
__device__ __forceinline__ void copy_run(double *const dx[3], double *const du[3], double *dw,
                                         int64_t *did, int64_t d0, const double *const sx[3],
                                         const double *const su[3], const double *sw,
                                         const int64_t *sid, int64_t s0, int64_t c) {
  constexpr int kB = 4;
  const int64_t nt = blockDim.x;
  for (int64_t j0 = threadIdx.x; j0 < c; j0 += kB * nt) {
    double x[kB][DIM], u[kB][3], w[kB];
    int64_t id[kB];
#pragma unroll
    for (int b = 0; b < kB; b++) {
      const int64_t j = j0 + b * nt;
      if (j < c) {
#pragma unroll
        for (int a = 0; a < DIM; a++) x[b][a] = sx[a][s0 + j];
        u[b][0] = su[0][s0 + j];
        u[b][1] = su[1][s0 + j];
        u[b][2] = su[2][s0 + j];
        w[b] = sw[s0 + j];
        id[b] = sid[s0 + j];
      }
    }
#pragma unroll
    for (int b = 0; b < kB; b++) {
      const int64_t j = j0 + b * nt;
      if (j < c) {
#pragma unroll
        for (int a = 0; a < DIM; a++) dx[a][d0 + j] = x[b][a];
        du[0][d0 + j] = u[b][0];
        du[1][d0 + j] = u[b][1];
        du[2][d0 + j] = u[b][2];
        dw[d0 + j] = w[b];
        did[d0 + j] = id[b];
      }
    }
  }
}

// Slab plan from the dense offsets (one workgroup of 1024 per species).
__global__ void __launch_bounds__(1024) k_slab_plan(GridDev g, SlabArgs sa, int *err) {
  __shared__ int64_t part[1024];
  const SlabDev &S = sa.s[blockIdx.x];
  const int n = g.npatch;
  for (int P = threadIdx.x; P < n; P += blockDim.x) {
    const int64_t c = S.off[P + 1] - S.off[P];
    S.cnt[P] = (int32_t)c;
    S.cap[P] = (int32_t)slab_room(c);
    S.tmp[P] = slab_room(c);
    S.arr[P] = 0;
  }
  __syncthreads();
  block_scan_1024(S.tmp, S.sb, n, part);
  if (threadIdx.x == 0) {
    S.ctl[1] = 0;
    if (S.sb[n] > S.capacity) {
      S.ctl[1] = 2;  // does not fit: every later kernel of the call stands still
      atomicOr(err, kErrCap);
    }
  }
}

// Dense -> slabs (grid: patches x species).
template <int DIM>
__global__ void __launch_bounds__(256) k_slab_in(GridDev g, SlabArgs sa) {
  const SlabDev &S = sa.s[blockIdx.y];
  if (S.ctl[1] == 2) return;
  const int P = blockIdx.x;
  const int64_t b = S.off[P], c = S.off[P + 1] - b;
  copy_run<DIM>(S.xs, S.us, S.ws, S.ids, S.sb[P], S.x, S.u, S.w, S.id, b, c);
}

// Fused step on particles [r0, r1) of the slab of patch P, in place: each
// wave takes 64-particle blocks r0 + 64 (wv + j nw) and prefetches the next
// block's particles while it computes the current one; every global access
// of a full block is unconditional (a prefetch past the range reloads its
// last particle), so the memory-counter waits stay exact.  The neighbour code
// of each particle goes to code[].  from_dense (the first step of a call):
// particle j of the patch is read from the dense layout at off[P] + j and
// written, with its weight and id, to slot j of the slab, so the call needs
// no separate copy into the slabs.
template <int DIM, bool WALLS, bool FROM_DENSE>
__device__ __forceinline__ void ipp_slab(const GridDev &g, const SlabDev &S, const TileGeom &t,
                                         const double *tEB, double *tJ, int P, uint32_t r0,
                                         uint32_t r1, int &bad, uint32_t *bits) {
  constexpr bool from_dense = FROM_DENSE;
  constexpr int CENTER = DIM == 2 ? 4 : 13;
  const int nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const uint32_t sbP = (uint32_t)S.sb[P];
  const uint32_t srcP = from_dense ? (uint32_t)S.off[P] : sbP;
  const double q = S.q, alpha = S.alpha;
  uint32_t base = r0 + 64u * (uint32_t)wv;
  if (base >= r1) return;
  const uint32_t step = 64u * (uint32_t)nw;
  auto slot = [&](uint32_t b) -> uint32_t {
    const uint32_t i = b + (uint32_t)lane;
    return srcP + (i < r1 ? i : r1 - 1);
  };
  const double *sx[DIM], *su[3], *sw;
#pragma unroll
  for (int a = 0; a < DIM; a++) sx[a] = from_dense ? S.x[a] : S.xs[a];
#pragma unroll
  for (int a = 0; a < 3; a++) su[a] = from_dense ? S.u[a] : S.us[a];
  sw = from_dense ? S.w : S.ws;
  struct PartS {
    double x[DIM], u[3], w;
    int64_t id;
  };
  auto load = [&](uint32_t k, PartS &p) {
#pragma unroll
    for (int a = 0; a < DIM; a++) p.x[a] = at(sx[a], k);
    p.u[0] = at(su[0], k);
    p.u[1] = at(su[1], k);
    p.u[2] = at(su[2], k);
    p.w = at(sw, k);
    if constexpr (FROM_DENSE) p.id = at(S.id, k);
  };
  PartS pc, pn;
  load(slot(base), pc);
  while (base + 64 <= r1) {
    const uint32_t nb = base + step;
    load(slot(nb), pn);
    const uint32_t i = sbP + base + (uint32_t)lane;
    double x[3], u[3];
#pragma unroll
    for (int a = 0; a < DIM; a++) x[a] = pc.x[a];
    u[0] = pc.u[0];
    u[1] = pc.u[1];
    u[2] = pc.u[2];
    const int code = step_particle<DIM, WALLS>(g, t, tEB, tJ, q, alpha, pc.w, x, u, bad);
#pragma unroll
    for (int a = 0; a < DIM; a++) at(S.xs[a], i) = x[a];
    at(S.us[0], i) = u[0];
    at(S.us[1], i) = u[1];
    at(S.us[2], i) = u[2];
    at(S.code, i) = (uint8_t)code;
    if constexpr (FROM_DENSE) {
      at(S.ws, i) = pc.w;
      at(S.ids, i) = pc.id;
    }
    if (bits && __ballot(code != CENTER)) {  // mark departures (slab-relative slot)
      const uint32_t j = base + (uint32_t)lane;
      if (code != CENTER) atomicOr(&bits[j >> 5], 1u << (j & 31));
    }
    base = nb;
    pc = pn;
  }
  if (base < r1) {  // partial last block
    const uint32_t i = sbP + base + (uint32_t)lane;
    if (base + (uint32_t)lane < r1) {
      double x[3], u[3];
#pragma unroll
      for (int a = 0; a < DIM; a++) x[a] = pc.x[a];
      u[0] = pc.u[0];
      u[1] = pc.u[1];
      u[2] = pc.u[2];
      const int code = step_particle<DIM, WALLS>(g, t, tEB, tJ, q, alpha, pc.w, x, u, bad);
#pragma unroll
      for (int a = 0; a < DIM; a++) at(S.xs[a], i) = x[a];
      at(S.us[0], i) = u[0];
      at(S.us[1], i) = u[1];
      at(S.us[2], i) = u[2];
      at(S.code, i) = (uint8_t)code;
      if constexpr (FROM_DENSE) {
        at(S.ws, i) = pc.w;
        at(S.ids, i) = pc.id;
      }
      if (bits && code != CENTER) {
        const uint32_t j = base + (uint32_t)lane;
        atomicOr(&bits[j >> 5], 1u << (j & 31));
      }
    }
  }
}

constexpr int kBitSlots = 16384;           // largest patch whose departures the fused
constexpr int kBitWords = kBitSlots / 32;  // kernel handles itself
// the departures kernel's bitmap path: slabs of up to this many particles
// (2D: the 32768-particle bins of large patches; 3D: a small bitmap, so
// that more of the many small bins' workgroups fit in a CU's LDS)
template <int DIM>
constexpr int kExchBitSlots = DIM == 2 ? 65536 : 16384;
template <int DIM>
constexpr int kExchBitWords = kExchBitSlots<DIM> / 32;

// Exclusive prefix sum of v over the workgroup (any size up to 1024, a
// multiple of 64); total in tot.  wtot: 16 shared ints.
__device__ __forceinline__ int block_excl_sum(int v, int &tot, int *wtot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) wtot[wv] = x;
  __syncthreads();
  int base = 0, all = 0;
  for (int k = 0; k < nw; k++) {
    const int t = wtot[k];
    if (k < wv) base += t;
    all += t;
  }
  tot = all;
  return base + x - v;
}

// The slot of the n-th set bit of a bitmap whose words hold pre[i] set bits
// before word i (words 0 .. W-1).
__device__ __forceinline__ int nth_set(const uint32_t *bits, const int *pre, int W, int n) {
  int lo = 0, hi = W - 1;  // the last word with pre <= n holds it
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= n)
      lo = mid;
    else
      hi = mid - 1;
  }
  uint32_t b = bits[lo];
  for (int d = n - pre[lo]; d > 0; d--) b &= b - 1;
  return 32 * lo + __ffs(b) - 1;
}

// The slot of the n-th particle that stays among slots [c2, c) (bit clear),
// given the H departures below c2.
__device__ __forceinline__ int nth_tail_stayer(const uint32_t *bits, const int *pre, int W, int c2,
                                               int c, int H, int n) {
  // stayers of [c2, 32 w) for a word w past c2's: 32 w - c2 - (pre[w] - H)
  int lo = c2 >> 5, hi = W - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (32 * mid - c2 - (pre[mid] - H) <= n)
      lo = mid;
    else
      hi = mid - 1;
  }
  uint32_t b = ~bits[lo];
  int before = 0;
  if (lo == (c2 >> 5))
    b &= ~((1u << (c2 & 31)) - 1u);  // (c2 & 31 == 0 keeps the word)
  else
    before = 32 * lo - c2 - (pre[lo] - H);
  if (lo == W - 1 && (c & 31)) b &= (1u << (c & 31)) - 1u;
  for (int d = n - before; d > 0; d--) b &= b - 1;
  return 32 * lo + __ffs(b) - 1;
}

// Departures of patch P from its departure bitmap (`bits`: bit j set if
// slot j leaves; `pre` receives the departures before each word): the q-th
// departure (slot order) goes to entry q of the patch's outbox region with
// its destination patch, and the departures below c2 = c - departures are
// the holes that the stayers of the slab's tail [c2, c) fill, the q-th
// stayer taking the q-th hole.  Each thread takes departures q, q + threads,
// ...: it loads the departure and, for a hole, its stayer before any store
// (one memory round trip per departure; the hole's old contents are read
// by the thread that overwrites them).
template <int DIM>
__device__ void depart_in_kernel(const GridDev &g, const SlabDev &S, int P, int c,
                                 const uint32_t *bits, int *pre, int *wtot) {
  const int64_t sbP = S.sb[P];
  const int nt = blockDim.x;
  const int W = (c + 31) >> 5;
  const int per = (W + nt - 1) / nt;
  const int w0 = min(W, (int)threadIdx.x * per), w1 = min(W, w0 + per);
  int k = 0;
  for (int i = w0; i < w1; i++) k += __popc(bits[i]);
  int m = 0;
  int r = block_excl_sum(k, m, wtot);
  for (int i = w0; i < w1; i++) {
    pre[i] = r;
    r += __popc(bits[i]);
  }
  if (threadIdx.x == 0) S.dep[P] = m;
  if (m == 0) {
    if (threadIdx.x == 0) S.cnt2[P] = c;
    return;
  }
  __syncthreads();  // pre[] complete
  const int c2 = c - m;
  // departures below c2
  const int H = (c2 >> 5) < W ? pre[c2 >> 5] + __popc(bits[c2 >> 5] & ((1u << (c2 & 31)) - 1u)) : m;
  int pc[3];
  patch_coords(g, P, pc);
  for (int q = threadIdx.x; q < m; q += nt) {
    const int h = nth_set(bits, pre, W, q);
    const int j = q < H ? nth_tail_stayer(bits, pre, W, c2, c, H, q) : -1;
    const int64_t sh = sbP + h;
    double xh[DIM], uh[3], xj[DIM], uj[3], wj = 0.0;
    int64_t idj = 0;
#pragma unroll
    for (int a = 0; a < DIM; a++) xh[a] = S.xs[a][sh];
    uh[0] = S.us[0][sh];
    uh[1] = S.us[1][sh];
    uh[2] = S.us[2][sh];
    const double wh = S.ws[sh];
    const int64_t idh = S.ids[sh];
    const int cd = (int)S.code[sh];
    if (j >= 0) {
      const int64_t sj = sbP + j;
#pragma unroll
      for (int a = 0; a < DIM; a++) xj[a] = S.xs[a][sj];
      uj[0] = S.us[0][sj];
      uj[1] = S.us[1][sj];
      uj[2] = S.us[2][sj];
      wj = S.ws[sj];
      idj = S.ids[sj];
    }
    const int64_t o = sbP + q;
#pragma unroll
    for (int a = 0; a < DIM; a++) S.ox[a][o] = xh[a];
    S.ou[0][o] = uh[0];
    S.ou[1][o] = uh[1];
    S.ou[2][o] = uh[2];
    S.ow[o] = wh;
    S.oid[o] = idh;
    S.odest[o] = dest_patch(g, pc, cd);
    if (j >= 0) {
#pragma unroll
      for (int a = 0; a < DIM; a++) S.xs[a][sh] = xj[a];
      S.us[0][sh] = uj[0];
      S.us[1][sh] = uj[1];
      S.us[2][sh] = uj[2];
      S.ws[sh] = wj;
      S.ids[sh] = idj;
    }
  }
  if (threadIdx.x == 0) S.cnt2[P] = c2;
}

// Waves per SIMD the per-patch kernel's registers allow (four in 2D: five,
// at 96 registers, measured slower).
template <int DIM>
constexpr int kSlabMinWaves = DIM == 2 ? 4 : 2;

// Per-patch launch: one workgroup per (patch, species).  WALLS: instance
// with reflecting walls (the periodic one compiles them out).
template <int DIM, bool WALLS, bool FD>
__global__ void __launch_bounds__(kMaxWgSlab<DIM>, kSlabMinWaves<DIM>) k_ipp_slab(GridDev g, SlabArgs sa, Fields f, int *err) {
  extern __shared__ __align__(16) double lds[];
  __shared__ uint32_t bits[kBitWords];
  __shared__ int pre[kBitWords];
  __shared__ int wtot[16];
  const int P = blockIdx.x;
  const SlabDev &S = sa.s[blockIdx.y];
  const uint64_t t0 = sa.trace ? __builtin_amdgcn_s_memrealtime() : 0;
  const int flag = S.ctl[1];
  const int c = S.cnt[P];  // (loaded with the flag)
  if (flag == 2) return;
  const TileGeom t = tile_geom<DIM>(g, P);
  double *tEB = lds;
  double *tJ = lds + 6 * t.TE;
  const bool mark = c <= kBitSlots;
  stage_eb<DIM>(g, t, f, tEB);
  zero_tile<DIM>(tJ, 3 * t.TJ);
  for (int k = threadIdx.x; k < kBitWords; k += blockDim.x) bits[k] = 0u;
  __syncthreads();
  int bad = 0;
  ipp_slab<DIM, WALLS, FD>(g, S, t, tEB, tJ, P, 0u, (uint32_t)c, bad, mark ? bits : nullptr);
  if (bad) atomicOr(err, bad);
  __syncthreads();
  flush_j<DIM>(g, t, tJ, f.j);
  if (mark)
    depart_in_kernel<DIM>(g, S, P, c, bits, pre, wtot);
  else if (threadIdx.x == 0)
    S.dep[P] = -1;  // left to the departures kernel
  if (sa.trace) {
    __syncthreads();  // every thread's work is done
    if (threadIdx.x == 0) {
      TraceRec *rec = reinterpret_cast<TraceRec *>(sa.trace + 4);
      TraceRec r;
      r.patch = P;
      r.unit = (int)blockIdx.y;
      r.block = (int)(blockIdx.y * gridDim.x + blockIdx.x);
      r.species = (int)blockIdx.y;
      r.t0 = t0;
      r.t1 = __builtin_amdgcn_s_memrealtime();
      rec[blockIdx.y * gridDim.x + blockIdx.x] = r;
      if (blockIdx.x == 0 && blockIdx.y == 0) sa.trace[0] = (uint64_t)gridDim.x * gridDim.y;
    }
  }
}

// Persistent launch: workgroups pop (patch, particle range) units of each
// species in turn (ticket qctl[2s], count qctl[2s+1], list at units +
// ubase), or, with combined, from one list whose units range over the
// particles of every species of the patch (ticket qctl[0], count qctl[1],
// list at units); E/B is restaged and J flushed only when the patch changes.
template <int DIM, bool WALLS, bool COMBINED, bool FD>
__global__ void __launch_bounds__(kMaxWgSlab<DIM>, kSlabMinWaves<DIM>) k_ipp_slab_persistent(GridDev g, SlabArgs sa, Fields f, int *err,
                                                                    const Unit *units, int *qctl) {
  constexpr bool combined = COMBINED;
  extern __shared__ __align__(16) double lds[];
  __shared__ int s_unit;
  int curP = -1;
  TileGeom t = tile_geom<DIM>(g, 0);
  double *tEB = lds;
  double *tJ = lds + 6 * t.TE;
  int bad = 0;
  const int nlist = combined ? 1 : sa.nsp;
  for (int s = 0; s < nlist; s++) {
    const SlabDev &S = sa.s[s];
    if (!combined && S.ctl[1] == 2) continue;
    const int n_units = qctl[2 * s + 1];
    const Unit *ul = units + (combined ? 0 : S.ubase);
    for (;;) {
      if (threadIdx.x == 0) s_unit = atomicAdd(&qctl[2 * s], 1);
      __syncthreads();
      const int u = __builtin_amdgcn_readfirstlane(s_unit);
      __syncthreads();  // every thread has read s_unit before the next pop
      const uint64_t t0 = sa.trace ? __builtin_amdgcn_s_memrealtime() : 0;
      if (u >= n_units) {
        if (sa.trace && threadIdx.x == 0 && u == n_units) sa.trace[0] = (uint64_t)n_units;
        break;
      }
      const Unit un = ul[u];
      if (un.P != curP) {
        if (curP >= 0) {
          flush_j<DIM>(g, t, tJ, f.j);
          __syncthreads();  // flush has read the J tile before it is zeroed
        }
        t = tile_geom<DIM>(g, un.P);
        stage_eb<DIM>(g, t, f, tEB);
        zero_tile<DIM>(tJ, 3 * t.TJ);
        __syncthreads();
        curP = un.P;
      }
      if constexpr (COMBINED) {
        // the unit's share of each species: [k0, k1) of the concatenation
        int base = 0;
        for (int r = 0; r < sa.nsp; r++) {
          const SlabDev &R = sa.s[r];
          if (R.ctl[1] == 2) continue;
          const int c = R.cnt[un.P];
          const int r0 = min(max(un.k0 - base, 0), c), r1 = min(max(un.k1 - base, 0), c);
          if (r0 < r1)
            ipp_slab<DIM, WALLS, FD>(g, R, t, tEB, tJ, un.P, (uint32_t)r0, (uint32_t)r1, bad,
                                     nullptr);
          base += c;
        }
      } else {
        ipp_slab<DIM, WALLS, FD>(g, S, t, tEB, tJ, un.P, (uint32_t)un.k0, (uint32_t)un.k1, bad,
                                 nullptr);
      }
      __syncthreads();  // this unit's deposits are done before any flush
      if (sa.trace && threadIdx.x == 0) {
        TraceRec r;
        r.patch = un.P;
        r.unit = u;
        r.block = (int)blockIdx.x;
        r.species = combined ? -1 : s;
        r.t0 = t0;
        r.t1 = __builtin_amdgcn_s_memrealtime();
        reinterpret_cast<TraceRec *>(sa.trace + 4)[u] = r;
      }
    }
  }
  if (curP >= 0) flush_j<DIM>(g, t, tJ, f.j);
  if (bad) atomicOr(err, bad);
}

constexpr int kExchPer = 64;  // slab slots per thread and tile of the large-patch path
// threads per workgroup of the departures kernel: its large 2D patches
// need many lanes in flight; the 3D bins' small slabs need few
constexpr int kExchWgMax = 1024;
constexpr int kExchWg2 = 256, kExchWg3 = 64;

// The 64 codes of this thread's slots j0 .. j0+63 as 16 words; slots at or
// past c read as CENTER.  Slabs start on 16-slot boundaries and j0 is a
// multiple of 64, so the 16-byte loads are aligned.
template <int CENTER>
__device__ __forceinline__ void load_codes(const uint8_t *code, int64_t sbP, int j0, int c,
                                           uint32_t w[16]) {
  if (j0 + kExchPer <= c) {
    const uint4 *p = reinterpret_cast<const uint4 *>(code + sbP + j0);
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint4 v = p[k];
      w[4 * k] = v.x;
      w[4 * k + 1] = v.y;
      w[4 * k + 2] = v.z;
      w[4 * k + 3] = v.w;
    }
  } else {
    constexpr uint32_t kC = CENTER * 0x01010101u;
#pragma unroll
    for (int k = 0; k < 16; k++) w[k] = kC;
    for (int j = j0; j < c && j < j0 + kExchPer; j++) {
      const int k = j - j0;
      w[k >> 2] = (w[k >> 2] & ~(0xffu << (8 * (k & 3)))) | ((uint32_t)code[sbP + j] << (8 * (k & 3)));
    }
  }
}

__device__ __forceinline__ int code_at(const uint32_t w[16], int k) {
  return (int)((w[k >> 2] >> (8 * (k & 3))) & 0xffu);
}

// Departure bitmap of a slab of c <= kExchBitSlots<DIM> particles from its code
// bytes: bit j of word j/32 set if slot j leaves the patch.  Slabs start on
// 16-slot boundaries, so the 16-byte loads are aligned; the last word's
// loads stay inside the slab's room (at least c + 64 slots).
template <int CENTER>
__device__ __forceinline__ void code_bits(const uint8_t *code, int c, uint32_t *bits) {
  constexpr uint32_t kC = CENTER * 0x01010101u;
  const int W = (c + 31) >> 5;
  const int nt = blockDim.x;
  auto word = [&](const uint4 &a, const uint4 &b, int i) {
    const uint32_t v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const uint32_t d = v[k] ^ kC;  // zero byte: code CENTER
#pragma unroll
      for (int y = 0; y < 4; y++) m |= (uint32_t)(((d >> (8 * y)) & 0xffu) != 0u) << (4 * k + y);
    }
    const int valid = c - 32 * i;
    bits[i] = valid >= 32 ? m : m & ((1u << valid) - 1u);
  };
  // two words per thread and memory round trip
  for (int i = threadIdx.x; i < W; i += 2 * nt) {
    const uint4 *p = reinterpret_cast<const uint4 *>(code) + 2 * i;
    const uint4 a0 = p[0], b0 = p[1];
    const int i1 = i + nt;
    uint4 a1 = a0, b1 = b0;
    if (i1 < W) {
      a1 = p[2 * nt];
      b1 = p[2 * nt + 1];
    }
    word(a0, b0, i);
    if (i1 < W) word(a1, b1, i1);
  }
}

// Departures of patch P (grid: patches x species, kExchWg2 or kExchWg3
// threads; with only_marked, only the patches the fused kernel left,
// dep[P] < 0): the particles whose code leaves the patch are copied to the
// patch's outbox region (from sb[P]) with their destination patch; the
// stayers in the slab's tail [c2, c) then fill the holes the departures left
// below c2 = c - departures.  Up to kExchBitSlots<DIM> particles: the
// departure bitmap in LDS and the fused kernel's epilogue.  Larger patches:
// tiles of kExchPer slots per thread, each thread copying its own
// departures and movers in turn.
template <int DIM>
__global__ void __launch_bounds__(kExchWgMax) k_exch_out(GridDev g, SlabArgs sa, int only_marked,
                                                        int in_order) {
  constexpr int CENTER = DIM == 2 ? 4 : 13;
  const SlabDev &S = sa.s[blockIdx.y];
  // persistent mode with one species: the crowded patches first (porder)
  const int P = in_order ? S.porder[blockIdx.x] : (int)blockIdx.x;
  __shared__ uint32_t bits[kExchBitWords<DIM>];
  __shared__ int pre[kExchBitWords<DIM>];
  __shared__ int wtot[16];
  // the patch's words are loaded together, before the tests that use them
  const int flag = S.ctl[1];
  const int dp = S.dep[P];
  const int c = S.cnt[P];
  const int64_t sbP = S.sb[P];
  if (flag == 2) return;
  if (P == 0 && threadIdx.x == 0) S.ctl[1] = 0;  // the previous step's overflow is resolved
  if (only_marked && dp >= 0) return;           // done by the fused kernel
  if (c <= kExchBitSlots<DIM>) {
    code_bits<CENTER>(S.code + sbP, c, bits);
    __syncthreads();
    depart_in_kernel<DIM>(g, S, P, c, bits, pre, wtot);
    return;
  }
  int pc[3];
  patch_coords(g, P, pc);
  uint32_t w[16];
  int tot = 0;
  // Large case: tiles of kExchPer slots per thread; each thread copies its
  // own departures and movers in slot order.
  const int tile = (int)blockDim.x * kExchPer;
  int m = 0;
  for (int t0 = 0; t0 < c; t0 += tile) {
    load_codes<CENTER>(S.code, sbP, t0 + kExchPer * (int)threadIdx.x, c, w);
    int k = 0;
#pragma unroll
    for (int i = 0; i < kExchPer; i++) k += code_at(w, i) != CENTER;
    (void)block_excl_sum(k, tot, wtot);
    m += tot;
  }
  if (threadIdx.x == 0) S.dep[P] = m;
  if (m == 0) {
    if (threadIdx.x == 0) S.cnt2[P] = c;
    return;
  }
  const int c2 = c - m;
  int run = 0;
  for (int t0 = 0; t0 < c; t0 += tile) {
    const int j0 = t0 + kExchPer * (int)threadIdx.x;
    load_codes<CENTER>(S.code, sbP, j0, c, w);
    int k = 0;
#pragma unroll
    for (int i = 0; i < kExchPer; i++) k += code_at(w, i) != CENTER;
    int r = run + block_excl_sum(k, tot, wtot);
    run += tot;
    for (int i = 0; i < kExchPer && k > 0; i++) {
      const int cd = code_at(w, i);
      if (cd == CENTER) continue;
      const int j = j0 + i;
      const int64_t o = sbP + r;
      copy_particle<DIM>(S.ox, S.ou, S.ow, S.oid, o, S.xs, S.us, S.ws, S.ids, sbP + j);
      S.odest[o] = dest_patch(g, pc, cd);
      if (j < c2) S.hole[sbP + r] = j;  // departures in slot order: the first lie below c2
      r++;
      k--;
    }
  }
  __threadfence_block();
  __syncthreads();  // departures copied and holes listed before the tail moves in
  run = 0;
  for (int t0 = c2 / tile * tile; t0 < c; t0 += tile) {
    const int j0 = t0 + kExchPer * (int)threadIdx.x;
    load_codes<CENTER>(S.code, sbP, j0, c, w);
    int k = 0;
#pragma unroll
    for (int i = 0; i < kExchPer; i++) k += j0 + i >= c2 && j0 + i < c && code_at(w, i) == CENTER;
    int r = run + block_excl_sum(k, tot, wtot);
    run += tot;
    for (int i = 0; i < kExchPer && k > 0; i++) {
      const int j = j0 + i;
      if (j < c2 || j >= c || code_at(w, i) != CENTER) continue;
      const int h = S.hole[sbP + r];
      copy_particle<DIM>(S.xs, S.us, S.ws, S.ids, sbP + h, S.xs, S.us, S.ws, S.ids, sbP + j);
      r++;
      k--;
    }
  }
  if (threadIdx.x == 0) S.cnt2[P] = c2;
}

// Arrivals (grid: source patches x species, kExchInWg threads): each
// departure of patch Q takes the next free slot of its destination slab; one
// that finds the slab full stays in the outbox, marked, and raises the
// overflow flag.  A wave's departures to one destination take their slots
// with one atomic add (a patch's departures go to at most 8 or 26
// neighbours), so the arrival counters see a few adds per source wave.
constexpr int kExchInWg = 128;

template <int DIM>
__global__ void __launch_bounds__(kExchInWg) k_exch_in(GridDev g, SlabArgs sa) {
  const SlabDev &S = sa.s[blockIdx.y];
  const int Q = blockIdx.x;
  // the state flag, the departure count and the outbox start are read
  // together; a standing species leaves after the reads
  const int flag = S.ctl[1];
  const int m = S.dep[Q];
  const int64_t ob = S.sb[Q];
  if (flag == 2) return;
  const int lane = threadIdx.x & 63;
  // whole waves iterate together (the ballots below need every lane)
  for (int rb = (int)threadIdx.x - lane; rb < m; rb += blockDim.x) {
    const int r = rb + lane;
    const bool valid = r < m;
    const int64_t e = ob + (valid ? r : 0);
    // the departure's state is loaded with its destination, so only the
    // stores wait for the slot the destination's arrival counter hands out
    double x[DIM], u[3], w = 0.0;
    int64_t id = 0;
    int D = -1;
    if (valid) {
#pragma unroll
      for (int a = 0; a < DIM; a++) x[a] = S.ox[a][e];
      u[0] = S.ou[0][e];
      u[1] = S.ou[1][e];
      u[2] = S.ou[2][e];
      w = S.ow[e];
      id = S.oid[e];
      D = S.odest[e];  // < 0: deleted at a removing wall
    }
    const bool live = D >= 0;
    // group the live lanes by destination; the group's first lane leads
    uint64_t todo = __ballot(live);
    uint64_t group = 0;
    while (todo) {
      const int l = __ffsll((unsigned long long)todo) - 1;
      const int Dl = __shfl(D, l, 64);
      const uint64_t mk = __ballot(live && D == Dl);
      if (live && D == Dl) group = mk;
      todo &= ~mk;
    }
    const int leader = live ? __ffsll((unsigned long long)group) - 1 : lane;
    int got = 0;
    if (live && leader == lane) got = atomicAdd(&S.arr[D], __popcll(group));
    const int gbase = __shfl(got, leader, 64);
    if (!live) continue;
    const int pos = S.cnt2[D] + gbase + __popcll(group & ((1ull << lane) - 1ull));
    if (pos < S.cap[D]) {
      const int64_t d = S.sb[D] + pos;
#pragma unroll
      for (int a = 0; a < DIM; a++) S.xs[a][d] = x[a];
      S.us[0][d] = u[0];
      S.us[1][d] = u[1];
      S.us[2][d] = u[2];
      S.ws[d] = w;
      S.ids[d] = id;
    } else {
      S.odest[e] = D | kUnplaced;
      atomicOr(&S.ctl[1], 1);
    }
  }
}

// Persistent mode: work units of chunk particles for the patch counts (one
// workgroup of at most kUnitsWg threads, each a contiguous run of patches):
// every full unit first, then the remainders from the largest to the
// smallest in kRemClasses size classes, each class in patch order.  A
// worker pops the next unit when it finishes one, so the list's end sets
// the launch's tail: with the smallest units last, the workers finish
// nearly together (largest units first is the classic list-scheduling
// rule).  count(P) loads patch P's count; keep(P, c) stores what the
// caller derives from it (for a thread's first kUnitsCached patches: all
// loads first, the stores after the scans); again(P) gives the count a
// second time, after keep.  The list goes to ul (units tagged with species
// s), its length to q[1] (0 if the species stands still) and a zero ticket
// to q[0].  kUnitsCached: counts a thread keeps in registers; cls:
// kRemClasses x kUnitsWg ints of LDS.  porder (if not null): the patches
// with at least chunk/2 particles, then the others, each in patch order --
// the order in which the departures kernel takes them, so that the
// crowded patches' workgroups, its longest, start first.
constexpr int kRemClasses = 8, kUnitsWg = 1024;

template <int kUnitsCached, class Count, class Keep, class Again>
__device__ void make_units(int s, int n, int chunk, bool still, Count count, Keep keep,
                           Again again, Unit *ul, int *q, int *wtot, int *cls,
                           int32_t *porder = nullptr) {
  const int nt = blockDim.x, t = threadIdx.x;
  const int per = (n + nt - 1) / nt;
  const int p0 = min(n, t * per), p1 = min(n, p0 + per);
  // size class of a remainder: 0 for the largest
  auto klass = [&](int c) { return (int)((int64_t)(chunk - c % chunk) * kRemClasses - 1) / chunk; };
  int cc[kUnitsCached];
  int nf = 0, nh = 0, nr[kRemClasses];
  const int heavy = max(chunk / 2, 1);
#pragma unroll
  for (int k = 0; k < kRemClasses; k++) nr[k] = 0;
#pragma unroll
  for (int k = 0; k < kUnitsCached; k++) cc[k] = p0 + k < p1 ? count(p0 + k) : 0;
#pragma unroll
  for (int k = 0; k < kUnitsCached; k++) {
    nf += cc[k] / chunk;
    nh += cc[k] >= heavy;
    if (cc[k] % chunk) nr[klass(cc[k])]++;
  }
  for (int P = p0 + kUnitsCached; P < p1; P++) {
    const int c = count(P);
    keep(P, c);
    nf += c / chunk;
    nh += c >= heavy;
    if (c % chunk) nr[klass(c)]++;
  }
  int tf = 0, tr = 0, th = 0;
  int rf = block_excl_sum(nf, tf, wtot);
  // crowded patches before this thread's; the others before it: p0 - that
  int hp = porder ? block_excl_sum(nh, th, wtot) : 0;
  int lp = th + (p0 - hp);
  // the remainders' starts: an exclusive scan of the class-major array
  // [class][thread] through LDS, each thread summing kRemClasses
  // consecutive elements of it
#pragma unroll
  for (int k = 0; k < kRemClasses; k++) cls[k * nt + t] = nr[k];
  __syncthreads();
  int v[kRemClasses], sum = 0;
#pragma unroll
  for (int j = 0; j < kRemClasses; j++) {
    v[j] = cls[t * kRemClasses + j];
    sum += v[j];
  }
  int base = block_excl_sum(sum, tr, wtot);  // (its barriers order the reads before the writes)
#pragma unroll
  for (int j = 0; j < kRemClasses; j++) {
    cls[t * kRemClasses + j] = base;
    base += v[j];
  }
  __syncthreads();
  int rr[kRemClasses];
#pragma unroll
  for (int k = 0; k < kRemClasses; k++) rr[k] = tf + cls[k * nt + t];
  // the cached patches' stores after the scans, whose barriers then need
  // not wait for them
#pragma unroll
  for (int k = 0; k < kUnitsCached; k++)
    if (p0 + k < p1) keep(p0 + k, cc[k]);
  auto emit = [&](int P, int c) {
    if (porder) porder[c >= heavy ? hp++ : lp++] = P;
    Unit un;
    un.s = s;
    un.P = P;
    for (int j = 0; j < c / chunk; j++) {
      un.k0 = j * chunk;
      un.k1 = un.k0 + chunk;
      ul[rf++] = un;
    }
    if (c % chunk) {
      un.k0 = c / chunk * chunk;
      un.k1 = c;
      const int k = klass(c);
#pragma unroll
      for (int x = 0; x < kRemClasses; x++)  // (a register index known at run time)
        if (x == k) ul[rr[x]++] = un;
    }
  };
#pragma unroll
  for (int k = 0; k < kUnitsCached; k++)
    if (p0 + k < p1) emit(p0 + k, cc[k]);
  for (int P = p0 + kUnitsCached; P < p1; P++) emit(P, again(P));
  if (threadIdx.x == 0) {
    q[1] = still ? 0 : tf + tr;
    q[0] = 0;
  }
}

// End of the exchange (one workgroup of 1024 per species): new counts; on
// an overflow, a new slab plan for the counts every patch needs.  With
// units (persistent mode), also the next step's work units.
__global__ void __launch_bounds__(kUnitsWg) k_exch_fin(GridDev g, SlabArgs sa, int *err, Unit *units,
                                                       int *qctl, int chunk) {
  __shared__ int64_t part[1024];
  __shared__ int wtot[16];
  __shared__ int cls[kRemClasses * kUnitsWg];
  const int s = blockIdx.x;
  const SlabDev &S = sa.s[s];
  const int n = g.npatch;
  const int flag = S.ctl[1];
  if (flag == 2) return;
  if (flag == 0) {
    if (units) {  // the new counts, and the work units from them, in one pass
      make_units<8>(
          s, n, chunk, false, [&](int P) { return S.cnt2[P] + S.arr[P]; },
          [&](int P, int c) {
            S.cnt[P] = c;
            S.arr[P] = 0;
          },
          [&](int P) { return S.cnt[P]; }, units + S.ubase, qctl + 2 * s, wtot, cls,
          sa.nsp == 1 ? S.porder : nullptr);
      return;
    }
    // four patches per thread and memory round trip
    constexpr int kB = 4;
    const int nt = blockDim.x;
    for (int P0 = threadIdx.x; P0 < n; P0 += kB * nt) {
      int c[kB];
#pragma unroll
      for (int k = 0; k < kB; k++) {
        const int P = P0 + k * nt;
        c[k] = P < n ? S.cnt2[P] + S.arr[P] : 0;
      }
#pragma unroll
      for (int k = 0; k < kB; k++) {
        const int P = P0 + k * nt;
        if (P < n) {
          S.cnt[P] = c[k];
          S.arr[P] = 0;
        }
      }
    }
    return;
  }
  for (int P = threadIdx.x; P < n; P += blockDim.x) {
    const int64_t need = (int64_t)S.cnt2[P] + S.arr[P];
    S.cap2[P] = (int32_t)slab_room(need);
    S.tmp[P] = slab_room(need);
    S.arr2[P] = 0;
  }
  __syncthreads();
  block_scan_1024(S.tmp, S.sb2, n, part);
  const bool still = S.sb2[n] > S.capacity;
  if (threadIdx.x == 0 && still) {
    S.ctl[1] = 2;  // no room for a new plan: the species stands still
    atomicOr(err, kErrCap);
  }
  if (units) {  // the counts the new plan's copies will set
    auto need = [&](int P) { return S.cnt2[P] + S.arr[P]; };
    make_units<8>(s, n, chunk, still, need, [](int, int) {}, need, units + S.ubase, qctl + 2 * s,
                  wtot, cls, sa.nsp == 1 ? S.porder : nullptr);
  }
}

// The re-plan kernels return at once without an overflow, which is almost
// every step: they run on a small grid whose workgroups loop over the
// patches when there is one.
constexpr int kReslabGrid = 512;  // workgroups per species

// Overflow, part 1 (grid: up to kReslabGrid x species; workgroup b takes
// items b, b + gridDim.x, ... of 2 x patches): every particle goes to its
// place in the new plan, inside the first buffer set -- item P < patches
// copies slab P, item patches + Q the outbox entries of patch Q that found
// no room.
template <int DIM>
__global__ void __launch_bounds__(256) k_reslab_move(GridDev g, SlabArgs sa) {
  const SlabDev &S = sa.s[blockIdx.y];
  if (S.ctl[1] != 1) return;
  const int n = g.npatch;
  for (int v = blockIdx.x; v < 2 * n; v += gridDim.x) {
    if (v < n) {
      const int P = v;
      const int placed = min(S.arr[P], S.cap[P] - S.cnt2[P]);
      const int64_t c = (int64_t)S.cnt2[P] + placed;
      copy_run<DIM>(S.x, S.u, S.w, S.id, S.sb2[P], S.xs, S.us, S.ws, S.ids, S.sb[P], c);
      continue;
    }
    const int Q = v - n;  // the outbox of patch Q
    const int m = S.dep[Q];
    const int64_t ob = S.sb[Q];
    for (int r = threadIdx.x; r < m; r += blockDim.x) {
      const int64_t e = ob + r;
      const int dv = S.odest[e];
      if (dv < 0 || !(dv & kUnplaced)) continue;  // deleted, or placed
      const int D = dv & ~kUnplaced;
      const int placed = min(S.arr[D], S.cap[D] - S.cnt2[D]);
      const int64_t pos = (int64_t)S.cnt2[D] + placed + atomicAdd(&S.arr2[D], 1);
      copy_particle<DIM>(S.x, S.u, S.w, S.id, S.sb2[D] + pos, S.ox, S.ou, S.ow, S.oid, e);
    }
  }
}

// Overflow, part 2 (grid: up to kReslabGrid x species, looping over the
// patches): back into the slab buffers at the new plan's places; the plan
// becomes current.
template <int DIM>
__global__ void __launch_bounds__(256) k_reslab_back(GridDev g, SlabArgs sa) {
  const SlabDev &S = sa.s[blockIdx.y];
  if (S.ctl[1] != 1) return;
  for (int P = blockIdx.x; P < g.npatch; P += gridDim.x) {
    const int64_t c = (int64_t)S.cnt2[P] + S.arr[P], d0 = S.sb2[P];
    copy_run<DIM>(S.xs, S.us, S.ws, S.ids, d0, S.x, S.u, S.w, S.id, d0, c);
    __syncthreads();  // every thread has read arr[P] before it is cleared
    if (threadIdx.x == 0) {
      S.cnt[P] = (int32_t)c;
      S.cap[P] = S.cap2[P];
      S.sb[P] = d0;
      S.arr[P] = 0;
      if (P == 0) S.sb[g.npatch] = S.sb2[g.npatch];
    }
  }
}

// Persistent mode, start of a call: work units from the slab counts (one
// workgroup of 1024 per species).
__global__ void __launch_bounds__(kUnitsWg) k_slab_units(GridDev g, SlabArgs sa, int chunk,
                                                         Unit *units, int *qctl) {
  __shared__ int wtot[16];
  __shared__ int cls[kRemClasses * kUnitsWg];
  const int s = blockIdx.x;
  const SlabDev &S = sa.s[s];
  auto count = [&](int P) { return S.cnt[P]; };
  make_units<16>(s, g.npatch, chunk, S.ctl[1] == 2, count, [](int, int) {}, count,
                 units + S.ubase, qctl + 2 * s, wtot, cls, sa.nsp == 1 ? S.porder : nullptr);
}

// Persistent mode with several species: one list of units over every
// species of a patch (the patch's particles of species 0, then of species
// 1, ...: a unit may span species), so a workgroup stages a patch's fields
// and flushes its current once for all species.  From the slab counts
// after the exchange (one workgroup of 1024); a species that stands still
// counts zero.  List at units, length in qctl[1], zero ticket in qctl[0].
__global__ void __launch_bounds__(kUnitsWg) k_units_all(GridDev g, SlabArgs sa, int chunk,
                                                        Unit *units, int *qctl) {
  __shared__ int wtot[16];
  __shared__ int cls[kRemClasses * kUnitsWg];
  auto count = [&](int P) {
    int c = 0;
    for (int s = 0; s < sa.nsp; s++)
      if (sa.s[s].ctl[1] != 2) c += sa.s[s].cnt[P];
    return c;
  };
  make_units<16>(-1, g.npatch, chunk, false, count, [](int, int) {}, count, units, qctl, wtot, cls);
}

// End of a call: dense offsets from the slab counts (one workgroup of 1024
// per species) ...
__global__ void __launch_bounds__(1024) k_slab_offsets(GridDev g, SlabArgs sa) {
  __shared__ int64_t part[1024];
  const SlabDev &S = sa.s[blockIdx.x];
  if (S.ctl[1] == 2) return;
  const int n = g.npatch;
  for (int P = threadIdx.x; P < n; P += blockDim.x) S.tmp[P] = S.cnt[P];
  __syncthreads();
  block_scan_1024(S.tmp, S.off, n, part);
}

// ... and slabs -> dense (grid: patches x species).
template <int DIM>
__global__ void __launch_bounds__(256) k_slab_out(GridDev g, SlabArgs sa) {
  const SlabDev &S = sa.s[blockIdx.y];
  if (S.ctl[1] == 2) return;
  const int P = blockIdx.x;
  copy_run<DIM>(S.x, S.u, S.w, S.id, S.off[P], S.xs, S.us, S.ws, S.ids, S.sb[P], S.cnt[P]);
}

}  // namespace

hipError_t launch_slab_begin(const GridDev &g, const SlabArgs &sa, int *err, hipStream_t st,
                             bool copy) {
  hipLaunchKernelGGL(k_slab_plan, dim3(sa.nsp), dim3(1024), 0, st, g, sa, err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !copy) return e;
  if (g.dim == 2)
    hipLaunchKernelGGL(k_slab_in<2>, dim3(g.npatch, sa.nsp), dim3(256), 0, st, g, sa);
  else
    hipLaunchKernelGGL(k_slab_in<3>, dim3(g.npatch, sa.nsp), dim3(256), 0, st, g, sa);
  return hipGetLastError();
}

template <int DIM, bool WALLS>
void ipp_slab_t(const GridDev &g, const SlabArgs &sa, const Fields &f, int *err, int wg, size_t lds,
                hipStream_t st) {
  // the call's first step reads the dense layout (its own instance, so the
  // steps after it keep the in-place kernel's registers)
  if (sa.from_dense) {
    if (DIM == 3)
      (void)hipFuncSetAttribute((const void *)k_ipp_slab<DIM, WALLS, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_ipp_slab<DIM, WALLS, true>), dim3(g.npatch, sa.nsp), dim3(wg), lds, st, g,
                       sa, f, err);
    return;
  }
  if (DIM == 3)
    (void)hipFuncSetAttribute((const void *)k_ipp_slab<DIM, WALLS, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_ipp_slab<DIM, WALLS, false>), dim3(g.npatch, sa.nsp), dim3(wg), lds, st, g,
                     sa, f, err);
}

hipError_t launch_ipp_slab(const GridDev &g, const SlabArgs &sa, const double *const e[3],
                           const double *const b[3], double *const j[3], int *err, int wg,
                           hipStream_t st) {
  const Fields f = mkfields(e, b, j);
  const size_t lds = lds_bytes_ipp(g);
  if (g.dim == 2)
    has_walls(g) ? ipp_slab_t<2, true>(g, sa, f, err, wg, lds, st)
              : ipp_slab_t<2, false>(g, sa, f, err, wg, lds, st);
  else
    has_walls(g) ? ipp_slab_t<3, true>(g, sa, f, err, wg, lds, st)
              : ipp_slab_t<3, false>(g, sa, f, err, wg, lds, st);
  return hipGetLastError();
}

template <int DIM, bool WALLS, bool COMBINED, bool FD>
void ipp_slab_pers_one(const GridDev &g, const SlabArgs &sa, const Fields &f, int *err,
                       const Unit *units, int *qctl, int grid, int wg, size_t lds,
                       hipStream_t st) {
  if (DIM == 3)
    (void)hipFuncSetAttribute((const void *)k_ipp_slab_persistent<DIM, WALLS, COMBINED, FD>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_ipp_slab_persistent<DIM, WALLS, COMBINED, FD>), dim3(grid), dim3(wg), lds,
                     st, g, sa, f, err, units, qctl);
}

template <int DIM, bool WALLS>
void ipp_slab_pers_t(const GridDev &g, const SlabArgs &sa, const Fields &f, int *err,
                     const Unit *units, int *qctl, int grid, int wg, size_t lds, hipStream_t st) {
  // several species: the instance whose units range over all of them; the
  // call's first step reads the dense layout
  if (sa.nsp > 1)
    sa.from_dense ? ipp_slab_pers_one<DIM, WALLS, true, true>(g, sa, f, err, units, qctl, grid, wg, lds, st)
                  : ipp_slab_pers_one<DIM, WALLS, true, false>(g, sa, f, err, units, qctl, grid, wg, lds, st);
  else
    sa.from_dense ? ipp_slab_pers_one<DIM, WALLS, false, true>(g, sa, f, err, units, qctl, grid, wg, lds, st)
                  : ipp_slab_pers_one<DIM, WALLS, false, false>(g, sa, f, err, units, qctl, grid, wg, lds, st);
}

hipError_t launch_ipp_slab_persistent(const GridDev &g, const SlabArgs &sa,
                                      const double *const e[3], const double *const b[3],
                                      double *const j[3], int *err, const Unit *units, int *qctl,
                                      int grid, int wg, hipStream_t st) {
  const Fields f = mkfields(e, b, j);
  const size_t lds = lds_bytes_ipp(g);
  if (g.dim == 2)
    has_walls(g) ? ipp_slab_pers_t<2, true>(g, sa, f, err, units, qctl, grid, wg, lds, st)
              : ipp_slab_pers_t<2, false>(g, sa, f, err, units, qctl, grid, wg, lds, st);
  else
    has_walls(g) ? ipp_slab_pers_t<3, true>(g, sa, f, err, units, qctl, grid, wg, lds, st)
              : ipp_slab_pers_t<3, false>(g, sa, f, err, units, qctl, grid, wg, lds, st);
  return hipGetLastError();
}

template <int DIM, bool WALLS, bool COMBINED, bool FD>
int slab_blocks_one(int wg, size_t lds) {
  if (DIM == 3)
    (void)hipFuncSetAttribute((const void *)k_ipp_slab_persistent<DIM, WALLS, COMBINED, FD>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, k_ipp_slab_persistent<DIM, WALLS, COMBINED, FD>, wg, lds) != hipSuccess)
    return 0;
  return n;
}

// resident workgroups per CU of every instance (one species or several;
// first step of a call or not): the grid must fit all of them
template <int DIM, bool WALLS>
int slab_blocks_t(int wg, size_t lds) {
  return std::min(std::min(slab_blocks_one<DIM, WALLS, false, false>(wg, lds),
                           slab_blocks_one<DIM, WALLS, true, false>(wg, lds)),
                  std::min(slab_blocks_one<DIM, WALLS, false, true>(wg, lds),
                           slab_blocks_one<DIM, WALLS, true, true>(wg, lds)));
}

int slab_persistent_blocks_per_cu(const GridDev &g, int wg) {
  const size_t lds = lds_bytes_ipp(g);
  const int n = g.dim == 2 ? (has_walls(g) ? slab_blocks_t<2, true>(wg, lds)
                                        : slab_blocks_t<2, false>(wg, lds))
                           : (has_walls(g) ? slab_blocks_t<3, true>(wg, lds)
                                        : slab_blocks_t<3, false>(wg, lds));
  return n > 0 ? n : 1;
}

hipError_t launch_exchange(const GridDev &g, const SlabArgs &sa, int *err, Unit *units, int *qctl,
                           int chunk, hipStream_t st) {
  const dim3 pg(g.npatch, sa.nsp);
  const int only_marked = units ? 0 : 1;  // the per-patch fused kernel did the departures
  const int in_order = units && sa.nsp == 1 ? 1 : 0;  // porder made by the unit list
  if (g.dim == 2) {
    hipLaunchKernelGGL(k_exch_out<2>, pg, dim3(kExchWg2), 0, st, g, sa, only_marked, in_order);
    hipLaunchKernelGGL(k_exch_in<2>, pg, dim3(kExchInWg), 0, st, g, sa);
  } else {
    hipLaunchKernelGGL(k_exch_out<3>, pg, dim3(kExchWg3), 0, st, g, sa, only_marked, in_order);
    hipLaunchKernelGGL(k_exch_in<3>, pg, dim3(kExchInWg), 0, st, g, sa);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // several species: one combined unit list, made once the counts are final
  const bool combined = units && sa.nsp > 1;
  hipLaunchKernelGGL(k_exch_fin, dim3(sa.nsp), dim3(kUnitsWg), 0, st, g, sa, err,
                     combined ? nullptr : units, qctl, chunk);
  const dim3 mg(std::min(2 * g.npatch, kReslabGrid), sa.nsp);
  const dim3 bg(std::min(g.npatch, kReslabGrid), sa.nsp);
  if (g.dim == 2) {
    hipLaunchKernelGGL(k_reslab_move<2>, mg, dim3(256), 0, st, g, sa);
    hipLaunchKernelGGL(k_reslab_back<2>, bg, dim3(256), 0, st, g, sa);
  } else {
    hipLaunchKernelGGL(k_reslab_move<3>, mg, dim3(256), 0, st, g, sa);
    hipLaunchKernelGGL(k_reslab_back<3>, bg, dim3(256), 0, st, g, sa);
  }
  if (combined)
    hipLaunchKernelGGL(k_units_all, dim3(1), dim3(kUnitsWg), 0, st, g, sa, chunk, units, qctl);
  return hipGetLastError();
}

hipError_t launch_slab_units(const GridDev &g, const SlabArgs &sa, int chunk, Unit *units,
                             int *qctl, hipStream_t st) {
  if (sa.nsp > 1)
    hipLaunchKernelGGL(k_units_all, dim3(1), dim3(kUnitsWg), 0, st, g, sa, chunk, units, qctl);
  else
    hipLaunchKernelGGL(k_slab_units, dim3(1), dim3(kUnitsWg), 0, st, g, sa, chunk, units, qctl);
  return hipGetLastError();
}

hipError_t launch_slab_end(const GridDev &g, const SlabArgs &sa, hipStream_t st) {
  hipLaunchKernelGGL(k_slab_offsets, dim3(sa.nsp), dim3(1024), 0, st, g, sa);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_slab_out<2>, dim3(g.npatch, sa.nsp), dim3(256), 0, st, g, sa);
  else
    hipLaunchKernelGGL(k_slab_out<3>, dim3(g.npatch, sa.nsp), dim3(256), 0, st, g, sa);
  return hipGetLastError();
}

}  // namespace pic
