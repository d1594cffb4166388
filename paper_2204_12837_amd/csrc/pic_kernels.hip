// HIP kernels (gfx950) for the per-step macro-particle operators of an
// electromagnetic PIC loop: Interpolation, Push, pre-BC and Projection
// (arXiv 2204.12837, section "Parallelization without tasks"), plus the
// sort by patch of the synchronisation phase.
//
// Design (one workgroup per patch and species, as the paper's per-patch
// loop, with the CPU thread replaced by a workgroup):
//  * the patch's E and B with one ghost layer on each side -- everything an
//    order-2 stencil can touch from a particle inside the patch -- are staged
//    once into LDS, so the gather reads LDS only;
//  * J is accumulated in a private LDS tile covering the patch plus the
//    two-cell reach of the five-point Esirkepov stencil, with LDS float64
//    atomics, then added to the grid with one global atomic per tile entry.
//    This is the paper's local sub-grid per patch followed by a reduction
//    into the patch grid "with the appropriate shift" (section
//    "Parallelization with OpenMP task");
//  * particles are read and written in structure-of-arrays order, so a wave
//    reads 64 consecutive doubles per array;
//  * pre-BC computes the destination patch of every particle as one of the
//    3^dim neighbour codes, and a stable per-code rank from wave ballots.
//    Each wave ranks its own contiguous share of the patch (a "ranking
//    unit"), so the particle loop has no workgroup barrier; the sort is then a
//    counting sort over (unit, code) (no global atomics).
//
// Floating point: this file is compiled with -ffp-contract=off.  The
// interpolation, the push and the patch key repeat the CPU oracle's
// operation sequence exactly (quadratic B-spline weights, x-then-y-then-z
// accumulation, Boris rotation form), so particle coordinates come out bit
// for bit equal; J differs from the oracle only through the order of the
// atomic additions.
#include <hip/hip_runtime.h>

#include "pic_common.h"
#include "pic_device.h"

namespace pic {

namespace {
// ---------------------------------------------------------------------------
// Fused step: Interpolation, Push, pre-BC and Projection of ranking segments
// [k0, k1) of patch P (each segment kSeg consecutive particles; the waves of
// the workgroup take segments in turn, 64 particles per block, and rank each
// segment on their own, so the loop has no barrier).  The E/B tile of P is in
// tEB, the J tile tJ accumulates.  GATHER: slot i of the patch takes the
// particle at perm[i] of the other buffer set (the previous sort's layout)
// and is written to this set; otherwise particles are updated in place.
//
// Each wave runs a software pipeline over its blocks: while block n is
// computed, the particles of block n+1 are being loaded and the permutation
// entries of block n+2 as well, so the dependent global loads (permutation,
// then particle) do not stall the wave.  Every global access of a full block
// is issued unconditionally (prefetches past the wave's end reload its last
// block), which keeps the memory-counter waits exact; only a partial last
// block runs masked.
template <int DIM, bool GATHER, bool WALLS>
__device__ __forceinline__ void ipp_segments(const GridDev &g, const SpDev &S, const TileGeom &t,
                                             const double *tEB, double *tJ, int P, int k0, int k1,
                                             int &bad) {
  const uint32_t beg = (uint32_t)S.off[P], end = (uint32_t)S.off[P + 1];
  const int nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int sbase = S.sstart[P];
  const double q = S.q, alpha = S.alpha;
  Blk cur;
  cur.start(k0 + wv, beg, end);
  if (cur.k >= k1) return;
  Blk nxt = cur;
  nxt.next(nw, k1, beg, end);
  auto src_of = [&](const Blk &b) -> uint32_t {
    const uint32_t i = b.slot(lane);
    return GATHER ? (uint32_t)at(S.perm, i) : i;
  };
  Part<DIM, GATHER> pc, pn;
  load_part<DIM, GATHER>(S, src_of(cur), pc);
  uint32_t srcn = src_of(nxt);
  double *const *xo = GATHER ? S.xa : S.x;
  double *const *uo = GATHER ? S.ua : S.u;
  int run = 0;
  // full blocks
  while (!cur.dead && cur.full()) {
    Blk nn = nxt;
    nn.next(nw, k1, beg, end);
    load_part<DIM, GATHER>(S, srcn, pn);
    const uint32_t srcnn = src_of(nn);
    const uint32_t i = cur.base + lane;
    double x[3], u[3];
#pragma unroll
    for (int a = 0; a < DIM; a++) x[a] = pc.x[a];
    u[0] = pc.u[0];
    u[1] = pc.u[1];
    u[2] = pc.u[2];
    const int code = step_particle<DIM, WALLS>(g, t, tEB, tJ, q, alpha, pc.w, x, u, bad);
#pragma unroll
    for (int a = 0; a < DIM; a++) at(xo[a], i) = x[a];
    at(uo[0], i) = u[0];
    at(uo[1], i) = u[1];
    at(uo[2], i) = u[2];
    if (GATHER) {
      at(S.wa, i) = pc.w;
      at(S.ida, i) = pc.id;
    }
    const uint32_t rank = wave_rank(true, code, lane, run);
    at(S.tag, i) = ((uint32_t)code << 27) | rank;
    // lanes >= 3^dim hold zero: the row is kCntRow wide
    S.cnt[(int64_t)(sbase + cur.k) * kCntRow + lane] = run;
    if (cur.base + 64 >= cur.se) run = 0;
    cur = nxt;
    nxt = nn;
    pc = pn;
    srcn = srcnn;
  }
  // partial last block
  if (!cur.dead) {
    const uint32_t i = cur.base + lane;
    const bool valid = i < cur.se;
    int code = DIM == 2 ? 4 : 13;
    if (valid) {
      double x[3], u[3];
#pragma unroll
      for (int a = 0; a < DIM; a++) x[a] = pc.x[a];
      u[0] = pc.u[0];
      u[1] = pc.u[1];
      u[2] = pc.u[2];
      code = step_particle<DIM, WALLS>(g, t, tEB, tJ, q, alpha, pc.w, x, u, bad);
#pragma unroll
      for (int a = 0; a < DIM; a++) at(xo[a], i) = x[a];
      at(uo[0], i) = u[0];
      at(uo[1], i) = u[1];
      at(uo[2], i) = u[2];
      if (GATHER) {
        at(S.wa, i) = pc.w;
        at(S.ida, i) = pc.id;
      }
    }
    const uint32_t rank = wave_rank(valid, code, lane, run);
    if (valid) at(S.tag, i) = ((uint32_t)code << 27) | rank;
    S.cnt[(int64_t)(sbase + cur.k) * kCntRow + lane] = run;
  }
}

// Per-patch launch: one workgroup per (patch, species), all its segments.
// WALLS: instance with reflecting walls (the periodic one compiles them out).
// With sa.jt (PIC_FLAG_DETERMINISTIC) every wave deposits into a J tile of
// its own, so no two waves race on a node: the LDS atomics of one wave
// apply in program order.  The tiles are then added in wave order and the
// sum is stored as this (species, patch)'s tile in sa.jt instead of being
// added to the grid with atomics.
template <int DIM, bool GATHER, bool WALLS>
__global__ void __launch_bounds__(kMaxWg<DIM>, kMinWaves<DIM>) k_ipp(GridDev g, SpArgs sa, Fields f, int *err) {
  extern __shared__ __align__(16) double lds[];
  const int P = blockIdx.x;
  const SpDev &S = sa.s[blockIdx.y];
  const TileGeom t = tile_geom<DIM>(g, P);
  const int nw = blockDim.x >> 6;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double *tEB = lds;
  double *tJ0 = lds + 6 * t.TE;
  double *tJ = sa.jt ? tJ0 + (size_t)wv * 3 * t.TJ : tJ0;
  stage_eb<DIM>(g, t, f, tEB);
  zero_tile<DIM>(tJ0, 3 * t.TJ * (sa.jt ? nw : 1));
  __syncthreads();
  int bad = 0;
  ipp_segments<DIM, GATHER, WALLS>(g, S, t, tEB, tJ, P, 0, S.sstart[P + 1] - S.sstart[P], bad);
  if (bad) atomicOr(err, bad);
  __syncthreads();
  if (sa.jt) {
    const int n3 = 3 * t.TJ;
    double *out = sa.jt + ((size_t)blockIdx.y * g.npatch + P) * n3;
    for (int r = threadIdx.x; r < n3; r += blockDim.x) {
      double v = tJ0[r];
      for (int k = 1; k < nw; k++) v += tJ0[(size_t)k * n3 + r];
      out[r] = v;
    }
    return;
  }
  flush_j<DIM>(g, t, tJ, f.j);
}

// PIC_FLAG_DETERMINISTIC: J at every node = the sum of the tile entries that
// cover it, species by species, the covering patches in a fixed order.  A
// patch's J tile spans nodes [P p - 2, P p + p + 3) along each axis, so a
// node is covered by the patch of (node + 2) / p at tile index
// r = (node + 2) - P p, and by the k-th patch before it (at r + k p) while
// r + k p < p + 5 (x-bins can be as narrow as one cell: up to six patches;
// with few patches along the axis, one patch may cover the node twice).
template <int DIM>
__global__ void __launch_bounds__(256) k_j_gather(GridDev g, SpArgs sa, Fields f) {
  const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
  const int Jx = g.patch[0] + 5, Jy = g.patch[1] + 5, Jz = DIM == 3 ? g.patch[2] + 5 : 1;
  const int64_t TJ = (int64_t)Jx * Jy * Jz;
  for (int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; node < ncell;
       node += (int64_t)gridDim.x * blockDim.x) {
    int gc[3];
    gc[0] = (int)(node % g.n[0]);
    const int64_t rest = node / g.n[0];
    gc[1] = (int)(rest % g.n[1]);
    gc[2] = (int)(rest / g.n[1]);
    constexpr int kCover = 6;
    int cp[3][kCover], cr[3][kCover], nc[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      nc[a] = 1;
      cp[a][0] = 0;
      cr[a][0] = 0;
      if (a >= DIM) continue;
      const int p = g.patch[a];
      int q = (gc[a] + 2) / p;
      int r = gc[a] + 2 - q * p;
      if (q >= g.np[a]) q -= g.np[a];
      nc[a] = 0;
      while (nc[a] < kCover && r < p + 5) {
        cp[a][nc[a]] = q;
        cr[a][nc[a]] = r;
        nc[a]++;
        q = q == 0 ? g.np[a] - 1 : q - 1;
        r += p;
      }
    }
    double v[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < sa.nsp; s++)
      for (int kz = 0; kz < nc[2]; kz++)
        for (int ky = 0; ky < nc[1]; ky++)
          for (int kx = 0; kx < nc[0]; kx++) {
            const int64_t P = cp[0][kx] + (int64_t)g.np[0] * (cp[1][ky] + (int64_t)g.np[1] * cp[2][kz]);
            const int64_t r = cr[0][kx] + (int64_t)Jx * (cr[1][ky] + (int64_t)Jy * cr[2][kz]);
            const double *T = sa.jt + ((int64_t)s * g.npatch + P) * 3 * TJ + r;
#pragma unroll
            for (int c = 0; c < 3; c++) v[c] += T[c * TJ];
          }
#pragma unroll
    for (int c = 0; c < 3; c++) f.j[c][node] = v[c];
  }
}

// Persistent launch: a fixed grid of workgroups pops (patch, segment range)
// units of each species in turn from a device ticket (qctl[2s], with
// qctl[2s+1] units listed at units + ubase) until every list is exhausted.
// The E/B tile is restaged and the J tile flushed only when the patch changes
// between a workgroup's consecutive units (E/B and J do not depend on the
// species).
template <int DIM, bool GATHER, bool WALLS>
__global__ void __launch_bounds__(kMaxWg<DIM>, kMinWaves<DIM>) k_ipp_persistent(GridDev g, SpArgs sa, Fields f, int *err,
                                                        const Unit *units, int *qctl) {
  extern __shared__ __align__(16) double lds[];
  __shared__ int s_unit;
  int curP = -1;
  TileGeom t = tile_geom<DIM>(g, 0);
  double *tEB = lds;
  double *tJ = lds + 6 * t.TE;
  int bad = 0;
  for (int s = 0; s < sa.nsp; s++) {
    const int n_units = qctl[2 * s + 1];
    const Unit *ul = units + sa.s[s].ubase;
    for (;;) {
      if (threadIdx.x == 0) s_unit = atomicAdd(&qctl[2 * s], 1);
      __syncthreads();
      const int u = __builtin_amdgcn_readfirstlane(s_unit);  // wave-uniform
      __syncthreads();  // every thread has read s_unit before the next pop
      if (u >= n_units) break;
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
      ipp_segments<DIM, GATHER, WALLS>(g, sa.s[s], t, tEB, tJ, un.P, un.k0, un.k1, bad);
      __syncthreads();  // this unit's deposits are done before any flush
    }
  }
  if (curP >= 0) flush_j<DIM>(g, t, tJ, f.j);
  if (bad) atomicOr(err, bad);
}

// Split path, first half: Interpolation + Push (and the walls: the mirror at
// reflecting walls, so that the Projection deposits along the mirrored move);
// saves the start positions.
template <int DIM>
__global__ void __launch_bounds__(kMaxWg<DIM>) k_interp_push(GridDev g, SpArgs sa, Fields f, int *err) {
  extern __shared__ __align__(16) double lds[];
  const int P = blockIdx.x;
  const SpDev &S = sa.s[blockIdx.y];
  const TileGeom t = tile_geom<DIM>(g, P);
  stage_eb<DIM>(g, t, f, lds);
  __syncthreads();
  const int64_t beg = S.off[P], end = S.off[P + 1];
  int bad = 0;
  for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
    double x[3], xi[3], u[3], v[3], F[6];
#pragma unroll
    for (int a = 0; a < DIM; a++) {
      x[a] = S.x[a][i];
      xi[a] = x[a] * g.inv_d[a];
      S.x0[a][i] = x[a];
    }
    if (!in_patch<DIM>(t, xi)) {
      bad |= kErrUnsorted;
      continue;
    }
    u[0] = S.u[0][i];
    u[1] = S.u[1][i];
    u[2] = S.u[2][i];
    const Shapes sh = shapes_at<DIM>(xi, t.org);
    interp6<DIM>(lds, t.TE, t.Tx, t.Txy, sh, F);
    boris(S.alpha, F, u, v);
    double x1[3];
#pragma unroll
    for (int a = 0; a < DIM; a++) x1[a] = x[a] + g.dt * v[a];
    // a particle leaving through a removing wall keeps its position outside
    // the box: the Projection skips it and pic_bin deletes it
    if (g.reflect | g.remove) wall_bc<DIM>(g, x1, u);
#pragma unroll
    for (int a = 0; a < DIM; a++) S.x[a][i] = x1[a];
    S.u[0][i] = u[0];
    S.u[1][i] = u[1];
    S.u[2][i] = u[2];
  }
  if (bad) atomicOr(err, bad);
}

// Split path, second half: Projection from the saved start positions.
template <int DIM>
__global__ void __launch_bounds__(kMaxWg<DIM>) k_project(GridDev g, SpArgs sa, Fields f, int *err) {
  extern __shared__ __align__(16) double lds[];
  const int P = blockIdx.x;
  const SpDev &S = sa.s[blockIdx.y];
  const TileGeom t = tile_geom<DIM>(g, P);
  double *tJ = lds;
  zero_tile<DIM>(tJ, 3 * t.TJ);
  __syncthreads();
  const int64_t beg = S.off[P], end = S.off[P + 1];
  int bad = 0;
  for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
    double xi0[3];
#pragma unroll
    for (int a = 0; a < DIM; a++) xi0[a] = S.x0[a][i] * g.inv_d[a];
    if (!in_patch<DIM>(t, xi0)) {
      bad |= kErrUnsorted;
      continue;
    }
    if (g.remove) {  // left through a removing wall: deleted, deposits nothing
      double x1[3];
#pragma unroll
      for (int a = 0; a < DIM; a++) x1[a] = S.x[a][i];
      if (outside_removing<DIM>(g, x1)) continue;
    }
    const double u0 = S.u[0][i], u1 = S.u[1][i], u2 = S.u[2][i];
    const double gam = sqrt(1.0 + ((u0 * u0 + u1 * u1) + u2 * u2));
    const double ig = 1.0 / gam;
    const double vz = u2 * ig;
    Win win[DIM];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < DIM; a++) {
      const Sh p0 = axis_shape<0>(xi0[a], t.org[a]);
      ok = ok && esk_win(p0, S.x[a][i] * g.inv_d[a], p0.i + 1 + t.org[a], win[a]);
    }
    if (ok)
      deposit<DIM>(g, tJ, t.TJ, t.Jx, t.Jxy, S.q * S.w[i], win, vz);
    else
      bad |= kErrCFL;
  }
  if (bad) atomicOr(err, bad);
  __syncthreads();
  flush_j<DIM>(g, t, tJ, f.j);
}

// Split path pre-BC: wrap, neighbour code and stable rank (per ranking
// segment, as in the fused kernel) of particles that moved at most one cell
// since the last sort.
template <int DIM>
__global__ void __launch_bounds__(kMaxWg<DIM>) k_tag(GridDev g, SpArgs sa, int *err) {
  constexpr int NC = DIM == 2 ? 9 : 27;
  constexpr int CENTER = (NC - 1) / 2;
  const int P = blockIdx.x;
  const SpDev &S = sa.s[blockIdx.y];
  const TileGeom t = tile_geom<DIM>(g, P);
  const int64_t beg = S.off[P], end = S.off[P + 1];
  const int nw = blockDim.x >> 6, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sbase = S.sstart[P], nseg = S.sstart[P + 1] - sbase;
  int bad = 0;
  for (int k = wv; k < nseg; k += nw) {
    const int64_t sb = beg + (int64_t)k * kSeg;
    const int64_t se = sb + kSeg < end ? sb + kSeg : end;
    int run = 0;
    for (int64_t base = sb; base < se; base += 64) {
      const int64_t i = base + lane;
      const bool valid = i < se;
      int code = CENTER;
      if (valid) {
        double x[3];
#pragma unroll
        for (int a = 0; a < DIM; a++) x[a] = S.x[a][i];
        const int c = dest_code<DIM>(g, t.lo, x);
        if (c < 0) {
          bad |= kErrPos;
        } else {
          code = c;
#pragma unroll
          for (int a = 0; a < DIM; a++) S.x[a][i] = x[a];
        }
      }
      const uint32_t rank = wave_rank(valid, code, lane, run);
      if (valid) S.tag[i] = ((uint32_t)code << 27) | rank;
    }
    if (lane < NC) S.cnt[(int64_t)(sbase + k) * kCntRow + lane] = run;
  }
  if (bad) atomicOr(err, bad);
}

// Sort, step 0: per (patch, code), the running count over the patch's
// segments (pre) and the total (tot).  One thread per patch and code.
__global__ void k_seg_prefix(GridDev g, SpArgs sa) {
  const SpDev &S = sa.s[blockIdx.y];
  const int nc = g.nc;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= g.npatch * nc) return;
  const int P = id / nc, c = id - P * nc;
  const int s0 = S.sstart[P], s1 = S.sstart[P + 1];
  int run = 0;
  for (int k = s0; k < s1; k++) {
    const int64_t at = (int64_t)k * nc + c;
    const int v = S.cnt[(int64_t)k * kCntRow + c];
    S.pre[at] = run;
    run += v;
  }
  S.tot[id] = run;
}

// Sort, step 1: for every destination patch D, the particles arriving from
// each (source patch, code) pair, ordered by source patch; gives each pair
// its start inside D and D's total.
__global__ void k_dest_bases(GridDev g, SpArgs sa) {
  const int D = blockIdx.x * blockDim.x + threadIdx.x;
  if (D >= g.npatch) return;
  const SpDev &S = sa.s[blockIdx.y];
  const int nc = g.nc;
  int dc[3];
  patch_coords(g, D, dc);
  int src[27], code[27], num[27];
  for (int c = 0; c < nc; c++) {
    int cc = c, Psrc = 0, mul = 1;
    for (int a = 0; a < 3; a++) {
      int delta = 0;
      if (a < g.dim) {
        delta = cc % 3 - 1;
        cc /= 3;
      }
      int q = dc[a] - delta;
      if (q < 0) q += g.np[a];
      if (q >= g.np[a]) q -= g.np[a];
      Psrc += q * mul;
      mul *= g.np[a];
    }
    // insertion by source patch (stable in c)
    int k = c;
    while (k > 0 && src[k - 1] > Psrc) {
      src[k] = src[k - 1];
      code[k] = code[k - 1];
      num[k] = num[k - 1];
      k--;
    }
    src[k] = Psrc;
    code[k] = c;
    num[k] = S.tot[(int64_t)Psrc * nc + c];
  }
  int64_t run = 0;
  for (int k = 0; k < nc; k++) {
    S.rbase[(int64_t)src[k] * nc + code[k]] = run;
    run += num[k];
  }
  S.in[D] = run;
}

// Sort, step 2: new patch offsets and the new layout's ranking-segment
// starts (one workgroup per species).
__global__ void __launch_bounds__(1024) k_scan_offsets(GridDev g, SpArgs sa) {
  const SpDev &S = sa.s[blockIdx.x];
  __shared__ int64_t part[1024];
  const int n = g.npatch;
  block_scan_1024(S.in, S.noff, n, part);
  for (int P = threadIdx.x; P < n; P += blockDim.x) S.in[P] = (S.in[P] + kSeg - 1) / kSeg;
  __syncthreads();
  block_scan_1024(S.in, S.tmp, n, part);
  for (int P = threadIdx.x; P <= n; P += blockDim.x) S.snext[P] = (int32_t)S.tmp[P];
}

// Sort, step 3: the new slot of every particle: destination start + start
// of (patch, code) inside it + the code's count in the patch's earlier
// segments + the particle's rank in its segment.  A workgroup of kSeg threads
// takes kPlaceSegs consecutive ranking segments (their patches found by
// binary search in the segment starts).  TO_PERM records the slot's source
// in perm[]; otherwise the particle is copied into the other buffer set.
constexpr int kPlaceSegs = 4;

template <bool TO_PERM>
__global__ void __launch_bounds__(kSeg) k_place(GridDev g, SpArgs sa, int *err) {
  const SpDev &S = sa.s[blockIdx.y];
  const int nseg = S.sstart[g.npatch];
  const int seg0 = blockIdx.x * kPlaceSegs;
  if (seg0 >= nseg) return;
  const int nc = g.nc;
  __shared__ int s_patch[kPlaceSegs];
  __shared__ int64_t base[kPlaceSegs][27];
  if (threadIdx.x < kPlaceSegs) {
    const int seg = seg0 + threadIdx.x;
    int lo = 0, hi = g.npatch;  // largest P with sstart[P] <= seg
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (S.sstart[mid] <= seg)
        lo = mid;
      else
        hi = mid;
    }
    s_patch[threadIdx.x] = seg < nseg ? lo : -1;
  }
  __syncthreads();
  if (threadIdx.x < (unsigned)(kPlaceSegs * nc)) {
    const int k = threadIdx.x / nc, c = threadIdx.x - k * nc;
    const int P = s_patch[k];
    if (P >= 0) {
      int pc[3];
      patch_coords(g, P, pc);
      const int D = dest_patch(g, pc, c);
      base[k][c] = S.noff[D] + S.rbase[(int64_t)P * nc + c] + S.pre[(int64_t)(seg0 + k) * nc + c];
    }
  }
  __syncthreads();
  int bad = 0;
  for (int k = 0; k < kPlaceSegs; k++) {
    const int P = s_patch[k];
    if (P < 0) break;
    const int64_t i = S.off[P] + (int64_t)(seg0 + k - S.sstart[P]) * kSeg + threadIdx.x;
    if (i >= S.off[P + 1]) continue;
    const uint32_t tg = S.tag[i];
    const int c = (int)(tg >> 27);
    int64_t dst = S.n;
    if (c < nc) dst = base[k][c] + (int64_t)(tg & ((1u << 27) - 1));
    if (dst >= S.n) {
      bad |= kErrPos;
      continue;
    }
    if (TO_PERM) {
      S.perm[dst] = (int32_t)i;  // the particle moves at the next fused kernel
    } else {
      for (int a = 0; a < g.dim; a++) S.xa[a][dst] = S.x[a][i];
      S.ua[0][dst] = S.u[0][i];
      S.ua[1][dst] = S.u[1][i];
      S.ua[2][dst] = S.u[2][i];
      S.wa[dst] = S.w[i];
      S.ida[dst] = S.id[i];
    }
  }
  if (bad) atomicOr(err, bad);
}

// Sort, step 4: publish the new offsets and segment starts.
__global__ void k_copy_offsets(GridDev g, SpArgs sa) {
  const SpDev &S = sa.s[blockIdx.y];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k <= g.npatch; k += gridDim.x * blockDim.x) {
    S.off[k] = S.noff[k];
    S.sstart[k] = S.snext[k];
  }
}

// Layout after any sort (one workgroup per species): segment starts from the
// patch offsets; in persistent mode also the work units: every patch's full
// units (spc segments each) first, in patch order, then the patches'
// remainder units (fewer segments), so the queue ends with the small units
// and the last workgroups to finish wait less.  Their number goes to
// qctl[2s+1] and a zero ticket to qctl[2s].  Uses the species' in, noff and
// tmp arrays as scratch.
__global__ void __launch_bounds__(1024) k_layout(GridDev g, SpArgs sa, Unit *units, int *qctl) {
  __shared__ int64_t part[1024];
  const int s = blockIdx.x;
  const SpDev &S = sa.s[s];
  const int n = g.npatch;
  for (int P = threadIdx.x; P < n; P += blockDim.x)
    S.in[P] = (S.off[P + 1] - S.off[P] + kSeg - 1) / kSeg;
  __syncthreads();
  block_scan_1024(S.in, S.noff, n, part);
  for (int P = threadIdx.x; P <= n; P += blockDim.x) S.sstart[P] = (int32_t)S.noff[P];
  if (!units) return;
  __syncthreads();
  // full units per patch -> noff (scan); remainder flags -> tmp (scan)
  for (int P = threadIdx.x; P < n; P += blockDim.x) {
    const int nseg = S.sstart[P + 1] - S.sstart[P];
    S.in[P] = nseg / g.spc;
  }
  __syncthreads();
  block_scan_1024(S.in, S.noff, n, part);
  for (int P = threadIdx.x; P < n; P += blockDim.x) {
    const int nseg = S.sstart[P + 1] - S.sstart[P];
    S.in[P] = nseg % g.spc != 0;
  }
  __syncthreads();
  block_scan_1024(S.in, S.tmp, n, part);
  const int64_t nfull = S.noff[n];
  for (int P = threadIdx.x; P < n; P += blockDim.x) {
    const int nseg = S.sstart[P + 1] - S.sstart[P];
    const int nf = nseg / g.spc;
    Unit un;
    un.s = s;
    un.P = P;
    for (int j = 0; j < nf; j++) {
      un.k0 = j * g.spc;
      un.k1 = un.k0 + g.spc;
      units[S.ubase + S.noff[P] + j] = un;
    }
    if (nseg % g.spc) {
      un.k0 = nf * g.spc;
      un.k1 = nseg;
      units[S.ubase + nfull + S.tmp[P]] = un;
    }
  }
  if (threadIdx.x == 0) {
    qctl[2 * s + 1] = (int)(nfull + S.tmp[n]);
    qctl[2 * s] = 0;
  }
}

__global__ void k_zero(double *a, double *b, double *c, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    a[k] = 0.0;
    b[k] = 0.0;
    c[k] = 0.0;
  }
}

// x-bins: patch offsets from bin offsets.
__global__ void __launch_bounds__(256) k_api_offsets(const int64_t *boff, int64_t *off, int64_t n,
                                                     int nb) {
  const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P < n) off[P] = boff[P * nb];
}

}  // namespace

size_t lds_bytes_ipp(const GridDev &g) { return tile_eb_bytes(g) + tile_j_bytes(g); }

hipError_t launch_zero(double *const j[3], int64_t ncell, hipStream_t st) {
  const int blocks = (int)std::min<int64_t>((ncell + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, j[0], j[1], j[2], ncell);
  return hipGetLastError();
}

template <int DIM, bool GATHER, bool WALLS>
void launch_ipp_t(const GridDev &g, const SpArgs &sa, const Fields &f, int *err, int wg,
                  size_t lds, hipStream_t st) {
  if (DIM == 3 || sa.jt)
    (void)hipFuncSetAttribute((const void *)k_ipp<DIM, GATHER, WALLS>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_ipp<DIM, GATHER, WALLS>), dim3(g.npatch, sa.nsp), dim3(wg), lds, st, g,
                     sa, f, err);
}

int det_waves(const GridDev &g, int wg) {
  const size_t room = (size_t)160 * 1024 - 4352 - tile_eb_bytes(g);
  const int fit = (int)(room / tile_j_bytes(g));
  return std::max(1, std::min(wg / 64, fit));
}

hipError_t launch_j_gather(const GridDev &g, const SpArgs &sa, double *const j[3], hipStream_t st) {
  const Fields f = mkfields(nullptr, nullptr, j);
  const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
  const int blocks = (int)std::min<int64_t>((ncell + 255) / 256, 8192);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_j_gather<2>, dim3(blocks), dim3(256), 0, st, g, sa, f);
  else
    hipLaunchKernelGGL(k_j_gather<3>, dim3(blocks), dim3(256), 0, st, g, sa, f);
  return hipGetLastError();
}

hipError_t launch_ipp(const GridDev &g, const SpArgs &sa, const double *const e[3],
                      const double *const b[3], double *const j[3], int *err, int wg,
                      hipStream_t st) {
  const Fields f = mkfields(e, b, j);
  // deterministic mode: one J tile per wave
  const size_t lds = sa.jt ? tile_eb_bytes(g) + (size_t)(wg / 64) * tile_j_bytes(g)
                           : lds_bytes_ipp(g);
  const int v = (g.dim == 3 ? 4 : 0) + (sa.gather ? 2 : 0) + (has_walls(g) ? 1 : 0);
  switch (v) {
    case 0: launch_ipp_t<2, false, false>(g, sa, f, err, wg, lds, st); break;
    case 1: launch_ipp_t<2, false, true>(g, sa, f, err, wg, lds, st); break;
    case 2: launch_ipp_t<2, true, false>(g, sa, f, err, wg, lds, st); break;
    case 3: launch_ipp_t<2, true, true>(g, sa, f, err, wg, lds, st); break;
    case 4: launch_ipp_t<3, false, false>(g, sa, f, err, wg, lds, st); break;
    case 5: launch_ipp_t<3, false, true>(g, sa, f, err, wg, lds, st); break;
    case 6: launch_ipp_t<3, true, false>(g, sa, f, err, wg, lds, st); break;
    default: launch_ipp_t<3, true, true>(g, sa, f, err, wg, lds, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_interp_push(const GridDev &g, const SpArgs &sa, const double *const e[3],
                              const double *const b[3], int *err, int wg, hipStream_t st) {
  const Fields f = mkfields(e, b, nullptr);
  const dim3 grid(g.npatch, sa.nsp);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_interp_push<2>, grid, dim3(wg), tile_eb_bytes(g), st, g, sa, f, err);
  else
    hipLaunchKernelGGL(k_interp_push<3>, grid, dim3(wg), tile_eb_bytes(g), st, g, sa, f, err);
  return hipGetLastError();
}

hipError_t launch_project(const GridDev &g, const SpArgs &sa, double *const j[3], int *err, int wg,
                          hipStream_t st) {
  const Fields f = mkfields(nullptr, nullptr, j);
  const dim3 grid(g.npatch, sa.nsp);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_project<2>, grid, dim3(wg), tile_j_bytes(g), st, g, sa, f, err);
  else
    hipLaunchKernelGGL(k_project<3>, grid, dim3(wg), tile_j_bytes(g), st, g, sa, f, err);
  return hipGetLastError();
}

hipError_t launch_tag(const GridDev &g, const SpArgs &sa, int *err, int wg, hipStream_t st) {
  const dim3 grid(g.npatch, sa.nsp);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_tag<2>, grid, dim3(wg), 0, st, g, sa, err);
  else
    hipLaunchKernelGGL(k_tag<3>, grid, dim3(wg), 0, st, g, sa, err);
  return hipGetLastError();
}

hipError_t launch_rebin(const GridDev &g, const SpArgs &sa, int *err, int64_t maxseg, bool to_perm,
                        hipStream_t st) {
  const int pc = g.npatch * g.nc;
  hipLaunchKernelGGL(k_seg_prefix, dim3((pc + 255) / 256, sa.nsp), dim3(256), 0, st, g, sa);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dest_bases, dim3((g.npatch + 127) / 128, sa.nsp), dim3(128), 0, st, g, sa);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_offsets, dim3(sa.nsp), dim3(1024), 0, st, g, sa);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const dim3 grid((unsigned)((maxseg + kPlaceSegs - 1) / kPlaceSegs), sa.nsp);
  if (to_perm)
    hipLaunchKernelGGL(k_place<true>, grid, dim3(kSeg), 0, st, g, sa, err);
  else
    hipLaunchKernelGGL(k_place<false>, grid, dim3(kSeg), 0, st, g, sa, err);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_copy_offsets, dim3((g.npatch + 256) / 256, sa.nsp), dim3(256), 0, st, g, sa);
  return hipGetLastError();
}

hipError_t launch_api_offsets(const int64_t *boff, int64_t *off, int64_t npatch, int nb,
                              hipStream_t st) {
  const int64_t n = npatch + 1;
  hipLaunchKernelGGL(k_api_offsets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, boff, off,
                     n, nb);
  return hipGetLastError();
}

hipError_t launch_layout(const GridDev &g, const SpArgs &sa, Unit *units, int *qctl,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_layout, dim3(sa.nsp), dim3(1024), 0, st, g, sa, units, qctl);
  return hipGetLastError();
}

template <int DIM, bool GATHER, bool WALLS>
int blocks_per_cu(int wg, size_t lds) {
  if (DIM == 3)
    (void)hipFuncSetAttribute((const void *)k_ipp_persistent<DIM, GATHER, WALLS>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_ipp_persistent<DIM, GATHER, WALLS>, wg,
                                                   lds) != hipSuccess)
    return 1;
  return n;
}

template <int DIM, bool WALLS>
int blocks_per_cu_both(int wg, size_t lds) {
  return std::min(blocks_per_cu<DIM, true, WALLS>(wg, lds), blocks_per_cu<DIM, false, WALLS>(wg, lds));
}

int persistent_grid(const GridDev &g, int wg) {
  const size_t lds = lds_bytes_ipp(g);
  int per_cu = g.dim == 2 ? (has_walls(g) ? blocks_per_cu_both<2, true>(wg, lds)
                                       : blocks_per_cu_both<2, false>(wg, lds))
                          : (has_walls(g) ? blocks_per_cu_both<3, true>(wg, lds)
                                       : blocks_per_cu_both<3, false>(wg, lds));
  int dev = 0, ncu = 0;
  if (per_cu < 1) per_cu = 1;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      ncu < 1)
    ncu = 1;
  return per_cu * ncu;
}

template <int DIM, bool GATHER, bool WALLS>
void launch_pers_t(const GridDev &g, const SpArgs &sa, const Fields &f, int *err,
                   const Unit *units, int *qctl, int grid, int wg, size_t lds, hipStream_t st) {
  if (DIM == 3)
    (void)hipFuncSetAttribute((const void *)k_ipp_persistent<DIM, GATHER, WALLS>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_ipp_persistent<DIM, GATHER, WALLS>), dim3(grid), dim3(wg), lds, st, g, sa,
                     f, err, units, qctl);
}

hipError_t launch_ipp_persistent(const GridDev &g, const SpArgs &sa, const double *const e[3],
                                 const double *const b[3], double *const j[3], int *err,
                                 const Unit *units, int *qctl, int grid, int wg, hipStream_t st) {
  const Fields f = mkfields(e, b, j);
  const size_t lds = lds_bytes_ipp(g);
  const int v = (g.dim == 3 ? 4 : 0) + (sa.gather ? 2 : 0) + (has_walls(g) ? 1 : 0);
  switch (v) {
    case 0: launch_pers_t<2, false, false>(g, sa, f, err, units, qctl, grid, wg, lds, st); break;
    case 1: launch_pers_t<2, false, true>(g, sa, f, err, units, qctl, grid, wg, lds, st); break;
    case 2: launch_pers_t<2, true, false>(g, sa, f, err, units, qctl, grid, wg, lds, st); break;
    case 3: launch_pers_t<2, true, true>(g, sa, f, err, units, qctl, grid, wg, lds, st); break;
    case 4: launch_pers_t<3, false, false>(g, sa, f, err, units, qctl, grid, wg, lds, st); break;
    case 5: launch_pers_t<3, false, true>(g, sa, f, err, units, qctl, grid, wg, lds, st); break;
    case 6: launch_pers_t<3, true, false>(g, sa, f, err, units, qctl, grid, wg, lds, st); break;
    default: launch_pers_t<3, true, true>(g, sa, f, err, units, qctl, grid, wg, lds, st); break;
  }
  return hipGetLastError();
}

}  // namespace pic
