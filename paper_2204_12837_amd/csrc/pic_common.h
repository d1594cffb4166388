// Internal declarations shared by the host side of the library and its
// kernels.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int kMaxSpecies = 8;
constexpr int kSeg = 256;   // particles per ranking segment (multiple of 64)
constexpr int kCntRow = 64; // row length of the per-segment code counts (one per lane)
constexpr int kErrCFL = 1;  // device error bits
constexpr int kErrPos = 2;
constexpr int kErrCap = 4;  // the slab layout does not fit the particle buffers
constexpr int kErrUnsorted = 8;  // a particle outside the patch its offsets give it

// Grid geometry as the kernels see it.  All derived values (inverse cell
// sizes, box lengths, Esirkepov factors) are computed once on the host.
struct GridDev {
  int dim;
  int n[3];       // cells per axis (1 for an absent axis)
  int patch[3];   // patch size per axis (1 for an absent axis)
  int np[3];      // patches per axis
  int npatch;     // total patches
  int nc;         // neighbour codes: 3^dim
  int spc;        // persistent mode: ranking segments per work unit
  double inv_d[3];
  double L[3];    // n * d
  double dt;
  double d_over_dt[3];
  int reflect;    // bit a set: reflecting particle walls at 0 and L on axis a
  int remove;     // bit a set: removing particle walls at 0 and L on axis a
};

// Neighbour code of a particle deleted at a removing wall (no destination).
constexpr int kGone = 31;

// Whether any axis has particle walls (the kernels' WALLS instances).
__host__ __device__ inline bool has_walls(const GridDev &g) { return (g.reflect | g.remove) != 0; }

// Whether x lies outside [0, L) on an axis with removing walls.
template <int DIM>
__device__ __forceinline__ bool outside_removing(const GridDev &g, const double x[3]) {
  bool out = false;
#pragma unroll
  for (int a = 0; a < DIM; a++)
    if ((g.remove >> a) & 1) out = out || !(x[a] >= 0.0 && x[a] < g.L[a]);
  return out;
}

// pre-BC at walls.  A pushed position x1 outside [0, L) on an axis with
// removing walls marks the particle for deletion: -1 is returned and nothing
// changes (the particle deposits no current and the synchronisation drops
// it).  Otherwise, on an axis with reflecting walls, a position that left
// [0, L) is mirrored back inside about the wall it crossed (x -> -x or
// x -> 2L - x; both exact in floating point, as x and 2L lie within a factor
// two of each other) and the momentum component along that axis changes
// sign.  The one position that lands on L itself (x1 = L) goes to the
// largest double below L.  Returns the mirrored axes as bits.
template <int DIM>
__device__ __forceinline__ int wall_bc(const GridDev &g, double x1[3], double u[3]) {
  if (g.remove && outside_removing<DIM>(g, x1)) return -1;
  int hit = 0;
#pragma unroll
  for (int a = 0; a < DIM; a++) {
    if (!((g.reflect >> a) & 1)) continue;
    double v = x1[a];
    if (v < 0.0) {
      v = -v;
    } else if (v >= g.L[a]) {
      v = 2.0 * g.L[a] - v;
      if (v >= g.L[a]) v = nextafter(g.L[a], 0.0);
    } else {
      continue;
    }
    x1[a] = v;
    u[a] = -u[a];
    hit |= 1 << a;
  }
  return hit;
}

// One species as the kernels see it (device pointers).
struct SpDev {
  double alpha;   // (q/m) * (dt/2)
  double q;
  int64_t n;
  double *x[3], *u[3], *w;
  int64_t *id;
  double *xa[3], *ua[3], *wa;  // sort target
  int64_t *ida;
  int64_t *off;     // [npatch+1] current patch offsets
  int64_t *noff;    // [npatch+1] scratch: offsets after the sort
  uint32_t *tag;    // [capacity] neighbour code << 27 | rank inside (segment, code)
  int32_t *sstart;  // [npatch+1] first ranking segment of each patch (kSeg particles each)
  int32_t *cnt;     // [max segments * kCntRow] particles per (segment, code)
  int32_t *pre;     // [max segments * nc] earlier segments' count of the code, same patch
  int32_t *tot;     // [npatch * nc] particles per (patch, code)
  int64_t *rbase;   // [npatch * nc] start of (patch, code) inside its destination
  int64_t *in;      // [npatch] particles arriving in each destination patch
  double *x0[3];    // saved start-of-step positions (split path)
  int32_t *snext;   // [npatch+1] segment starts of the layout after the sort
  int64_t *tmp;     // [npatch+1] scan scratch
  int32_t *perm;    // [capacity] gather index: slot j of the next layout takes the
                    // particle at perm[j] of the current one
  int32_t ubase;    // persistent mode: first work unit of this species
};

// A persistent-mode work unit of species s and patch P: ranking segments
// [k0, k1) in the dense layout, particles [k0, k1) of the slab in the slab
// layout.
struct Unit {
  int32_t s, P, k0, k1;
};

// One species in the slab layout of a pic_step call: patch P owns slots
// [sb[P], sb[P] + cap[P]) of the second buffer set, cnt[P] of them live.
struct SlabDev {
  double alpha, q;
  int64_t capacity;
  double *x[3], *u[3], *w;      // dense layout (first buffer set): the call's input and
  int64_t *id;                  // output, and scratch of a new slab plan
  double *xs[3], *us[3], *ws;   // slabs (second buffer set)
  int64_t *ids;
  int64_t *off;                 // [npatch+1] dense patch offsets
  int64_t *sb, *sb2;            // [npatch+1] slab starts (current, new plan)
  int32_t *cap, *cap2;          // [npatch] slab room (current, new plan)
  int32_t *cnt, *cnt2;          // [npatch] live particles (after the step, after departures)
  int32_t *arr, *arr2;          // [npatch] arrivals of the step, arrivals of a new plan
  int32_t *dep;                 // [npatch] departures of the step
  int32_t *porder;              // [npatch] persistent mode, one species: the patches in the
                                // departures kernel's order (crowded ones first)
  uint8_t *code;                // [capacity] neighbour code of each slab slot
  int32_t *hole;                // [capacity] hole lists (patch P's at sb[P])
  double *ox[3], *ou[3], *ow;   // outbox of departures [capacity], patch P's
  int64_t *oid;                 // from sb[P]
  int32_t *odest;               // destination patch of each outbox entry
  int32_t *ctl;                 // [2] unused, overflow state (0 none, 1 new plan, 2 fatal)
  int64_t *tmp;                 // [npatch+1] scan scratch
  int32_t ubase;                // persistent mode: first work unit of this species
};

// One traced work item of a fused-kernel launch (PIC_FLAG_TRACE): its
// patch, unit (persistent mode; the species in per-patch mode), workgroup,
// and start and end times of the device's constant 100 MHz clock.  The
// buffer holds the count of the last launch's records in its first word,
// then the records from byte 32.
struct TraceRec {
  int32_t patch, unit, block, species;
  uint64_t t0, t1;
};

struct SlabArgs {
  int nsp;
  SlabDev s[kMaxSpecies];
  uint64_t *trace;  // trace buffer, or null when tracing is off
  int from_dense;   // first step of a call: the fused kernel reads each patch's
                    // particles from the dense layout (offsets off) and writes
                    // them, updated, into the slabs (with weights and ids)
};
static_assert(sizeof(SlabArgs) <= 4096, "kernel argument block too large");

// Slab-layout launchers (pic_slab.hip).
// copy = false: only the slab plan (the caller fills the slabs).
hipError_t launch_slab_begin(const GridDev &g, const SlabArgs &sa, int *err, hipStream_t st,
                             bool copy = true);
hipError_t launch_ipp_slab(const GridDev &g, const SlabArgs &sa, const double *const e[3],
                           const double *const b[3], double *const j[3], int *err, int wg,
                           hipStream_t st);
hipError_t launch_ipp_slab_persistent(const GridDev &g, const SlabArgs &sa,
                                      const double *const e[3], const double *const b[3],
                                      double *const j[3], int *err, const Unit *units,
                                      int *qctl, int grid, int wg, hipStream_t st);
int slab_persistent_blocks_per_cu(const GridDev &g, int wg);
// Departures left by the fused kernel, arrivals, counts (and, on an
// overflow, a new slab plan); with units != nullptr (persistent mode) also
// the next step's work units of chunk particles.
hipError_t launch_exchange(const GridDev &g, const SlabArgs &sa, int *err, Unit *units,
                           int *qctl, int chunk, hipStream_t st);
hipError_t launch_slab_units(const GridDev &g, const SlabArgs &sa, int chunk, Unit *units,
                             int *qctl, hipStream_t st);
hipError_t launch_slab_end(const GridDev &g, const SlabArgs &sa, hipStream_t st);

// Adjoint (reverse-mode derivative) of a segment of 2D steps.
constexpr int kAdjMaxSteps = 8;  // steps per recomputed segment

struct AdjSp {
  double alpha, q;
  int64_t n;        // particles in the checkpoint arrays
  int64_t nid;      // length of the cotangent arrays (ids lie in [0, nid))
  const double *x[3], *u[3], *w;
  const int64_t *id;
  const int64_t *off;     // [npatch+1] patch offsets if the checkpoint is sorted, else null
  double *xb[3], *ub[3];  // cotangents of the state, indexed by id
};

struct AdjArgs {
  int nsp;
  AdjSp s[kMaxSpecies];
};

hipError_t launch_adjoint(const GridDev &g, const AdjArgs &aa, const double *const e[3],
                          const double *const b[3], const double *const jb[3],
                          double *const eb[3], double *const bb[3], int nsteps, int with_dep,
                          int *err, hipStream_t st);


struct SpArgs {
  int nsp;
  int gather;  // fused kernel: read particle j from perm[j] of the other buffer set
               // (the layout the previous sort computed) and write slot j
  SpDev s[kMaxSpecies];
  double *jt;  // PIC_FLAG_DETERMINISTIC: each (species, patch)'s J tile
               // [nsp][npatch][3][TJ], summed into J by k_j_gather; null otherwise
};

// Launch helpers (implemented in pic_kernels.hip).  Each returns the HIP
// error of its launch.
hipError_t launch_zero(double *const j[3], int64_t ncell, hipStream_t st);
hipError_t launch_ipp(const GridDev &g, const SpArgs &sa, const double *const e[3],
                      const double *const b[3], double *const j[3], int *err, int wg,
                      hipStream_t st);
// PIC_FLAG_DETERMINISTIC: waves of the per-patch fused kernel whose private
// J tiles fit beside the E/B tile (at most wg / 64), and J <- the tiles in
// sa.jt summed per node in a fixed order.
int det_waves(const GridDev &g, int wg);
hipError_t launch_j_gather(const GridDev &g, const SpArgs &sa, double *const j[3], hipStream_t st);
// Persistent variant: `grid` workgroups pop units from units[0 .. qctl[1]) with
// the ticket qctl[0] (reset by launch_layout).
hipError_t launch_ipp_persistent(const GridDev &g, const SpArgs &sa, const double *const e[3],
                                 const double *const b[3], double *const j[3], int *err,
                                 const Unit *units, int *qctl, int grid, int wg, hipStream_t st);
int persistent_grid(const GridDev &g, int wg);
// Segment starts (and, if units != nullptr, the work-unit list, its length in
// qctl[1] and a zero ticket in qctl[0]) from the current patch offsets.
hipError_t launch_layout(const GridDev &g, const SpArgs &sa, Unit *units, int *qctl,
                         hipStream_t st);
// x-bins: off[P] = boff[nb * P] for P in [0, npatch] (the offsets of the
// patches, each made of nb consecutive bins).
hipError_t launch_api_offsets(const int64_t *boff, int64_t *off, int64_t npatch, int nb,
                              hipStream_t st);
hipError_t launch_interp_push(const GridDev &g, const SpArgs &sa, const double *const e[3],
                              const double *const b[3], int *err, int wg, hipStream_t st);
hipError_t launch_project(const GridDev &g, const SpArgs &sa, double *const j[3], int *err,
                          int wg, hipStream_t st);
hipError_t launch_tag(const GridDev &g, const SpArgs &sa, int *err, int wg, hipStream_t st);
// Counting sort from the tags: with to_perm the particles stay where they are
// and perm[] records the new layout (applied by the next gathering fused
// kernel); otherwise they are copied into the other buffer set.  maxseg
// bounds the number of ranking segments of any species.
hipError_t launch_rebin(const GridDev &g, const SpArgs &sa, int *err, int64_t maxseg, bool to_perm,
                        hipStream_t st);

// General sort (pic_sort.hip): wrap + key + stable radix sort of unsorted
// input, gather into the second buffer set, patch offsets.
struct SortScratch {
  uint32_t *keys = nullptr, *keys_out = nullptr;
  uint32_t *idx = nullptr, *idx_out = nullptr;
  uint32_t *hist = nullptr;  // per radix pass: digit counts of every tile
  int64_t cap = 0;
};
hipError_t general_sort(const GridDev &g, SpDev &s, SortScratch &scr, int *err, hipStream_t st);
void free_sort_scratch(SortScratch &scr);
// x-bins (pic_sort.hip): stable counting sort of the n particles sorted by
// API patch (offsets off_api, npatch_api patches of nb bins each) into bin
// order in the second buffer set; writes the bin offsets to s.off and uses
// s.sstart, s.cnt, s.tmp, s.in and s.noff as scratch (sized for the bins and
// a capacity of at least n).  For at most 256 bins per patch
// (bin_order_supported).
bool bin_order_supported(int nb);
hipError_t bin_order(const GridDev &g, SpDev &s, const int64_t *off_api, int64_t npatch_api, int nb,
                     int64_t n, int *err, hipStream_t st);
// Its two halves: bin counts and offsets (s.off), then the placement with
// dst0[bin] as each bin's first slot in the second buffer set (s.off for
// the dense bin order, the slab starts for pic_step's slab layout, whose
// fit flag ctl[1] is checked first; ctl may be null).
hipError_t bin_count(const GridDev &g, SpDev &s, const int64_t *off_api, int64_t npatch_api, int nb,
                     int64_t n, int *err, hipStream_t st);
hipError_t bin_place(const GridDev &g, SpDev &s, const int64_t *off_api, int64_t npatch_api, int nb,
                     int64_t n, const int64_t *dst0, const int32_t *ctl, hipStream_t st);

size_t lds_bytes_ipp(const GridDev &g);

}  // namespace pic
