// C ABI of the library (declared in include/pic.h): configuration checks,
// context lifetime, scratch management and the launch sequences of the
// entry points.  All arithmetic on particles and fields happens in the
// kernels; this file only validates, sizes and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "pic.h"
#include "pic_common.h"
#include "pic_fields.h"

using namespace pic;

// Device scratch of pic_step_noalloc: one copy per GPU, held from the
// library's load on that GPU until the process ends.  In host code this name
// stands for a host-side symbol, not a device address: pic_init looks up
// the address of the current GPU's copy with hipGetSymbolAddress once per
// device, and only that address is ever passed to kernels.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of the static scratch (the device must
// be current); nullptr if the lookup fails.
void *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_noalloc_ptr[device] = p;
  }
  return g_noalloc_ptr[device];
}

struct SpScratch {
  int64_t cap = 0;      // particle capacity the buffers below were sized for
  int64_t maxseg = 0;   // ranking segments the count arrays hold
  uint32_t *tag = nullptr;
  int32_t *sstart = nullptr, *cnt = nullptr, *pre = nullptr, *tot = nullptr;
  int32_t *snext = nullptr, *perm = nullptr;
  int64_t *tmp = nullptr;
  int64_t *rbase = nullptr, *in = nullptr, *noff = nullptr;
  int64_t x0cap = 0;
  double *x0[3] = {nullptr, nullptr, nullptr};
  int64_t ubase = 0, maxunits = 0;  // persistent mode: place in the unit list
};

// Slab-layout scratch of one species (the per-patch arrays, the outbox and
// the control words; the code and hole lists reuse the sort's tag and
// permutation arrays).
struct SlabScratch {
  int64_t cap = 0;  // particle capacity the outbox was sized for
  int64_t *sb = nullptr, *sb2 = nullptr;
  int32_t *room = nullptr, *room2 = nullptr, *cnt = nullptr, *cnt2 = nullptr;
  int32_t *arr = nullptr, *arr2 = nullptr, *dep = nullptr, *ctl = nullptr, *porder = nullptr;
  double *ox[3] = {nullptr, nullptr, nullptr}, *ou[3] = {nullptr, nullptr, nullptr};
  double *ow = nullptr;
  int64_t *oid = nullptr;
  int32_t *odest = nullptr;
};

// Static LDS budget kept free beside the tiles when a configuration is
// validated: 2 x 2048 words (the per-patch fused kernel's departure bitmap
// and prefix take 2 x 512 of them) plus control words and slack, so the
// tile sizes accepted leave room to grow those arrays.
constexpr size_t kStaticLds = 2 * 2048 * 4 + 256;

}  // namespace

// Event pairs around timed launches, per kernel class.
struct Timing {
  bool on = false;
  std::vector<hipEvent_t> pool;   // reusable events
  size_t used = 0;
  std::vector<std::pair<int, size_t>> marks;  // (kernel class, index of start event)
  double ms[PIC_KERNEL_COUNT] = {0};
  int64_t launches[PIC_KERNEL_COUNT] = {0};
};

// Steps one captured slab-layout graph holds (a call replays it, then a
// one-step graph for the remainder): fewer graph launches per step.
constexpr int kGraphSteps = 8;

// A captured graph and the pointers/counts it was captured with.
struct GraphCache {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<uintptr_t> key;
};

struct pic_ctx {
  pic_config cfg;
  Timing tm;
  GraphCache gc[2];  // one per buffer parity (the step swaps the buffer sets)
  int gc_next = 0;
  hipStream_t cap_stream = nullptr;  // stream used only to capture graphs
  GridDev g;
  int device = 0;
  int wg = 256;           // threads per workgroup of the slab-layout kernels
  int wgd = 256;          // ... of the dense-layout kernels (at most 512 in 3D)
  int *err_dev = nullptr;
  bool poisoned = false;
  bool moved = false;   // pic_interp_push ran since the last sort
  int moved_nsp = 0;
  char msg[512] = {0};
  SpScratch sp[kMaxSpecies];
  SortScratch sort[kMaxSpecies];
  Unit *units = nullptr;  // persistent mode: work-unit list of all species
  int64_t units_cap = 0;
  int *qctl = nullptr;    // per species: ticket, number of units
  int pgrid = 0;          // persistent grid size
  SlabScratch slab[kMaxSpecies];
  GraphCache slab_gc[2];  // slab-layout graphs: [0] kGraphSteps steps, [1] one step
  int pgrid_slab = 0;     // persistent grid size of the slab-layout kernel
  // x-bins: the kernels' "patches" (GridDev) are the bins; with more than one
  // bin per patch the bin offsets live here and the caller's offset arrays
  // receive every nb-th entry.
  int nb = 1;                           // bins per patch
  int64_t npatch_api = 0;               // patches of the configuration
  int64_t *boff[kMaxSpecies] = {};      // [bins + 1] per species
  // pic_cycle: every step ends with a field step on the step's fields
  bool cycle = false;
  // PIC_FLAG_RESIDENT: the particles of these species live in their slabs
  // (second buffer set) since the last pic_step; the first set and the
  // offsets are stale until resident_flush
  bool resident = false;
  int32_t res_nsp = 0;
  pic_species res_sp[kMaxSpecies];
  YeeArgs yee{};
  // pic_step_noalloc: this device's static scratch; layout_stale: the
  // segment starts and work units in sp[] do not describe the particles
  // (pic_step_noalloc sorted them with its own scratch)
  void *noalloc = nullptr;
  bool layout_stale = false;
  // PIC_FLAG_TRACE: header (record count of the last launch) and records
  uint64_t *trace = nullptr;
  int64_t trace_cap = 0;  // records
  // PIC_FLAG_DETERMINISTIC: every (species, patch)'s J tile
  double *jt = nullptr;
  size_t jt_cap = 0;  // doubles
};

static_assert(sizeof(pic_trace_record) == sizeof(TraceRec), "trace record layout");

namespace {

void set_msg(char *buf, size_t len, const char *fmt, ...) {
  if (!buf || !len) return;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, len, fmt, ap);
  va_end(ap);
}

pic_status fail(pic_ctx *c, pic_status st, const char *fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->msg, sizeof(c->msg), fmt, ap);
    va_end(ap);
  }
  return st;
}

pic_status hip_fail(pic_ctx *c, hipError_t e, const char *what) {
  return fail(c, PIC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int axes(const pic_config *c) { return c->dim == 3 ? 3 : 2; }

size_t tiles_bytes(const pic_config *c, int bx) {
  size_t te = 1, tj = 1;
  for (int a = 0; a < axes(c); a++) {
    const int p = a == 0 ? bx : c->patch[a];
    te *= (size_t)(p + 3);
    tj *= (size_t)(p + 5);
  }
  return (6 * te + 3 * tj) * sizeof(double);
}

constexpr size_t kLdsMax = 160 * 1024;  // LDS of one CU

bool tiles_fit(const pic_config *c, int bx) { return tiles_bytes(c, bx) + kStaticLds <= kLdsMax; }

// Width of the x-bins: bin_x if set, else patch[0] or its widest divisor
// whose tiles fit (0 if none does).
int choose_bin(const pic_config *c) {
  if (c->bin_x > 0) return c->bin_x;
  for (int b = c->patch[0]; b >= 1; b--)
    if (c->patch[0] % b == 0 && tiles_fit(c, b)) return b;
  return 0;
}

// Default threads per workgroup of the slab-layout kernels: 1024 in 3D; in
// 2D 256 when the LDS admits three or more workgroups per CU, else enough
// threads for 16 waves per CU (the 128-register budget): 512 for two, 1024
// for one.  The per-patch fused kernel's static LDS (departure bitmap and
// prefix) is about 4 KB.
int default_wg(const pic_config *c) {
  if (c->dim == 3) return 1024;
  const size_t per_wg = tiles_bytes(c, choose_bin(c)) + 4352;
  const size_t per_cu = kLdsMax / per_wg;
  return per_cu >= 3 ? 256 : per_cu == 2 ? 512 : 1024;
}

// Derived geometry of the kernels, whose patches are the x-bins; cfg must
// be valid.
GridDev make_grid(const pic_config *c) {
  GridDev g{};
  g.dim = c->dim;
  g.npatch = 1;
  g.nc = c->dim == 3 ? 27 : 9;
  const int bx = choose_bin(c);
  for (int a = 0; a < 3; a++) {
    const bool on = a < c->dim;
    g.n[a] = on ? c->n[a] : 1;
    g.patch[a] = on ? (a == 0 ? bx : c->patch[a]) : 1;
    g.np[a] = g.n[a] / g.patch[a];
    g.npatch *= g.np[a];
    const double d = on ? c->d[a] : 1.0;
    g.inv_d[a] = 1.0 / d;
    g.L[a] = (double)g.n[a] * d;
    g.d_over_dt[a] = d / c->dt;
  }
  g.dt = c->dt;
  for (int a = 0; a < c->dim; a++) {
    if (c->particle_bc[a] == PIC_BC_REFLECT) g.reflect |= 1 << a;
    if (c->particle_bc[a] == PIC_BC_REMOVE) g.remove |= 1 << a;
  }
  return g;
}

pic_status check_species(pic_ctx *c, const pic_species *sp, int32_t nsp, bool need_sorted) {
  (void)need_sorted;
  if (!c) return PIC_ERR_ARG;
  if (c->poisoned) return fail(c, PIC_ERR_STATE, "context unusable after a device error");
  if (!sp || nsp < 1) return fail(c, PIC_ERR_ARG, "no species");
  if (nsp > kMaxSpecies) return fail(c, PIC_ERR_CAPACITY, "at most %d species", kMaxSpecies);
  for (int s = 0; s < nsp; s++) {
    const pic_species &p = sp[s];
    if (p.n < 0 || p.capacity < 0) return fail(c, PIC_ERR_ARG, "species %d: negative size", s);
    if (p.n > p.capacity)
      return fail(c, PIC_ERR_CAPACITY, "species %d: n=%lld above capacity=%lld", s,
                  (long long)p.n, (long long)p.capacity);
    if (p.n >= (int64_t)1 << 29)
      return fail(c, PIC_ERR_CAPACITY, "species %d: n must stay below 2^29", s);
    if (!(p.m > 0) || !std::isfinite(p.m) || !std::isfinite(p.q))
      return fail(c, PIC_ERR_ARG, "species %d: bad charge or mass", s);
    for (int a = 0; a < c->cfg.dim; a++)
      if (!p.x[a] || !p.x_alt[a]) return fail(c, PIC_ERR_ARG, "species %d: null position", s);
    for (int a = 0; a < 3; a++)
      if (!p.u[a] || !p.u_alt[a]) return fail(c, PIC_ERR_ARG, "species %d: null momentum", s);
    if (!p.w || !p.w_alt || !p.id || !p.id_alt || !p.offset)
      return fail(c, PIC_ERR_ARG, "species %d: null weight/id/offset array", s);
  }
  return PIC_OK;
}

template <typename T>
hipError_t realloc_dev(T *&p, size_t n) {
  if (p) {
    hipError_t e = hipFree(p);
    if (e != hipSuccess) return e;
    p = nullptr;
  }
  return hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T));
}

// Per-species scratch for the sort (and, if x0, the saved positions); in
// persistent mode also the work-unit list.
pic_status ensure_scratch(pic_ctx *c, const pic_species *sp, int32_t nsp, bool x0,
                          hipStream_t st) {
  bool synced = false;
  bool units_changed = false;
  for (int s = 0; s < nsp; s++) {
    SpScratch &S = c->sp[s];
    const int64_t cap = sp[s].capacity;
    const bool need_tag = cap > S.cap || !S.tag;
    const bool need_x0 = x0 && (cap > S.x0cap || !S.x0[0]);
    if ((need_tag || need_x0) && !synced) {
      hipError_t e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
      synced = true;
    }
    if (need_tag) {
      hipError_t e;
      const size_t np = (size_t)c->g.npatch, nc = (size_t)c->g.nc;
      const int64_t maxseg = (int64_t)np + cap / kSeg + 1;
      if ((e = realloc_dev(S.tag, (size_t)cap)) != hipSuccess) return hip_fail(c, e, "hipMalloc");
      if ((e = realloc_dev(S.perm, (size_t)cap)) != hipSuccess) return hip_fail(c, e, "hipMalloc");

      if ((e = realloc_dev(S.cnt, (size_t)maxseg * kCntRow)) != hipSuccess)
        return hip_fail(c, e, "hipMalloc");
      if ((e = realloc_dev(S.pre, (size_t)maxseg * nc)) != hipSuccess)
        return hip_fail(c, e, "hipMalloc");
      if (!S.rbase) {
        if ((e = realloc_dev(S.sstart, np + 1)) != hipSuccess) return hip_fail(c, e, "hipMalloc");
        if ((e = realloc_dev(S.snext, np + 1)) != hipSuccess) return hip_fail(c, e, "hipMalloc");
        if ((e = realloc_dev(S.tmp, np + 1)) != hipSuccess) return hip_fail(c, e, "hipMalloc");
        if ((e = realloc_dev(S.tot, np * nc)) != hipSuccess) return hip_fail(c, e, "hipMalloc");
        if ((e = realloc_dev(S.rbase, np * nc)) != hipSuccess) return hip_fail(c, e, "hipMalloc");
        if ((e = realloc_dev(S.in, np)) != hipSuccess) return hip_fail(c, e, "hipMalloc");
        if ((e = realloc_dev(S.noff, np + 1)) != hipSuccess) return hip_fail(c, e, "hipMalloc");
      }
      S.cap = cap;
      S.maxseg = maxseg;
      const int64_t mu = (int64_t)np + (maxseg + c->g.spc - 1) / c->g.spc + 1;
      if (mu != S.maxunits) units_changed = true;
      S.maxunits = mu;
    }
    if (need_x0) {
      for (int a = 0; a < c->cfg.dim; a++) {
        hipError_t e = realloc_dev(S.x0[a], (size_t)cap);
        if (e != hipSuccess) return hip_fail(c, e, "hipMalloc");
      }
      S.x0cap = cap;
    }
  }
  if (c->cfg.mode == PIC_MODE_PERSISTENT && (units_changed || !c->units)) {
    int64_t tot = 0;
    for (int s = 0; s < nsp; s++) {
      c->sp[s].ubase = tot;
      tot += c->sp[s].maxunits;
    }
    if (tot > c->units_cap) {
      if (!synced) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
      }
      hipError_t e = realloc_dev(c->units, (size_t)tot);
      if (e != hipSuccess) return hip_fail(c, e, "hipMalloc");
      c->units_cap = tot;
    }
  }
  return PIC_OK;
}

int64_t max_segments(const SpScratch *scr, int32_t nsp) {
  int64_t m = 1;
  for (int s = 0; s < nsp; s++) m = std::max(m, scr[s].maxseg);
  return m;
}

// Kernel arguments of the species with their scratch from scr (the
// context's own, c->sp, unless a caller passes another set).
SpArgs make_args(pic_ctx *c, const pic_species *sp, int32_t nsp, const SpScratch *scr = nullptr) {
  if (!scr) scr = c->sp;
  SpArgs a{};
  a.nsp = nsp;
  for (int s = 0; s < nsp; s++) {
    const pic_species &p = sp[s];
    SpDev &d = a.s[s];
    d.alpha = (p.q / p.m) * (0.5 * c->cfg.dt);
    d.q = p.q;
    d.n = p.n;
    for (int k = 0; k < 3; k++) {
      d.x[k] = k < c->cfg.dim ? p.x[k] : nullptr;
      d.xa[k] = k < c->cfg.dim ? p.x_alt[k] : nullptr;
      d.u[k] = p.u[k];
      d.ua[k] = p.u_alt[k];
      d.x0[k] = scr[s].x0[k];
    }
    d.w = p.w;
    d.wa = p.w_alt;
    d.id = p.id;
    d.ida = p.id_alt;
    d.off = c->nb > 1 ? c->boff[s] : p.offset;
    d.noff = scr[s].noff;
    d.tag = scr[s].tag;
    d.sstart = scr[s].sstart;
    d.cnt = scr[s].cnt;
    d.pre = scr[s].pre;
    d.tot = scr[s].tot;
    d.rbase = scr[s].rbase;
    d.in = scr[s].in;
    d.ubase = (int32_t)scr[s].ubase;
    d.snext = scr[s].snext;
    d.tmp = scr[s].tmp;
    d.perm = scr[s].perm;
  }
  return a;
}

void swap_buffers(pic_species &p) {
  for (int k = 0; k < 3; k++) {
    std::swap(p.x[k], p.x_alt[k]);
    std::swap(p.u[k], p.u_alt[k]);
  }
  std::swap(p.w, p.w_alt);
  std::swap(p.id, p.id_alt);
}

// Fold finished event pairs into the totals (waits for them).
void timing_collect(pic_ctx *c) {
  Timing &t = c->tm;
  for (auto &m : t.marks) {
    float ms = 0.f;
    if (hipEventSynchronize(t.pool[m.second + 1]) == hipSuccess &&
        hipEventElapsedTime(&ms, t.pool[m.second], t.pool[m.second + 1]) == hipSuccess) {
      t.ms[m.first] += ms;
      t.launches[m.first] += 1;
    }
  }
  t.marks.clear();
  t.used = 0;
}

// Record one event of a timed launch; returns its pool index (or -1).
long timing_event(pic_ctx *c, hipStream_t st) {
  Timing &t = c->tm;
  if (!t.on) return -1;
  if (t.used == t.pool.size()) {
    if (t.pool.size() >= 4096) timing_collect(c);
    if (t.used == t.pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      t.pool.push_back(e);
    }
  }
  const size_t k = t.used++;
  if (hipEventRecord(t.pool[k], st) != hipSuccess) return -1;
  return (long)k;
}

// Bracket the launches made by fn() with events when timing is on.
template <typename F>
hipError_t timed(pic_ctx *c, int kind, hipStream_t st, F &&fn) {
  const long a = timing_event(c, st);
  hipError_t e = fn();
  const long b = timing_event(c, st);
  if (a >= 0 && b == a + 1) c->tm.marks.push_back({kind, (size_t)a});
  return e;
}

pic_status finish(pic_ctx *c, hipStream_t st) {
  if (c->cfg.flags & PIC_FLAG_CHECK) return pic_check(c, st);
  return PIC_OK;
}

// Removing walls: the particles that survive a call are the first
// offset[npatch] of each species; wait for the stream and hand the caller
// the new counts.
pic_status update_counts(pic_ctx *c, pic_species *sp, int32_t nsp, hipStream_t st) {
  if (!c->g.remove) return PIC_OK;
  for (int s = 0; s < nsp; s++) {
    int64_t n = 0;
    hipError_t e = hipMemcpyAsync(&n, sp[s].offset + c->npatch_api, sizeof(n),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(c, e, "reading the surviving count");
    if (n < 0 || n > sp[s].n) return fail(c, PIC_ERR_STATE, "species %d: bad surviving count", s);
    sp[s].n = n;
  }
  return PIC_OK;
}

bool fields_ok(const pic_ctx *c, const pic_fields *f, bool eb, bool j) {
  if (!f) return false;
  for (int k = 0; k < 3; k++) {
    if (eb && (!f->e[k] || !f->b[k])) return false;
    if (j && !f->j[k]) return false;
  }
  (void)c;
  return true;
}

// Enqueue one whole step (J <- 0, fused kernel, sort, layout) on st for the
// buffer assignment in sp.  gather: the fused kernel reads the particles
// through the previous sort's permutation and writes the other buffer set.
// materialize: the sort copies the particles into the other buffer set;
// otherwise it only records the permutation.  The caller swaps the buffer
// sets once per gather and once per materialize.
// scr and units: the scratch and persistent work-unit list the kernels use.
hipError_t enqueue_step(pic_ctx *c, const pic_species *sp, int32_t nsp, const pic_fields *f,
                        hipStream_t st, bool gather, bool materialize, const SpScratch *scr,
                        Unit *units) {
  int64_t ncell = 1;
  for (int a = 0; a < c->cfg.dim; a++) ncell *= c->cfg.n[a];
  SpArgs a = make_args(c, sp, nsp, scr);
  a.gather = gather ? 1 : 0;
  // deterministic: the per-patch launch with per-wave J tiles, then J from
  // the tiles in a fixed order (no J <- 0 needed: the gather writes J)
  const bool det = (c->cfg.flags & PIC_FLAG_DETERMINISTIC) != 0;
  const bool pers = c->cfg.mode == PIC_MODE_PERSISTENT && !det;
  a.jt = det ? c->jt : nullptr;
  hipError_t e = hipSuccess;
  if (!det) e = timed(c, PIC_KERNEL_ZERO, st, [&] { return launch_zero(f->j, ncell, st); });
  if (e == hipSuccess)
    e = timed(c, PIC_KERNEL_IPP, st, [&] {
      if (det) {
        hipError_t r2 = launch_ipp(c->g, a, f->e, f->b, f->j, c->err_dev, c->wgd, st);
        return r2 == hipSuccess ? launch_j_gather(c->g, a, f->j, st) : r2;
      }
      return pers ? launch_ipp_persistent(c->g, a, f->e, f->b, f->j, c->err_dev, units, c->qctl,
                                          c->pgrid, c->wgd, st)
                  : launch_ipp(c->g, a, f->e, f->b, f->j, c->err_dev, c->wgd, st);
    });
  if (e != hipSuccess) return e;
  // the sort reads the particles where the fused kernel wrote them
  SpArgs r = make_args(c, sp, nsp, scr);
  if (gather)
    for (int s = 0; s < nsp; s++) {
      std::swap(r.s[s].x, r.s[s].xa);
      std::swap(r.s[s].u, r.s[s].ua);
      std::swap(r.s[s].w, r.s[s].wa);
      std::swap(r.s[s].id, r.s[s].ida);
    }
  e = timed(c, PIC_KERNEL_REBIN, st, [&] {
    hipError_t r2 = launch_rebin(c->g, r, c->err_dev, max_segments(scr, nsp), !materialize, st);
    if (r2 == hipSuccess && pers) r2 = launch_layout(c->g, r, units, c->qctl, st);
    return r2;
  });
  if (e == hipSuccess && c->cycle)
    e = timed(c, PIC_KERNEL_MAXWELL, st, [&] { return launch_yee_step(c->yee, st); });
  return e;
}

// Everything a captured graph depends on.
std::vector<uintptr_t> graph_key(const pic_ctx *c, const pic_species *sp, int32_t nsp,
                                 const pic_fields *f) {
  std::vector<uintptr_t> k;
  k.push_back((uintptr_t)nsp);
  k.push_back((uintptr_t)c->cycle);
  for (int s = 0; s < nsp; s++) {
    const pic_species &p = sp[s];
    k.push_back((uintptr_t)p.n);
    for (int a = 0; a < 3; a++) {
      k.push_back((uintptr_t)p.x[a]);
      k.push_back((uintptr_t)p.x_alt[a]);
      k.push_back((uintptr_t)p.u[a]);
      k.push_back((uintptr_t)p.u_alt[a]);
    }
    k.push_back((uintptr_t)p.w);
    k.push_back((uintptr_t)p.w_alt);
    k.push_back((uintptr_t)p.id);
    k.push_back((uintptr_t)p.id_alt);
    k.push_back((uintptr_t)p.offset);
    k.push_back((uintptr_t)c->sp[s].tag);
    k.push_back((uintptr_t)c->sp[s].cnt);
    uint64_t qb, mb;
    std::memcpy(&qb, &p.q, sizeof qb);
    std::memcpy(&mb, &p.m, sizeof mb);
    k.push_back((uintptr_t)qb);
    k.push_back((uintptr_t)mb);
  }
  for (int a = 0; a < 3; a++) {
    k.push_back((uintptr_t)f->e[a]);
    k.push_back((uintptr_t)f->b[a]);
    k.push_back((uintptr_t)f->j[a]);
  }
  k.push_back((uintptr_t)c->units);
  return k;
}

// Capture two middle steps of a run (gathering fused kernel A->B with a
// permutation-only sort, then B->A) into a graph, unless one of the two
// cached graphs was captured with the same pointers; returns it.
pic_status ensure_graph(pic_ctx *c, const pic_species *sp, int32_t nsp, const pic_fields *f,
                        hipGraphExec_t *out) {
  std::vector<uintptr_t> key = graph_key(c, sp, nsp, f);
  for (GraphCache &gc : c->gc)
    if (gc.exec && key == gc.key) {
      *out = gc.exec;
      return PIC_OK;
    }
  GraphCache &slot = c->gc[c->gc_next];
  c->gc_next ^= 1;
  if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
  if (slot.graph) (void)hipGraphDestroy(slot.graph);
  slot = GraphCache{};
  hipError_t e;
  if (!c->cap_stream && (e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) !=
                            hipSuccess)
    return hip_fail(c, e, "hipStreamCreate");
  pic_species tmp[kMaxSpecies];
  for (int s = 0; s < nsp; s++) tmp[s] = sp[s];
  if ((e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return hip_fail(c, e, "hipStreamBeginCapture");
  hipError_t eq = hipSuccess;
  for (int k = 0; k < 2 && eq == hipSuccess; k++) {
    eq = enqueue_step(c, tmp, nsp, f, c->cap_stream, true, false, c->sp, c->units);
    for (int s = 0; s < nsp; s++) swap_buffers(tmp[s]);
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->cap_stream, &g);
  if (eq != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(c, eq != hipSuccess ? eq : e, "graph capture");
  }
  hipGraphExec_t x = nullptr;
  if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(c, e, "hipGraphInstantiate");
  }
  slot.graph = g;
  slot.exec = x;
  slot.key = std::move(key);
  *out = x;
  return PIC_OK;
}

// The slab layout fits when every species' buffers hold its particles plus
// the room the plan adds (n/8 + 79 per patch, see slab_room) and stay below
// 2^29 elements (32-bit byte offsets in the kernels).
bool slab_fits(const pic_ctx *c, const pic_species *sp, int32_t nsp) {
  const int64_t np = c->g.npatch;
  for (int s = 0; s < nsp; s++) {
    const int64_t n = sp[s].n, cap = sp[s].capacity;
    if (cap >= ((int64_t)1 << 29)) return false;
    if (cap < n + n / 8 + 80 * np) return false;
  }
  return true;
}

pic_status ensure_slab(pic_ctx *c, const pic_species *sp, int32_t nsp, hipStream_t st) {
  const size_t np = (size_t)c->g.npatch;
  bool synced = false;
  auto sync = [&]() -> hipError_t {
    if (synced) return hipSuccess;
    synced = true;
    return hipStreamSynchronize(st);
  };
  for (int s = 0; s < nsp; s++) {
    SlabScratch &L = c->slab[s];
    hipError_t e = hipSuccess;
    if (!L.sb) {
      if ((e = sync()) != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
      if ((e = realloc_dev(L.sb, np + 1)) != hipSuccess ||
          (e = realloc_dev(L.sb2, np + 1)) != hipSuccess ||
          (e = realloc_dev(L.room, np)) != hipSuccess ||
          (e = realloc_dev(L.room2, np)) != hipSuccess ||
          (e = realloc_dev(L.cnt, np)) != hipSuccess ||
          (e = realloc_dev(L.cnt2, np)) != hipSuccess ||
          (e = realloc_dev(L.arr, np)) != hipSuccess ||
          (e = realloc_dev(L.arr2, np)) != hipSuccess || (e = realloc_dev(L.dep, np)) != hipSuccess ||
          (e = realloc_dev(L.porder, np)) != hipSuccess ||
          (e = realloc_dev(L.ctl, 2)) != hipSuccess)
        return hip_fail(c, e, "hipMalloc");
      // a valid patch order before any unit list writes one
      std::vector<int32_t> ident(np);
      for (size_t P = 0; P < np; P++) ident[P] = (int32_t)P;
      if ((e = hipMemcpy(L.porder, ident.data(), np * sizeof(int32_t), hipMemcpyHostToDevice)) !=
          hipSuccess)
        return hip_fail(c, e, "hipMemcpy");
    }
    const int64_t cap = sp[s].capacity;
    if (cap > L.cap) {
      if ((e = sync()) != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
      for (int a = 0; a < 3; a++) {
        if (a < c->cfg.dim && (e = realloc_dev(L.ox[a], (size_t)cap)) != hipSuccess)
          return hip_fail(c, e, "hipMalloc");
        if ((e = realloc_dev(L.ou[a], (size_t)cap)) != hipSuccess) return hip_fail(c, e, "hipMalloc");
      }
      if ((e = realloc_dev(L.ow, (size_t)cap)) != hipSuccess ||
          (e = realloc_dev(L.oid, (size_t)cap)) != hipSuccess ||
          (e = realloc_dev(L.odest, (size_t)cap)) != hipSuccess)
        return hip_fail(c, e, "hipMalloc");
      L.cap = cap;
    }
  }
  return PIC_OK;
}

SlabArgs make_slab_args(pic_ctx *c, const pic_species *sp, int32_t nsp) {
  SlabArgs a{};
  a.nsp = nsp;
  a.trace = (c->cfg.flags & PIC_FLAG_TRACE) ? c->trace : nullptr;
  for (int s = 0; s < nsp; s++) {
    const pic_species &p = sp[s];
    const SlabScratch &L = c->slab[s];
    SlabDev &d = a.s[s];
    d.alpha = (p.q / p.m) * (0.5 * c->cfg.dt);
    d.q = p.q;
    d.capacity = p.capacity;
    for (int k = 0; k < 3; k++) {
      const bool on = k < c->cfg.dim;
      d.x[k] = on ? p.x[k] : nullptr;
      d.xs[k] = on ? p.x_alt[k] : nullptr;
      d.ox[k] = on ? L.ox[k] : nullptr;
      d.u[k] = p.u[k];
      d.us[k] = p.u_alt[k];
      d.ou[k] = L.ou[k];
    }
    d.w = p.w;
    d.ws = p.w_alt;
    d.ow = L.ow;
    d.id = p.id;
    d.ids = p.id_alt;
    d.oid = L.oid;
    d.odest = L.odest;
    d.off = c->nb > 1 ? c->boff[s] : p.offset;
    d.sb = L.sb;
    d.sb2 = L.sb2;
    d.cap = L.room;
    d.cap2 = L.room2;
    d.cnt = L.cnt;
    d.cnt2 = L.cnt2;
    d.arr = L.arr;
    d.arr2 = L.arr2;
    d.dep = L.dep;
    d.porder = L.porder;
    d.ctl = L.ctl;
    d.code = reinterpret_cast<uint8_t *>(c->sp[s].tag);
    d.hole = c->sp[s].perm;
    d.tmp = c->sp[s].tmp;
    d.ubase = (int32_t)c->sp[s].ubase;
  }
  return a;
}

// One step in the slab layout: J <- 0, the in-place fused kernel, the
// exchange of the particles that changed patch.
hipError_t enqueue_slab_step(pic_ctx *c, const SlabArgs &a, const pic_fields *f, hipStream_t st) {
  int64_t ncell = 1;
  for (int d = 0; d < c->cfg.dim; d++) ncell *= c->cfg.n[d];
  const bool pers = c->cfg.mode == PIC_MODE_PERSISTENT;
  hipError_t e = timed(c, PIC_KERNEL_ZERO, st, [&] { return launch_zero(f->j, ncell, st); });
  // the call's first fused kernel also fills the slabs from the dense
  // layout: it is timed with the layout copies
  if (e == hipSuccess)
    e = timed(c, a.from_dense ? PIC_KERNEL_SLAB : PIC_KERNEL_IPP, st, [&] {
      return pers ? launch_ipp_slab_persistent(c->g, a, f->e, f->b, f->j, c->err_dev, c->units,
                                               c->qctl, c->pgrid_slab, c->wg, st)
                  : launch_ipp_slab(c->g, a, f->e, f->b, f->j, c->err_dev, c->wg, st);
    });
  if (e == hipSuccess)
    e = timed(c, PIC_KERNEL_EXCHANGE, st, [&] {
      return launch_exchange(c->g, a, c->err_dev, pers ? c->units : nullptr, c->qctl,
                             c->g.spc * kSeg, st);
    });
  if (e == hipSuccess && c->cycle)
    e = timed(c, PIC_KERNEL_MAXWELL, st, [&] { return launch_yee_step(c->yee, st); });
  return e;
}

// The captured run of `steps` slab steps (kGraphSteps or one) for these
// arguments (captured anew when any pointer, count or field differs from
// the cached one).
pic_status ensure_slab_graph(pic_ctx *c, const SlabArgs &a, const pic_fields *f, int steps,
                             hipGraphExec_t *out) {
  std::vector<uintptr_t> key((sizeof(SlabArgs) + sizeof(uintptr_t) - 1) / sizeof(uintptr_t), 0);
  std::memcpy(key.data(), &a, sizeof(SlabArgs));
  for (int k = 0; k < 3; k++) {
    key.push_back((uintptr_t)f->e[k]);
    key.push_back((uintptr_t)f->b[k]);
    key.push_back((uintptr_t)f->j[k]);
  }
  key.push_back((uintptr_t)c->units);
  key.push_back((uintptr_t)c->pgrid_slab);
  key.push_back((uintptr_t)c->cycle);
  key.push_back((uintptr_t)steps);
  GraphCache &gc = c->slab_gc[steps == 1 ? 1 : 0];
  if (gc.exec && key == gc.key) {
    *out = gc.exec;
    return PIC_OK;
  }
  if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
  if (gc.graph) (void)hipGraphDestroy(gc.graph);
  gc = GraphCache{};
  hipError_t e;
  if (!c->cap_stream && (e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) !=
                            hipSuccess)
    return hip_fail(c, e, "hipStreamCreate");
  if ((e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return hip_fail(c, e, "hipStreamBeginCapture");
  hipError_t eq = hipSuccess;
  for (int k = 0; k < steps && eq == hipSuccess; k++) eq = enqueue_slab_step(c, a, f, c->cap_stream);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->cap_stream, &g);
  if (eq != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(c, eq != hipSuccess ? eq : e, "graph capture");
  }
  hipGraphExec_t x = nullptr;
  if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(c, e, "hipGraphInstantiate");
  }
  gc.graph = g;
  gc.exec = x;
  gc.key = std::move(key);
  *out = x;
  return PIC_OK;
}

// x-bins: the bin offsets of each species, allocated on first use.
pic_status ensure_boff(pic_ctx *c, int32_t nsp) {
  if (c->nb == 1) return PIC_OK;
  for (int s = 0; s < nsp; s++)
    if (!c->boff[s]) {
      hipError_t e = realloc_dev(c->boff[s], (size_t)c->g.npatch + 1);
      if (e != hipSuccess) return hip_fail(c, e, "hipMalloc");
    }
  return PIC_OK;
}

// pic_step in the slab layout: dense -> slabs, nsteps slab steps, slabs ->
// dense (new offsets); the caller's first buffer set holds the result.
// Enqueues only (the caller finishes the call).
// cont: the particles are already in the slabs (a resident call after a
// resident call on the same species): no slab plan and no first step from
// the dense layout.  keep: leave them there (no slabs -> dense copy).
pic_status step_slab(pic_ctx *c, pic_species *sp, int32_t nsp, pic_fields *f, int32_t nsteps,
                     hipStream_t st, bool cont, bool keep) {
  pic_status r = ensure_slab(c, sp, nsp, st);
  if (r != PIC_OK) return r;
  if (c->cfg.flags & PIC_FLAG_TRACE) {
    // one record per (patch, species) workgroup or per unit of the list
    const int64_t need = std::max<int64_t>((int64_t)c->g.npatch * nsp, c->units_cap);
    if (need > c->trace_cap) {
      hipError_t e = hipStreamSynchronize(st);
      if (e == hipSuccess) e = realloc_dev(c->trace, 4 + 4 * (size_t)need);
      if (e == hipSuccess) e = hipMemset(c->trace, 0, 4 * sizeof(uint64_t));
      if (e != hipSuccess) return hip_fail(c, e, "trace buffer");
      c->trace_cap = need;
    }
  }
  const bool pers = c->cfg.mode == PIC_MODE_PERSISTENT;
  if (pers && !c->pgrid_slab) {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu < 1)
      ncu = 1;
    c->pgrid_slab = slab_persistent_blocks_per_cu(c->g, c->wg) * ncu;
  }
  // x-bins: the particles arrive sorted by patch; the copy into the slabs
  // puts them in bin order (bin counts first, then the slab plan, then each
  // particle straight into its bin's slab)
  const bool bins = c->nb > 1 && bin_order_supported(c->nb);
  if (bins && !cont) {
    if ((r = ensure_boff(c, nsp)) != PIC_OK) return r;
    for (int s = 0; s < nsp; s++) {
      SpDev d = make_args(c, sp, nsp).s[s];
      d.off = c->boff[s];
      const hipError_t e = timed(c, PIC_KERNEL_SORT, st, [&] {
        return bin_count(c->g, d, sp[s].offset, c->npatch_api, c->nb, sp[s].n, c->err_dev, st);
      });
      if (e != hipSuccess) return hip_fail(c, e, "bin count");
    }
  }
  const SlabArgs a = make_slab_args(c, sp, nsp);
  // without x-bins the first step's fused kernel reads the dense layout
  // itself and fills the slabs (the call makes no separate copy into them)
  SlabArgs first = a;
  first.from_dense = bins || cont ? 0 : 1;
  hipError_t e = cont ? hipSuccess : timed(c, PIC_KERNEL_SLAB, st, [&] {
    hipError_t r2 = launch_slab_begin(c->g, a, c->err_dev, st, false);
    for (int s = 0; bins && s < nsp && r2 == hipSuccess; s++) {
      SpDev d = make_args(c, sp, nsp).s[s];
      d.off = c->boff[s];
      r2 = bin_place(c->g, d, sp[s].offset, c->npatch_api, c->nb, sp[s].n, c->slab[s].sb,
                     c->slab[s].ctl, st);
    }
    return r2;
  });
  // (a continued call's units are the last step's, made for the next one)
  if (e == hipSuccess && pers && !cont)
    e = timed(c, PIC_KERNEL_EXCHANGE, st, [&] {
      return launch_slab_units(c->g, a, c->g.spc * kSeg, c->units, c->qctl, st);
    });
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  int k0 = 0;
  if (first.from_dense && nsteps > 0) {
    if ((e = enqueue_slab_step(c, first, f, st)) != hipSuccess)
      return hip_fail(c, e, "kernel launch");
    k0 = 1;
  }
  if ((c->cfg.flags & PIC_FLAG_GRAPH) && !c->tm.on && k0 < nsteps) {
    // graphs of kGraphSteps steps, then one-step graphs for the rest
    int k = k0;
    if (nsteps - k >= kGraphSteps) {
      hipGraphExec_t x = nullptr;
      if ((r = ensure_slab_graph(c, a, f, kGraphSteps, &x)) != PIC_OK) return r;
      for (; nsteps - k >= kGraphSteps; k += kGraphSteps)
        if ((e = hipGraphLaunch(x, st)) != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
    }
    if (k < nsteps) {
      hipGraphExec_t x = nullptr;
      if ((r = ensure_slab_graph(c, a, f, 1, &x)) != PIC_OK) return r;
      for (; k < nsteps; k++)
        if ((e = hipGraphLaunch(x, st)) != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
    }
  } else {
    for (int k = k0; k < nsteps; k++)
      if ((e = enqueue_slab_step(c, a, f, st)) != hipSuccess) return hip_fail(c, e, "kernel launch");
  }
  if (keep) return PIC_OK;
  e = timed(c, PIC_KERNEL_SLAB, st, [&] {
    hipError_t r2 = launch_slab_end(c->g, a, st);
    // the dense layout's segment starts (and persistent work units) for
    // whatever runs next on these particles
    if (r2 == hipSuccess)
      r2 = launch_layout(c->g, make_args(c, sp, nsp), pers ? c->units : nullptr, c->qctl, st);
    return r2;
  });
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  return PIC_OK;
}

// x-bins: the caller's patch offsets (every nb-th bin offset).
hipError_t api_offsets(pic_ctx *c, const pic_species *sp, int32_t nsp, hipStream_t st) {
  if (c->nb == 1) return hipSuccess;
  for (int s = 0; s < nsp; s++) {
    const hipError_t e = launch_api_offsets(c->boff[s], sp[s].offset, c->npatch_api, c->nb, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// PIC_FLAG_RESIDENT: the resident species' slabs -> dense layout, offsets,
// segment starts (and work units) -- what pic_step's slab layout does at the
// end of a call -- enqueued on st; then nothing is resident.
pic_status resident_flush(pic_ctx *c, hipStream_t st) {
  if (!c->resident) return PIC_OK;
  c->resident = false;
  const pic_species *sp = c->res_sp;
  const int32_t nsp = c->res_nsp;
  const SlabArgs a = make_slab_args(c, sp, nsp);
  const bool pers = c->cfg.mode == PIC_MODE_PERSISTENT;
  hipError_t e = timed(c, PIC_KERNEL_SLAB, st, [&] {
    hipError_t r2 = launch_slab_end(c->g, a, st);
    if (r2 == hipSuccess)
      r2 = launch_layout(c->g, make_args(c, sp, nsp), pers ? c->units : nullptr, c->qctl, st);
    return r2;
  });
  if (e == hipSuccess) e = api_offsets(c, sp, nsp, st);
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  return PIC_OK;
}

// The same species arrays (and counts) as the resident ones.
bool same_as_resident(const pic_ctx *c, const pic_species *sp, int32_t nsp) {
  if (!c->resident || nsp != c->res_nsp) return false;
  for (int s = 0; s < nsp; s++) {
    const pic_species &a = sp[s], &b = c->res_sp[s];
    bool same = a.n == b.n && a.capacity == b.capacity && a.q == b.q && a.m == b.m &&
                a.w == b.w && a.id == b.id && a.w_alt == b.w_alt && a.id_alt == b.id_alt &&
                a.offset == b.offset;
    for (int k = 0; k < 3; k++)
      same = same && a.x[k] == b.x[k] && a.u[k] == b.u[k] && a.x_alt[k] == b.x_alt[k] &&
             a.u_alt[k] == b.u_alt[k];
    if (!same) return false;
  }
  return true;
}

// The synchronisation-phase sort of pic_bin: with general, wrap + key +
// stable sort of particles in any order; otherwise the neighbour-code sort
// after pic_interp_push.  Then segment starts (and work units), the buffer
// swap and, with x-bins, the caller's patch offsets.
pic_status sort_species(pic_ctx *c, pic_species *sp, int32_t nsp, bool general, hipStream_t st) {
  pic_status r;
  if ((r = ensure_scratch(c, sp, nsp, false, st)) != PIC_OK) return r;
  if ((r = ensure_boff(c, nsp)) != PIC_OK) return r;
  if (!general) {
    // particles moved at most one cell since the last sort: neighbour-code sort
    const SpArgs a = make_args(c, sp, nsp);
    hipError_t e =
        timed(c, PIC_KERNEL_TAG, st, [&] { return launch_tag(c->g, a, c->err_dev, c->wgd, st); });
    if (e == hipSuccess)
      e = timed(c, PIC_KERNEL_REBIN, st, [&] {
        return launch_rebin(c->g, a, c->err_dev, max_segments(c->sp, nsp), false, st);
      });
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  } else {
    for (int s = 0; s < nsp; s++) {
      const SpArgs a = make_args(c, sp + s, 1);
      SpDev d = a.s[0];
      d.off = c->nb > 1 ? c->boff[s] : sp[s].offset;
      hipError_t e = timed(c, PIC_KERNEL_SORT, st,
                           [&] { return general_sort(c->g, d, c->sort[s], c->err_dev, st); });
      if (e != hipSuccess) return hip_fail(c, e, "general sort");
    }
  }
  {
    const SpArgs a = make_args(c, sp, nsp);
    hipError_t e = launch_layout(c->g, a, c->cfg.mode == PIC_MODE_PERSISTENT ? c->units : nullptr,
                                 c->qctl, st);
    if (e == hipSuccess) e = api_offsets(c, sp, nsp, st);
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  }
  for (int s = 0; s < nsp; s++) swap_buffers(sp[s]);
  c->moved = false;
  return PIC_OK;
}

// pic_step in the dense layout: the first step updates the particles in
// place and records the sort as a permutation; middle steps gather through
// it into the other buffer set; the last step's sort copies the particles
// into their sorted places, so between calls the arrays are always sorted.
// scr and units: the scratch and work-unit list the kernels use; graphs:
// middle steps may replay a captured graph (PIC_FLAG_GRAPH).
pic_status step_dense(pic_ctx *c, pic_species *sp, int32_t nsp, const pic_fields *f,
                      int32_t nsteps, hipStream_t st, const SpScratch *scr, Unit *units,
                      bool graphs) {
  pic_status r;
  auto step = [&](bool gather, bool materialize) -> pic_status {
    hipError_t e = enqueue_step(c, sp, nsp, f, st, gather, materialize, scr, units);
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
    for (int s = 0; s < nsp; s++) {
      if (gather) swap_buffers(sp[s]);
      if (materialize) swap_buffers(sp[s]);
    }
    return PIC_OK;
  };
  if ((r = step(false, nsteps == 1)) != PIC_OK) return r;
  int middle = nsteps - 2;  // steps 1 .. nsteps-2
  if (graphs && (c->cfg.flags & PIC_FLAG_GRAPH) && !c->tm.on && middle >= 2) {
    hipGraphExec_t x = nullptr;
    if ((r = ensure_graph(c, sp, nsp, f, &x)) != PIC_OK) return r;
    for (; middle >= 2; middle -= 2) {
      hipError_t e = hipGraphLaunch(x, st);
      if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
    }
  }
  for (; middle > 0; middle--)
    if ((r = step(true, false)) != PIC_OK) return r;
  if (nsteps >= 2 && (r = step(true, true)) != PIC_OK) return r;
  return PIC_OK;
}

// The context's segment starts (and persistent work units) are recomputed
// from the caller's offsets when another scratch set last sorted the
// particles (pic_step_noalloc).
pic_status refresh_layout(pic_ctx *c, const pic_species *sp, int32_t nsp, hipStream_t st) {
  if (!c->layout_stale) return PIC_OK;
  const SpArgs a = make_args(c, sp, nsp);
  const hipError_t e = launch_layout(
      c->g, a, c->cfg.mode == PIC_MODE_PERSISTENT ? c->units : nullptr, c->qctl, st);
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  c->layout_stale = false;
  return PIC_OK;
}

// x-bins: particles sorted by patch put into bin order inside each patch
// (a stable counting sort per patch), then segment starts (and work
// units) and the buffer swap.  More bins per patch than the counting sort
// serves: the general sort.
pic_status order_bins(pic_ctx *c, pic_species *sp, int32_t nsp, hipStream_t st) {
  if (!bin_order_supported(c->nb)) return sort_species(c, sp, nsp, true, st);
  pic_status r;
  if ((r = ensure_boff(c, nsp)) != PIC_OK) return r;
  for (int s = 0; s < nsp; s++) {
    SpDev d = make_args(c, sp, nsp).s[s];
    d.off = c->boff[s];
    hipError_t e = timed(c, PIC_KERNEL_SORT, st, [&] {
      return bin_order(c->g, d, sp[s].offset, c->npatch_api, c->nb, sp[s].n, c->err_dev, st);
    });
    if (e != hipSuccess) return hip_fail(c, e, "bin order");
  }
  const SpArgs a = make_args(c, sp, nsp);
  const hipError_t e = launch_layout(
      c->g, a, c->cfg.mode == PIC_MODE_PERSISTENT ? c->units : nullptr, c->qctl, st);
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  for (int s = 0; s < nsp; s++) swap_buffers(sp[s]);
  return PIC_OK;
}

// Field steps (forward, j read) or their reverse mode (j accumulated into).
pic_status yee_steps(pic_ctx *c, double *const e[3], double *const b[3], double *const j[3],
                     int32_t nsteps, bool adjoint, void *stream) {
  if (!c) return PIC_ERR_ARG;
  if (c->poisoned) return fail(c, PIC_ERR_STATE, "context unusable after a device error");
  if (!e || !b || !j) return fail(c, PIC_ERR_ARG, "null field array");
  for (int k = 0; k < 3; k++)
    if (!e[k] || !b[k] || !j[k]) return fail(c, PIC_ERR_ARG, "null field pointer");
  if (nsteps < 0) return fail(c, PIC_ERR_ARG, "nsteps < 0");
  if (c->g.n[1] > 65535 || c->g.n[2] > 65535)
    return fail(c, PIC_ERR_ARG, "the field solver takes at most 65535 cells along y and z");
  hipStream_t st = (hipStream_t)stream;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, PIC_ERR_HIP, "hipSetDevice");
  YeeArgs a{};
  a.dim = c->cfg.dim;
  for (int k = 0; k < 3; k++) {
    a.n[k] = c->g.n[k];
    a.c[k] = k < c->cfg.dim ? c->cfg.dt / c->cfg.d[k] : 0.0;
    a.e[k] = e[k];
    a.b[k] = b[k];
    a.j[k] = j[k];
  }
  a.dt = c->cfg.dt;
  for (int s = 0; s < nsteps; s++) {
    const hipError_t x = timed(c, PIC_KERNEL_MAXWELL, st, [&] {
      return adjoint ? launch_yee_adjoint_step(a, st) : launch_yee_step(a, st);
    });
    if (x != hipSuccess) return hip_fail(c, x, "kernel launch");
  }
  return finish(c, st);
}

}  // namespace

extern "C" {

pic_status pic_validate_config(const pic_config *c, char *msg, size_t len) {
  if (msg && len) msg[0] = 0;
  if (!c) {
    set_msg(msg, len, "null config");
    return PIC_ERR_ARG;
  }
  if (c->dim != 2 && c->dim != 3) {
    set_msg(msg, len, "dim must be 2 or 3 (got %d)", c->dim);
    return PIC_ERR_ARG;
  }
  if (c->shape_order != 2) {
    set_msg(msg, len, "shape_order must be 2 (quadratic shapes), got %d", c->shape_order);
    return PIC_ERR_ARG;
  }
  long long npatch = 1;
  double inv2 = 0.0;
  for (int a = 0; a < c->dim; a++) {
    if (c->n[a] < 1 || c->n[a] > (1 << 30)) {
      set_msg(msg, len, "n[%d]=%d out of range", a, c->n[a]);
      return PIC_ERR_ARG;
    }
    if (c->patch[a] < 6) {
      set_msg(msg, len, "patch[%d]=%d below 6 cells (three-point stencil plus ghosts)", a,
              c->patch[a]);
      return PIC_ERR_ARG;
    }
    if (c->n[a] % c->patch[a]) {
      set_msg(msg, len, "patch[%d]=%d does not divide n[%d]=%d", a, c->patch[a], a, c->n[a]);
      return PIC_ERR_ARG;
    }
    if (!(c->d[a] > 0) || !std::isfinite(c->d[a])) {
      set_msg(msg, len, "d[%d] must be positive and finite", a);
      return PIC_ERR_ARG;
    }
    npatch *= c->n[a] / c->patch[a];
    inv2 += 1.0 / (c->d[a] * c->d[a]);
  }
  if (c->dim == 2 && ((c->n[2] != 1 && c->n[2] != 0) || (c->patch[2] != 1 && c->patch[2] != 0))) {
    set_msg(msg, len, "2D configuration needs n[2] = patch[2] = 1");
    return PIC_ERR_ARG;
  }
  if (npatch > (1ll << 30)) {
    set_msg(msg, len, "too many patches (%lld)", npatch);
    return PIC_ERR_ARG;
  }
  long long ncell = 1;
  for (int a = 0; a < c->dim; a++) ncell *= c->n[a];
  if (ncell > (1ll << 40)) {
    set_msg(msg, len, "grid too large");
    return PIC_ERR_ARG;
  }
  const double cfl = 1.0 / std::sqrt(inv2);
  if (!(c->dt > 0) || !std::isfinite(c->dt) || c->dt > cfl) {
    set_msg(msg, len, "dt=%.17g must be in (0, %.17g] (Courant limit)", c->dt, cfl);
    return PIC_ERR_ARG;
  }
  if (c->mode != PIC_MODE_PER_PATCH && c->mode != PIC_MODE_PERSISTENT) {
    set_msg(msg, len, "unknown mode %d", c->mode);
    return PIC_ERR_ARG;
  }
  if (c->chunk < 0 || c->chunk % kSeg) {
    set_msg(msg, len, "chunk must be 0 (auto) or a positive multiple of %d", kSeg);
    return PIC_ERR_ARG;
  }
  if (c->wg_size != 0 && (c->wg_size < 64 || c->wg_size > 1024 || c->wg_size % 64)) {
    set_msg(msg, len, "wg_size must be 0 or a multiple of 64 in [64, 1024]");
    return PIC_ERR_ARG;
  }
  if (c->flags &
      ~(uint32_t)(PIC_FLAG_CHECK | PIC_FLAG_GRAPH | PIC_FLAG_TRACE | PIC_FLAG_DETERMINISTIC |
                  PIC_FLAG_RESIDENT)) {
    set_msg(msg, len, "unknown flag bits 0x%x", c->flags);
    return PIC_ERR_ARG;
  }
  for (int a = 0; a < c->dim; a++)
    if (c->particle_bc[a] < PIC_BC_PERIODIC || c->particle_bc[a] > PIC_BC_REMOVE) {
      set_msg(msg, len, "particle_bc[%d]=%d must be PIC_BC_PERIODIC, PIC_BC_REFLECT or PIC_BC_REMOVE",
              a, c->particle_bc[a]);
      return PIC_ERR_ARG;
    }
  if (c->flags & PIC_FLAG_DETERMINISTIC)
    for (int a = 0; a < c->dim; a++)
      if (c->particle_bc[a] == PIC_BC_REMOVE) {
        set_msg(msg, len,
                "PIC_FLAG_DETERMINISTIC keeps the dense layout, which cannot delete particles "
                "(removing walls on axis %d)", a);
        return PIC_ERR_ARG;
      }
  if (c->flags & PIC_FLAG_RESIDENT) {
    if (c->flags & PIC_FLAG_DETERMINISTIC) {
      set_msg(msg, len, "PIC_FLAG_RESIDENT keeps the slab layout, PIC_FLAG_DETERMINISTIC the dense one");
      return PIC_ERR_ARG;
    }
    for (int a = 0; a < c->dim; a++)
      if (c->particle_bc[a] == PIC_BC_REMOVE) {
        set_msg(msg, len,
                "PIC_FLAG_RESIDENT: removing walls change the counts that each call reports "
                "(removing walls on axis %d)", a);
        return PIC_ERR_ARG;
      }
  }
  if (c->bin_x < 0 || (c->bin_x > 0 && c->patch[0] % c->bin_x)) {
    set_msg(msg, len, "bin_x=%d must be 0 (auto) or divide patch[0]=%d", c->bin_x, c->patch[0]);
    return PIC_ERR_ARG;
  }
  const int bx = choose_bin(c);
  if (bx == 0 || !tiles_fit(c, bx)) {
    const int b = bx ? bx : 1;
    set_msg(msg, len,
            "patch too large: E/B and J tiles of x-bins of %d cells need %zu bytes of LDS "
            "(max %zu)",
            b, tiles_bytes(c, b) + kStaticLds, kLdsMax);
    return PIC_ERR_ARG;
  }
  return PIC_OK;
}

int64_t pic_num_patches(const pic_config *c) {
  if (pic_validate_config(c, nullptr, 0) != PIC_OK) return 0;
  int64_t n = 1;
  for (int a = 0; a < c->dim; a++) n *= c->n[a] / c->patch[a];
  return n;
}

int32_t pic_bin_width(const pic_config *c) {
  if (pic_validate_config(c, nullptr, 0) != PIC_OK) return 0;
  return choose_bin(c);
}

pic_status pic_init(const pic_config *cfg, int32_t device, pic_ctx **out) {
  if (!out) return PIC_ERR_ARG;
  *out = nullptr;
  char m[256];
  if (pic_validate_config(cfg, m, sizeof m) != PIC_OK) return PIC_ERR_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PIC_ERR_HIP;
  if (hipSetDevice(device) != hipSuccess) return PIC_ERR_HIP;
  pic_ctx *c = new pic_ctx();
  c->cfg = *cfg;
  if (c->cfg.dim == 2) {
    c->cfg.n[2] = 1;
    c->cfg.patch[2] = 1;
    c->cfg.d[2] = 1.0;
  }
  c->g = make_grid(&c->cfg);
  c->nb = c->cfg.patch[0] / c->g.patch[0];
  c->npatch_api = c->g.npatch / c->nb;
  c->device = device;
  c->wg = cfg->wg_size ? cfg->wg_size : default_wg(&c->cfg);
  c->wgd = std::min(c->wg, c->cfg.dim == 2 ? 256 : 512);
  // deterministic: as many waves as private J tiles fit beside the E/B tile
  if (c->cfg.flags & PIC_FLAG_DETERMINISTIC) c->wgd = 64 * det_waves(c->g, c->wgd);
  const int chunk = cfg->chunk ? cfg->chunk : 2048;
  c->g.spc = std::max(1, chunk / kSeg);
  if (hipMalloc(&c->err_dev, sizeof(int)) != hipSuccess ||
      hipMemset(c->err_dev, 0, sizeof(int)) != hipSuccess ||
      hipMalloc(&c->qctl, 2 * kMaxSpecies * sizeof(int)) != hipSuccess ||
      hipMemset(c->qctl, 0, 2 * kMaxSpecies * sizeof(int)) != hipSuccess) {
    (void)hipFree(c->err_dev);
    (void)hipFree(c->qctl);
    delete c;
    return PIC_ERR_HIP;
  }
  if (c->cfg.mode == PIC_MODE_PERSISTENT) c->pgrid = persistent_grid(c->g, c->wgd);
  c->noalloc = noalloc_scratch(device);  // checked by pic_step_noalloc
  *out = c;
  return PIC_OK;
}

void pic_free(pic_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  // (resident particles are not written back: their buffers may be gone)
  for (int s = 0; s < kMaxSpecies; s++) {
    SpScratch &S = c->sp[s];
    (void)hipFree(S.tag);
    (void)hipFree(S.cnt);
    (void)hipFree(S.snext);
    (void)hipFree(S.tmp);
    (void)hipFree(S.perm);
    (void)hipFree(S.pre);
    (void)hipFree(S.tot);
    (void)hipFree(S.sstart);
    (void)hipFree(S.rbase);
    (void)hipFree(S.in);
    (void)hipFree(S.noff);
    for (int a = 0; a < 3; a++) (void)hipFree(S.x0[a]);
    free_sort_scratch(c->sort[s]);
    (void)hipFree(c->boff[s]);
    SlabScratch &L = c->slab[s];
    for (void *p : {(void *)L.sb, (void *)L.sb2, (void *)L.room, (void *)L.room2, (void *)L.cnt,
                    (void *)L.cnt2, (void *)L.arr, (void *)L.arr2, (void *)L.dep, (void *)L.porder,
                    (void *)L.ctl, (void *)L.ow, (void *)L.oid, (void *)L.odest})
      (void)hipFree(p);
    for (int a = 0; a < 3; a++) {
      (void)hipFree(L.ox[a]);
      (void)hipFree(L.ou[a]);
    }
  }
  for (GraphCache &gc : c->slab_gc) {
    if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
    if (gc.graph) (void)hipGraphDestroy(gc.graph);
  }
  for (hipEvent_t e : c->tm.pool) (void)hipEventDestroy(e);
  for (GraphCache &gc : c->gc) {
    if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
    if (gc.graph) (void)hipGraphDestroy(gc.graph);
  }
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  (void)hipFree(c->units);
  (void)hipFree(c->trace);
  (void)hipFree(c->jt);
  (void)hipFree(c->qctl);
  (void)hipFree(c->err_dev);
  delete c;
}

pic_status pic_timing_enable(pic_ctx *c, int32_t on) {
  if (!c) return PIC_ERR_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, PIC_ERR_HIP, "hipSetDevice");
  timing_collect(c);
  for (int k = 0; k < PIC_KERNEL_COUNT; k++) {
    c->tm.ms[k] = 0;
    c->tm.launches[k] = 0;
  }
  c->tm.on = on != 0;
  return PIC_OK;
}

pic_status pic_timing_read(pic_ctx *c, int32_t kernel, double *total_ms, int64_t *launches) {
  if (!c || kernel < 0 || kernel >= PIC_KERNEL_COUNT) return PIC_ERR_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, PIC_ERR_HIP, "hipSetDevice");
  timing_collect(c);
  if (total_ms) *total_ms = c->tm.ms[kernel];
  if (launches) *launches = c->tm.launches[kernel];
  return PIC_OK;
}

pic_status pic_trace_read(pic_ctx *c, pic_trace_record *out, int64_t cap, int64_t *n) {
  if (!c || !n || cap < 0 || (cap > 0 && !out)) return PIC_ERR_ARG;
  *n = 0;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, PIC_ERR_HIP, "hipSetDevice");
  if (!c->trace) return PIC_OK;
  hipError_t e = hipDeviceSynchronize();
  uint64_t count = 0;
  if (e == hipSuccess) e = hipMemcpy(&count, c->trace, sizeof(count), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "reading the trace");
  const int64_t m = std::min<int64_t>({(int64_t)count, cap, c->trace_cap});
  if (m > 0 && (e = hipMemcpy(out, c->trace + 4, (size_t)m * sizeof(pic_trace_record),
                              hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(c, e, "reading the trace");
  *n = std::min<int64_t>((int64_t)count, c->trace_cap);
  return PIC_OK;
}

pic_status pic_check(pic_ctx *c, void *stream) {
  if (!c) return PIC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  int h = 0;
  e = hipMemcpy(&h, c->err_dev, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy");
  if (h) {
    c->poisoned = true;
    if (h & kErrCFL)
      return fail(c, PIC_ERR_CFL, "a particle moved more than one cell in one step");
    if (h & kErrCap)
      return fail(c, PIC_ERR_CAPACITY, "the per-patch slabs outgrew the particle buffers");
    if (h & kErrUnsorted)
      return fail(c, PIC_ERR_UNSORTED,
                  "a particle lies outside the patch its offsets assign it to (not sorted by patch)");
    return fail(c, PIC_ERR_POS,
                "a position lies more than one period outside the box (or outside a walled axis)");
  }
  if (c->poisoned) return PIC_ERR_STATE;
  return PIC_OK;
}

const char *pic_last_error(const pic_ctx *c) { return c ? c->msg : "null context"; }

pic_status pic_sync(pic_ctx *c, void *stream) {
  if (!c) return PIC_ERR_ARG;
  if (c->poisoned) return fail(c, PIC_ERR_STATE, "context unusable after a device error");
  hipStream_t st = (hipStream_t)stream;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, PIC_ERR_HIP, "hipSetDevice");
  const pic_status r = resident_flush(c, st);
  if (r != PIC_OK) return r;
  return finish(c, st);
}

pic_status pic_bin(pic_ctx *c, pic_species *sp, int32_t nsp, void *stream) {
  pic_status r = check_species(c, sp, nsp, false);
  if (r != PIC_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, PIC_ERR_HIP, "hipSetDevice");
  if ((r = resident_flush(c, st)) != PIC_OK) return r;  // PIC_FLAG_RESIDENT: dense layout first
  if (c->moved && nsp != c->moved_nsp)
    return fail(c, PIC_ERR_STATE, "pic_bin after pic_interp_push needs the same species");
  // removing walls: the general sort, whose keys drop deleted particles past
  // the last patch (the neighbour-code sort keeps every particle)
  if ((r = sort_species(c, sp, nsp, !c->moved || c->g.remove, st)) != PIC_OK) return r;
  if ((r = finish(c, st)) != PIC_OK) return r;
  return update_counts(c, sp, nsp, st);
}

pic_status pic_interp_push(pic_ctx *c, pic_species *sp, int32_t nsp, const pic_fields *f,
                           void *stream) {
  pic_status r = check_species(c, sp, nsp, true);
  if (r != PIC_OK) return r;
  if (!fields_ok(c, f, true, false)) return fail(c, PIC_ERR_ARG, "null field pointer");
  if (c->moved) return fail(c, PIC_ERR_STATE, "pic_interp_push twice without a sort");
  hipStream_t st = (hipStream_t)stream;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, PIC_ERR_HIP, "hipSetDevice");
  if ((r = resident_flush(c, st)) != PIC_OK) return r;  // PIC_FLAG_RESIDENT: dense layout first
  if ((r = ensure_scratch(c, sp, nsp, true, st)) != PIC_OK) return r;
  if ((r = refresh_layout(c, sp, nsp, st)) != PIC_OK) return r;
  // x-bins: the particles arrive sorted by patch; the kernels need them by bin
  if (c->nb > 1 && (r = order_bins(c, sp, nsp, st)) != PIC_OK) return r;
  const SpArgs a = make_args(c, sp, nsp);
  hipError_t e = timed(c, PIC_KERNEL_INTERP_PUSH, st, [&] {
    return launch_interp_push(c->g, a, f->e, f->b, c->err_dev, c->wgd, st);
  });
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  c->moved = true;
  c->moved_nsp = nsp;
  return finish(c, st);
}

pic_status pic_project(pic_ctx *c, const pic_species *sp, int32_t nsp, pic_fields *f,
                       void *stream) {
  pic_status r = check_species(c, sp, nsp, true);
  if (r != PIC_OK) return r;
  if (!fields_ok(c, f, false, true)) return fail(c, PIC_ERR_ARG, "null J pointer");
  if (!c->moved || nsp != c->moved_nsp)
    return fail(c, PIC_ERR_STATE, "pic_project needs a preceding pic_interp_push");
  hipStream_t st = (hipStream_t)stream;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, PIC_ERR_HIP, "hipSetDevice");
  if ((r = resident_flush(c, st)) != PIC_OK) return r;  // PIC_FLAG_RESIDENT: dense layout first
  const SpArgs a = make_args(c, sp, nsp);
  hipError_t e = timed(c, PIC_KERNEL_PROJECT, st,
                       [&] { return launch_project(c->g, a, f->j, c->err_dev, c->wgd, st); });
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  return finish(c, st);
}

pic_status pic_step(pic_ctx *c, pic_species *sp, int32_t nsp, pic_fields *f, int32_t nsteps,
                    void *stream) {
  pic_status r = check_species(c, sp, nsp, true);
  if (r != PIC_OK) return r;
  if (!fields_ok(c, f, true, true)) return fail(c, PIC_ERR_ARG, "null field pointer");
  if (nsteps < 0) return fail(c, PIC_ERR_ARG, "nsteps < 0");
  if (c->moved) return fail(c, PIC_ERR_STATE, "pic_step with a sort pending (call pic_bin)");
  hipStream_t st = (hipStream_t)stream;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, PIC_ERR_HIP, "hipSetDevice");
  // PIC_FLAG_RESIDENT: a call on the resident species continues in their
  // slabs; any other call first writes the resident species back
  const bool res = (c->cfg.flags & PIC_FLAG_RESIDENT) && (c->nb == 1 || bin_order_supported(c->nb));
  const bool cont = res && same_as_resident(c, sp, nsp);
  if (c->resident && !cont && (r = resident_flush(c, st)) != PIC_OK) return r;
  if ((r = ensure_scratch(c, sp, nsp, false, st)) != PIC_OK) return r;
  if (!cont && (r = refresh_layout(c, sp, nsp, st)) != PIC_OK) return r;
  if (nsteps == 0) return finish(c, st);
  // removing walls delete particles only in the slab layout's exchange, so
  // every call takes it there
  if (c->g.remove && !slab_fits(c, sp, nsp))
    return fail(c, PIC_ERR_CAPACITY,
                "removing walls need buffers with the slab layout's room (n + n/8 + 80 per slab)");
  const bool det = (c->cfg.flags & PIC_FLAG_DETERMINISTIC) != 0;
  const bool slab = !det && (nsteps >= 3 || c->g.remove || res) && slab_fits(c, sp, nsp);
  if (det) {
    // one J tile per (species, patch)
    size_t tj = 3;
    for (int a = 0; a < c->cfg.dim; a++) tj *= (size_t)(c->g.patch[a] + 5);
    const size_t need = tj * (size_t)c->g.npatch * (size_t)nsp;
    if (need > c->jt_cap) {
      hipError_t e = hipStreamSynchronize(st);
      if (e == hipSuccess) e = realloc_dev(c->jt, need);
      if (e != hipSuccess) return hip_fail(c, e, "hipMalloc");
      c->jt_cap = need;
    }
  }
  // x-bins: the particles arrive sorted by patch; the kernels need them by
  // bin (the slab layout's first copy orders them itself)
  if (c->nb > 1 && !(slab && bin_order_supported(c->nb)) &&
      (r = order_bins(c, sp, nsp, st)) != PIC_OK)
    return r;
  if (slab) {
    if ((r = step_slab(c, sp, nsp, f, nsteps, st, cont, res)) != PIC_OK) return r;
    if (res) {  // the particles stay in the slabs (offsets and first set stale)
      c->resident = true;
      c->res_nsp = nsp;
      for (int s = 0; s < nsp; s++) c->res_sp[s] = sp[s];
      return finish(c, st);
    }
  } else {
    if ((r = step_dense(c, sp, nsp, f, nsteps, st, c->sp, c->units, true)) != PIC_OK) return r;
  }
  const hipError_t e = api_offsets(c, sp, nsp, st);
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  if ((r = finish(c, st)) != PIC_OK) return r;
  return update_counts(c, sp, nsp, st);
}


pic_status pic_step_noalloc(pic_ctx *c, pic_species *sp, int32_t nsp, pic_fields *f,
                            int32_t nsteps, void *stream) {
  pic_status r = check_species(c, sp, nsp, true);
  if (r != PIC_OK) return r;
  if (!fields_ok(c, f, true, true)) return fail(c, PIC_ERR_ARG, "null field pointer");
  if (nsteps < 0) return fail(c, PIC_ERR_ARG, "nsteps < 0");
  if (c->moved) return fail(c, PIC_ERR_STATE, "pic_step_noalloc with a sort pending (call pic_bin)");
  if (c->nb > 1)
    return fail(c, PIC_ERR_ARG, "pic_step_noalloc: x-bins need the per-call bin sort (pic_step)");
  if (c->g.remove)
    return fail(c, PIC_ERR_ARG, "pic_step_noalloc: removing walls need the slab layout (pic_step)");
  if (c->cfg.flags & PIC_FLAG_DETERMINISTIC)
    return fail(c, PIC_ERR_ARG, "pic_step_noalloc: PIC_FLAG_DETERMINISTIC needs its tile buffer (pic_step)");
  if (!c->noalloc) return fail(c, PIC_ERR_HIP, "pic_step_noalloc: no static scratch on this device");
  // the dense layout's scratch, carved from the static array in 256-byte
  // aligned pieces: per species the tags and permutation (n each), the
  // per-segment code counts and prefixes, the per-patch arrays; in
  // persistent mode the work units of every species after them
  const size_t np = (size_t)c->g.npatch, nc = (size_t)c->g.nc;
  char *base = static_cast<char *>(c->noalloc);
  size_t used = 0;
  auto take = [&](size_t bytes) -> void * {
    used = (used + 255) & ~(size_t)255;
    void *p = base + used;
    used += std::max<size_t>(bytes, 1);
    return p;
  };
  SpScratch v[kMaxSpecies];
  int64_t nunits = 0;
  for (int s = 0; s < nsp; s++) {
    SpScratch &S = v[s];
    const size_t n = (size_t)sp[s].n;
    const size_t maxseg = np + n / kSeg + 1;
    S.cap = (int64_t)n;
    S.maxseg = (int64_t)maxseg;
    S.tag = static_cast<uint32_t *>(take(n * sizeof(uint32_t)));
    S.perm = static_cast<int32_t *>(take(n * sizeof(int32_t)));
    S.cnt = static_cast<int32_t *>(take(maxseg * kCntRow * sizeof(int32_t)));
    S.pre = static_cast<int32_t *>(take(maxseg * nc * sizeof(int32_t)));
    S.sstart = static_cast<int32_t *>(take((np + 1) * sizeof(int32_t)));
    S.snext = static_cast<int32_t *>(take((np + 1) * sizeof(int32_t)));
    S.tmp = static_cast<int64_t *>(take((np + 1) * sizeof(int64_t)));
    S.tot = static_cast<int32_t *>(take(np * nc * sizeof(int32_t)));
    S.rbase = static_cast<int64_t *>(take(np * nc * sizeof(int64_t)));
    S.in = static_cast<int64_t *>(take(np * sizeof(int64_t)));
    S.noff = static_cast<int64_t *>(take((np + 1) * sizeof(int64_t)));
    S.maxunits = (int64_t)np + ((int64_t)maxseg + c->g.spc - 1) / c->g.spc + 1;
    S.ubase = nunits;
    nunits += S.maxunits;
  }
  const bool pers = c->cfg.mode == PIC_MODE_PERSISTENT;
  Unit *units = pers ? static_cast<Unit *>(take((size_t)nunits * sizeof(Unit))) : nullptr;
  if (used > kNoAllocBytes)
    return fail(c, PIC_ERR_CAPACITY,
                "pic_step_noalloc: these particles need %zu bytes of scratch, the static "
                "array holds %zu",
                used, kNoAllocBytes);
  hipStream_t st = (hipStream_t)stream;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, PIC_ERR_HIP, "hipSetDevice");
  if ((r = resident_flush(c, st)) != PIC_OK) return r;  // PIC_FLAG_RESIDENT: dense layout first
  if (nsteps == 0) return finish(c, st);
  // the static array holds whatever the last call on this GPU left there:
  // segment starts (and work units, with a zero ticket) from the offsets
  hipError_t e = launch_layout(c->g, make_args(c, sp, nsp, v), units, c->qctl, st);
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  // no timing events (their creation may allocate), no graph capture
  const bool timing = c->tm.on;
  c->tm.on = false;
  r = step_dense(c, sp, nsp, f, nsteps, st, v, units, false);
  c->tm.on = timing;
  c->layout_stale = true;  // the context's own scratch no longer matches
  if (r != PIC_OK) return r;
  return finish(c, st);
}

pic_status pic_rho(pic_ctx *c, const pic_species *sp, int32_t nsp, double *rho, void *stream) {
  if (!c) return PIC_ERR_ARG;
  if (c->poisoned) return fail(c, PIC_ERR_STATE, "context unusable after a device error");
  if (!rho) return fail(c, PIC_ERR_ARG, "null rho");
  if (!sp || nsp < 1) return fail(c, PIC_ERR_ARG, "no species");
  if (nsp > kRhoMaxSpecies) return fail(c, PIC_ERR_CAPACITY, "at most %d species", kRhoMaxSpecies);
  RhoArgs a{};
  a.dim = c->cfg.dim;
  for (int k = 0; k < 3; k++) {
    a.n[k] = c->g.n[k];
    a.patch[k] = k < c->cfg.dim ? c->cfg.patch[k] : 1;
    a.np[k] = a.n[k] / a.patch[k];
    a.inv_d[k] = c->g.inv_d[k];
  }
  a.nsp = nsp;
  for (int s = 0; s < nsp; s++) {
    const pic_species &p = sp[s];
    if (p.n < 0 || p.n > p.capacity) return fail(c, PIC_ERR_CAPACITY, "species %d: bad n", s);
    for (int k = 0; k < c->cfg.dim; k++)
      if (!p.x[k]) return fail(c, PIC_ERR_ARG, "species %d: null position", s);
    if (!p.w || !p.offset) return fail(c, PIC_ERR_ARG, "species %d: null weight/offset", s);
    a.s[s].q = p.q;
    for (int k = 0; k < 3; k++) a.s[s].x[k] = k < c->cfg.dim ? p.x[k] : nullptr;
    a.s[s].w = p.w;
    a.s[s].off = p.offset;
  }
  a.rho = rho;
  size_t tile = sizeof(double);
  for (int k = 0; k < c->cfg.dim; k++) tile *= (size_t)(a.patch[k] + 3);
  hipStream_t st = (hipStream_t)stream;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, PIC_ERR_HIP, "hipSetDevice");
  if (const pic_status r = resident_flush(c, st); r != PIC_OK) return r;  // PIC_FLAG_RESIDENT: dense layout first
  const hipError_t e =
      timed(c, PIC_KERNEL_RHO, st, [&] { return launch_rho(a, c->err_dev, tile, st); });
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  return finish(c, st);
}

pic_status pic_maxwell(pic_ctx *c, double *const e[3], double *const b[3],
                       const double *const j[3], int32_t nsteps, void *stream) {
  // the forward step only reads the current
  double *jr[3] = {const_cast<double *>(j ? j[0] : nullptr), const_cast<double *>(j ? j[1] : nullptr),
                   const_cast<double *>(j ? j[2] : nullptr)};
  return yee_steps(c, e, b, j ? jr : nullptr, nsteps, false, stream);
}

pic_status pic_cycle(pic_ctx *c, pic_species *sp, int32_t nsp, double *const e[3],
                     double *const b[3], double *const j[3], int32_t nsteps, void *stream) {
  if (!c) return PIC_ERR_ARG;
  if (!e || !b || !j) return fail(c, PIC_ERR_ARG, "null field array");
  if (c->g.n[1] > 65535 || c->g.n[2] > 65535)
    return fail(c, PIC_ERR_ARG, "the field solver takes at most 65535 cells along y and z");
  pic_fields f{};
  YeeArgs y{};
  y.dim = c->cfg.dim;
  for (int k = 0; k < 3; k++) {
    f.e[k] = e[k];
    f.b[k] = b[k];
    f.j[k] = j[k];
    y.n[k] = c->g.n[k];
    y.c[k] = k < c->cfg.dim ? c->cfg.dt / c->cfg.d[k] : 0.0;
    y.e[k] = e[k];
    y.b[k] = b[k];
    y.j[k] = j[k];
  }
  y.dt = c->cfg.dt;
  c->cycle = true;
  c->yee = y;
  const pic_status r = pic_step(c, sp, nsp, &f, nsteps, stream);
  c->cycle = false;
  return r;
}

pic_status pic_maxwell_adjoint(pic_ctx *c, double *const eb[3], double *const bb[3],
                               double *const jb[3], int32_t nsteps, void *stream) {
  return yee_steps(c, eb, bb, jb, nsteps, true, stream);
}

pic_status pic_adjoint(pic_ctx *c, const pic_species *ck, int32_t nsp, const pic_fields *f,
                       const double *const jbar[3], int32_t nsteps, int32_t with_deposit,
                       pic_cotangent *cot, double *const ebar[3], double *const bbar[3],
                       void *stream) {
  if (!c) return PIC_ERR_ARG;
  if (c->poisoned) return fail(c, PIC_ERR_STATE, "context unusable after a device error");
  if (c->cfg.dim != 2) return fail(c, PIC_ERR_ARG, "pic_adjoint supports 2D3V only");
  if (!ck || nsp < 1 || nsp > kMaxSpecies || !cot)
    return fail(c, PIC_ERR_ARG, "bad species or cotangent arguments");
  if (nsteps < 1 || nsteps > kAdjMaxSteps)
    return fail(c, PIC_ERR_ARG, "nsteps must be in [1, %d]", kAdjMaxSteps);
  if (!fields_ok(c, f, true, false)) return fail(c, PIC_ERR_ARG, "null field pointer");
  if (!ebar || !bbar) return fail(c, PIC_ERR_ARG, "null field cotangent");
  for (int k = 0; k < 3; k++)
    if (!ebar[k] || !bbar[k]) return fail(c, PIC_ERR_ARG, "null field cotangent");
  if (with_deposit < 0 || with_deposit > 2)
    return fail(c, PIC_ERR_ARG, "with_deposit must be 0, 1 or 2");
  if (with_deposit && (!jbar || !jbar[0] || !jbar[1] || !jbar[2]))
    return fail(c, PIC_ERR_ARG, "with_deposit needs jbar");
  AdjArgs a{};
  a.nsp = nsp;
  for (int s = 0; s < nsp; s++) {
    const pic_species &p = ck[s];
    const pic_cotangent &q = cot[s];
    if (p.n < 0 || p.n > p.capacity) return fail(c, PIC_ERR_CAPACITY, "species %d: bad n", s);
    if (!(p.m > 0) || !std::isfinite(p.q)) return fail(c, PIC_ERR_ARG, "species %d: q, m", s);
    if (!p.x[0] || !p.x[1] || !p.u[0] || !p.u[1] || !p.u[2] || !p.w || !p.id)
      return fail(c, PIC_ERR_ARG, "species %d: null particle array", s);
    if (q.n < 0 || !q.x[0] || !q.x[1] || !q.u[0] || !q.u[1] || !q.u[2])
      return fail(c, PIC_ERR_ARG, "species %d: null cotangent array", s);
    AdjSp &d = a.s[s];
    d.alpha = (p.q / p.m) * (0.5 * c->cfg.dt);
    d.q = p.q;
    d.n = p.n;
    d.nid = q.n;
    for (int k = 0; k < 3; k++) {
      d.x[k] = k < 2 ? p.x[k] : nullptr;
      d.u[k] = p.u[k];
      d.xb[k] = k < 2 ? q.x[k] : nullptr;
      d.ub[k] = q.u[k];
    }
    d.w = p.w;
    d.id = p.id;
    d.off = c->nb > 1 ? nullptr : p.offset;  // x-bins: the untiled kernel
  }
  hipStream_t st = (hipStream_t)stream;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, PIC_ERR_HIP, "hipSetDevice");
  if (const pic_status r = resident_flush(c, st); r != PIC_OK) return r;  // PIC_FLAG_RESIDENT: dense layout first
  hipError_t e = timed(c, PIC_KERNEL_ADJOINT, st, [&] {
    return launch_adjoint(c->g, a, f->e, f->b, with_deposit ? jbar : nullptr, ebar, bbar, nsteps,
                          with_deposit, c->err_dev, st);
  });
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  return finish(c, st);
}

}  // extern "C"
