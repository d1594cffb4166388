/* pic.h -- C ABI of the MI355X (gfx950) library for the per-step
 * macro-particle operators of an electromagnetic particle-in-cell loop:
 * field Interpolation, Push, pre-boundary-condition operations (pre-BC) and
 * current Projection (arXiv 2204.12837, section "Parallelization without
 * tasks": the four operators applied per patch and species, followed by a
 * synchronisation phase that applies particle boundary conditions and sorts
 * the particles).  The paper names the operators and the order-2 shape; the
 * formulas are those of the published methods it relies on: quadratic
 * B-spline shapes on Yee's staggered grid, Boris's relativistic push and
 * Esirkepov's charge-conserving current deposit.
 *
 * Conventions shared by every entry point
 *   Units     normalised: c = 1, charge in e, mass in m_e, u = p/(m c).
 *   Grid      periodic fields, n[a] cells of size d[a] per axis
 *             (particles see periodic, reflecting or removing boundaries
 *             per axis, pic_config.particle_bc); each field
 *             component is a device array of prod(n) float64 values, x
 *             fastest, entry (i,j,k) at ((i+sx/2)d_x, (j+sy/2)d_y,
 *             (k+sz/2)d_z) with stagger bits Ex(1,0,0) Ey(0,1,0) Ez(0,0,1)
 *             Bx(0,1,1) By(1,0,1) Bz(1,1,0) (J as E); in 2D (2D3V) the z
 *             bit and the z axis are dropped.
 *   Patches   the grid is split into patches of patch[a] cells (paper,
 *             section "Parallelization without tasks"); patch id
 *             Px + NPx (Py + NPy Pz); particles are stored sorted by patch:
 *             patch P owns entries [offset[P], offset[P+1]) of every particle
 *             array.  Inside a patch the order is that of the previous step
 *             (the sort is stable), except where pic_step (slab layout) or
 *             x-bins (pic_config.bin_x) state otherwise.
 *   Particles structure of arrays per species, float64 x/u/w and int64 id,
 *             all on the context's device, each of `capacity` elements.
 *   Memory    the caller owns every particle, field and offset array and
 *             never hands ownership to the library; the context owns its
 *             scratch (keys, counts, saved positions, error word).
 *   Streams   work is enqueued on the given HIP stream (NULL = the null
 *             stream) and returns without waiting, except where stated.
 *             The calls on one context share its scratch: issue them on
 *             one stream (or order the streams), never concurrently.
 *   Errors    host-detectable errors (bad config, null pointer, count above
 *             capacity, wrong call order) return at once with nothing
 *             enqueued.  Errors found by kernels (a particle moving more than
 *             one cell, a position outside the box, a particle outside the
 *             patch its offsets give it) set a sticky error word
 *             in the context; pic_check (or any call when PIC_FLAG_CHECK is
 *             set) waits for the stream and reports it.  After a device
 *             error the context refuses further work until pic_free.
 *             Nothing throws or aborts across the ABI.  One context per host
 *             thread.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_ctx pic_ctx;

typedef enum {
  PIC_OK = 0,
  PIC_ERR_ARG = 1,      /* invalid argument or configuration */
  PIC_ERR_HIP = 2,      /* a HIP runtime call failed */
  PIC_ERR_CAPACITY = 3, /* n above capacity, or too many patches/species */
  PIC_ERR_CFL = 4,      /* a particle moved more than one cell in a step */
  PIC_ERR_POS = 5,      /* a position more than one period outside the box, or
                           outside [0, L) on an axis with reflecting walls */
  PIC_ERR_STATE = 6,    /* wrong call order, or context poisoned by an error */
  PIC_ERR_UNSORTED = 7  /* a particle lies outside the patch its offsets
                           assign it to: the input was not sorted by patch */
} pic_status;

enum { PIC_MODE_PER_PATCH = 0, PIC_MODE_PERSISTENT = 1 };

/* particle boundary condition of an axis (pic_config.particle_bc) */
enum { PIC_BC_PERIODIC = 0, PIC_BC_REFLECT = 1, PIC_BC_REMOVE = 2 };

enum {
  PIC_FLAG_CHECK = 1, /* every call waits for its stream and reports device errors */
  PIC_FLAG_GRAPH = 2, /* pic_step replays captured HIP graphs of its steps
                         (in the slab layout one of eight steps as often as
                         the call allows, then one of one step for the rest;
                         in the dense layout one of two steps, whose buffer
                         swap makes two steps the period); a graph is
                         recaptured when any array pointer or count changes */
  PIC_FLAG_DETERMINISTIC = 8, /* pic_step and pic_cycle give the same bits on
                         every run: the dense layout (its counting sort is
                         stable), the per-patch launch (also in persistent
                         mode), every wave of a patch's workgroup depositing
                         into a J tile of its own, the tiles summed in wave
                         order and J at every node summed from the covering
                         tiles in a fixed order (no float64 atomics).  Costs
                         a tile buffer of npatch x species x 3 (p+5)^dim
                         doubles and fewer waves per workgroup where the
                         tiles do not fit (3D).  Not with removing walls
                         (PIC_ERR_ARG).  pic_project and pic_rho keep their
                         order-dependent float64 atomic sums. */
  PIC_FLAG_RESIDENT = 16, /* pic_step (and pic_cycle) leave the particles in
                         their slabs (second buffer set) at the end of the
                         call, and the next pic_step on the same species
                         arrays continues from there: no slab plan, no first
                         step from the dense layout and no slabs -> dense
                         copy per call, so calls of one or two steps cost
                         what a step of a long call costs.  Every call of
                         one step or more takes the slab layout (buffers
                         with its room; otherwise the call runs in the
                         dense layout and nothing stays resident).  While
                         resident, the first buffer set and the offsets are
                         stale and the caller must not write any of the
                         species' arrays: pic_sync writes them (the dense
                         layout, in the first set, as a call without the
                         flag leaves it), and so does every other entry
                         point that takes particles, and pic_step on other
                         arrays, before it starts.  pic_free writes nothing
                         back.
                         Not with PIC_FLAG_DETERMINISTIC or removing walls
                         (PIC_ERR_ARG). */
  PIC_FLAG_TRACE = 4  /* the fused kernel of pic_step's slab layout records,
                         for every work item of each launch (a (patch,
                         species) workgroup in per-patch mode, a popped unit
                         in persistent mode), its patch, workgroup and start
                         and end times; pic_trace_read returns the last
                         launch's records (the GPU counterpart of the
                         paper's per-operation scheduling diagnostics,
                         section "Task scheduling visualization") */
};

typedef struct {
  int32_t dim;         /* 2 = 2D3V, 3 = 3D3V */
  int32_t n[3];        /* cells per axis; n[2] = 1 in 2D */
  double d[3];         /* cell sizes (d[2] ignored in 2D) */
  double dt;           /* time step; must satisfy dt < 1/sqrt(sum 1/d^2) */
  int32_t patch[3];    /* patch size in cells: divides n, >= 6 (three-point
                          stencil plus ghosts); patch[2] = 1 in 2D */
  int32_t shape_order; /* interpolation/projection order: must be 2 */
  int32_t mode;        /* PIC_MODE_PER_PATCH: one workgroup per patch and
                          species; PIC_MODE_PERSISTENT: a fixed grid pulls
                          (patch, species, chunk) units from a device queue */
  int32_t chunk;       /* persistent mode: particles per work unit, a multiple
                          of 256 (0 = auto: 2048) */
  int32_t wg_size;     /* threads per workgroup, a multiple of 64 up to 1024
                          (0 = auto: 1024 in 3D; in 2D 256, or up to 1024 when
                          the LDS tiles admit fewer than four workgroups per
                          CU, as with x-bins of tall patches); the
                          dense-layout kernels use at most 256 in 2D and 512
                          in 3D */
  uint32_t flags;      /* PIC_FLAG_* */
  int32_t bin_x;       /* x-bins: width in cells of the bins a patch is cut
                          into along x (paper, sections "Parallelization
                          without tasks" and "Parallelization with OpenMP
                          task": bins of bin_x_size cells, each with its own
                          local sub-grid whose current is added to the grid
                          with a shift of a multiple of bin_x_size).  The
                          kernels stage fields and accumulate J per bin, so a
                          patch whose tiles do not fit in the 160 KB of LDS
                          can still be used.  Must divide patch[0].  0 = auto:
                          patch[0] if its tiles fit, else the widest divisor
                          of patch[0] whose tiles fit.  With more than one
                          bin per patch, the particles inside a patch are
                          ordered by bin: pic_step and pic_interp_push first
                          put them in bin order with a stable counting sort
                          inside each patch (in pic_step's slab layout, as
                          part of the copy into the slabs). */
  int32_t particle_bc[3]; /* particle boundary per axis, PIC_BC_* (ignored
                          for z in 2D); walls sit at 0 and L = n d.  Fields
                          and current stay periodic arrays: nodes beyond a
                          wall are read and written at their periodic
                          images.
                          PIC_BC_REFLECT: the paper's reflective particle
                          condition (section "Basic performance
                          benchmarks", its radiation-pressure case).  In the
                          pre-BC operation, which writes positions and
                          momenta (section "Parallelization with OpenMP
                          task"), a particle pushed across a wall is
                          mirrored back inside (x -> -x, x -> 2L - x; x = L
                          exactly goes to the largest double below L) and
                          its momentum component along the axis changes
                          sign, before its current is projected: the
                          deposit follows the mirrored move and stays
                          charge-conserving.  pic_bin reports PIC_ERR_POS
                          for a position outside [0, L) on such an axis
                          instead of wrapping it.  pic_adjoint
                          differentiates through the mirror.
                          PIC_BC_REMOVE: the paper's "delete" condition
                          (section "Parallelization without tasks": pre-BC
                          flags the particles, the synchronisation applies
                          the condition).  A particle pushed outside
                          [0, L) on such an axis deposits no current in
                          that step and is deleted; pic_bin deletes a
                          position outside [0, L) on it.  pic_step,
                          pic_cycle and pic_bin then wait for their stream
                          and set each species' n to the surviving count
                          (its particles are the first n of the arrays, as
                          always); pic_step and pic_cycle need buffers with
                          the slab layout's room for every call length
                          (PIC_ERR_CAPACITY otherwise).  In pic_adjoint a
                          particle deleted inside the segment contributes
                          nothing: its cotangents are zero. */
} pic_config;

typedef struct {
  double q, m;         /* charge, mass */
  int64_t n;           /* particles in the arrays, below 2^29 (element offsets
                          of every array fit in 32 bits as byte offsets) */
  int64_t capacity;    /* length of every particle array */
  double *x[3];        /* positions (x[2] = NULL in 2D) */
  double *u[3];        /* momenta u^{n-1/2} */
  double *w;           /* weights (density carried by one macro-particle) */
  int64_t *id;         /* particle ids (carried along, never read) */
  double *x_alt[3];    /* second buffer set: target of the sort; */
  double *u_alt[3];    /*   pic_bin and pic_step swap it with the */
  double *w_alt;       /*   first set in this struct after sorting */
  int64_t *id_alt;
  int64_t *offset;     /* [n_patches + 1] patch offsets, written by the sort */
} pic_species;

typedef struct {
  const double *e[3];  /* Ex, Ey, Ez */
  const double *b[3];  /* Bx, By, Bz */
  double *j[3];        /* Jx, Jy, Jz (accumulated into) */
} pic_fields;

/* Check a configuration without touching a device.  Pure host code.
 * Writes a reason into msg (if msg != NULL, at most len bytes with the NUL).
 * Returns PIC_OK or PIC_ERR_ARG. */
pic_status pic_validate_config(const pic_config *cfg, char *msg, size_t len);

/* Number of patches of a valid configuration (0 if invalid).  Pure host. */
int64_t pic_num_patches(const pic_config *cfg);

/* Width in cells of the x-bins a valid configuration uses (bin_x, or the
 * automatic choice when bin_x = 0); 0 if the configuration is invalid.
 * Pure host. */
int32_t pic_bin_width(const pic_config *cfg);

/* Create a context on HIP device `device`: validates cfg, allocates the
 * context's scratch.  *out is NULL on failure. */
pic_status pic_init(const pic_config *cfg, int32_t device, pic_ctx **out);

/* Release a context and its scratch (waits for the device).  NULL is a no-op. */
void pic_free(pic_ctx *ctx);

/* Synchronisation-phase sort (paper, section "Parallelization without
 * tasks": boundary conditions are applied and particles sorted after the
 * operators).  For each species: periodic wrap of every position, patch
 * key, stable counting sort by patch into the *_alt arrays, offset[]
 * written, then the two buffer sets are swapped in *sp.  Accepts particles
 * in any order and anywhere within one period of the box (within the box on
 * a reflecting axis; outside it on a removing axis they are deleted and
 * sp[s].n is updated, see pic_config.particle_bc). */
pic_status pic_bin(pic_ctx *ctx, pic_species *sp, int32_t nsp, void *stream);

/* Interpolation + Push (paper: the first two operators).  Particles must be
 * sorted by patch (offset[] valid, e.g. after pic_bin).  Gathers E and B at
 * each position with the quadratic shape, advances u by the relativistic
 * Boris push and x by dt*v.  Positions are left unwrapped (the boundary
 * condition belongs to the sort), except that they are mirrored at
 * reflecting walls; the start-of-step positions are kept in the context
 * for pic_project.  J is not touched. */
pic_status pic_interp_push(pic_ctx *ctx, pic_species *sp, int32_t nsp, const pic_fields *f,
                           void *stream);

/* Projection (paper: the fourth operator): J += Esirkepov deposit of every
 * particle's move from the positions saved by the preceding pic_interp_push
 * on this context to the current (unwrapped) positions.  Does not zero J.
 * A particle outside a removing axis deposits nothing (pic_bin deletes it).
 * PIC_ERR_STATE without a preceding pic_interp_push. */
pic_status pic_project(pic_ctx *ctx, const pic_species *sp, int32_t nsp, pic_fields *f,
                       void *stream);

/* nsteps whole steps (paper, section "Parallelization without tasks": the
 * per-patch operators, then the synchronisation phase): J <- 0, then the
 * fused Interpolation, Push, pre-BC and Projection of every species (J
 * accumulated in on-chip tiles per patch and added to the grid), then the
 * particles regrouped by patch.  Equals the sequence {zero J;
 * pic_interp_push; pic_project; pic_bin} per step, up to the order of the
 * particles inside a patch.  J holds the last step's current.  Particles
 * must be sorted (offset[] valid, e.g. by pic_bin on this context); on
 * return they are sorted again, in the first buffer set or the second
 * (follow the pointers in sp).
 *
 * Layout: with nsteps >= 3 and, for every species, capacity >=
 * n + n/8 + 80 * (number of x-bins: patches times patch[0] / bin width) and
 * capacity < 2^29, the call keeps the
 * particles in per-bin slabs of the second buffer set, updates them in
 * place and moves only those that change patch; the order inside a patch is
 * then arbitrary and the result is in the first set.  Otherwise every step
 * sorts by neighbour code (stable: the order inside a patch is the previous
 * order).  In persistent mode the fused kernel runs on a fixed grid that pulls
 * (patch, particle range) units from a device queue.  With PIC_FLAG_GRAPH
 * (and timing off) the steps replay captured HIP graphs (of eight steps and
 * of one in the slab layout, of two otherwise).  With PIC_FLAG_RESIDENT the
 * particles stay in the slabs between calls (see the flag).  The context owns an outbox of capacity
 * particles per species for the slab layout.  With removing walls every
 * call takes the slab layout and updates sp[s].n on return. */
pic_status pic_step(pic_ctx *ctx, pic_species *sp, int32_t nsp, pic_fields *f, int32_t nsteps,
                    void *stream);

/* PIC_FLAG_RESIDENT: write the particles that pic_step left in their slabs
 * back to the dense layout (first buffer set, offsets, as a pic_step
 * without the flag leaves them), enqueued on stream.  No-op when nothing is
 * resident.  With PIC_FLAG_CHECK it waits for the stream. */
pic_status pic_sync(pic_ctx *ctx, void *stream);

/* pic_step without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same computation and result as pic_step in the
 * dense layout (every step sorts by neighbour code; the order inside a patch
 * stays that of the previous step), in the same buffers and with the same
 * swap of the two buffer sets in *sp.  Its scratch (per species: 4 + 4
 * bytes per particle, the per-segment code counts, per-patch arrays; in
 * persistent mode the work units) is carved from a static device array of
 * 64 MiB that the library holds on every GPU it runs on until the process
 * ends -- about 6 million 2D particles in total (the exact need is
 * reported in the error message).  Beyond that, PIC_ERR_CAPACITY with
 * nothing enqueued.  Not for configurations with x-bins or removing walls
 * (PIC_ERR_ARG: those need pic_step's allocating paths); PIC_FLAG_GRAPH is
 * ignored and pic_timing_* do not cover these launches.
 * Every call on one GPU shares that GPU's array, and each call starts by
 * rebuilding what it needs there from the offsets: calls that overlap on
 * one GPU (other contexts, other streams, other host threads) race and
 * must be ordered by the caller.  Afterwards the other entry points on this
 * context rebuild their own segment starts from the offsets. */
pic_status pic_step_noalloc(pic_ctx *ctx, pic_species *sp, int32_t nsp, pic_fields *f,
                            int32_t nsteps, void *stream);

/* Field solver of the PIC loop (the paper's loop solves Maxwell's equations
 * on the grid with the current densities of the Projection as sources,
 * section "Parallelization without tasks"): nsteps steps of Yee's
 * finite-difference time-domain scheme, normalised units (c = 1), periodic,
 * with the same current j in every step:
 *   E <- E + dt (curl B - j)   (Ampere: B is at the half step),
 *   B <- B - dt curl E         (Faraday: with the new E).
 * Curls are differences of neighbouring staggered values divided by the
 * cell size (backward differences of B at E's positions, forward
 * differences of E at B's positions); with c_a = dt / d_a every component
 * is evaluated in one fixed order without contraction:
 *   Ex <- ((Ex + c_y dyBz) - c_z dzBy) - dt Jx, Ey <- ((Ey + c_z dzBx) -
 *   c_x dxBz) - dt Jy, Ez <- ((Ez + c_x dxBy) - c_y dyBx) - dt Jz,
 *   Bx <- (Bx - c_y dyEz) + c_z dzEy, By <- (By - c_z dzEx) + c_x dxEz,
 *   Bz <- (Bz - c_x dxEy) + c_y dyEx
 * (no z terms in 2D).  e and b (device, prod(n) values per component, x
 * fastest, the staggering of the file header) are updated in place; j is
 * read.  With the current of a pic_step step (Esirkepov's charge-conserving
 * deposit) the update keeps Gauss's law.  At most 65535 cells along y and
 * along z.  Timed as PIC_KERNEL_MAXWELL. */
pic_status pic_maxwell(pic_ctx *ctx, double *const e[3], double *const b[3],
                       const double *const j[3], int32_t nsteps, void *stream);

/* The self-consistent PIC loop: nsteps times {the pic_step step on E and B
 * (J <- its current), then one pic_maxwell field step of E and B with that
 * J}.  Same layouts, modes, graphs and conditions as pic_step (a captured
 * slab-layout step includes the field step); e and b are updated in place,
 * j holds the last step's current.  Equals alternating pic_step(.., 1) and
 * pic_maxwell(.., 1), up to the order of the particles inside a patch and
 * the rounding of J's float64 atomic sums. */
pic_status pic_cycle(pic_ctx *ctx, pic_species *sp, int32_t nsp, double *const e[3],
                     double *const b[3], double *const j[3], int32_t nsteps, void *stream);

/* Charge density (the charge-density projection that accompanies the
 * current projection, section "Parallelization with OpenMP task"):
 * rho += sum over species and particles of q w S(x - node) on the primal
 * nodes (prod(n) values, x fastest), S the quadratic B-spline of the
 * Interpolation operator.  Particles must be sorted by patch (offset[]
 * valid) with positions inside the box; a particle outside its patch sets
 * the sticky position error.  Each term is (q w)(Sx Sy [Sz]); per patch the
 * terms are summed in an on-chip tile, then added to rho with float64
 * atomics.  Timed as PIC_KERNEL_RHO. */
pic_status pic_rho(pic_ctx *ctx, const pic_species *sp, int32_t nsp, double *rho, void *stream);

/* Reverse mode of pic_maxwell: eb and bb hold, on entry, the cotangents of
 * E and B after nsteps field steps (d L / d E_final, d L / d B_final) and on
 * return those of E and B before them; jb (device, accumulated +=) receives
 * the cotangent of the current used in every step.  The transpose of one
 * step, applied nsteps times: the transposed Faraday update (the discrete
 * curls of the staggered grid are each other's transposes) of eb with the
 * current's cotangent jb -= dt eb, then the transposed Ampere update of bb:
 *   Ebx <- (Ebx - c_y dyBbz) + c_z dzBby, Eby <- (Eby - c_z dzBbx) +
 *   c_x dxBbz, Ebz <- (Ebz - c_x dxBby) + c_y dyBbx, Jb <- Jb - dt Eb,
 *   Bbx <- (Bbx + c_y dyEbz) - c_z dzEby, Bby <- (Bby + c_z dzEbx) -
 *   c_x dxEbz, Bbz <- (Bbz + c_x dxEby) - c_y dyEbx
 * (backward differences of Bb, forward differences of Eb).  Timed as
 * PIC_KERNEL_MAXWELL. */
pic_status pic_maxwell_adjoint(pic_ctx *ctx, double *const eb[3], double *const bb[3],
                               double *const jb[3], int32_t nsteps, void *stream);

/* Cotangents of one species' particle state, indexed by particle id. */
typedef struct {
  double *x[3]; /* d L / d position (x[2] unused in 2D) */
  double *u[3]; /* d L / d momentum */
  int64_t n;    /* length of every array; particle ids must lie in [0, n) */
} pic_cotangent;

/* Reverse-mode derivative of a segment of nsteps (1..8) 2D3V steps, for a
 * loss L = sum Jbar . J_final that depends on the current deposited by the
 * last step (fields static, J rebuilt every step, so only the final deposit
 * enters L and particles do not interact).  The gradient of the Boris push,
 * the quadratic-shape interpolation and Esirkepov's deposit, written by hand.
 *   ckpt      particle state at the segment start (any order; ids index the
 *             cotangents).  Not modified.
 *   f         E and B (read); f->j unused.
 *   with_deposit  1: the segment's last step is the final step, its deposit
 *             contracted with jbar seeds the cotangents; 0: cot holds, on
 *             entry, the cotangents of the state after the segment; 2: both
 *             (the last step's deposit enters the loss through jbar and the
 *             later state through cot, as in a self-consistent loop where
 *             the current drives the field solver).
 *   cot       on return: cotangents of the state at the segment start.
 *   ebar,bbar d L / d E and d L / d B, accumulated (+=).
 * The segment is recomputed from ckpt with the forward kernels' operation
 * sequence (checkpointing: the caller keeps states every few steps and calls
 * this for each segment from the last to the first).  2D only. */
pic_status pic_adjoint(pic_ctx *ctx, const pic_species *ckpt, int32_t nsp, const pic_fields *f,
                       const double *const jbar[3], int32_t nsteps, int32_t with_deposit,
                       pic_cotangent *cot, double *const ebar[3], double *const bbar[3],
                       void *stream);

/* Kernel classes whose launches the context can time. */
enum {
  PIC_KERNEL_ZERO = 0,        /* J <- 0 */
  PIC_KERNEL_IPP = 1,         /* fused Interpolation + Push + pre-BC + Projection */
  PIC_KERNEL_REBIN = 2,       /* neighbour-code counting sort (bases, scan, scatter) */
  PIC_KERNEL_INTERP_PUSH = 3, /* split path: Interpolation + Push */
  PIC_KERNEL_PROJECT = 4,     /* split path: Projection */
  PIC_KERNEL_TAG = 5,         /* split path: pre-BC codes and ranks */
  PIC_KERNEL_SORT = 6,        /* general sort of unsorted input */
  PIC_KERNEL_ADJOINT = 7,     /* adjoint segment */
  PIC_KERNEL_EXCHANGE = 8,    /* slab layout: departures, arrivals, counts, work units */
  PIC_KERNEL_SLAB = 9,        /* slab layout, once per call: the slab plan, the first
                                 step's fused kernel (which fills the slabs from the
                                 dense layout; with x-bins, the bin placement), and
                                 slabs -> dense */
  PIC_KERNEL_MAXWELL = 10,    /* field solver step (Ampere and Faraday) */
  PIC_KERNEL_RHO = 11,        /* charge density */
  PIC_KERNEL_COUNT = 12
};

/* Observability: when on, every later launch of a kernel class is bracketed
 * by HIP events recorded on the caller's stream.  Turning it on clears the
 * totals.  Costs two event records per launch. */
pic_status pic_timing_enable(pic_ctx *ctx, int32_t on);

/* Total milliseconds and number of launches of a kernel class since timing
 * was enabled.  Waits for the recorded events. */
pic_status pic_timing_read(pic_ctx *ctx, int32_t kernel, double *total_ms, int64_t *launches);

/* One work item of a traced fused-kernel launch (PIC_FLAG_TRACE). */
typedef struct {
  int32_t patch;   /* the kernels' patch (x-bin when patches are cut into bins) */
  int32_t unit;    /* persistent mode: index of the unit in the launch's work
                      list; per-patch mode: the species */
  int32_t block;   /* workgroup that ran it (persistent mode: the worker) */
  int32_t species; /* species, or -1 for a unit spanning every species */
  uint64_t t0, t1; /* start and end, ticks of the device's constant 100 MHz
                      clock (s_memrealtime) */
} pic_trace_record;

/* Records of the last traced fused-kernel launch on this context (the last
 * step of the last pic_step or pic_cycle call in the slab layout with
 * PIC_FLAG_TRACE): waits for the device, copies at most cap records to out
 * (host memory; may be NULL when cap = 0) and sets *n to the launch's
 * record count (0 before any traced launch).  The dense layout's kernels and
 * the split entry points are not traced. */
pic_status pic_trace_read(pic_ctx *ctx, pic_trace_record *out, int64_t cap, int64_t *n);

/* Wait for `stream` and report the sticky device error word. */
pic_status pic_check(pic_ctx *ctx, void *stream);

/* Text of the last error on this context ("" if none). */
const char *pic_last_error(const pic_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
