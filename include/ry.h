/*
 * ry.h -- C ABI of the MI355X (gfx950) octree hydro library.
 *
 * The library advances the ideal-gas Euler equations on a Peano-Hilbert
 * ordered octree (RAMSES-yOMP, Sec. 1: octs of 2x2x2 cells, each level
 * halving the cell size, octs ordered along the Hilbert curve) with the
 * per-oct unsplit MUSCL-Hancock update (MinMod slopes, half-step predictor,
 * HLLC fluxes, conservative update with coarse-fine flux correction) that
 * the paper's godunov_fine routine performs (Table 1), and level
 * subcycling with dt(l+1) = dt(l)/2 (Sec. 2.3, next to Eq. 1).
 *
 * Conventions for every call:
 *   - Plain C types only; no C++ types or exceptions cross the ABI.
 *   - Host pointers are borrowed for the duration of the call only.
 *   - Device memory belongs to the context; it is obtained through the
 *     config's dev_alloc hook (NULL -> hipMalloc) and released on destroy.
 *   - Every call returns an ry_status; RY_EINVAL leaves the state untouched;
 *     ry_last_error() gives a per-context message.
 *   - Device-side numeric faults (non-finite state, rho <= 0 or E <= 0 in a
 *     leaf cell) are latched in a device error word and reported as
 *     RY_ENUMERIC by the next syncing call (ry_cfl_dt, ry_advance,
 *     ry_conserved_totals, ry_download, ry_batch_run).
 *   - No thread safety per context; distinct contexts are independent.
 *   - Work is enqueued on cfg.stream (a hipStream_t; NULL = the library's
 *     own stream).  Calls marked "syncs" wait for that stream.
 *
 * State layout (also the ry_download / ry_upload layout): per level, octs in
 * ascending Hilbert key order; nv = 5 + nscalar planes (rho, rho u, rho v,
 * rho w, E, then rho s_k for each passive scalar s_k) of 8*n_oct FP64
 * values; cell index = 8*oct + (ix + 2*iy + 4*iz).
 */
#ifndef RY_H
#define RY_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct ry_ctx ry_ctx;

typedef enum {
  RY_OK = 0,
  RY_EINVAL = -1,    /* invalid argument or configuration                 */
  RY_ENOMEM = -2,    /* device or host allocation failed (nothing leaked) */
  RY_EHIP = -3,      /* a HIP runtime call failed                         */
  RY_ESTATE = -4,    /* call out of the subcycling order, or not built    */
  RY_ENUMERIC = -5   /* numeric fault latched on the device               */
} ry_status;

enum { RY_FP64 = 0, RY_MIXED = 1 };               /* precision form           */
enum { RY_BC_PERIODIC = 0, RY_BC_OUTFLOW = 1 };
enum { RY_REFINE_NONE = 0, RY_REFINE_GRAD = 1, RY_REFINE_MASS = 2 };
#define RY_MAX_LEVELS 16
#define RY_MAX_SCALARS 4

typedef struct {
  int32_t level_min, level_max; /* level numbers; dx(l) = boxlen / (nbase[0] 2^(l-level_min)) */
  int32_t nbase[3];             /* cells per axis at level_min; even, at least 2             */
  double boxlen, gamma, cfl;    /* gamma > 1, cfl > 0                                        */
  int32_t bc[6];                /* -x,+x,-y,+y,-z,+z: RY_BC_*; periodic pairs must match      */
  int32_t precision;            /* RY_FP64 | RY_MIXED                                         */
  int32_t refine;               /* RY_REFINE_*                                                */
  double refine_param;          /* theta (GRAD) or rho_thr (MASS)                             */
  double rho_floor, p_floor;    /* > 0                                                        */
  void* stream;                 /* hipStream_t borrowed from the caller; NULL = own stream   */
  void* (*dev_alloc)(size_t bytes, void* user);  /* NULL = hipMalloc                      */
  void (*dev_free)(void* p, void* user);
  void* alloc_user;
  int32_t nscalar;              /* passive scalars (metals, chemistry, dust) advected with    */
                                /* the mass flux, 0..RY_MAX_SCALARS; not in batched boxes     */
} ry_config;

/* Host callback filling newly created cells of `level`: ijk holds 3*ncell
 * integer cell coordinates (x,y,z interleaved), U receives nv planes of
 * ncell conserved values.  Called during ry_amr_build only. */
typedef void (*ry_fill_fn)(void* user, int32_t level, int64_t ncell, const int32_t* ijk, double* U);

/* Create a context (validates cfg; allocates nothing on the device). */
ry_status ry_create(const ry_config* cfg, ry_ctx** out);
void ry_destroy(ry_ctx* ctx);

/* Build the octree from the level_min field U_base (host, nv planes of
 * nbase[0]*nbase[1]*nbase[2] values, x fastest): refinement flags by the
 * configured criterion on leaf cells, the neighbour rule (a cell is refined
 * only when its 26 neighbours exist at its level), Hilbert ordering, values
 * of new cells from `fill`, restriction of refined cells, upload.
 * RY_EINVAL if a level's octs plus ghost octs reach 2^29 (the kernels index
 * a level's cells in 32 bits).  Syncs. */
ry_status ry_amr_build(ry_ctx* ctx, const double* U_base, ry_fill_fn fill, void* user);

ry_status ry_level_info(const ry_ctx* ctx, int32_t level, int64_t* n_oct, int64_t* n_leaf_cells);
/* Hilbert keys (n_oct) and refined-cell masks (n_oct bytes, bit c = cell c)
 * copied from the device (syncs; RY_EHIP on a copy failure). */
ry_status ry_get_mesh(const ry_ctx* ctx, int32_t level, uint64_t* keys, uint8_t* refined);

/* dt of the next coarse step: min over levels of 2^(l-level_min) * cfl *
 * dx(l) / max over leaf cells of (|u|+|v|+|w|+3c).  Syncs. */
ry_status ry_cfl_dt(ry_ctx* ctx, double* dt_coarse);

/* One step of `level` with time step dt (async on the stream).  Order rule
 * (fine-first subcycling): a step of l < level_max is legal only after
 * exactly two steps of l+1 since l's previous step (when l+1 is non-empty),
 * each of dt/2 exactly; otherwise RY_ESTATE / RY_EINVAL. */
ry_status ry_hydro_step(ry_ctx* ctx, int32_t level, double dt);

/* Up to n_coarse coarse steps, each with dt from the CFL rule clipped to
 * reach t_end exactly; dt stays on the device (no host sync per step);
 * steps are replayed from a captured hipGraph.  *t_io: time in/out.  Syncs. */
ry_status ry_advance(ry_ctx* ctx, int32_t n_coarse, double t_end, double* t_io);

/* Regrid between coarse steps (dynamic refinement, the refine_fine step of
 * the paper's Table 1).  Top-down over l = level_min .. level_max-1: every
 * cell of level l is re-flagged on its current density by the configured
 * criterion, under the build's neighbour rule (26 neighbours at level l);
 * level l+1 becomes the children of the refined cells in Hilbert order --
 * surviving octs keep their state, new octs take the MinMod-linear
 * interpolation of their parent cell and its six face neighbours (the
 * coarse-fine ghost formula), octs whose parent is no longer refined
 * disappear with their descendants.  Then refined cells are restricted
 * bottom-up.  By default every step runs on the device (flags, child
 * levels, state remap, tile tables, ghost octs); only counts cross PCIe.
 * RY_ESTATE inside a coarse step; RY_EINVAL (mesh unchanged) if a source
 * the neighbour rule guarantees is missing, a level's octs plus ghost octs
 * would reach 2^29, or, on the device path, a level reaches 2^28 octs or
 * 2^25 tiles (its counts are 32-bit).  Counts of created / destroyed
 * octs (either may be NULL).  Syncs. */
ry_status ry_regrid(ry_ctx* ctx, int64_t* n_created, int64_t* n_destroyed);
/* on = 0: later regrids evaluate flags and build tables on the host from
 * the densities (8 B per cell crosses PCIe) and keep only the state remap on
 * the device; on != 0 (the default): all on the device.  Both give the same
 * mesh and state bit for bit. */
ry_status ry_set_regrid_device(ry_ctx* ctx, int32_t on);
/* Change the refinement parameter (theta or rho_thr) used by later regrids. */
ry_status ry_set_refine_param(ry_ctx* ctx, double value);

/* Sum over leaf cells of U * dx^3 (nv values: mass, momentum, energy, then
 * the scalar masses), deterministic reduction order.  Syncs. */
ry_status ry_conserved_totals(ry_ctx* ctx, double* tot);

/* Copy one level's state (all cells of all octs) to / from the host.
 * ry_download syncs; ry_upload syncs and recomputes the stored CFL data. */
ry_status ry_download(ry_ctx* ctx, int32_t level, double* U);
ry_status ry_upload(ry_ctx* ctx, int32_t level, const double* U);

/* Batched independent boxes (single level, periodic or outflow each):
 * cfgs[b] describes box b (level_min == level_max), U0[b] its field as for
 * ry_amr_build.  All boxes share one tile list (and, with a persistent
 * tuning, one work queue).  Default tuning {1, 0, 4, 1, 1, 4}; ry_autotune
 * picks among the plain and the persistent queue-fed launches.  RY_EINVAL
 * if the boxes' octs together reach 2^29. */
ry_status ry_batch_create(const ry_config* cfgs, int32_t nbox, const double* const* U0, ry_ctx** out);
/* nsteps steps of every box, each box with its own CFL dt computed on the
 * device, as one captured graph (reused while nsteps and the state parity
 * repeat) of one hydro launch per step over the tiles of all boxes.
 * Syncs. */
ry_status ry_batch_run(ry_ctx* ctx, int32_t nsteps);
ry_status ry_batch_box_info(const ry_ctx* ctx, int32_t box, int64_t* n_oct, double* t);
ry_status ry_batch_download(ry_ctx* ctx, int32_t box, double* U);

/* Tuning of the hydro kernel launch (see ry_tuning fields).  Results in FP64
 * do not depend on the tuning. */
typedef struct {
  int32_t tiles_per_wg;   /* tiles per workgroup: 1, 2 or 4 (tile_cells 4); 1 (tile_cells 8) */
  int32_t persistent;     /* 0: one workgroup per tile group; 1: work queue (tile_cells 4)  */
  int32_t waves_per_cu;   /* persistent grid = CUs * waves_per_cu / waves per workgroup     */
  int32_t batch;          /* tile groups popped per queue access                            */
  int32_t waves_per_tile; /* tile_cells 4: 1, 2 or 4 wavefronts per tile (8, 16, 32 threads */
                          /* per oct), tiles_per_wg * waves_per_tile <= 4; with passive     */
                          /* scalars only {1,0,*,*,1}, {1,0,*,*,2} and {2,0,*,*,1};         */
                          /* tile_cells 8: 8 (one thread per cell) or 4 (two cells per      */
                          /* thread) (else RY_EINVAL)                                        */
  int32_t tile_cells;     /* tile edge in cells: 4 (a 2x2x2-oct tile, 64 cells) or 8 (a     */
                          /* 4x4x4-oct tile, 512 cells: fewer halo cells converted,          */
                          /* predicted and solved per cell; hydro variables alone)           */
} ry_tuning;
/* ry_set_tuning sets the tuning of every level; ry_get_tuning returns the
 * tuning of level_min.  RY_EINVAL for a combination without a kernel (see
 * the fields).  Choosing the 8^3-cell tile builds its tile tables on the
 * device (syncs). */
ry_status ry_set_tuning(ry_ctx* ctx, const ry_tuning* t);
ry_status ry_get_tuning(const ry_ctx* ctx, ry_tuning* t);
/* Tuning of one level (RY_EINVAL outside level_min..level_max).  Choosing
 * the 8^3-cell tile for a level builds that level's tile tables on the
 * device (syncs). */
ry_status ry_set_level_tuning(ry_ctx* ctx, int32_t level, const ry_tuning* t);
ry_status ry_get_level_tuning(const ry_ctx* ctx, int32_t level, ry_tuning* t);
/* Per level, time every candidate tuning (small tiles with 1-4 tiles per
 * workgroup and 1-4 wavefronts per tile, plain or queue-fed; the 8^3-cell
 * tile) on the current state (state unchanged): each candidate once, then
 * the three fastest and the default {1, 0, 4, 1, 1, 4} again in six
 * interleaved rounds; the lowest median wins, but the default stays unless
 * beaten by more than 2%.  Each level keeps its winner; *best = the winner
 * of level_min.  times_ms[i] (n_cand of them) = the hydro time of one
 * coarse step if candidate i ran on every level (level l weighted by its
 * 2^(l - level_min) substeps).  Syncs. */
ry_status ry_autotune(ry_ctx* ctx, ry_tuning* best, double* times_ms, int32_t max_cand, int32_t* n_cand);

/* Diagnostics. */
/* Floor activations (density and pressure floors counted separately) since
 * the build, each event of a step counted once, however often the kernels
 * recompute the value: a leaf cell's own primitive conversion; both face
 * states of each face an update uses (counted by the face's upper cell when
 * that is a leaf, else by its lower cell); once per parent step, every
 * ghost cell of a refined level (the cells of the oct positions next to the
 * level's octs that hold no oct of the level).  The time-step computation
 * is not counted.  Syncs. */
int64_t ry_floor_count(ry_ctx* ctx);
/* Per-kernel timing with HIP events on the launch stream (0 = off).  While
 * on, ry_advance launches eagerly instead of replaying graphs. */
ry_status ry_set_timing(ry_ctx* ctx, int32_t on);
ry_status ry_kernel_time(ry_ctx* ctx, const char* kernel, int64_t* launches, double* total_ms);
/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): the CFL time step
 * of one level held in the caller's device memory, the same reduction as
 * ry_cfl_dt's for one level, dt = cfl * dx / max over leaf cells of
 * (|u|+|v|+|w|+3c) (+inf when no cell is a leaf).  U: device, 5 planes of
 * `plane` doubles (plane >= 8 * n_oct), cell index 8*oct + (ix + 2 iy +
 * 4 iz) as in ry_download; refined: device, n_oct bytes, bit c = cell c
 * refined (refined cells are left out); dt: host, written on RY_OK; stream:
 * a hipStream_t or NULL.  Allocates nothing: the partial maxima live in a
 * 512 KiB array in device memory that every GPU the library runs on holds
 * for the life of the process; n_oct above 2,097,152 (what it covers) ->
 * RY_EINVAL before any launch.  Calls that overlap on one GPU share that
 * array and race.  RY_ENUMERIC if a leaf cell is non-finite or has rho <= 0
 * or E <= 0.  Syncs the stream. */
ry_status ry_cfl_dt_noalloc(const double* U, int64_t plane, int64_t n_oct, const uint8_t* refined, double gamma,
                            double cfl, double dx, double rho_floor, double p_floor, double* dt, void* stream);

/* Device bandwidth probe: copy `bytes` within device memory `reps` times,
 * returns the average kernel time in ms.  Used to calibrate counters. */
ry_status ry_copy_probe(ry_ctx* ctx, size_t bytes, int32_t reps, double* ms);
const char* ry_last_error(const ry_ctx* ctx);

/* Host-only mesh inspection (no device work, usable without a GPU): runs the
 * library's own octree builder -- refinement criterion, neighbour rule,
 * Hilbert order -- exactly as ry_amr_build does, and exposes the result.
 * ry_mesh_level with keys/refined NULL returns only n_oct. */
typedef struct ry_mesh ry_mesh;
ry_status ry_mesh_build(const ry_config* cfg, const double* U_base, ry_fill_fn fill, void* user, ry_mesh** out);
ry_status ry_mesh_level(const ry_mesh* m, int32_t level, int64_t* n_oct, uint64_t* keys, uint8_t* refined,
                        int64_t* n_ghost);
void ry_mesh_free(ry_mesh* m);
/* Peano-Hilbert key of oct coordinates with `bits` bits per axis. */
uint64_t ry_hilbert_key(int32_t bits, uint32_t x, uint32_t y, uint32_t z);

#ifdef __cplusplus
}
#endif
#endif
