/*
 * ryo.h -- C interface of the FP64 CPU oracle for the octree
 * MUSCL-Hancock / MinMod / HLLC hydro step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this library; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the GPU
 * library (its own header, its own mesh builder, its own Hilbert curve).
 *
 * What the paper fixes (RAMSES-yOMP, Sec. 1 and Sec. 2.3, Eq. 1):
 *   - the mesh is an octree: octs of 2x2x2 cells, each level halving the
 *     cell size (Sec. 1, octree description);
 *   - octs are ordered along the Peano-Hilbert curve (Sec. 1, domain
 *     decomposition paragraph);
 *   - level l+1 takes two steps of half the time step per step of level l
 *     (Sec. 2.3, the subcycling weight next to Eq. 1);
 *   - the hydro routine (godunov_fine, Table 1) is the loop over octs.
 * The numerical scheme itself is not given in the paper; the oracle follows
 * the published textbook methods named in oracle/ryo.c for each step.
 */
#ifndef RYO_H
#define RYO_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { RYO_OK = 0, RYO_EINVAL = -1, RYO_ENOMEM = -2, RYO_ESTATE = -4, RYO_ENUMERIC = -5 };
enum { RYO_BC_PERIODIC = 0, RYO_BC_OUTFLOW = 1 };
enum { RYO_REFINE_NONE = 0, RYO_REFINE_GRAD = 1, RYO_REFINE_MASS = 2 };
#define RYO_MAX_LEVELS 16
#define RYO_MAX_SCALARS 4

typedef struct {
  int32_t level_min, level_max;  /* levels are numbered like the paper's l  */
  int32_t nbase[3];              /* cells per axis at level_min (even)       */
  double boxlen, gamma, cfl;
  int32_t bc[6];                 /* -x,+x,-y,+y,-z,+z                         */
  int32_t refine;                /* RYO_REFINE_*                              */
  double refine_param;           /* theta (GRAD) or rho_thr (MASS)            */
  double rho_floor, p_floor;
  int32_t nscalar;               /* passive scalars advected with the mass
                                  * flux (0..RYO_MAX_SCALARS); the state then
                                  * has 5 + nscalar planes, the scalars
                                  * conserved as rho*s                       */
} ryo_config;

/* Fill callback: values U (5 + nscalar planes of ncell, SoA) of new cells at `level`,
 * given their integer cell coordinates ijk (3*ncell, x,y,z interleaved). */
typedef void (*ryo_fill_fn)(void* user, int32_t level, int64_t ncell,
                            const int32_t* ijk, double* U);

typedef struct ryo_ctx ryo_ctx;

int  ryo_create(const ryo_config* cfg, ryo_ctx** out);
void ryo_destroy(ryo_ctx* c);
/* U_base: host, 5 + nscalar planes of nbase[0]*nbase[1]*nbase[2] values, x fastest. */
int  ryo_amr_build(ryo_ctx* c, const double* U_base, ryo_fill_fn fill, void* user);
int  ryo_level_info(const ryo_ctx* c, int32_t level, int64_t* n_oct, int64_t* n_leaf_cells);
int  ryo_get_mesh(const ryo_ctx* c, int32_t level, uint64_t* keys, uint8_t* refined);
int  ryo_get_coords(const ryo_ctx* c, int32_t level, int32_t* oct_xyz);
/* U: 5 + nscalar planes of 8*n_oct values; cell index = 8*oct + (ix + 2 iy + 4 iz). */
int  ryo_download(const ryo_ctx* c, int32_t level, double* U);
int  ryo_upload(ryo_ctx* c, int32_t level, const double* U);
/* Regrid between coarse steps: re-flag every cell of levels level_min ..
 * level_max-1 top-down with the build's criterion and neighbour rule; kept
 * child octs keep their values, new ones take the MinMod-linear
 * interpolation of their parent cell, orphaned octs disappear; then
 * restriction bottom-up.  Counts of created / destroyed octs. */
int  ryo_regrid(ryo_ctx* c, int64_t* n_created, int64_t* n_destroyed);
/* Change the refinement criterion's parameter (theta or rho_thr) for later
 * regrids. */
int  ryo_set_refine_param(ryo_ctx* c, double value);
int  ryo_cfl_dt(ryo_ctx* c, double* dt_coarse);
int  ryo_coarse_step(ryo_ctx* c, double dt_coarse);
int  ryo_advance(ryo_ctx* c, int32_t n_coarse, double t_end, double* t_io, int32_t* n_done);
/* tot: 5 + nscalar sums over leaf cells of U dx^3. */
int  ryo_conserved_totals(const ryo_ctx* c, double* tot);
/* Floor activations (density and pressure counted separately) since the
 * build, each event of a step counted once: a leaf cell's own primitive
 * conversion; both face states of each face an update uses (counted by the
 * face's upper cell when that is a leaf, else by its lower cell); once per
 * parent step, every ghost cell of a refined level that an update reads
 * (a ghost cell with a leaf cell one step away along an axis, two steps
 * along an axis, or one step along each of two axes).  The time-step
 * computation is not counted. */
int64_t ryo_floor_count(const ryo_ctx* c);
void ryo_reset_floor_count(ryo_ctx* c);
const char* ryo_last_error(const ryo_ctx* c);
int  ryo_num_threads(void);
void ryo_set_num_threads(int n);

/* The Hilbert key of oct coordinates (x,y,z) with `bits` bits per axis. */
uint64_t ryo_hilbert_key(int32_t bits, uint32_t x, uint32_t y, uint32_t z);
/* Single-face HLLC flux in direction d (0,1,2) for primitive states
 * W = (rho, u, v, w, p); exposed for unit pins. */
void ryo_hllc(const double WL[5], const double WR[5], int32_t d, double gamma, double F[5]);
/* The same with nscalar passive scalars appended to W and F. */
void ryo_hllc_scalars(const double* WL, const double* WR, int32_t nscalar, int32_t d, double gamma, double* F);
double ryo_minmod(double a, double b);

#ifdef __cplusplus
}
#endif
#endif
