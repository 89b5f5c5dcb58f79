/*
 * ry_poisson.h -- C ABI of the uniform-level Poisson solver of the MI355X
 * library: the preconditioned pipelined conjugate-gradient method (PPCG,
 * Ghysels & Vanroose 2014, Algorithm 4) that the paper adopts in place of
 * plain CG for the cell-level Poisson equation (Sec. 2.3), with the paper's
 * seven-point preconditioner (13/12 at the centre, 1/6 on each face
 * neighbour, Sec. 2.3) and its error measure eps_i = sqrt((r_i.u_i) /
 * (r_0.u_0)), u = M^-1 r (Eq. 3, Sec. 3.2).
 *
 * Problem: A x = b on an n0 x n1 x n2 grid (x fastest), A = the 7-point
 * negative Laplacian with unit spacing (6 on the diagonal, -1 to each face
 * neighbour), boundary periodic or zero Dirichlet.  The preconditioner is
 * applied as the matrix M^-1 with the same boundary rule; RY_PC_NONE gives
 * the pipelined form of plain CG (M^-1 = I).  A periodic problem is
 * singular: b must have zero sum for the iteration to converge.
 *
 * Conventions: every function returns a ry_status (include/ry.h); host
 * pointers are borrowed for the duration of the call; device memory belongs
 * to the solver and comes from cfg->dev_alloc (hipMalloc when NULL); calls
 * marked "syncs" wait for the solver's stream.  No thread safety per
 * solver.  Arithmetic is FP64 throughout.
 */
#ifndef RY_POISSON_H
#define RY_POISSON_H
#include <stddef.h>
#include <stdint.h>

#include "ry.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { RY_PBC_PERIODIC = 0, RY_PBC_DIRICHLET = 1 };
enum { RY_PC_NONE = 0, RY_PC_STENCIL7 = 1 };
/* vectors of the pipelined recurrences, for ry_poisson_download */
enum { RY_PV_X = 0, RY_PV_R, RY_PV_U, RY_PV_W, RY_PV_Z, RY_PV_Q, RY_PV_S, RY_PV_P, RY_PV_COUNT };

typedef struct {
  int32_t n[3];                                   /* cells per axis, each >= 1, product < 2^31 */
  int32_t bc;                                     /* RY_PBC_*                                    */
  int32_t precond;                                /* RY_PC_*                                     */
  void* stream;                                   /* hipStream_t; NULL = library-owned stream    */
  void* (*dev_alloc)(size_t bytes, void* user);   /* NULL = hipMalloc                            */
  void (*dev_free)(void* p, void* user);
  void* alloc_user;
} ry_poisson_config;

typedef struct ry_poisson ry_poisson;

/* Allocates nine FP64 grid vectors (x, r, u, w twice, z, q, s, p) plus
 * reduction scratch and an eps history of RY_POISSON_HIST entries.
 * RY_EINVAL: bad sizes or enums; RY_ENOMEM: allocation failed (nothing
 * leaks); RY_EHIP: no device. */
#define RY_POISSON_HIST 65536
ry_status ry_poisson_create(const ry_poisson_config* cfg, ry_poisson** out);
void ry_poisson_destroy(ry_poisson* p);

/* Start a solve: b (host, n0*n1*n2, x fastest) and the initial guess x0
 * (host, NULL = 0).  Sets r0 = b - A x0, u0 = M^-1 r0, w0 = A u0, clears the
 * direction vectors and the history (eps_0 = 1, or 0 when r0.u0 = 0).
 * Async on the solver's stream. */
ry_status ry_poisson_set_rhs(ry_poisson* p, const double* b, const double* x0);

/* Iterate until eps_i <= eps or i == max_iter (i counts iterations since
 * ry_poisson_set_rhs); *n_iter = the i reached.  The test runs on the
 * device; the host looks at it once every batch of 16 iterations.  Syncs.
 * RY_ESTATE before ry_poisson_set_rhs; RY_EINVAL for max_iter outside
 * [0, RY_POISSON_HIST - 1]. */
ry_status ry_poisson_solve(ry_poisson* p, double eps, int32_t max_iter, int32_t* n_iter);

/* Exactly n more iterations with no convergence test (timing, step-by-step
 * checks).  Async. */
ry_status ry_poisson_iterate(ry_poisson* p, int32_t n);

/* eps_0 .. eps_k of the current solve (k = iterations done); *n = k + 1
 * entries written, at most cap.  Syncs. */
ry_status ry_poisson_eps_history(ry_poisson* p, double* eps, int32_t cap, int32_t* n);

/* Copy one recurrence vector (RY_PV_*) to the host (n0*n1*n2 doubles, x
 * fastest).  RY_PV_X is the current iterate.  Syncs. */
ry_status ry_poisson_download(ry_poisson* p, int32_t which, double* host);

/* Scalars carried between iterations: alpha_{i-1}, gamma_{i-1} and i.  Syncs. */
ry_status ry_poisson_scalars(ry_poisson* p, double* alpha_prev, double* gamma_prev, int32_t* iter);

/* Kernel timing: when on, every iteration kernel is bracketed by HIP events
 * on the solver's stream; ry_poisson_kernel_time returns the number of
 * timed launches and their summed duration (ms) since timing was switched
 * on.  Syncs. */
ry_status ry_poisson_set_timing(ry_poisson* p, int32_t on);
ry_status ry_poisson_kernel_time(ry_poisson* p, int32_t* launches, double* total_ms);

const char* ry_poisson_last_error(const ry_poisson* p);

#ifdef __cplusplus
}
#endif
#endif
