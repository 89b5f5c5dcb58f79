/*
 * poisson.h -- C interface of the FP64 CPU oracle for the Poisson solver on
 * one uniform level: plain and preconditioned conjugate gradients, and the
 * preconditioned pipelined conjugate-gradient method (PPCG).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this code; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the GPU
 * library.
 *
 * What the paper fixes (Sec. 2.3, "Additional improvements"; Sec. 3.2 and
 * the equation defining the solution error):
 *   - the cell-level Poisson equation is solved by conjugate gradients in
 *     RAMSES and by PPCG (Ghysels & Vanroose 2014, Algorithm 4: pipelined
 *     PCG) in RAMSES-yOMP;
 *   - the preconditioner is a seven-point stencil, 13/12 at the centre and
 *     1/6 on each of the six face neighbours (a 1-D stencil of the cited
 *     preconditioner paper, generalised to 3-D);
 *   - convergence is measured by eps_i = sqrt((r_i . u_i) / (r_0 . u_0)),
 *     u = M^-1 r (u = r for plain CG), with 1e-4 the usual target.
 *
 * Operator: A = the 7-point negative Laplacian with unit spacing, 6 on the
 * diagonal and -1 towards each face neighbour, on an n0 x n1 x n2 grid (x
 * fastest).  Boundary: periodic, or zero Dirichlet (a neighbour outside the
 * grid holds 0).  The preconditioner stencil is applied as the matrix M^-1
 * with the same boundary rule.
 */
#ifndef RYO_POISSON_H
#define RYO_POISSON_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { RYO_PBC_PERIODIC = 0, RYO_PBC_DIRICHLET = 1 };
enum { RYO_PC_NONE = 0, RYO_PC_STENCIL7 = 1 };

/* y = A x */
void ryo_poisson_apply_A(const int32_t n[3], int32_t bc, const double* x, double* y);
/* y = M^-1 x (RYO_PC_NONE: y = x) */
void ryo_poisson_apply_Minv(const int32_t n[3], int32_t bc, int32_t pc, const double* x, double* y);

/* Textbook PCG (Hestenes-Stiefel recurrences).  x: in x0, out the iterate
 * reached.  eps_hist[0..k]: eps of every iterate.  Stops at the first k with
 * eps_k <= eps or k == max_iter; returns k, or -1 on bad arguments, -2 when
 * memory runs out. */
int32_t ryo_pcg(const int32_t n[3], int32_t bc, int32_t pc, const double* b, double* x, double eps,
                int32_t max_iter, double* eps_hist);

/* PPCG state: the eight vectors of the pipelined recurrences plus the
 * scalars of the previous iteration. */
typedef struct {
  double *x, *r, *u, *w, *z, *q, *s, *p;   /* each n0*n1*n2, caller-owned */
  double alpha_prev, gamma_prev;
  int32_t i;                               /* iterations done */
} ryo_ppcg_state;

/* r0 = b - A x0, u0 = M^-1 r0, w0 = A u0; z, q, s, p = 0; i = 0. */
void ryo_ppcg_init(const int32_t n[3], int32_t bc, int32_t pc, const double* b, const double* x0,
                   ryo_ppcg_state* st);
/* gamma_i = r.u and delta_i = w.u of the current state. */
void ryo_ppcg_dots(const int32_t n[3], const ryo_ppcg_state* st, double* gamma, double* delta);
/* One PPCG iteration i -> i+1 given gamma_i, delta_i of the current state. */
void ryo_ppcg_step(const int32_t n[3], int32_t bc, int32_t pc, ryo_ppcg_state* st, double gamma, double delta);
/* Full PPCG solve, same contract as ryo_pcg. */
int32_t ryo_ppcg(const int32_t n[3], int32_t bc, int32_t pc, const double* b, double* x, double eps,
                 int32_t max_iter, double* eps_hist);

#ifdef __cplusplus
}
#endif
#endif
