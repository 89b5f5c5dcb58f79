/*
 * poisson.c -- FP64 CPU oracle of the Poisson solvers on one uniform level
 * (interface and sources in poisson.h).
 *
 * TEST INFRASTRUCTURE ONLY: the checker of the GPU library, never part of
 * the product path.  Everything is plain loops in the order the methods
 * state them; dot products are summed sequentially in cell order.
 *
 *   - Operator and preconditioner: the paper, Sec. 2.3 (seven-point
 *     preconditioner stencil 13/12 centre, 1/6 neighbours); the operator is
 *     the standard 7-point negative Laplacian.
 *   - PCG: Hestenes & Stiefel (1952) with a preconditioner (e.g. Saad 2003,
 *     Iterative Methods for Sparse Linear Systems, Alg. 9.1).
 *   - PPCG: Ghysels & Vanroose (2014), Algorithm 4, the method the paper
 *     adopts (Sec. 2.3).
 *   - Stopping rule: the paper's error measure eps_i = sqrt(gamma_i /
 *     gamma_0), gamma = r.u (Eq. 3, Sec. 3.2).
 */
#include "poisson.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static int64_t ncell(const int32_t n[3]) { return (int64_t)n[0] * n[1] * n[2]; }

/* Value of x at (i, j, k) under the boundary rule; `inside` says whether
 * the position is a grid cell at all (Dirichlet: outside values are 0). */
static double at(const int32_t n[3], int32_t bc, const double* x, int64_t i, int64_t j, int64_t k) {
  if (bc == RYO_PBC_PERIODIC) {
    i = (i + n[0]) % n[0];
    j = (j + n[1]) % n[1];
    k = (k + n[2]) % n[2];
  } else if (i < 0 || i >= n[0] || j < 0 || j >= n[1] || k < 0 || k >= n[2]) {
    return 0.0;
  }
  return x[i + (int64_t)n[0] * (j + (int64_t)n[1] * k)];
}

/* Sum of the six face neighbours of (i, j, k), in the fixed order
 * x-, x+, y-, y+, z-, z+. */
static double nb_sum(const int32_t n[3], int32_t bc, const double* x, int64_t i, int64_t j, int64_t k) {
  double s = at(n, bc, x, i - 1, j, k);
  s += at(n, bc, x, i + 1, j, k);
  s += at(n, bc, x, i, j - 1, k);
  s += at(n, bc, x, i, j + 1, k);
  s += at(n, bc, x, i, j, k - 1);
  s += at(n, bc, x, i, j, k + 1);
  return s;
}

void ryo_poisson_apply_A(const int32_t n[3], int32_t bc, const double* x, double* y) {
  for (int64_t k = 0; k < n[2]; ++k)
    for (int64_t j = 0; j < n[1]; ++j)
      for (int64_t i = 0; i < n[0]; ++i) {
        const int64_t c = i + (int64_t)n[0] * (j + (int64_t)n[1] * k);
        y[c] = 6.0 * x[c] - nb_sum(n, bc, x, i, j, k);
      }
}

void ryo_poisson_apply_Minv(const int32_t n[3], int32_t bc, int32_t pc, const double* x, double* y) {
  const int64_t N = ncell(n);
  if (pc == RYO_PC_NONE) {
    memcpy(y, x, sizeof(double) * (size_t)N);
    return;
  }
  for (int64_t k = 0; k < n[2]; ++k)
    for (int64_t j = 0; j < n[1]; ++j)
      for (int64_t i = 0; i < n[0]; ++i) {
        const int64_t c = i + (int64_t)n[0] * (j + (int64_t)n[1] * k);
        y[c] = (13.0 / 12.0) * x[c] + (1.0 / 6.0) * nb_sum(n, bc, x, i, j, k);
      }
}

static double dot(int64_t N, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t c = 0; c < N; ++c) s += a[c] * b[c];
  return s;
}

static int bad_args(const int32_t n[3], int32_t bc, int32_t pc) {
  if (!n || n[0] < 1 || n[1] < 1 || n[2] < 1) return 1;
  if (bc != RYO_PBC_PERIODIC && bc != RYO_PBC_DIRICHLET) return 1;
  if (pc != RYO_PC_NONE && pc != RYO_PC_STENCIL7) return 1;
  return 0;
}

int32_t ryo_pcg(const int32_t n[3], int32_t bc, int32_t pc, const double* b, double* x, double eps,
                int32_t max_iter, double* eps_hist) {
  if (bad_args(n, bc, pc) || !b || !x || max_iter < 0) return -1;
  const int64_t N = ncell(n);
  double* r = malloc(sizeof(double) * (size_t)N);
  double* z = malloc(sizeof(double) * (size_t)N);
  double* p = malloc(sizeof(double) * (size_t)N);
  double* Ap = malloc(sizeof(double) * (size_t)N);
  if (!r || !z || !p || !Ap) {
    free(r); free(z); free(p); free(Ap);
    return -2;
  }
  /* r0 = b - A x0, z0 = M^-1 r0, p0 = z0 */
  ryo_poisson_apply_A(n, bc, x, Ap);
  for (int64_t c = 0; c < N; ++c) r[c] = b[c] - Ap[c];
  ryo_poisson_apply_Minv(n, bc, pc, r, z);
  memcpy(p, z, sizeof(double) * (size_t)N);
  double rz = dot(N, r, z);
  const double rz0 = rz;
  int32_t k = 0;
  for (;; ++k) {
    const double e = (rz0 > 0.0) ? sqrt(rz / rz0) : 0.0;
    if (eps_hist) eps_hist[k] = e;
    if (e <= eps || k == max_iter) break;
    /* alpha = (r, z) / (p, A p); x += alpha p; r -= alpha A p */
    ryo_poisson_apply_A(n, bc, p, Ap);
    const double alpha = rz / dot(N, p, Ap);
    for (int64_t c = 0; c < N; ++c) {
      x[c] += alpha * p[c];
      r[c] -= alpha * Ap[c];
    }
    /* z = M^-1 r; beta = (r_new, z_new) / (r, z); p = z + beta p */
    ryo_poisson_apply_Minv(n, bc, pc, r, z);
    const double rz_new = dot(N, r, z);
    const double beta = rz_new / rz;
    rz = rz_new;
    for (int64_t c = 0; c < N; ++c) p[c] = z[c] + beta * p[c];
  }
  free(r); free(z); free(p); free(Ap);
  return k;
}

void ryo_ppcg_init(const int32_t n[3], int32_t bc, int32_t pc, const double* b, const double* x0,
                   ryo_ppcg_state* st) {
  const int64_t N = ncell(n);
  if (x0) memcpy(st->x, x0, sizeof(double) * (size_t)N);
  else memset(st->x, 0, sizeof(double) * (size_t)N);
  /* r0 = b - A x0; u0 = M^-1 r0; w0 = A u0 */
  ryo_poisson_apply_A(n, bc, st->x, st->w);
  for (int64_t c = 0; c < N; ++c) st->r[c] = b[c] - st->w[c];
  ryo_poisson_apply_Minv(n, bc, pc, st->r, st->u);
  ryo_poisson_apply_A(n, bc, st->u, st->w);
  memset(st->z, 0, sizeof(double) * (size_t)N);
  memset(st->q, 0, sizeof(double) * (size_t)N);
  memset(st->s, 0, sizeof(double) * (size_t)N);
  memset(st->p, 0, sizeof(double) * (size_t)N);
  st->alpha_prev = 0.0;
  st->gamma_prev = 0.0;
  st->i = 0;
}

void ryo_ppcg_dots(const int32_t n[3], const ryo_ppcg_state* st, double* gamma, double* delta) {
  const int64_t N = ncell(n);
  *gamma = dot(N, st->r, st->u);
  *delta = dot(N, st->w, st->u);
}

void ryo_ppcg_step(const int32_t n[3], int32_t bc, int32_t pc, ryo_ppcg_state* st, double gamma, double delta) {
  const int64_t N = ncell(n);
  double* m = malloc(sizeof(double) * (size_t)N);
  double* nv = malloc(sizeof(double) * (size_t)N);
  if (!m || !nv) {
    free(m); free(nv);
    return;
  }
  /* m_i = M^-1 w_i, n_i = A m_i */
  ryo_poisson_apply_Minv(n, bc, pc, st->w, m);
  ryo_poisson_apply_A(n, bc, m, nv);
  /* the step length and direction weight */
  double alpha, beta;
  if (st->i > 0) {
    beta = gamma / st->gamma_prev;
    alpha = gamma / (delta - beta * gamma / st->alpha_prev);
  } else {
    beta = 0.0;
    alpha = gamma / delta;
  }
  /* the four direction recurrences, then the four state updates */
  for (int64_t c = 0; c < N; ++c) {
    st->z[c] = nv[c] + beta * st->z[c];
    st->q[c] = m[c] + beta * st->q[c];
    st->s[c] = st->w[c] + beta * st->s[c];
    st->p[c] = st->u[c] + beta * st->p[c];
    st->x[c] = st->x[c] + alpha * st->p[c];
    st->r[c] = st->r[c] - alpha * st->s[c];
    st->u[c] = st->u[c] - alpha * st->q[c];
    st->w[c] = st->w[c] - alpha * st->z[c];
  }
  st->alpha_prev = alpha;
  st->gamma_prev = gamma;
  st->i += 1;
  free(m);
  free(nv);
}

int32_t ryo_ppcg(const int32_t n[3], int32_t bc, int32_t pc, const double* b, double* x, double eps,
                 int32_t max_iter, double* eps_hist) {
  if (bad_args(n, bc, pc) || !b || !x || max_iter < 0) return -1;
  const int64_t N = ncell(n);
  ryo_ppcg_state st;
  double* buf = malloc(sizeof(double) * (size_t)N * 7);
  if (!buf) return -2;
  st.x = x;
  st.r = buf;
  st.u = buf + N;
  st.w = buf + 2 * N;
  st.z = buf + 3 * N;
  st.q = buf + 4 * N;
  st.s = buf + 5 * N;
  st.p = buf + 6 * N;
  double* x0 = malloc(sizeof(double) * (size_t)N);
  if (!x0) {
    free(buf);
    return -2;
  }
  memcpy(x0, x, sizeof(double) * (size_t)N);
  ryo_ppcg_init(n, bc, pc, b, x0, &st);
  free(x0);
  double gamma0 = 0.0;
  int32_t k = 0;
  for (;; ++k) {
    double gamma, delta;
    ryo_ppcg_dots(n, &st, &gamma, &delta);
    if (k == 0) gamma0 = gamma;
    const double e = (gamma0 > 0.0) ? sqrt(gamma / gamma0) : 0.0;
    if (eps_hist) eps_hist[k] = e;
    if (e <= eps || k == max_iter) break;
    ryo_ppcg_step(n, bc, pc, &st, gamma, delta);
  }
  free(buf);
  return k;
}
