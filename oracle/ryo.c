/*
 * ryo.c -- FP64 CPU oracle for the octree MUSCL-Hancock / MinMod / HLLC
 * hydro step with level subcycling and coarse-fine flux correction.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline leg of the benchmark; never by the product path.  Built with
 * gcc -O2 -ffp-contract=off (no fused multiply-add, no fast-math), so every
 * expression below is evaluated in IEEE double in the order written.
 *
 * The paper (RAMSES-yOMP) fixes the mesh (octree of 2^3-cell octs, level
 * l+1 halves the cell size: Sec. 1), the Hilbert ordering of octs (Sec. 1),
 * the subcycling rule dt(l+1) = dt(l)/2 (Sec. 2.3, next to Eq. 1) and the
 * OpenMP static schedule over grid loops (Sec. 2.2).  It does not state the
 * hydro scheme; each step below follows the published method it names:
 *   - primitive variables and floors ............ ideal gas, E = p/(g-1)+rho v^2/2
 *   - MinMod-limited slopes, half-step predictor  van Leer (1979); Toro (2009) ch. 13-14
 *   - HLLC Riemann flux, Davis wave speeds ...... Toro, Spruce & Speares (1994);
 *                                                  Toro (2009) ch. 10; Davis (1988)
 *   - coarse-fine refluxing ...................... Berger & Colella (1989)
 *   - Hilbert curve .............................. Skilling (2004), transpose form
 * The oracle is deliberately plain: every cell re-gathers its own stencil,
 * every position is resolved through a hash lookup, nothing is blocked,
 * fused or cached across cells.
 */
#include "ryo.h"
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* NV: array bound (5 hydro variables + the most passive scalars); c->nv:
 * the variables of this context (5 + nscalar). */
#define NV (5 + RYO_MAX_SCALARS)

typedef struct {
  int64_t n;          /* number of octs                                   */
  uint64_t* key;      /* Hilbert keys, ascending                          */
  int32_t* oc;        /* oct coordinates, 3 per oct                       */
  uint8_t* refined;   /* bit c set when cell c has a child oct            */
  double* U;          /* state, nv planes of 8n                           */
  double* Un;         /* next state                                       */
  double* reg;        /* flux registers: [oct][face 6][var nv][substep 2] */
  uint64_t* hkey;     /* hash table: packed coords + 1 (0 = empty)        */
  int64_t* hval;
  uint64_t hmask;
} level_t;

struct ryo_ctx {
  ryo_config cfg;
  int nv;                    /* 5 + passive scalars                       */
  int nlev;
  int bits0;                 /* Hilbert bits per axis at level_min        */
  level_t lev[RYO_MAX_LEVELS];
  int built;
  int64_t floors;
  int numeric_error;
  char err[256];
};

static void set_err(ryo_ctx* c, const char* m) {
  snprintf(c->err, sizeof c->err, "%s", m);
}

/* ------------------------------------------------------------------------ */
/* Hilbert curve: Skilling (2004), "Programming the Hilbert curve",           */
/* AIP Conf. Proc. 707.  Coordinates are turned into the "transposed" index   */
/* (undo the excess work, then Gray-encode), then the bits are interleaved    */
/* with x as the most significant axis of every 3-bit group.                  */
/* ------------------------------------------------------------------------ */
uint64_t ryo_hilbert_key(int32_t bits, uint32_t x, uint32_t y, uint32_t z) {
  uint32_t X[3] = {x, y, z};
  if (bits <= 0) return 0;
  uint32_t M = 1u << (bits - 1);
  for (uint32_t Q = M; Q > 1; Q >>= 1) {
    uint32_t P = Q - 1;
    for (int i = 0; i < 3; i++) {
      if (X[i] & Q) {
        X[0] ^= P;                       /* invert low bits of x */
      } else {
        uint32_t t = (X[0] ^ X[i]) & P;  /* exchange low bits of x and X[i] */
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  for (int i = 1; i < 3; i++) X[i] ^= X[i - 1];  /* Gray encode */
  uint32_t t = 0;
  for (uint32_t Q = M; Q > 1; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1;
  for (int i = 0; i < 3; i++) X[i] ^= t;
  uint64_t h = 0;
  for (int b = bits - 1; b >= 0; b--)
    for (int i = 0; i < 3; i++) h = (h << 1) | ((X[i] >> b) & 1u);
  return h;
}

/* ------------------------------------------------------------------------ */
/* Per-level hash of oct coordinates -> oct index.                           */
/* ------------------------------------------------------------------------ */
static uint64_t pack3(int64_t x, int64_t y, int64_t z) {
  return (uint64_t)x | ((uint64_t)y << 21) | ((uint64_t)z << 42);
}
static uint64_t mix64(uint64_t k) {
  k += 0x9E3779B97F4A7C15ull;
  k = (k ^ (k >> 30)) * 0xBF58476D1CE4E5B9ull;
  k = (k ^ (k >> 27)) * 0x94D049BB133111EBull;
  return k ^ (k >> 31);
}
static int build_hash(level_t* L) {
  uint64_t cap = 16;
  while (cap < (uint64_t)(2 * L->n + 16)) cap <<= 1;
  free(L->hkey); free(L->hval);
  L->hkey = (uint64_t*)calloc(cap, sizeof(uint64_t));
  L->hval = (int64_t*)malloc(cap * sizeof(int64_t));
  if (!L->hkey || !L->hval) return -1;
  L->hmask = cap - 1;
  for (int64_t o = 0; o < L->n; o++) {
    uint64_t k = pack3(L->oc[3 * o], L->oc[3 * o + 1], L->oc[3 * o + 2]) + 1;
    uint64_t s = mix64(k) & L->hmask;
    while (L->hkey[s]) s = (s + 1) & L->hmask;
    L->hkey[s] = k;
    L->hval[s] = o;
  }
  return 0;
}
static int64_t find_oct(const level_t* L, int64_t ox, int64_t oy, int64_t oz) {
  if (L->n == 0) return -1;
  uint64_t k = pack3(ox, oy, oz) + 1;
  uint64_t s = mix64(k) & L->hmask;
  while (L->hkey[s]) {
    if (L->hkey[s] == k) return L->hval[s];
    s = (s + 1) & L->hmask;
  }
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Geometry helpers.                                                          */
/* ------------------------------------------------------------------------ */
static int64_t ncells(const ryo_ctx* c, int l, int a) {
  return (int64_t)c->cfg.nbase[a] << (l - c->cfg.level_min);
}
static double dx_of(const ryo_ctx* c, int l) {
  return c->cfg.boxlen / (double)ncells(c, l, 0);
}
static level_t* LV(ryo_ctx* c, int l) { return &c->lev[l - c->cfg.level_min]; }
static const level_t* LVc(const ryo_ctx* c, int l) { return &c->lev[l - c->cfg.level_min]; }

/* Boundary conditions on a cell position of level l: periodic wrap or
 * outflow clamp to the nearest interior cell (zero gradient). */
static void bc_cell(const ryo_ctx* c, int l, int64_t p[3]) {
  for (int a = 0; a < 3; a++) {
    int64_t N = ncells(c, l, a);
    if (p[a] < 0) {
      if (c->cfg.bc[2 * a] == RYO_BC_PERIODIC) p[a] = ((p[a] % N) + N) % N;
      else p[a] = 0;
    } else if (p[a] >= N) {
      if (c->cfg.bc[2 * a + 1] == RYO_BC_PERIODIC) p[a] = p[a] % N;
      else p[a] = N - 1;
    }
  }
}
static int cell_of(const int64_t p[3]) {
  return (int)((p[0] & 1) + 2 * (p[1] & 1) + 4 * (p[2] & 1));
}

/* ------------------------------------------------------------------------ */
/* MinMod limiter (sign-test form).                                          */
/* ------------------------------------------------------------------------ */
double ryo_minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

/* ------------------------------------------------------------------------ */
/* Stencil resolution.                                                        */
/* ------------------------------------------------------------------------ */
/* Value of the finest existing cell covering position q of level l. */
static void cover_value(const ryo_ctx* c, int l, const int64_t q_in[3], double U[NV]) {
  int64_t q[3] = {q_in[0], q_in[1], q_in[2]};
  bc_cell(c, l, q);
  for (;;) {
    const level_t* L = LVc(c, l);
    int64_t o = find_oct(L, q[0] >> 1, q[1] >> 1, q[2] >> 1);
    if (o >= 0) {
      int64_t cell = 8 * o + cell_of(q);
      for (int v = 0; v < c->nv; v++) U[v] = L->U[(int64_t)v * 8 * L->n + cell];
      return;
    }
    /* not at this level: go to the parent cell one level up */
    q[0] >>= 1; q[1] >>= 1; q[2] >>= 1;
    l -= 1;
  }
}

/* Conserved state at cell position (x,y,z) of level l: the cell itself when
 * it exists at l; otherwise a ghost made by MinMod-limited linear
 * interpolation of the conserved variables of the covering level l-1 cell Q:
 *   U = U_Q + sum_d sigma_d * 0.25 * minmod(U_Q - U_{Q-e_d}, U_{Q+e_d} - U_Q),
 * sigma_d = +1 / -1 for the upper / lower child of Q along d. */
static void coarse_interp(const ryo_ctx* c, int l, const int64_t p[3], double U[NV]);

static void value_at(const ryo_ctx* c, int l, int64_t x, int64_t y, int64_t z, double U[NV]) {
  int64_t p[3] = {x, y, z};
  bc_cell(c, l, p);
  const level_t* L = LVc(c, l);
  int64_t o = find_oct(L, p[0] >> 1, p[1] >> 1, p[2] >> 1);
  if (o >= 0) {
    int64_t cell = 8 * o + cell_of(p);
    for (int v = 0; v < c->nv; v++) U[v] = L->U[(int64_t)v * 8 * L->n + cell];
    return;
  }
  coarse_interp(c, l, p, U);
}

/* The MinMod-linear interpolation of cell p of level l (inside the domain)
 * from its covering level l-1 cell and that cell's six neighbours. */
static void coarse_interp(const ryo_ctx* c, int l, const int64_t p[3], double U[NV]) {
  int64_t q[3] = {p[0] >> 1, p[1] >> 1, p[2] >> 1};
  double UQ[NV], Um[NV], Up[NV], s[3][NV];
  cover_value(c, l - 1, q, UQ);
  for (int d = 0; d < 3; d++) {
    int64_t qm[3] = {q[0], q[1], q[2]}, qp[3] = {q[0], q[1], q[2]};
    qm[d] -= 1;
    qp[d] += 1;
    cover_value(c, l - 1, qm, Um);
    cover_value(c, l - 1, qp, Up);
    for (int v = 0; v < c->nv; v++) s[d][v] = ryo_minmod(UQ[v] - Um[v], Up[v] - UQ[v]);
  }
  double sg[3];
  for (int d = 0; d < 3; d++) sg[d] = (p[d] & 1) ? 1.0 : -1.0;
  for (int v = 0; v < c->nv; v++)
    U[v] = UQ[v] + (sg[0] * 0.25 * s[0][v] + sg[1] * 0.25 * s[1][v] + sg[2] * 0.25 * s[2][v]);
}

/* ------------------------------------------------------------------------ */
/* Primitive variables with floors.                                           */
/* ------------------------------------------------------------------------ */
static void cons_to_prim(const ryo_ctx* c, const double U[NV], double W[NV], int64_t* fl) {
  double g = c->cfg.gamma;
  double rho = U[0];
  if (rho < c->cfg.rho_floor) { rho = c->cfg.rho_floor; (*fl)++; }
  double ke = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / rho;
  double p = (g - 1.0) * (U[4] - ke);
  if (p < c->cfg.p_floor) { p = c->cfg.p_floor; (*fl)++; }
  W[0] = rho;
  W[1] = U[1] / rho;
  W[2] = U[2] / rho;
  W[3] = U[3] / rho;
  W[4] = p;
  /* passive scalars: conserved rho*s, primitive s */
  for (int v = 5; v < c->nv; v++) W[v] = U[v] / rho;
}

/* ------------------------------------------------------------------------ */
/* MUSCL-Hancock: limited slopes and the half-step predictor of the          */
/* primitive-variable Euler equations (unsplit, all three slopes).           */
/* ------------------------------------------------------------------------ */
typedef struct {
  double Wt[NV];     /* predicted primitive state at t + dt/2 */
  double D[3][NV];   /* undivided MinMod slopes per axis       */
} pred_t;

static void predict(const ryo_ctx* c, int l, int64_t x, int64_t y, int64_t z, double h,
                    pred_t* P, int64_t* fl) {
  double U[NV], W0[NV], Wm[NV], Wp[NV];
  value_at(c, l, x, y, z, U);
  cons_to_prim(c, U, W0, fl);
  for (int d = 0; d < 3; d++) {
    int64_t m[3] = {x, y, z}, pp[3] = {x, y, z};
    m[d] -= 1;
    pp[d] += 1;
    value_at(c, l, m[0], m[1], m[2], U);
    cons_to_prim(c, U, Wm, fl);
    value_at(c, l, pp[0], pp[1], pp[2], U);
    cons_to_prim(c, U, Wp, fl);
    for (int v = 0; v < c->nv; v++) P->D[d][v] = ryo_minmod(W0[v] - Wm[v], Wp[v] - W0[v]);
  }
  double g = c->cfg.gamma;
  double r = W0[0], u = W0[1], v = W0[2], w = W0[3], p = W0[4];
  const double* Dx = P->D[0];
  const double* Dy = P->D[1];
  const double* Dz = P->D[2];
  P->Wt[0] = r - h * (u * Dx[0] + r * Dx[1] + v * Dy[0] + r * Dy[2] + w * Dz[0] + r * Dz[3]);
  P->Wt[1] = u - h * (u * Dx[1] + v * Dy[1] + w * Dz[1] + Dx[4] / r);
  P->Wt[2] = v - h * (u * Dx[2] + v * Dy[2] + w * Dz[2] + Dy[4] / r);
  P->Wt[3] = w - h * (u * Dx[3] + v * Dy[3] + w * Dz[3] + Dz[4] / r);
  P->Wt[4] = p - h * (u * Dx[4] + v * Dy[4] + w * Dz[4] + g * p * (Dx[1] + Dy[2] + Dz[3]));
  /* a passive scalar is advected: s~ = s - h (u Dx s + v Dy s + w Dz s) */
  for (int k = 5; k < c->nv; k++) P->Wt[k] = W0[k] - h * (u * Dx[k] + v * Dy[k] + w * Dz[k]);
}

/* ------------------------------------------------------------------------ */
/* HLLC flux (Toro, Spruce & Speares 1994; Davis 1988 wave speeds).          */
/* ------------------------------------------------------------------------ */
/* nv = 5 + passive scalars; a passive scalar s is carried like a transverse
 * velocity: flux rho u s, star state r (rho_K s_K) (Toro 2009, Sec. 10.6). */
static void hllc_nv(const double* WL, const double* WR, int nv, int32_t d, double g, double* F) {
  int t1 = (d == 0) ? 1 : 0;   /* tangential axes in increasing order */
  int t2 = (d == 2) ? 1 : 2;
  double rl = WL[0], ul = WL[1 + d], al = WL[1 + t1], bl = WL[1 + t2], pl = WL[4];
  double rr = WR[0], ur = WR[1 + d], ar = WR[1 + t1], br = WR[1 + t2], pr = WR[4];
  double cl = sqrt(g * pl / rl);
  double cr = sqrt(g * pr / rr);
  double SL = fmin(ul - cl, ur - cr);
  double SR = fmax(ul + cl, ur + cr);
  double El = pl / (g - 1.0) + 0.5 * rl * (ul * ul + al * al + bl * bl);
  double Er = pr / (g - 1.0) + 0.5 * rr * (ur * ur + ar * ar + br * br);
  double num = pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur);
  double den = rl * (SL - ul) - rr * (SR - ur);
  double Ss = num / den;
  double FL[NV] = {rl * ul, rl * ul * ul + pl, rl * ul * al, rl * ul * bl, (El + pl) * ul};
  double FR[NV] = {rr * ur, rr * ur * ur + pr, rr * ur * ar, rr * ur * br, (Er + pr) * ur};
  for (int k = 5; k < nv; k++) {
    FL[k] = rl * ul * WL[k];
    FR[k] = rr * ur * WR[k];
  }
  double Fn[NV] = {0.0};
  if (SL >= 0.0) {
    for (int i = 0; i < nv; i++) Fn[i] = FL[i];
  } else if (Ss >= 0.0) {
    double r = (SL - ul) / (SL - Ss);
    double Us[NV] = {r * rl, r * (rl * Ss), r * (rl * al), r * (rl * bl),
                     r * (El + rl * (Ss - ul) * (Ss + pl / (rl * (SL - ul))))};
    double Uk[NV] = {rl, rl * ul, rl * al, rl * bl, El};
    for (int k = 5; k < nv; k++) {
      Us[k] = r * (rl * WL[k]);
      Uk[k] = rl * WL[k];
    }
    for (int i = 0; i < nv; i++) Fn[i] = FL[i] + SL * (Us[i] - Uk[i]);
  } else if (SR > 0.0) {
    double r = (SR - ur) / (SR - Ss);
    double Us[NV] = {r * rr, r * (rr * Ss), r * (rr * ar), r * (rr * br),
                     r * (Er + rr * (Ss - ur) * (Ss + pr / (rr * (SR - ur))))};
    double Uk[NV] = {rr, rr * ur, rr * ar, rr * br, Er};
    for (int k = 5; k < nv; k++) {
      Us[k] = r * (rr * WR[k]);
      Uk[k] = rr * WR[k];
    }
    for (int i = 0; i < nv; i++) Fn[i] = FR[i] + SR * (Us[i] - Uk[i]);
  } else {
    for (int i = 0; i < nv; i++) Fn[i] = FR[i];
  }
  /* rotate back: normal momentum to axis d, tangential to t1, t2 */
  F[0] = Fn[0];
  F[1 + d] = Fn[1];
  F[1 + t1] = Fn[2];
  F[1 + t2] = Fn[3];
  F[4] = Fn[4];
  for (int k = 5; k < nv; k++) F[k] = Fn[k];
}

void ryo_hllc(const double WL[5], const double WR[5], int32_t d, double g, double F[5]) {
  hllc_nv(WL, WR, 5, d, g, F);
}

void ryo_hllc_scalars(const double* WL, const double* WR, int32_t nscalar, int32_t d, double g, double* F) {
  hllc_nv(WL, WR, 5 + nscalar, d, g, F);
}

/* Flux through the face between cells A (lower) and B (upper) along d, from
 * their predictions: W_L = Wt_A + D_A/2, W_R = Wt_B - D_B/2, floors applied. */
static void face_flux(const ryo_ctx* c, const pred_t* A, const pred_t* B, int d, double F[NV],
                      int64_t* fl) {
  double WL[NV], WR[NV];
  for (int v = 0; v < c->nv; v++) {
    WL[v] = A->Wt[v] + 0.5 * A->D[d][v];
    WR[v] = B->Wt[v] - 0.5 * B->D[d][v];
  }
  if (WL[0] < c->cfg.rho_floor) { WL[0] = c->cfg.rho_floor; (*fl)++; }
  if (WR[0] < c->cfg.rho_floor) { WR[0] = c->cfg.rho_floor; (*fl)++; }
  if (WL[4] < c->cfg.p_floor) { WL[4] = c->cfg.p_floor; (*fl)++; }
  if (WR[4] < c->cfg.p_floor) { WR[4] = c->cfg.p_floor; (*fl)++; }
  hllc_nv(WL, WR, c->nv, d, c->cfg.gamma, F);
}

/* Is position p (level l, after boundary conditions) a refined cell of l?
 * Returns the child oct index at l+1, or -1. */
static int64_t refined_child(const ryo_ctx* c, int l, const int64_t p_in[3]) {
  if (l >= c->cfg.level_max) return -1;
  int64_t p[3] = {p_in[0], p_in[1], p_in[2]};
  bc_cell(c, l, p);
  const level_t* L = LVc(c, l);
  int64_t o = find_oct(L, p[0] >> 1, p[1] >> 1, p[2] >> 1);
  if (o < 0) return -1;
  if (!(L->refined[o] & (1u << cell_of(p)))) return -1;
  return find_oct(LVc(c, l + 1), p[0], p[1], p[2]);
}

/* Is cell position p of level l a leaf cell of l?  Positions outside an
 * outflow face (read through the zero-gradient clamp) are not, nor are
 * positions whose oct does not exist at l (ghosts) or refined cells. */
static int is_leaf_cell(const ryo_ctx* c, int l, const int64_t p_in[3]) {
  int64_t p[3] = {p_in[0], p_in[1], p_in[2]};
  for (int a = 0; a < 3; a++) {
    int64_t N = ncells(c, l, a);
    if ((p[a] < 0 && c->cfg.bc[2 * a] != RYO_BC_PERIODIC) || (p[a] >= N && c->cfg.bc[2 * a + 1] != RYO_BC_PERIODIC))
      return 0;
  }
  bc_cell(c, l, p);
  const level_t* L = LVc(c, l);
  int64_t o = find_oct(L, p[0] >> 1, p[1] >> 1, p[2] >> 1);
  return o >= 0 && !(L->refined[o] & (1u << cell_of(p)));
}

/* Time- and area-averaged flux of a coarse-fine face, from the registers of
 * the fine oct: Fbar = (q_1 + q_2) / 8 (Berger & Colella 1989). */
static void register_flux(const ryo_ctx* c, int lf, int64_t child, int face, double F[NV]) {
  const level_t* Lf = LVc(c, lf);
  for (int v = 0; v < c->nv; v++) {
    const double* q = &Lf->reg[((child * 6 + face) * c->nv + v) * 2];
    F[v] = 0.125 * (q[0] + q[1]);
  }
}

/* ------------------------------------------------------------------------ */
/* Flux computation and conservative update of one level (one substep).      */
/* ------------------------------------------------------------------------ */
/* Floor activations are counted once per event of the step, whatever the
 * order of the computation (this oracle recomputes every stencil value
 * for each use): a leaf cell's own primitive conversion, each face state of
 * a face that an update uses -- counted by the face's upper cell when that
 * is a leaf, otherwise by its lower cell -- and, once per parent step, each
 * ghost cell of the level (ghost_census). */
static void update_level(ryo_ctx* c, int l, double lam, int substep) {
  level_t* L = LV(c, l);
  const int64_t n = L->n;
  const double h = 0.5 * lam;
  int64_t floors = 0;
#pragma omp parallel for schedule(static) reduction(+ : floors)
  for (int64_t o = 0; o < n; o++) {
    int64_t fl = 0, rep = 0;   /* counted events; repeated evaluations (not counted) */
    for (int ci = 0; ci < 8; ci++) {
      if (L->refined[o] & (1u << ci)) continue;   /* refined cells: restriction */
      int64_t p[3] = {2 * (int64_t)L->oc[3 * o] + (ci & 1), 2 * (int64_t)L->oc[3 * o + 1] + ((ci >> 1) & 1),
                      2 * (int64_t)L->oc[3 * o + 2] + ((ci >> 2) & 1)};
      {
        double Uc[NV], Wc[NV];
        value_at(c, l, p[0], p[1], p[2], Uc);
        cons_to_prim(c, Uc, Wc, &fl);
      }
      pred_t P0, Pm[3], Pp[3];
      predict(c, l, p[0], p[1], p[2], h, &P0, &rep);
      double Fm[3][NV], Fp[3][NV];
      for (int d = 0; d < 3; d++) {
        int64_t m[3] = {p[0], p[1], p[2]}, q[3] = {p[0], p[1], p[2]};
        m[d] -= 1;
        q[d] += 1;
        int64_t chm = refined_child(c, l, m);
        if (chm >= 0) {
          register_flux(c, l + 1, chm, 2 * d + 1, Fm[d]);
        } else {
          predict(c, l, m[0], m[1], m[2], h, &Pm[d], &rep);
          face_flux(c, &Pm[d], &P0, d, Fm[d], &fl);
        }
        int64_t chp = refined_child(c, l, q);
        if (chp >= 0) {
          register_flux(c, l + 1, chp, 2 * d + 0, Fp[d]);
        } else {
          predict(c, l, q[0], q[1], q[2], h, &Pp[d], &rep);
          face_flux(c, &P0, &Pp[d], d, Fp[d], is_leaf_cell(c, l, q) ? &rep : &fl);
        }
      }
      int64_t cell = 8 * o + ci;
      for (int v = 0; v < c->nv; v++) {
        double acc = (Fm[0][v] - Fp[0][v]) + (Fm[1][v] - Fp[1][v]) + (Fm[2][v] - Fp[2][v]);
        L->Un[v * 8 * n + cell] = L->U[v * 8 * n + cell] + lam * acc;
      }
    }
    /* Coarse-fine faces of this oct: record q_s = (f1 + f2) + (f3 + f4), the
     * four fine-face fluxes in ascending in-oct cell order. */
    if (l > c->cfg.level_min) {
      for (int face = 0; face < 6; face++) {
        int d = face >> 1, up = face & 1;
        int64_t nb[3] = {L->oc[3 * o], L->oc[3 * o + 1], L->oc[3 * o + 2]};
        nb[d] += up ? 1 : -1;
        int64_t cp[3] = {2 * nb[0], 2 * nb[1], 2 * nb[2]};
        bc_cell(c, l, cp);
        if (find_oct(L, cp[0] >> 1, cp[1] >> 1, cp[2] >> 1) >= 0) continue;
        double f[4][NV];
        int k = 0;
        for (int ci = 0; ci < 8; ci++) {
          if (((ci >> d) & 1) != up) continue;
          int64_t p[3] = {2 * (int64_t)L->oc[3 * o] + (ci & 1), 2 * (int64_t)L->oc[3 * o + 1] + ((ci >> 1) & 1),
                          2 * (int64_t)L->oc[3 * o + 2] + ((ci >> 2) & 1)};
          int64_t q[3] = {p[0], p[1], p[2]};
          q[d] += up ? 1 : -1;
          pred_t Pa, Pb;
          predict(c, l, p[0], p[1], p[2], h, &Pa, &rep);
          predict(c, l, q[0], q[1], q[2], h, &Pb, &rep);
          if (up) face_flux(c, &Pa, &Pb, d, f[k], &rep);
          else face_flux(c, &Pb, &Pa, d, f[k], &rep);
          k++;
        }
        for (int v = 0; v < c->nv; v++)
          L->reg[((o * 6 + face) * c->nv + v) * 2 + substep] = (f[0][v] + f[1][v]) + (f[2][v] + f[3][v]);
      }
    }
    floors += fl;
  }
  c->floors += floors;
}

/* Refined cell of level l = mean of its 8 children (level l+1):
 * 0.125 * (((c0+c1)+(c2+c3)) + ((c4+c5)+(c6+c7))). Written into dst of l. */
static void restrict_level(ryo_ctx* c, int l, double* dst) {
  level_t* L = LV(c, l);
  level_t* F = LV(c, l + 1);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < F->n; k++) {
    int64_t p[3] = {F->oc[3 * k], F->oc[3 * k + 1], F->oc[3 * k + 2]};
    int64_t o = find_oct(L, p[0] >> 1, p[1] >> 1, p[2] >> 1);
    int64_t cell = 8 * o + cell_of(p);
    for (int v = 0; v < c->nv; v++) {
      const double* s = &F->U[v * 8 * F->n + 8 * k];
      dst[v * 8 * L->n + cell] = 0.125 * (((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])));
    }
  }
}

/* Whether an update of level l reads cell position p: whether a leaf cell
 * of l lies in the stencil around p -- one step along an axis, two steps
 * along an axis, or one step along each of two axes (the cells whose
 * predictions the fluxes of a cell use, and their neighbours). */
static int read_by_update(const ryo_ctx* c, int l, const int64_t p[3]) {
  for (int d = 0; d < 3; d++)
    for (int s = -2; s <= 2; s++) {
      if (s == 0) continue;
      int64_t q[3] = {p[0], p[1], p[2]};
      q[d] += s;
      if (is_leaf_cell(c, l, q)) return 1;
    }
  for (int d = 0; d < 3; d++)
    for (int e = d + 1; e < 3; e++)
      for (int sd = -1; sd <= 1; sd += 2)
        for (int se = -1; se <= 1; se += 2) {
          int64_t q[3] = {p[0], p[1], p[2]};
          q[d] += sd;
          q[e] += se;
          if (is_leaf_cell(c, l, q)) return 1;
        }
  return 0;
}

/* Floor activations of the ghost cells of level l (l > level_min) that the
 * updates of a parent step read, at its start: the cells of the oct
 * positions that a 26-neighbour of an existing level-l oct occupies but no
 * level-l oct does (inside the domain or across a periodic face) that lie
 * in the stencil of a leaf cell, each MinMod-linear interpolated state
 * converted once. */
static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}
static void ghost_census(ryo_ctx* c, int l) {
  const level_t* L = LVc(c, l);
  int64_t cap = 26 * L->n, m = 0;
  uint64_t* pos = (uint64_t*)malloc((cap ? cap : 1) * sizeof(uint64_t));
  if (!pos) return;
  for (int64_t o = 0; o < L->n; o++)
    for (int dz = -1; dz <= 1; dz++)
      for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
          if (!dx && !dy && !dz) continue;
          int64_t q[3] = {L->oc[3 * o] + dx, L->oc[3 * o + 1] + dy, L->oc[3 * o + 2] + dz};
          int out = 0;
          for (int a = 0; a < 3; a++) {
            int64_t N = ncells(c, l, a) / 2;
            if (q[a] < 0) {
              if (c->cfg.bc[2 * a] != RYO_BC_PERIODIC) out = 1;
              else q[a] += N;
            } else if (q[a] >= N) {
              if (c->cfg.bc[2 * a + 1] != RYO_BC_PERIODIC) out = 1;
              else q[a] -= N;
            }
          }
          if (out || find_oct(L, q[0], q[1], q[2]) >= 0) continue;
          pos[m++] = (uint64_t)q[0] | ((uint64_t)q[1] << 21) | ((uint64_t)q[2] << 42);
        }
  qsort(pos, (size_t)m, sizeof(uint64_t), cmp_u64);
  int64_t fl = 0;
  for (int64_t i = 0; i < m; i++) {
    if (i > 0 && pos[i] == pos[i - 1]) continue;
    int64_t q[3] = {(int64_t)(pos[i] & 0x1FFFFF), (int64_t)((pos[i] >> 21) & 0x1FFFFF), (int64_t)(pos[i] >> 42)};
    for (int ci = 0; ci < 8; ci++) {
      int64_t p[3] = {2 * q[0] + (ci & 1), 2 * q[1] + ((ci >> 1) & 1), 2 * q[2] + ((ci >> 2) & 1)};
      if (!read_by_update(c, l, p)) continue;
      double U[NV], W[NV];
      coarse_interp(c, l, p, U);
      cons_to_prim(c, U, W, &fl);
    }
  }
  free(pos);
  c->floors += fl;
}

/* Fine-first recursion: level l+1 takes two half steps, then level l takes
 * its step, then the refined cells of l are restricted from l+1. */
static void advance_level(ryo_ctx* c, int l, double dt, int substep) {
  if (l < c->cfg.level_max && LV(c, l + 1)->n > 0) {
    ghost_census(c, l + 1);
    advance_level(c, l + 1, 0.5 * dt, 0);
    advance_level(c, l + 1, 0.5 * dt, 1);
  }
  double lam = dt / dx_of(c, l);
  update_level(c, l, lam, substep);
  level_t* L = LV(c, l);
  if (l < c->cfg.level_max && LV(c, l + 1)->n > 0) restrict_level(c, l, L->Un);
  double* t = L->U;
  L->U = L->Un;
  L->Un = t;
}

/* ------------------------------------------------------------------------ */
/* Mesh build: refinement flags, the neighbour rule, Hilbert order.          */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t key; int32_t x, y, z; } okey_t;
static int cmp_okey(const void* a, const void* b) {
  uint64_t ka = ((const okey_t*)a)->key, kb = ((const okey_t*)b)->key;
  return ka < kb ? -1 : (ka > kb ? 1 : 0);
}

static int alloc_level(level_t* L, int64_t n, int nv) {
  L->n = n;
  L->key = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
  L->oc = (int32_t*)malloc((n ? n : 1) * 3 * sizeof(int32_t));
  L->refined = (uint8_t*)calloc(n ? n : 1, 1);
  L->U = (double*)calloc((n ? n : 1) * 8 * nv, sizeof(double));
  L->Un = (double*)calloc((n ? n : 1) * 8 * nv, sizeof(double));
  L->reg = (double*)calloc((n ? n : 1) * 12 * nv, sizeof(double));
  if (!L->key || !L->oc || !L->refined || !L->U || !L->Un || !L->reg) return -1;
  return 0;
}
static void free_level(level_t* L) {
  free(L->key); free(L->oc); free(L->refined); free(L->U); free(L->Un); free(L->reg);
  free(L->hkey); free(L->hval);
  memset(L, 0, sizeof *L);
}

/* Set octs of level l from an (unsorted) list of coordinates. */
static int set_octs(ryo_ctx* c, int l, okey_t* list, int64_t n) {
  int bits = c->bits0 + (l - c->cfg.level_min);
  for (int64_t i = 0; i < n; i++)
    list[i].key = ryo_hilbert_key(bits, (uint32_t)list[i].x, (uint32_t)list[i].y, (uint32_t)list[i].z);
  qsort(list, (size_t)n, sizeof(okey_t), cmp_okey);
  level_t* L = LV(c, l);
  free_level(L);
  if (alloc_level(L, n, c->nv)) return -1;
  for (int64_t i = 0; i < n; i++) {
    L->key[i] = list[i].key;
    L->oc[3 * i] = list[i].x;
    L->oc[3 * i + 1] = list[i].y;
    L->oc[3 * i + 2] = list[i].z;
  }
  return build_hash(L);
}

/* Density of the finest existing cell covering position p of level l. */
static double cover_rho(const ryo_ctx* c, int l, const int64_t p[3]) {
  double U[NV];
  cover_value(c, l, p, U);
  return U[0];
}

/* Refinement criterion on leaf cell p of level l. */
static int flag_cell(const ryo_ctx* c, int l, const int64_t p[3], double rho_c) {
  if (c->cfg.refine == RYO_REFINE_GRAD) {
    double g[3];
    for (int d = 0; d < 3; d++) {
      int64_t m[3] = {p[0], p[1], p[2]}, q[3] = {p[0], p[1], p[2]};
      m[d] -= 1;
      q[d] += 1;
      g[d] = 0.5 * (cover_rho(c, l, q) - cover_rho(c, l, m));
    }
    double th = c->cfg.refine_param;
    return g[0] * g[0] + g[1] * g[1] + g[2] * g[2] > (th * rho_c) * (th * rho_c);
  }
  if (c->cfg.refine == RYO_REFINE_MASS) {
    double thr = c->cfg.refine_param * ldexp(1.0, 3 * (l - c->cfg.level_min));
    return rho_c > thr;
  }
  return 0;
}

/* Neighbour rule: a flagged cell is refined only when all 26 neighbour cells
 * exist at its level (positions outside an outflow face count as existing). */
static int neighbours_exist(const ryo_ctx* c, int l, const int64_t p[3]) {
  const level_t* L = LVc(c, l);
  for (int dz = -1; dz <= 1; dz++)
    for (int dy = -1; dy <= 1; dy++)
      for (int dx = -1; dx <= 1; dx++) {
        if (!dx && !dy && !dz) continue;
        int64_t q[3] = {p[0] + dx, p[1] + dy, p[2] + dz};
        int out = 0;
        for (int a = 0; a < 3; a++) {
          int64_t N = ncells(c, l, a);
          if (q[a] < 0 && c->cfg.bc[2 * a] != RYO_BC_PERIODIC) out = 1;
          if (q[a] >= N && c->cfg.bc[2 * a + 1] != RYO_BC_PERIODIC) out = 1;
        }
        if (out) continue;
        bc_cell(c, l, q);
        if (find_oct(L, q[0] >> 1, q[1] >> 1, q[2] >> 1) < 0) return 0;
      }
  return 1;
}

int ryo_amr_build(ryo_ctx* c, const double* U_base, ryo_fill_fn fill, void* user) {
  if (!c || !U_base) return RYO_EINVAL;
  if (c->cfg.level_max > c->cfg.level_min && !fill && c->cfg.refine != RYO_REFINE_NONE) {
    set_err(c, "fill callback required when level_max > level_min");
    return RYO_EINVAL;
  }
  for (int i = 0; i < c->nlev; i++) free_level(&c->lev[i]);
  const int l0 = c->cfg.level_min;
  const int64_t nb0 = c->cfg.nbase[0], nb1 = c->cfg.nbase[1], nb2 = c->cfg.nbase[2];
  int64_t n0 = (nb0 / 2) * (nb1 / 2) * (nb2 / 2);
  okey_t* list = (okey_t*)malloc(n0 * sizeof(okey_t));
  if (!list) return RYO_ENOMEM;
  int64_t k = 0;
  for (int32_t z = 0; z < nb2 / 2; z++)
    for (int32_t y = 0; y < nb1 / 2; y++)
      for (int32_t x = 0; x < nb0 / 2; x++) {
        list[k].x = x; list[k].y = y; list[k].z = z; k++;
      }
  if (set_octs(c, l0, list, n0)) { free(list); return RYO_ENOMEM; }
  free(list);
  level_t* L = LV(c, l0);
  const int64_t ncell0 = nb0 * nb1 * nb2;
  for (int64_t o = 0; o < L->n; o++)
    for (int ci = 0; ci < 8; ci++) {
      int64_t x = 2 * (int64_t)L->oc[3 * o] + (ci & 1);
      int64_t y = 2 * (int64_t)L->oc[3 * o + 1] + ((ci >> 1) & 1);
      int64_t z = 2 * (int64_t)L->oc[3 * o + 2] + ((ci >> 2) & 1);
      for (int v = 0; v < c->nv; v++)
        L->U[v * 8 * L->n + 8 * o + ci] = U_base[v * ncell0 + x + nb0 * (y + nb1 * z)];
    }
  for (int l = l0; l < c->cfg.level_max; l++) {
    level_t* Lc = LV(c, l);
    uint8_t* flag = (uint8_t*)calloc(Lc->n ? Lc->n : 1, 1);
    if (!flag) return RYO_ENOMEM;
    int64_t nref = 0;
#pragma omp parallel for schedule(static) reduction(+ : nref)
    for (int64_t o = 0; o < Lc->n; o++)
      for (int ci = 0; ci < 8; ci++) {
        int64_t p[3] = {2 * (int64_t)Lc->oc[3 * o] + (ci & 1), 2 * (int64_t)Lc->oc[3 * o + 1] + ((ci >> 1) & 1),
                        2 * (int64_t)Lc->oc[3 * o + 2] + ((ci >> 2) & 1)};
        double rho_c = Lc->U[8 * o + ci];
        if (flag_cell(c, l, p, rho_c) && neighbours_exist(c, l, p)) {
          flag[o] |= (uint8_t)(1u << ci);
          nref++;
        }
      }
    if (nref == 0) { free(flag); break; }
    okey_t* nl = (okey_t*)malloc(nref * sizeof(okey_t));
    if (!nl) { free(flag); return RYO_ENOMEM; }
    int64_t m = 0;
    for (int64_t o = 0; o < Lc->n; o++) {
      Lc->refined[o] = flag[o];
      for (int ci = 0; ci < 8; ci++)
        if (flag[o] & (1u << ci)) {
          nl[m].x = 2 * Lc->oc[3 * o] + (ci & 1);
          nl[m].y = 2 * Lc->oc[3 * o + 1] + ((ci >> 1) & 1);
          nl[m].z = 2 * Lc->oc[3 * o + 2] + ((ci >> 2) & 1);
          m++;
        }
    }
    free(flag);
    if (set_octs(c, l + 1, nl, nref)) { free(nl); return RYO_ENOMEM; }
    free(nl);
    level_t* Lf = LV(c, l + 1);
    int32_t* ijk = (int32_t*)malloc(Lf->n * 8 * 3 * sizeof(int32_t));
    double* Uf = (double*)malloc(Lf->n * 8 * c->nv * sizeof(double));
    if (!ijk || !Uf) { free(ijk); free(Uf); return RYO_ENOMEM; }
    for (int64_t o = 0; o < Lf->n; o++)
      for (int ci = 0; ci < 8; ci++) {
        int64_t i = 8 * o + ci;
        ijk[3 * i] = 2 * Lf->oc[3 * o] + (ci & 1);
        ijk[3 * i + 1] = 2 * Lf->oc[3 * o + 1] + ((ci >> 1) & 1);
        ijk[3 * i + 2] = 2 * Lf->oc[3 * o + 2] + ((ci >> 2) & 1);
      }
    fill(user, l + 1, Lf->n * 8, ijk, Uf);
    memcpy(Lf->U, Uf, Lf->n * 8 * c->nv * sizeof(double));
    free(ijk);
    free(Uf);
  }
  /* restrict bottom-up so that every refined cell holds its children's mean */
  for (int l = c->cfg.level_max - 1; l >= l0; l--)
    if (LV(c, l + 1)->n > 0) restrict_level(c, l, LV(c, l)->U);
  c->built = 1;
  return RYO_OK;
}

/* ------------------------------------------------------------------------ */
/* Regrid between coarse steps (dynamic refinement).                          */
/*                                                                            */
/* Top-down over l = level_min .. level_max-1, with level l already final:    */
/*   1. every cell of level l (leaf or refined) is flagged by the build's     */
/*      criterion on its current value, and refined only when its 26          */
/*      neighbours exist at level l (the build's neighbour rule);              */
/*   2. level l+1 becomes the children of the refined cells, in Hilbert       */
/*      order: a child oct that existed keeps its values, a new one is         */
/*      filled by the MinMod-linear interpolation of its parent cell (the     */
/*      coarse-fine ghost formula); octs whose parent cell is no longer       */
/*      refined disappear with their descendants (the parent cell keeps its   */
/*      restricted value).                                                     */
/* Finally every refined cell is restricted bottom-up from its children.      */
/* ------------------------------------------------------------------------ */
int ryo_regrid(ryo_ctx* c, int64_t* n_created, int64_t* n_destroyed) {
  if (!c || !c->built) return RYO_EINVAL;
  int64_t created = 0, destroyed = 0;
  for (int l = c->cfg.level_min; l < c->cfg.level_max; l++) {
    level_t* Lc = LV(c, l);
    uint8_t* flag = (uint8_t*)calloc(Lc->n ? Lc->n : 1, 1);
    if (!flag) return RYO_ENOMEM;
    int64_t nref = 0;
    for (int64_t o = 0; o < Lc->n; o++)
      for (int ci = 0; ci < 8; ci++) {
        int64_t p[3] = {2 * (int64_t)Lc->oc[3 * o] + (ci & 1), 2 * (int64_t)Lc->oc[3 * o + 1] + ((ci >> 1) & 1),
                        2 * (int64_t)Lc->oc[3 * o + 2] + ((ci >> 2) & 1)};
        double rho_c = Lc->U[8 * o + ci];
        if (flag_cell(c, l, p, rho_c) && neighbours_exist(c, l, p)) {
          flag[o] |= (uint8_t)(1u << ci);
          nref++;
        }
      }
    okey_t* nl = (okey_t*)malloc((nref ? nref : 1) * sizeof(okey_t));
    if (!nl) { free(flag); return RYO_ENOMEM; }
    int64_t m = 0;
    for (int64_t o = 0; o < Lc->n; o++) {
      Lc->refined[o] = flag[o];
      for (int ci = 0; ci < 8; ci++)
        if (flag[o] & (1u << ci)) {
          nl[m].x = 2 * Lc->oc[3 * o] + (ci & 1);
          nl[m].y = 2 * Lc->oc[3 * o + 1] + ((ci >> 1) & 1);
          nl[m].z = 2 * Lc->oc[3 * o + 2] + ((ci >> 2) & 1);
          m++;
        }
    }
    free(flag);
    /* detach the old level l+1; build the new one */
    level_t old = *LV(c, l + 1);
    memset(LV(c, l + 1), 0, sizeof(level_t));
    if (set_octs(c, l + 1, nl, nref)) { free(nl); free_level(&old); return RYO_ENOMEM; }
    free(nl);
    level_t* Lf = LV(c, l + 1);
    for (int64_t o = 0; o < Lf->n; o++) {
      int64_t ko = find_oct(&old, Lf->oc[3 * o], Lf->oc[3 * o + 1], Lf->oc[3 * o + 2]);
      for (int ci = 0; ci < 8; ci++) {
        double U[NV];
        if (ko >= 0) {
          for (int v = 0; v < c->nv; v++) U[v] = old.U[(int64_t)v * 8 * old.n + 8 * ko + ci];
        } else {
          int64_t p[3] = {2 * (int64_t)Lf->oc[3 * o] + (ci & 1), 2 * (int64_t)Lf->oc[3 * o + 1] + ((ci >> 1) & 1),
                          2 * (int64_t)Lf->oc[3 * o + 2] + ((ci >> 2) & 1)};
          coarse_interp(c, l + 1, p, U);
        }
        for (int v = 0; v < c->nv; v++) Lf->U[(int64_t)v * 8 * Lf->n + 8 * o + ci] = U[v];
      }
      if (ko < 0) created++;
    }
    for (int64_t o = 0; o < old.n; o++)
      if (find_oct(Lf, old.oc[3 * o], old.oc[3 * o + 1], old.oc[3 * o + 2]) < 0) destroyed++;
    free_level(&old);
  }
  for (int l = c->cfg.level_max - 1; l >= c->cfg.level_min; l--)
    if (LV(c, l + 1)->n > 0) restrict_level(c, l, LV(c, l)->U);
  if (n_created) *n_created = created;
  if (n_destroyed) *n_destroyed = destroyed;
  return RYO_OK;
}

/* ------------------------------------------------------------------------ */
/* Time step, totals, driver.                                                 */
/* ------------------------------------------------------------------------ */
static int check_state(ryo_ctx* c) {
  int bad = 0;
  for (int i = 0; i < c->nlev; i++) {
    level_t* L = &c->lev[i];
    for (int64_t o = 0; o < L->n; o++)
      for (int ci = 0; ci < 8; ci++) {
        if (L->refined[o] & (1u << ci)) continue;
        int64_t cell = 8 * o + ci;
        double r = L->U[cell], E = L->U[4 * 8 * L->n + cell];
        int fin = 1;
        for (int v = 0; v < c->nv; v++) fin &= isfinite(L->U[v * 8 * L->n + cell]);
        if (!fin || !(r > 0.0) || !(E > 0.0)) bad = 1;
      }
  }
  if (bad) c->numeric_error = 1;
  return c->numeric_error;
}

int ryo_cfl_dt(ryo_ctx* c, double* dt_coarse) {
  if (!c || !dt_coarse || !c->built) return RYO_EINVAL;
  if (check_state(c)) { set_err(c, "non-finite or non-positive density/energy"); return RYO_ENUMERIC; }
  double g = c->cfg.gamma;
  double best = INFINITY;
  int64_t fl = 0;
  for (int l = c->cfg.level_min; l <= c->cfg.level_max; l++) {
    level_t* L = LV(c, l);
    if (L->n == 0) continue;
    double smax = 0.0;
    int any = 0;
    for (int64_t o = 0; o < L->n; o++)
      for (int ci = 0; ci < 8; ci++) {
        if (L->refined[o] & (1u << ci)) continue;
        double U[NV], W[NV];
        for (int v = 0; v < c->nv; v++) U[v] = L->U[v * 8 * L->n + 8 * o + ci];
        cons_to_prim(c, U, W, &fl);   /* the time step's conversions: not counted */
        double cs = sqrt(g * W[4] / W[0]);
        double s = fabs(W[1]) + fabs(W[2]) + fabs(W[3]) + 3.0 * cs;
        if (s > smax) smax = s;
        any = 1;
      }
    if (!any) continue;
    double dtl = c->cfg.cfl * dx_of(c, l) / smax;
    double cand = ldexp(dtl, l - c->cfg.level_min);
    if (cand < best) best = cand;
  }
  (void)fl;
  *dt_coarse = best;
  return RYO_OK;
}

int ryo_coarse_step(ryo_ctx* c, double dt) {
  if (!c || !c->built || !(dt > 0.0) || !isfinite(dt)) return RYO_EINVAL;
  advance_level(c, c->cfg.level_min, dt, 0);
  return RYO_OK;
}

int ryo_advance(ryo_ctx* c, int32_t n_coarse, double t_end, double* t_io, int32_t* n_done) {
  if (!c || !t_io || !c->built || n_coarse < 0) return RYO_EINVAL;
  double t = *t_io;
  int32_t k = 0;
  for (; k < n_coarse && t < t_end; k++) {
    double dt;
    int rc = ryo_cfl_dt(c, &dt);
    if (rc) { *t_io = t; if (n_done) *n_done = k; return rc; }
    int last = 0;
    if (dt >= t_end - t) { dt = t_end - t; last = 1; }
    advance_level(c, c->cfg.level_min, dt, 0);
    t = last ? t_end : t + dt;
  }
  *t_io = t;
  if (n_done) *n_done = k;
  if (check_state(c)) { set_err(c, "non-finite or non-positive density/energy"); return RYO_ENUMERIC; }
  return RYO_OK;
}

/* Sum over leaf cells of U * dx^3 (Neumaier compensated summation, levels
 * ascending, octs in Hilbert order, cells in in-oct order). */
int ryo_conserved_totals(const ryo_ctx* c, double* tot) {
  if (!c || !tot || !c->built) return RYO_EINVAL;
  for (int v = 0; v < c->nv; v++) {
    double s = 0.0, comp = 0.0;
    for (int l = c->cfg.level_min; l <= c->cfg.level_max; l++) {
      const level_t* L = LVc(c, l);
      double dx = dx_of(c, l);
      double vol = dx * dx * dx;
      for (int64_t o = 0; o < L->n; o++)
        for (int ci = 0; ci < 8; ci++) {
          if (L->refined[o] & (1u << ci)) continue;
          double x = L->U[v * 8 * L->n + 8 * o + ci] * vol;
          double t = s + x;
          if (fabs(s) >= fabs(x)) comp += (s - t) + x;
          else comp += (x - t) + s;
          s = t;
        }
    }
    tot[v] = s + comp;
  }
  return RYO_OK;
}

/* ------------------------------------------------------------------------ */
/* Lifetime and accessors.                                                   */
/* ------------------------------------------------------------------------ */
int ryo_create(const ryo_config* cfg, ryo_ctx** out) {
  if (!cfg || !out) return RYO_EINVAL;
  *out = NULL;
  if (cfg->level_min < 1 || cfg->level_max < cfg->level_min ||
      cfg->level_max - cfg->level_min + 1 > RYO_MAX_LEVELS || cfg->level_max > 20)
    return RYO_EINVAL;
  for (int a = 0; a < 3; a++)
    if (cfg->nbase[a] < 2 || (cfg->nbase[a] & 1)) return RYO_EINVAL;
  for (int a = 0; a < 3; a++) {
    int lo = cfg->bc[2 * a], hi = cfg->bc[2 * a + 1];
    if ((lo == RYO_BC_PERIODIC) != (hi == RYO_BC_PERIODIC)) return RYO_EINVAL;
    if ((lo != RYO_BC_PERIODIC && lo != RYO_BC_OUTFLOW) || (hi != RYO_BC_PERIODIC && hi != RYO_BC_OUTFLOW))
      return RYO_EINVAL;
  }
  if (!(cfg->gamma > 1.0) || !(cfg->cfl > 0.0) || !(cfg->boxlen > 0.0)) return RYO_EINVAL;
  if (!(cfg->rho_floor > 0.0) || !(cfg->p_floor > 0.0)) return RYO_EINVAL;
  if (cfg->refine < RYO_REFINE_NONE || cfg->refine > RYO_REFINE_MASS) return RYO_EINVAL;
  if (cfg->nscalar < 0 || cfg->nscalar > RYO_MAX_SCALARS) return RYO_EINVAL;
  ryo_ctx* c = (ryo_ctx*)calloc(1, sizeof(ryo_ctx));
  if (!c) return RYO_ENOMEM;
  c->cfg = *cfg;
  c->nv = 5 + cfg->nscalar;
  c->nlev = cfg->level_max - cfg->level_min + 1;
  int m = cfg->nbase[0];
  if (cfg->nbase[1] > m) m = cfg->nbase[1];
  if (cfg->nbase[2] > m) m = cfg->nbase[2];
  int noct = m / 2, bits = 0;
  while ((1 << bits) < noct) bits++;
  c->bits0 = bits;
  *out = c;
  return RYO_OK;
}

void ryo_destroy(ryo_ctx* c) {
  if (!c) return;
  for (int i = 0; i < c->nlev; i++) free_level(&c->lev[i]);
  free(c);
}

static int level_ok(const ryo_ctx* c, int32_t l) {
  return c && c->built && l >= c->cfg.level_min && l <= c->cfg.level_max;
}

int ryo_level_info(const ryo_ctx* c, int32_t l, int64_t* n_oct, int64_t* n_leaf) {
  if (!level_ok(c, l)) return RYO_EINVAL;
  const level_t* L = LVc(c, l);
  int64_t leaf = 0;
  for (int64_t o = 0; o < L->n; o++)
    for (int ci = 0; ci < 8; ci++) leaf += !(L->refined[o] & (1u << ci));
  if (n_oct) *n_oct = L->n;
  if (n_leaf) *n_leaf = leaf;
  return RYO_OK;
}

int ryo_get_mesh(const ryo_ctx* c, int32_t l, uint64_t* keys, uint8_t* refined) {
  if (!level_ok(c, l)) return RYO_EINVAL;
  const level_t* L = LVc(c, l);
  if (L->n == 0) return RYO_OK;   /* an empty level may hold no arrays */
  if (keys) memcpy(keys, L->key, L->n * sizeof(uint64_t));
  if (refined) memcpy(refined, L->refined, L->n);
  return RYO_OK;
}

int ryo_get_coords(const ryo_ctx* c, int32_t l, int32_t* xyz) {
  if (!level_ok(c, l) || !xyz) return RYO_EINVAL;
  const level_t* L = LVc(c, l);
  if (L->n) memcpy(xyz, L->oc, L->n * 3 * sizeof(int32_t));
  return RYO_OK;
}

int ryo_download(const ryo_ctx* c, int32_t l, double* U) {
  if (!level_ok(c, l) || !U) return RYO_EINVAL;
  const level_t* L = LVc(c, l);
  if (L->n) memcpy(U, L->U, L->n * 8 * c->nv * sizeof(double));
  return RYO_OK;
}

int ryo_upload(ryo_ctx* c, int32_t l, const double* U) {
  if (!level_ok(c, l) || !U) return RYO_EINVAL;
  level_t* L = LV(c, l);
  if (L->n) memcpy(L->U, U, L->n * 8 * c->nv * sizeof(double));
  c->numeric_error = 0;
  return RYO_OK;
}

int ryo_set_refine_param(ryo_ctx* c, double value) {
  if (!c || !(value == value)) return RYO_EINVAL;
  c->cfg.refine_param = value;
  return RYO_OK;
}

int64_t ryo_floor_count(const ryo_ctx* c) { return c ? c->floors : 0; }
void ryo_reset_floor_count(ryo_ctx* c) { if (c) c->floors = 0; }
const char* ryo_last_error(const ryo_ctx* c) { return c ? c->err : "null context"; }

int ryo_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
void ryo_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
