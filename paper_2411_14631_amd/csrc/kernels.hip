// HIP kernels (gfx950) of the octree MUSCL-Hancock / MinMod / HLLC hydro step.
//
// Work unit: a tile = an aligned 2x2x2 block of octs (4x4x4 cells, the octs
// sharing their Hilbert key except for the lowest 3 bits).  One 64-lane
// wavefront owns one tile; the tile's primitive-variable stencil (the 8x8x8
// box around the 4x4x4 core, of which 304 positions are used) is staged in
// LDS once and shared by the tile's 64 cells.  Phases per tile:
//   A  gather U of the 304 stencil positions through the tile's 4x4x4 table
//      of neighbouring octs (real or ghost), convert to primitives -> LDS
//   B  MinMod slopes and the half-step predictor for the 160 cells that
//      border a flux face (core + one layer per face) -> LDS
//   C  240 face fluxes (HLLC; normal slopes recomputed from LDS) -> LDS
//   D  per cell: coarse-fine register override, conservative FP64 update,
//      fused CFL reduction on the new state; fine-side flux registers.
// The scheme's definitions: ideal-gas primitives with floors; undivided
// MinMod slopes; unsplit primitive predictor with h = lambda/2 (van Leer
// 1979; Toro 2009 ch. 13-14); face states W~ +- D/2; HLLC with Davis wave
// speeds (Toro, Spruce & Speares 1994); Berger & Colella (1989) refluxing.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ry_internal.h"

namespace ry {

// ---------------------------------------------------------------------------
// Stencil position tables (compile-time): positions s in [-2,5]^3 relative to
// the tile's first cell, stored as (sx+2) + 8 (sy+2) + 64 (sz+2).
// ---------------------------------------------------------------------------
struct StencilTables {
  uint16_t a[304];   // positions whose primitives are needed
  uint16_t b[160];   // positions that get a predicted state
};

constexpr StencilTables make_tables() {
  StencilTables t{};
  int na = 0, nb = 0;
  for (int z = -2; z <= 5; ++z)
    for (int y = -2; y <= 5; ++y)
      for (int x = -2; x <= 5; ++x) {
        const int ox = (x < 0 || x > 3), oy = (y < 0 || y > 3), oz = (z < 0 || z > 3);
        const int nout = ox + oy + oz;
        const bool ex = (x == -1 || x == 4), ey = (y == -1 || y == 4), ez = (z == -1 || z == 4);
        bool needA = (nout <= 1);
        if (nout == 2) needA = (ox ? ex : true) && (oy ? ey : true) && (oz ? ez : true);
        bool needB = (nout == 0) || (nout == 1 && (ox ? ex : true) && (oy ? ey : true) && (oz ? ez : true));
        const uint16_t idx = uint16_t((x + 2) + 8 * (y + 2) + 64 * (z + 2));
        if (needA) t.a[na++] = idx;
        if (needB) t.b[nb++] = idx;
      }
  return t;
}
__constant__ StencilTables c_st = make_tables();

static_assert(make_tables().a[303] != 0, "stencil table A must hold 304 positions");

template <typename Real>
struct TileLDS {
  Real W[NVAR][512];      // primitives on the padded 8^3 stencil; reused for fluxes
  Real Wt[NVAR][216];     // predicted states on the padded 6^3 box [-1,4]^3
  int32_t tab[TILE_TAB];  // ext oct index of the 4x4x4 oct neighbourhood
  uint8_t ref[TILE_TAB];  // refined-cell bytes of those octs
};
static_assert(sizeof(double) * NVAR * 240 <= sizeof(float) * NVAR * 512, "flux alias");

// ---------------------------------------------------------------------------
// Scalar helpers.
// ---------------------------------------------------------------------------
template <typename Real>
__device__ __forceinline__ Real mmod(Real a, Real b) {
  // MinMod, sign-test form
  Real m = (a < b) ? a : b;
  Real M = (a > b) ? a : b;
  return (a > Real(0) && b > Real(0)) ? m : ((a < Real(0) && b < Real(0)) ? M : Real(0));
}

template <typename Real> __device__ __forceinline__ Real fdiv(Real a, Real b);
template <> __device__ __forceinline__ double fdiv<double>(double a, double b) { return a / b; }
template <> __device__ __forceinline__ float fdiv<float>(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
}
template <typename Real> __device__ __forceinline__ Real fsqrt(Real a);
template <> __device__ __forceinline__ double fsqrt<double>(double a) { return sqrt(a); }
template <> __device__ __forceinline__ float fsqrt<float>(float a) { return __builtin_amdgcn_sqrtf(a); }

// Primitive variables (FP64 in both forms) with floors.
__device__ __forceinline__ void cons2prim(const double U[NVAR], double W[NVAR], double g, double rf, double pf,
                                          int& nfl) {
  double rho = U[0];
  if (rho < rf) { rho = rf; ++nfl; }
  const double ke = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / rho;
  double p = (g - 1.0) * (U[4] - ke);
  if (p < pf) { p = pf; ++nfl; }
  W[0] = rho;
  W[1] = U[1] / rho;
  W[2] = U[2] / rho;
  W[3] = U[3] / rho;
  W[4] = p;
}

// CFL signal speed |u|+|v|+|w|+3c of a conserved state, in the same IEEE
// operations as the definition (no contraction), so dt is reproducible.
__device__ __forceinline__ double signal_speed(const double U[NVAR], double g, double rf, double pf) {
#pragma clang fp contract(off)
  double rho = U[0];
  if (rho < rf) rho = rf;
  const double ke = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / rho;
  double p = (g - 1.0) * (U[4] - ke);
  if (p < pf) p = pf;
  const double u = U[1] / rho, v = U[2] / rho, w = U[3] / rho;
  const double c = sqrt(g * p / rho);
  return fabs(u) + fabs(v) + fabs(w) + 3.0 * c;
}

// HLLC flux in the face-normal frame: (r, u, a, b, p) = density, normal and
// two tangential velocities, pressure of the left / right face state.  The
// star state is formed only for the side the branch selects.  Output Fn in
// the same frame (mass, normal momentum, tangential momenta, energy).
template <typename Real>
__device__ __forceinline__ void hllc_n(Real rl, Real ul, Real al, Real bl, Real pl, Real rr, Real ur, Real ar,
                                       Real br, Real pr, Real g, Real Fn[5]) {
  const Real cl = fsqrt<Real>(fdiv<Real>(g * pl, rl));
  const Real cr = fsqrt<Real>(fdiv<Real>(g * pr, rr));
  const Real SL = fmin(ul - cl, ur - cr);
  const Real SR = fmax(ul + cl, ur + cr);
  const Real num = pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur);
  const Real den = rl * (SL - ul) - rr * (SR - ur);
  const Real Ss = fdiv<Real>(num, den);
  const bool useL = (SL >= Real(0)) || (Ss >= Real(0));
  const Real rK = useL ? rl : rr, uK = useL ? ul : ur, aK = useL ? al : ar, bK = useL ? bl : br;
  const Real pK = useL ? pl : pr, SK = useL ? SL : SR;
  const bool star = useL ? !(SL >= Real(0)) : (SR > Real(0));
  const Real EK = fdiv<Real>(pK, g - Real(1)) + Real(0.5) * rK * (uK * uK + aK * aK + bK * bK);
  const Real mK = rK * uK;
  Fn[0] = mK;
  Fn[1] = mK * uK + pK;
  Fn[2] = mK * aK;
  Fn[3] = mK * bK;
  Fn[4] = (EK + pK) * uK;
  if (star) {
    const Real r = (SK - uK) / (SK - Ss);   // true division: r == 1 when S* == u_K
    const Real q = SK - uK;
    const Real Es = EK + rK * (Ss - uK) * (Ss + fdiv<Real>(pK, rK * q));
    Fn[0] = Fn[0] + SK * (r * rK - rK);
    Fn[1] = Fn[1] + SK * (r * (rK * Ss) - mK);
    Fn[2] = Fn[2] + SK * (r * (rK * aK) - rK * aK);
    Fn[3] = Fn[3] + SK * (r * (rK * bK) - rK * bK);
    Fn[4] = Fn[4] + SK * (r * Es - EK);
  }
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// XCD-aware mapping of a workgroup to a contiguous range of work items:
// workgroups are dealt round-robin to the 8 XCDs, so XCD x receives every
// 8th workgroup; give it the x-th contiguous slice of the items instead.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int x = bid & 7, j = bid >> 3;
  const int q = nblocks >> 3, r = nblocks & 7;
  return x * q + (x < r ? x : r) + j;
}

// ---------------------------------------------------------------------------
// The per-tile hydro update.
// ---------------------------------------------------------------------------
template <typename Real>
__device__ void hydro_tile(const HydroArgs& A, int tile, TileLDS<Real>& S, int lane, bool active) {
  // `active` is wave-uniform; an inactive wave only keeps the barrier count
  const double g = A.gamma, rf = A.rho_floor, pf = A.p_floor;
  const int64_t P = A.plane;
  int nfl = 0;
  const uint32_t fl = A.tflag[tile];
  const int box = A.tile_box ? A.tile_box[tile] : 0;
  const double lam = A.lam_dev ? A.lam_dev[box] : A.lam_host;
  const Real h = Real(0.5 * lam);

  // --- phase 0: the tile's oct table and refined bytes
  if (active) {
    const int32_t e = A.tab[size_t(tile) * TILE_TAB + lane];
    S.tab[lane] = e;
    S.ref[lane] = (e >= 0) ? A.refined[e] : uint8_t(0);
  }
  __syncthreads();

  // --- phase A: gather + primitives
  for (int i = lane; active && i < 304; i += 64) {
    const int iw = c_st.a[i];
    int sx = (iw & 7) - 2, sy = ((iw >> 3) & 7) - 2, sz = (iw >> 6) - 2;
    if ((fl & CL_LOX) && sx < 0) sx = 0;
    if ((fl & CL_HIX) && sx > 3) sx = 3;
    if ((fl & CL_LOY) && sy < 0) sy = 0;
    if ((fl & CL_HIY) && sy > 3) sy = 3;
    if ((fl & CL_LOZ) && sz < 0) sz = 0;
    if ((fl & CL_HIZ) && sz > 3) sz = 3;
    const int t = ((sx >> 1) + 1) + 4 * ((sy >> 1) + 1) + 16 * ((sz >> 1) + 1);
    const int32_t e = S.tab[t];
    double U[NVAR];
    if (e >= 0) {
      const int64_t cell = int64_t(e) * 8 + ((sx & 1) | ((sy & 1) << 1) | ((sz & 1) << 2));
#pragma unroll
      for (int v = 0; v < NVAR; ++v) U[v] = A.U[v * P + cell];
    } else {
      U[0] = 1.0; U[1] = 0.0; U[2] = 0.0; U[3] = 0.0; U[4] = 1.0;   // never read by a leaf update
    }
    double W[NVAR];
    cons2prim(U, W, g, rf, pf, nfl);
#pragma unroll
    for (int v = 0; v < NVAR; ++v) S.W[v][iw] = Real(W[v]);
  }
  __syncthreads();

  // --- phase B: slopes + predictor
  for (int i = lane; active && i < 160; i += 64) {
    const int iw = c_st.b[i];
    const int sx = (iw & 7) - 2, sy = ((iw >> 3) & 7) - 2, sz = (iw >> 6) - 2;
    Real W0[NVAR], D[3][NVAR];
#pragma unroll
    for (int v = 0; v < NVAR; ++v) W0[v] = S.W[v][iw];
    const int st[3] = {1, 8, 64};
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int v = 0; v < NVAR; ++v)
        D[d][v] = mmod<Real>(W0[v] - S.W[v][iw - st[d]], S.W[v][iw + st[d]] - W0[v]);
    const Real r = W0[0], u = W0[1], vv = W0[2], w = W0[3], p = W0[4];
    const Real ir = fdiv<Real>(Real(1), r);
    const Real gg = Real(g);
    Real Wt[NVAR];
    Wt[0] = r - h * (u * D[0][0] + r * D[0][1] + vv * D[1][0] + r * D[1][2] + w * D[2][0] + r * D[2][3]);
    Wt[1] = u - h * (u * D[0][1] + vv * D[1][1] + w * D[2][1] + D[0][4] * ir);
    Wt[2] = vv - h * (u * D[0][2] + vv * D[1][2] + w * D[2][2] + D[1][4] * ir);
    Wt[3] = w - h * (u * D[0][3] + vv * D[1][3] + w * D[2][3] + D[2][4] * ir);
    Wt[4] = p - h * (u * D[0][4] + vv * D[1][4] + w * D[2][4] + gg * p * (D[0][1] + D[1][2] + D[2][3]));
    const int ip = (sx + 1) + 6 * (sy + 1) + 36 * (sz + 1);
#pragma unroll
    for (int v = 0; v < NVAR; ++v) S.Wt[v][ip] = Wt[v];
  }
  __syncthreads();

  // --- phase C: face fluxes (kept in registers, then written over W)
  double Fr[4][NVAR];
#pragma unroll
  for (int rnd = 0; rnd < 4; ++rnd) {
    const int f = lane + 64 * rnd;
    if (active && f < 240) {
      const int d = f / 80;
      const int rem = f - 80 * d;
      const int pl_ = (rem >> 4) - 1, ta = rem & 3, tb = (rem >> 2) & 3;
      // lower cell of the face: coordinate pl_ along d, (ta, tb) along the
      // tangential axes in increasing order
      const int cx = (d == 0) ? pl_ : ta;
      const int cy = (d == 0) ? ta : ((d == 1) ? pl_ : tb);
      const int cz = (d == 2) ? pl_ : tb;
      const int stw = (d == 0) ? 1 : ((d == 1) ? 8 : 64);
      const int stp = (d == 0) ? 1 : ((d == 1) ? 6 : 36);
      const int iwA = (cx + 2) + 8 * (cy + 2) + 64 * (cz + 2);
      const int ipA = (cx + 1) + 6 * (cy + 1) + 36 * (cz + 1);
      Real WL[NVAR], WR[NVAR];
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        const Real wam = S.W[v][iwA - stw], wa = S.W[v][iwA], wb = S.W[v][iwA + stw], wbp = S.W[v][iwA + 2 * stw];
        const Real da = mmod<Real>(wa - wam, wb - wa);
        const Real db = mmod<Real>(wb - wa, wbp - wb);
        WL[v] = S.Wt[v][ipA] + Real(0.5) * da;
        WR[v] = S.Wt[v][ipA + stp] - Real(0.5) * db;
      }
      const Real rfr = Real(rf), pfr = Real(pf);
      if (WL[0] < rfr) { WL[0] = rfr; ++nfl; }
      if (WR[0] < rfr) { WR[0] = rfr; ++nfl; }
      if (WL[4] < pfr) { WL[4] = pfr; ++nfl; }
      if (WR[4] < pfr) { WR[4] = pfr; ++nfl; }
      const Real unl = (d == 0) ? WL[1] : ((d == 1) ? WL[2] : WL[3]);
      const Real unr = (d == 0) ? WR[1] : ((d == 1) ? WR[2] : WR[3]);
      const Real t1l = (d == 0) ? WL[2] : WL[1], t1r = (d == 0) ? WR[2] : WR[1];
      const Real t2l = (d == 2) ? WL[2] : WL[3], t2r = (d == 2) ? WR[2] : WR[3];
      Real Fn[5];
      hllc_n<Real>(WL[0], unl, t1l, t2l, WL[4], WR[0], unr, t1r, t2r, WR[4], Real(g), Fn);
      Fr[rnd][0] = double(Fn[0]);
      Fr[rnd][1] = double((d == 0) ? Fn[1] : Fn[2]);
      Fr[rnd][2] = double((d == 1) ? Fn[1] : ((d == 0) ? Fn[2] : Fn[3]));
      Fr[rnd][3] = double((d == 2) ? Fn[1] : Fn[3]);
      Fr[rnd][4] = double(Fn[4]);
    }
  }
  __syncthreads();
  double* SF = reinterpret_cast<double*>(&S.W[0][0]);   // [5][240]
#pragma unroll
  for (int rnd = 0; rnd < 4; ++rnd) {
    const int f = lane + 64 * rnd;
    if (active && f < 240) {
#pragma unroll
      for (int v = 0; v < NVAR; ++v) SF[v * 240 + f] = Fr[rnd][v];
    }
  }
  __syncthreads();

  // --- phase D: update of the cell owned by this lane
  {
    const int cx = lane & 3, cy = (lane >> 2) & 3, cz = lane >> 4;
    const int ts = ((cx >> 1) + 1) + 4 * ((cy >> 1) + 1) + 16 * ((cz >> 1) + 1);
    const int32_t e = active ? S.tab[ts] : -1;
    const int ci = (cx & 1) | ((cy & 1) << 1) | ((cz & 1) << 2);
    const bool leaf = (e >= 0) && (e < A.n_oct) && !((S.ref[ts] >> ci) & 1);
    double s = 0.0;
    if (leaf) {
      const int cc[3] = {cx, cy, cz};
      double acc[NVAR] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int ta = cc[d == 0 ? 1 : 0], tb = cc[d == 2 ? 1 : 2];
        const int fm = d * 80 + cc[d] * 16 + ta + 4 * tb;
        const int fp = fm + 16;
        double Fm[NVAR], Fp[NVAR];
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
          Fm[v] = SF[v * 240 + fm];
          Fp[v] = SF[v * 240 + fp];
        }
        if (A.child) {
          // a refined neighbour across a face: use its child oct's register
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            int n[3] = {cx, cy, cz};
            n[d] += side ? 1 : -1;
            const uint32_t lo = (d == 0) ? CL_LOX : ((d == 1) ? CL_LOY : CL_LOZ);
            const uint32_t hi = lo << 1;
            if ((n[d] < 0 && (fl & lo)) || (n[d] > 3 && (fl & hi))) continue;
            const int tn = ((n[0] >> 1) + 1) + 4 * ((n[1] >> 1) + 1) + 16 * ((n[2] >> 1) + 1);
            const int32_t en = S.tab[tn];
            const int cn = (n[0] & 1) | ((n[1] & 1) << 1) | ((n[2] & 1) << 2);
            if (en >= 0 && en < A.n_oct && ((S.ref[tn] >> cn) & 1)) {
              const int32_t ch = A.child[int64_t(en) * 8 + cn];
              const int face = 2 * d + (side ? 0 : 1);   // child's face toward this cell
              const double* q = A.reg_fine + (int64_t(ch) * 6 + face) * NVAR * 2;
#pragma unroll
              for (int v = 0; v < NVAR; ++v) {
                const double fb = 0.125 * (q[2 * v] + q[2 * v + 1]);
                if (side) Fp[v] = fb; else Fm[v] = fb;
              }
            }
          }
        }
#pragma unroll
        for (int v = 0; v < NVAR; ++v) acc[v] += (Fm[v] - Fp[v]);
      }
      const int64_t cell = int64_t(e) * 8 + ci;
      double Un[NVAR];
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        Un[v] = A.U[v * P + cell] + lam * acc[v];
        A.Un[v * P + cell] = Un[v];
      }
      if (A.smax || A.err) {
        s = signal_speed(Un, g, rf, pf);
        const bool bad = !(isfinite(Un[0]) && isfinite(Un[1]) && isfinite(Un[2]) && isfinite(Un[3]) &&
                           isfinite(Un[4])) || !(Un[0] > 0.0) || !(Un[4] > 0.0) || !isfinite(s);
        if (bad) {
          atomicOr(A.err, 1);
          s = 0.0;
        }
      }
    }
    if (active && A.smax) {
      const double m = wave_max(s);
      if (lane == 0 && m > 0.0) atomicMax(&A.smax[box], (unsigned long long)__double_as_longlong(m));
    }
  }

  // --- fine-side registers: q_s = (f1 + f2) + (f3 + f4) on coarse-fine faces
  if (active && A.record_reg && lane < 48) {
    const int b = lane / 6, face = lane - 6 * (lane / 6);
    const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
    const int tb_ = (bx + 1) + 4 * (by + 1) + 16 * (bz + 1);
    const int32_t eb = S.tab[tb_];
    const int d = face >> 1, up = face & 1;
    const int dd = up ? 1 : -1;
    const int rx = bx + (d == 0 ? dd : 0), ry_ = by + (d == 1 ? dd : 0), rz = bz + (d == 2 ? dd : 0);
    const int rd = (d == 0) ? rx : ((d == 1) ? ry_ : rz);
    const uint32_t lo = (d == 0) ? CL_LOX : ((d == 1) ? CL_LOY : CL_LOZ);
    const bool clamped = (rd < 0 && (fl & lo)) || (rd > 1 && (fl & (lo << 1)));
    if (eb >= 0 && eb < A.n_oct && !clamped) {
      const int tn = (rx + 1) + 4 * (ry_ + 1) + 16 * (rz + 1);
      if (S.tab[tn] >= A.n_oct) {
        // the 4 cells of the oct on this face, ascending in-oct index: insert
        // bit `up` at position d into j = 0..3
        const int m = (1 << d) - 1;
        int fi[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = (j & m) | (up << d) | ((j & ~m) << 1);
          const int ccx = 2 * bx + (c & 1), ccy = 2 * by + ((c >> 1) & 1), ccz = 2 * bz + ((c >> 2) & 1);
          const int cd = (d == 0) ? ccx : ((d == 1) ? ccy : ccz);
          const int ta = (d == 0) ? ccy : ccx;
          const int tbb = (d == 2) ? ccy : ccz;
          fi[j] = d * 80 + (cd + up) * 16 + ta + 4 * tbb;
        }
        double* q = A.reg_own + (int64_t(eb) * 6 + face) * NVAR * 2;
#pragma unroll
        for (int v = 0; v < NVAR; ++v)
          q[2 * v + A.substep] =
              (SF[v * 240 + fi[0]] + SF[v * 240 + fi[1]]) + (SF[v * 240 + fi[2]] + SF[v * 240 + fi[3]]);
      }
    }
  }
  if (active && A.floors) {
    const int tot = wave_sum(nfl);
    if (lane == 0 && tot) atomicAdd(A.floors, (unsigned long long)tot);
  }
  __syncthreads();
}

template <typename Real, int TPW>
__global__ __launch_bounds__(64 * TPW) void hydro_kernel(HydroArgs A) {
  __shared__ TileLDS<Real> S[TPW];
  if (A.skip && *A.skip) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ngroups = (A.n_tile + TPW - 1) / TPW;
  const int grp = xcd_remap(blockIdx.x, gridDim.x);
  if (grp >= ngroups) return;
  const int tile = grp * TPW + w;
  hydro_tile<Real>(A, tile < A.n_tile ? tile : 0, S[w], lane, tile < A.n_tile);
}

// Persistent variant: workgroups pop groups of tiles from 8 per-XCD queues
// (one contiguous slice of the Hilbert-ordered tile list per XCD; a
// workgroup whose own queue is empty takes from the next one).  Every
// workgroup exits once all 8 queues are exhausted.
template <typename Real, int TPW>
__global__ __launch_bounds__(64 * TPW) void hydro_kernel_persistent(HydroArgs A, int batch) {
  __shared__ TileLDS<Real> S[TPW];
  __shared__ int s_item;
  if (A.skip && *A.skip) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ngroups = (A.n_tile + TPW - 1) / TPW;
  const int nitems = (ngroups + batch - 1) / batch;
  const int q = nitems >> 3, r = nitems & 7;
  int cur = blockIdx.x & 7;
  int exhausted = 0;
  while (true) {
    if (threadIdx.x == 0) {
      int item = -1;
      while (exhausted < 8) {
        const int qlen = q + (cur < r ? 1 : 0);
        const unsigned int k = atomicAdd(&A.queue[cur], 1u);
        if (int(k) < qlen) {
          item = cur * q + (cur < r ? cur : r) + int(k);
          break;
        }
        cur = (cur + 1) & 7;
        ++exhausted;
      }
      s_item = item;
    }
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item < 0) break;
    for (int j = 0; j < batch; ++j) {
      const int grp = item * batch + j;
      if (grp >= ngroups) break;
      const int tile = grp * TPW + w;
      hydro_tile<Real>(A, tile < A.n_tile ? tile : 0, S[w], lane, tile < A.n_tile);
    }
  }
}

template <typename Real, int TPW>
static int launch_hydro_t(const HydroArgs& a, const ry_tuning& t, int num_cu, hipStream_t s) {
  const int ngroups = (a.n_tile + TPW - 1) / TPW;
  if (ngroups == 0) return 0;
  if (!t.persistent) {
    hipLaunchKernelGGL((hydro_kernel<Real, TPW>), dim3(ngroups), dim3(64 * TPW), 0, s, a);
  } else {
    const int batch = t.batch > 0 ? t.batch : 1;
    const int nitems = (ngroups + batch - 1) / batch;
    int grid = num_cu * (t.waves_per_cu > 0 ? t.waves_per_cu : 4) / TPW;
    if (grid < 8) grid = 8;
    if (grid > nitems) grid = ((nitems + 7) / 8) * 8;
    hipLaunchKernelGGL((hydro_kernel_persistent<Real, TPW>), dim3(grid), dim3(64 * TPW), 0, s, a, batch);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int hydro_max_tiles_per_wg() { return 4; }

int launch_hydro(const HydroArgs& a, int precision, const ry_tuning& t, int num_cu, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const int tpw = t.tiles_per_wg;
  if (precision == RY_MIXED) {
    if (tpw == 1) return launch_hydro_t<float, 1>(a, t, num_cu, s);
    if (tpw == 2) return launch_hydro_t<float, 2>(a, t, num_cu, s);
    return launch_hydro_t<float, 4>(a, t, num_cu, s);
  }
  if (tpw == 1) return launch_hydro_t<double, 1>(a, t, num_cu, s);
  if (tpw == 2) return launch_hydro_t<double, 2>(a, t, num_cu, s);
  return launch_hydro_t<double, 4>(a, t, num_cu, s);
}

// ---------------------------------------------------------------------------
// Ghost octs: MinMod-limited linear interpolation of the covering coarse
// cell's conserved variables, written into both state buffers.
// ---------------------------------------------------------------------------
__global__ void ghost_kernel(GhostArgs A) {
  if (A.skip && *A.skip) return;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= A.n_ghost * 8) return;
  const int64_t gi = i >> 3;
  const int c = int(i & 7);
  const double sx = (c & 1) ? 0.25 : -0.25, sy = (c & 2) ? 0.25 : -0.25, sz = (c & 4) ? 0.25 : -0.25;
  int64_t src[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) src[k] = A.gsrc[gi * 7 + k];
  const int64_t dst = (A.n_oct + gi) * 8 + c;
#pragma unroll
  for (int v = 0; v < NVAR; ++v) {
    double val[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      const int up = int(src[k] >> 48);
      const int64_t cell = src[k] & ((int64_t(1) << 48) - 1);
      val[k] = A.src[up][v * A.src_plane[up] + cell];
    }
    const double q = val[0];
    const double mx = mmod<double>(q - val[1], val[2] - q);
    const double my = mmod<double>(q - val[3], val[4] - q);
    const double mz = mmod<double>(q - val[5], val[6] - q);
    const double out = q + (sx * mx + sy * my + sz * mz);
    A.dst0[v * A.plane + dst] = out;
    A.dst1[v * A.plane + dst] = out;
  }
}

int launch_ghost(const GhostArgs& a, void* stream) {
  if (a.n_ghost == 0) return 0;
  const int64_t n = a.n_ghost * 8;
  hipLaunchKernelGGL(ghost_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// Restriction: refined cell of level l = mean of its 8 children.
// ---------------------------------------------------------------------------
__global__ void restrict_kernel(const double* __restrict__ Uf, int64_t pf, int64_t nf,
                                const int32_t* __restrict__ parent, double* __restrict__ Uc, int64_t pc,
                                const int32_t* skip) {
  if (skip && *skip) return;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nf * NVAR) return;
  const int64_t k = i / NVAR;
  const int v = int(i - k * NVAR);
  const double* s = Uf + v * pf + 8 * k;
  Uc[v * pc + parent[k]] = 0.125 * (((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])));
}

int launch_restrict(const double* Uf, int64_t pf, int64_t nf, const int32_t* parent, double* Uc, int64_t pc,
                    const int32_t* skip, void* stream) {
  if (nf == 0) return 0;
  const int64_t n = nf * NVAR;
  hipLaunchKernelGGL(restrict_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, Uf, pf,
                     nf, parent, Uc, pc, skip);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// CFL: max signal speed over the leaf cells of a level -> atomicMax slot.
// ---------------------------------------------------------------------------
__global__ void cfl_kernel(const double* __restrict__ U, int64_t plane, int64_t n_oct,
                           const uint8_t* __restrict__ refined, double g, double rf, double pf,
                           unsigned long long* slot, int32_t* err) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < n_oct * 8) {
    const int64_t o = i >> 3;
    const int c = int(i & 7);
    if (!((refined[o] >> c) & 1)) {
      double Uc[NVAR];
#pragma unroll
      for (int v = 0; v < NVAR; ++v) Uc[v] = U[v * plane + i];
      s = signal_speed(Uc, g, rf, pf);
      const bool bad = !(isfinite(Uc[0]) && isfinite(Uc[1]) && isfinite(Uc[2]) && isfinite(Uc[3]) &&
                         isfinite(Uc[4])) || !(Uc[0] > 0.0) || !(Uc[4] > 0.0) || !isfinite(s);
      if (bad) {
        atomicOr(err, 1);
        s = 0.0;
      }
    }
  }
  const double m = wave_max(s);
  if ((threadIdx.x & 63) == 0 && m > 0.0) atomicMax(slot, (unsigned long long)__double_as_longlong(m));
}

int launch_cfl(const double* U, int64_t plane, int64_t n_oct, const uint8_t* refined, double g, double rf, double pf,
               unsigned long long* slot, int32_t* err, void* stream) {
  if (n_oct == 0) return 0;
  const int64_t n = n_oct * 8;
  hipLaunchKernelGGL(cfl_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, U, plane, n_oct,
                     refined, g, rf, pf, slot, err);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// Time step on the device: dt from the CFL slots, clipped to t_end; lambda.
// ---------------------------------------------------------------------------
__global__ void finalize_kernel(FinalizeArgs A) {
#pragma clang fp contract(off)
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (!A.batch) {
    if (i != 0) return;
    if (*A.done) {
      *A.skip = 1;
      *A.lam = 0.0;
      return;
    }
    double best = INFINITY;
    for (int k = 0; k < A.nslot; ++k) {
      const double smax = __longlong_as_double((long long)A.smax[k]);
      if (!(smax > 0.0)) continue;
      const double dtl = A.cfl * A.dx[k] / smax;
      const double cand = ldexp(dtl, k);
      if (cand < best) best = cand;
    }
    for (int k = 0; k < A.nslot; ++k) A.clear[k] = 0ull;
    const double t = *A.t;
    double dt = best;
    int last = 0;
    if (dt >= A.t_end - t) {
      dt = A.t_end - t;
      last = 1;
    }
    if (!(dt > 0.0)) {
      *A.done = 1;
      *A.skip = 1;
      *A.lam = 0.0;
      return;
    }
    *A.lam = dt / A.dx[0];
    *A.t = last ? A.t_end : t + dt;
    *A.skip = 0;
    *A.nstep += 1;
    if (last) *A.done = 1;
  } else {
    if (i >= A.nslot) return;
    const double smax = __longlong_as_double((long long)A.smax[i]);
    A.clear[i] = 0ull;
    const double dx = A.dx_box[i];
    const double dt = A.cfl * dx / smax;
    A.lam[i] = dt / dx;
    A.t[i] = A.t[i] + dt;
    if (i == 0) *A.nstep += 1;
  }
}

int launch_finalize(const FinalizeArgs& a, void* stream) {
  const int n = a.batch ? a.nslot : 1;
  hipLaunchKernelGGL(finalize_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ void zero_u32_kernel(unsigned int* p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}
__global__ void zero_u64_kernel(unsigned long long* p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}
int launch_zero_u32(unsigned int* p, int64_t n, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(zero_u32_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, p, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int launch_zero_u64(unsigned long long* p, int64_t n, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(zero_u64_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, p, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// Conserved totals: fixed-shape two-pass reduction (deterministic).
// ---------------------------------------------------------------------------
constexpr int TOT_BLOCKS = 1024;
int totals_blocks() { return TOT_BLOCKS; }

__global__ void totals_kernel(const double* __restrict__ U, int64_t plane, int64_t n_oct,
                              const uint8_t* __restrict__ refined, double vol, double* __restrict__ partial) {
  __shared__ double red[NVAR][256];
  const int64_t ncell = n_oct * 8;
  const int64_t per = (ncell + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = int64_t(blockIdx.x) * per;
  const int64_t i1 = (i0 + per < ncell) ? i0 + per : ncell;
  double acc[NVAR] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    if ((refined[i >> 3] >> (i & 7)) & 1) continue;
#pragma unroll
    for (int v = 0; v < NVAR; ++v) acc[v] += U[v * plane + i] * vol;
  }
#pragma unroll
  for (int v = 0; v < NVAR; ++v) red[v][threadIdx.x] = acc[v];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s)
#pragma unroll
      for (int v = 0; v < NVAR; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int v = 0; v < NVAR; ++v) partial[v * TOT_BLOCKS + blockIdx.x] += red[v][0];
}

__global__ void totals_final_kernel(const double* __restrict__ partial, int nparts, double* out) {
  __shared__ double red[256];
  for (int v = 0; v < NVAR; ++v) {
    double a = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) a += partial[v * nparts + i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = red[0];
    __syncthreads();
  }
}

int launch_totals(const double* U, int64_t plane, int64_t n_oct, const uint8_t* refined, double vol, double* partial,
                  int nblocks, void* stream) {
  if (n_oct == 0) return 0;
  hipLaunchKernelGGL(totals_kernel, dim3(nblocks), dim3(256), 0, (hipStream_t)stream, U, plane, n_oct, refined, vol,
                     partial);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int launch_totals_final(const double* partial, int nparts, double* out, void* stream) {
  hipLaunchKernelGGL(totals_final_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, partial, nparts, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// Plain streaming copy (bandwidth reference for counter calibration).
// ---------------------------------------------------------------------------
__global__ void copy_kernel(const double2* __restrict__ src, double2* __restrict__ dst, int64_t n2) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n2; i += int64_t(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}
int launch_copy(const double* src, double* dst, int64_t n, void* stream) {
  const int64_t n2 = n / 2;
  hipLaunchKernelGGL(copy_kernel, dim3(8192), dim3(256), 0, (hipStream_t)stream, (const double2*)src, (double2*)dst,
                     n2);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ry
