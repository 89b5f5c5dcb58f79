// Per-tile hydro update of the octree MUSCL-Hancock / MinMod / HLLC step
// (gfx950 device code; included by kernels.hip and hydro.hip).
//
// Work unit: a tile = an aligned 2x2x2 block of octs (4x4x4 cells, the octs
// sharing their Hilbert key except for the lowest 3 bits), handled by 1, 2
// or 4 wavefronts of one workgroup; the tile's primitive-variable stencil
// (304 positions of the 8x8x8 box around the 4x4x4 core) is staged in LDS
// once and shared by the tile's 64 cells.  Phases per tile:
//   A  gather U of the 304 stencil positions through the tile's 4x4x4 table
//      of neighbouring octs (real or ghost), convert to primitives -> LDS
//   B1 MinMod slopes and the half-step predictor for the 160 cells that
//      border a flux face (the 64 core cells + one layer per face), kept in
//      registers by the thread that owns the cell
//   B2 the left states W~ + D/2 of the 240 faces replace the stencil in LDS
//   C  HLLC on each face by the thread owning its upper cell (the right
//      state W~ - D/2 never leaves registers); fluxes -> LDS
//   D  per core cell: coarse-fine register override, conservative FP64
//      update, fused CFL reduction on the new state; fine-side registers.
// The scheme's definitions: ideal-gas primitives with floors; undivided
// MinMod slopes; unsplit primitive predictor with h = lambda/2 (van Leer
// 1979; Toro 2009 ch. 13-14); face states W~ +- D/2; HLLC with Davis wave
// speeds (Toro, Spruce & Speares 1994); Berger & Colella (1989) refluxing.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ry_internal.h"

namespace ry {

// Multiply-adds written in one expression are fused (FMA) in the per-tile
// update: the same source expression compiles to the same fused operations
// wherever it is inlined, so a face flux computed by two tiles stays
// identical.  The code after this header (in the files that include it) is
// compiled without contraction again.
#pragma clang fp contract(on)

// ---------------------------------------------------------------------------
// Tile geometry.  Stencil positions s in [-2,5]^3 relative to the tile's
// first cell.  The primitives that are needed sit in LDS as the 6^3 box
// [-1,4]^3 (strides 1, WB, WBB) followed by the six 4x4 far planes at -2
// and 5 (x-, x+, y-, y+, z-, z+); only the one-layer cells next to a far
// plane read it.
// ---------------------------------------------------------------------------
constexpr int WB = 6, WBB = 36, NBOX = 216;
constexpr int WSIZE = NBOX + 6 * 16;   // primitives per variable
constexpr int NPOS_A = 304;   // positions whose primitives are needed
constexpr int NPOS_B = 160;   // positions that get a predicted state (core + one layer per face)
constexpr int NCORE = 64;     // B positions 0..63: the core cells, x fastest
constexpr int NUPPER = 48;    // B positions 64..111: the upper one-layer cells
constexpr int NFACE = 240;    // 3 directions x 5 planes x 16
__host__ __device__ constexpr int widx(int x, int y, int z) {
  return (x >= -1 && x <= 4 && y >= -1 && y <= 4 && z >= -1 && z <= 4)
             ? (x + 1) + WB * (y + 1) + WBB * (z + 1)
             : (x == -2  ? NBOX + y + 4 * z
                : x == 5  ? NBOX + 16 + y + 4 * z
                : y == -2 ? NBOX + 32 + x + 4 * z
                : y == 5  ? NBOX + 48 + x + 4 * z
                : z == -2 ? NBOX + 64 + x + 4 * y
                          : NBOX + 80 + x + 4 * y);
}
// Face index of the face along d whose upper cell is (x, y, z) (the plane
// coordinate runs 0..4, the transverse ones 0..3); x runs fastest in every
// direction so that neighbouring lanes touch neighbouring LDS words.
__host__ __device__ constexpr int fidx(int d, int x, int y, int z) {
  return d == 0 ? x + 5 * y + 20 * z : (d == 1 ? 80 + x + 4 * y + 20 * z : 160 + x + 4 * y + 16 * z);
}

// Per-item constants, computed at compile time:
//  a[i]: bits 0-9 LDS index, 10-15 oct-table slot, 16-18 in-oct cell,
//        19-27 raw (x+2)+8(y+2)+64(z+2) of stencil position i
//  b[i], i >= NCORE (one-layer cells: 48 upper ones at coordinate 4 along
//        their normal, then 48 lower ones at -1): bits 0-8 LDS index of the
//        cell, 9-17 LDS index of its outward neighbour (a far plane), 18-19
//        normal axis, 20 upper layer, 21-28 the face (fidx) between the cell
//        and the core.  b[i < NCORE] = LDS index of core cell i.
struct StencilTables {
  uint32_t a[NPOS_A];
  uint32_t b[NPOS_B];
};

constexpr StencilTables make_tables() {
  StencilTables t{};
  int na = 0;
  for (int z = -2; z <= 5; ++z)
    for (int y = -2; y <= 5; ++y)
      for (int x = -2; x <= 5; ++x) {
        const int ox = (x < 0 || x > 3), oy = (y < 0 || y > 3), oz = (z < 0 || z > 3);
        const int nout = ox + oy + oz;
        const bool ex = (x == -1 || x == 4), ey = (y == -1 || y == 4), ez = (z == -1 || z == 4);
        const bool edges = (ox ? ex : true) && (oy ? ey : true) && (oz ? ez : true);
        if ((nout <= 1) || (nout == 2 && edges)) {
          const int slot = ((x >> 1) + 1) + 4 * ((y >> 1) + 1) + 16 * ((z >> 1) + 1);
          const int cb = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2);
          const int raw = (x + 2) + 8 * (y + 2) + 64 * (z + 2);
          t.a[na++] = uint32_t(widx(x, y, z) | (slot << 10) | (cb << 16) | (raw << 19));
        }
      }
  for (int i = 0; i < NCORE; ++i) t.b[i] = uint32_t(widx(i & 3, (i >> 2) & 3, i >> 4));
  int nb = NCORE;
  for (int up = 1; up >= 0; --up)
    for (int d = 0; d < 3; ++d)
      for (int t2 = 0; t2 < 4; ++t2)
        for (int t1 = 0; t1 < 4; ++t1) {
          int c[3] = {0, 0, 0};
          c[d] = up ? 4 : -1;
          c[d == 0 ? 1 : 0] = t1;
          c[d == 2 ? 1 : 2] = t2;
          int o[3] = {c[0], c[1], c[2]};
          o[d] += up ? 1 : -1;
          int u[3] = {c[0], c[1], c[2]};
          if (!up) u[d] += 1;
          const int face = fidx(d, u[0], u[1], u[2]);
          t.b[nb++] = uint32_t(widx(c[0], c[1], c[2]) | (widx(o[0], o[1], o[2]) << 9) | (d << 18) | (up << 20) |
                               (face << 21));
        }
  return t;
}
static __constant__ StencilTables c_st = make_tables();
static_assert(make_tables().a[NPOS_A - 1] != 0 && make_tables().b[NPOS_B - 1] != 0, "stencil tables");
static_assert(WSIZE < 512 && NFACE < 256, "LDS indices must fit the table fields");

// One LDS buffer serves three phases in turn: primitives [NVAR][WSIZE] (A,
// B1), then the left face states [NVAR][NFACE] and the upper one-layer
// cells' right states [NVAR][NUPPER] (B2 -> C), then the face fluxes
// [NVAR][NFACE] (C -> D).  Fluxes are stored in Real: in the mixed
// form they are FP32 results, so FP32 storage loses nothing.
template <typename Real, int NV>
struct TileLDS {
  static constexpr int NW = NV * WSIZE, NF = NV * (NFACE + NUPPER);
  Real buf[NW > NF ? NW : NF];
  int32_t tab[TILE_TAB];  // ext oct index of the 4x4x4 oct neighbourhood
  uint8_t ref[TILE_TAB];  // refined-cell bytes of those octs
};

// ---------------------------------------------------------------------------
// Scalar helpers.
// ---------------------------------------------------------------------------
// MinMod: min(a,b) if both > 0, max(a,b) if both < 0, else 0 -- which is
// the median of (a, b, 0): max(min(a,b), min(max(a,b), 0)) in FP64 (four
// min/max), one v_med3 in FP32.
__device__ __forceinline__ double mmod(double a, double b) { return fmax(fmin(a, b), fmin(fmax(a, b), 0.0)); }
__device__ __forceinline__ float mmod(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }

// Reciprocal and quotient (operands here are normal numbers).  The hardware
// FP64 reciprocal is good to about 5e-8 relative; with e = 1 - b r one
// third-order step r (1 + e + e^2) leaves an error of order e^3, below an
// ulp (two Newton steps would cost one more operation).
__device__ __forceinline__ double rcp(double b) {
  const double r = __builtin_amdgcn_rcp(b);
  const double e = fma(-b, r, 1.0);
  return fma(r, fma(e, e, e), r);
}
__device__ __forceinline__ float rcp(float b) { return __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double qdiv(double a, double b) {
  const double r = rcp(b);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
// Sound speed sqrt(gp / rho) for gp = gamma p, written as gp / sqrt(gp rho):
// one hardware reciprocal square root (about 5e-8 relative) and one
// third-order step y (1 + e/2 + 3e^2/8), e = 1 - a y^2, in FP64.
__device__ __forceinline__ double sound_speed(double gp, double rho) {
  const double a = gp * rho;
  const double y = __builtin_amdgcn_rsq(a);
  const double e = fma(-(a * y), y, 1.0);
  return gp * fma(y, e * fma(0.375, e, 0.5), y);
}
__device__ __forceinline__ float sound_speed(float gp, float rho) { return gp * __builtin_amdgcn_rsqf(gp * rho); }

// Primitive variables (FP64 in both forms) with floors; nfl counts floor
// activations.  Passive scalars: s = (rho s) / rho.
template <int NS>
__device__ __forceinline__ void cons2prim(const double U[NVAR + NS], double W[NVAR + NS], double g, double rf,
                                          double pf, int& nfl) {
  // floors as max(): a non-finite state never gets here unnoticed (the CFL
  // pass flags it on upload, the update flags it where it is produced)
  const bool lo_r = U[0] < rf;
  const double rho = fmax(U[0], rf);
  const double ir = rcp(rho);
  const double ke = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) * ir;
  const double p0 = (g - 1.0) * (U[4] - ke);
  const bool lo_p = p0 < pf;
  nfl += int(lo_r) + int(lo_p);
  W[0] = rho;
  W[1] = U[1] * ir;
  W[2] = U[2] * ir;
  W[3] = U[3] * ir;
  W[4] = fmax(p0, pf);
#pragma unroll
  for (int k = 0; k < NS; ++k) W[NVAR + k] = U[NVAR + k] * ir;
}

// CFL signal speed |u|+|v|+|w|+3c of a conserved state (floors as for the
// primitives), with one refined reciprocal and one refined reciprocal
// square root: within a few ulp of the definition.
__device__ __forceinline__ double signal_speed(const double U[NVAR], double g, double rf, double pf) {
  const double rho = fmax(U[0], rf);
  const double ir = rcp(rho);
  const double ke = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) * ir;
  double p = (g - 1.0) * (U[4] - ke);
  p = fmax(p, pf);
  return (fabs(U[1]) + fabs(U[2]) + fabs(U[3])) * ir + 3.0 * sound_speed(g * p, rho);
}

// What a passive scalar's HLLC flux needs from the hydro solve: the side K
// and the mass flux.  A scalar is carried like a transverse velocity (Toro
// 2009, Sec. 10.6), so its flux is s_K times the mass flux.
template <typename Real>
struct HllcSide {
  bool useL;
  Real F0;
  __device__ __forceinline__ Real scalar_flux(Real sl, Real sr) const { return (useL ? sl : sr) * F0; }
};

// HLLC flux in the face-normal frame: (r, u, a, b, p) = density, normal and
// two tangential velocities, pressure of the left / right face state.  The
// branch picks a side K (L when S_L >= 0 or S* >= 0, else R) and whether the
// star state of K applies; only that side's star state is formed.  With
// x = (S* - u_K) / (S_K - S*) (so that rho*_K = rho_K (1 + x), and x is
// exactly 0 when S* = u_K: stationary contacts stay exact), the star flux
// F_K + S_K (U*_K - U_K) reads
//   mass      m_K + S_K rho_K x
//   normal    m_K u_K + p_K + S_K rho_K (S* - u_K + x S*)
//   tangent   a_K (mass flux), b_K (mass flux)
//   energy    (E_K + p_K) u_K + S_K (E' + x (E_K + E')),
//             E' = rho_K (S* - u_K) (S* + p_K / (rho_K (S_K - u_K))).
template <typename Real>
__device__ __forceinline__ void hllc_n(Real rl, Real ul, Real al, Real bl, Real pl, Real rr, Real ur, Real ar,
                                       Real br, Real pr, Real g, Real igm1, Real Fn[5], HllcSide<Real>& side) {
  const Real cl = sound_speed(g * pl, rl);
  const Real cr = sound_speed(g * pr, rr);
  const Real SL = fmin(ul - cl, ur - cr);
  const Real SR = fmax(ul + cl, ur + cr);
  const Real num = pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur);
  const Real den = rl * (SL - ul) - rr * (SR - ur);
  const Real Ss = qdiv(num, den);
  const bool useL = (SL >= Real(0)) || (Ss >= Real(0));
  const Real rK = useL ? rl : rr, uK = useL ? ul : ur, aK = useL ? al : ar, bK = useL ? bl : br;
  const Real pK = useL ? pl : pr, SK = useL ? SL : SR;
  const bool star = useL ? !(SL >= Real(0)) : (SR > Real(0));
  const Real EK = pK * igm1 + Real(0.5) * rK * (uK * uK + aK * aK + bK * bK);
  const Real mK = rK * uK;
  const Real dSu = Ss - uK;
  // rho_K (S_K - u_K) and S_K - S* (never 0 on a star face) share one
  // reciprocal; off star faces the weights below are 0 and the reciprocal
  // is of 1, so nothing non-finite enters
  const Real rq = rK * (SK - uK);
  const Real dq = SK - Ss;
  const Real inv = rcp(star ? dq * rq : Real(1));
  const Real x = dSu * (rq * inv);
  const Real Ep = rK * dSu * (Ss + pK * (dq * inv));
  const Real w = star ? SK : Real(0);
  const Real wr = w * rK;
  Fn[0] = mK + wr * x;
  Fn[1] = (mK * uK + pK) + wr * (dSu + x * Ss);
  Fn[2] = aK * Fn[0];
  Fn[3] = bK * Fn[0];
  Fn[4] = (EK + pK) * uK + w * (Ep + x * (EK + Ep));
  side.useL = useL;
  side.F0 = Fn[0];
}

// Unsplit half-step predictor of the primitives W0 with undivided slopes
// D[axis][var] and h = lambda / 2.
template <typename Real, int NS>
__device__ __forceinline__ void predict(const Real W0[NVAR + NS], const Real D[3][NVAR + NS], Real h, Real g,
                                        Real P[NVAR + NS]) {
  const Real r = W0[0], u = W0[1], vv = W0[2], w = W0[3], p = W0[4];
  const Real ir = rcp(r);
  P[0] = r - h * (u * D[0][0] + r * D[0][1] + vv * D[1][0] + r * D[1][2] + w * D[2][0] + r * D[2][3]);
  P[1] = u - h * (u * D[0][1] + vv * D[1][1] + w * D[2][1] + D[0][4] * ir);
  P[2] = vv - h * (u * D[0][2] + vv * D[1][2] + w * D[2][2] + D[1][4] * ir);
  P[3] = w - h * (u * D[0][3] + vv * D[1][3] + w * D[2][3] + D[2][4] * ir);
  P[4] = p - h * (u * D[0][4] + vv * D[1][4] + w * D[2][4] + g * p * (D[0][1] + D[1][2] + D[2][3]));
  // a passive scalar is advected: s~ = s - h (u Dx s + v Dy s + w Dz s)
#pragma unroll
  for (int k = NVAR; k < NVAR + NS; ++k) P[k] = W0[k] - h * (u * D[0][k] + vv * D[1][k] + w * D[2][k]);
}

// Floors of a face state; nfl counts activations.
template <typename Real>
__device__ __forceinline__ void floor_state(Real* s, Real rf, Real pf, int& nfl) {
  nfl += int(s[0] < rf) + int(s[4] < pf);
  s[0] = fmax(s[0], rf);
  s[4] = fmax(s[4], pf);
}

// Flux through the lower face along axis D of a core cell: the left state
// comes from LDS (FL[var * NFACE + f]), the right one, W~ - D/2, from the
// cell's predicted state Pw and slope Pdd along D.  The HLLC runs in the
// face-normal frame; F is returned in the global frame.
template <typename Real, int D, int NS>
__device__ __forceinline__ void core_face_flux(const Real* FL, int f, const Real Pw[NVAR + NS],
                                               const Real Pdd[NVAR + NS], Real rf, Real pf, Real g, Real igm1,
                                               int& nfl, Real F[NVAR + NS]) {
  constexpr int iu = 1 + D, i1 = (D == 0) ? 2 : 1, i2 = (D == 2) ? 2 : 3;
  Real wr[NVAR + NS];
#pragma unroll
  for (int v = 0; v < NVAR + NS; ++v) wr[v] = Pw[v] - Real(0.5) * Pdd[v];
  floor_state<Real>(wr, rf, pf, nfl);
  Real Fn[5];
  HllcSide<Real> side;
  hllc_n<Real>(FL[f], FL[iu * NFACE + f], FL[i1 * NFACE + f], FL[i2 * NFACE + f], FL[4 * NFACE + f], wr[0], wr[iu],
               wr[i1], wr[i2], wr[4], g, igm1, Fn, side);
  F[0] = Fn[0];
  F[iu] = Fn[1];
  F[i1] = Fn[2];
  F[i2] = Fn[3];
  F[4] = Fn[4];
#pragma unroll
  for (int k = NVAR; k < NVAR + NS; ++k) F[k] = side.scalar_flux(FL[k * NFACE + f], wr[k]);
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
// The per-tile hydro update.  NT = threads cooperating on one tile (64, 128
// or 256: 8, 16 or 32 threads per oct).  `active` is uniform over the NT
// threads; an inactive group only keeps the workgroup's barrier count.
// ---------------------------------------------------------------------------
// Hides a value from the optimiser so that per-thread table loads are issued
// per tile instead of being hoisted (and held in registers) across the tile
// loop of the persistent kernel.
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <typename Real, int NT, int NS>
__device__ void hydro_tile(const HydroArgs& A, int tile, TileLDS<Real, NVAR + NS>& S, int tid_in,
                           bool active) {
  constexpr int NV = NVAR + NS;
  const int tid = opaque(tid_in);
  const int lane = tid & 63;
  const double g = A.gamma, rf = A.rho_floor, pf = A.p_floor;
  const int64_t P = A.plane;
  int nfl = 0;
  const uint32_t fl = active ? A.tflag[tile] : 0u;
  const int box = (active && A.tile_box) ? A.tile_box[tile] : 0;
  const double lam = A.lam_dev ? A.lam_dev[box] : A.lam_host;
  const Real h = Real(0.5 * lam);
  const Real igm1 = Real(A.igm1);

  // The thread's stencil-table entries for phases A and B, loaded together up
  // front: a load issued inside a round would make that round wait for every
  // state load issued before it.
  constexpr int NRA = (NPOS_A + NT - 1) / NT;
  constexpr int NRB = (NPOS_B + NT - 1) / NT;
  uint32_t entA[NRA], entB[NRB];
#pragma unroll
  for (int rnd = 0; rnd < NRA; ++rnd) {
    const int i = tid + NT * rnd;
    entA[rnd] = c_st.a[uint32_t(i < NPOS_A ? i : 0)];
  }
#pragma unroll
  for (int rnd = 0; rnd < NRB; ++rnd) {
    const int i = tid + NT * rnd;
    entB[rnd] = c_st.b[uint32_t(i < NPOS_B ? i : 0)];
  }

  // --- phase 0: the tile's oct table (the refined bytes of its octs are
  // loaded in phase A behind the state loads; phase D is their first reader)
  int32_t e_tab = -1;
  if (active && tid < TILE_TAB) {
    e_tab = A.tab[size_t(tile) * TILE_TAB + tid];
    S.tab[tid] = e_tab;
  }
  __syncthreads();
  // Wait for the table entries here on every path: otherwise the gather's
  // conditional state loads leave the compiler's load counting unsure of them,
  // and each round would wait for the state loads of the rounds before it.
#pragma unroll
  for (int rnd = 0; rnd < NRA; ++rnd) asm volatile("" ::"v"(entA[rnd]));
#pragma unroll
  for (int rnd = 0; rnd < NRB; ++rnd) asm volatile("" ::"v"(entB[rnd]));

  // --- phase A: gather + primitives (all loads of the thread's positions are
  // issued before any conversion)
  Real* W = S.buf;                              // [NV][WSIZE]
  // the planes' base addresses, formed in scalar registers (an empty asm on
  // the plane offset keeps the compiler from folding it back into every
  // per-lane address)
  const double* Up[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    int64_t off = v * P;
    asm volatile("" : "+s"(off));
    Up[v] = A.U + off;
  }
  const bool off32 = P <= (int64_t(1) << 29);
  double Ua[NRA][NV];
  int iwa[NRA];
#pragma unroll
  for (int rnd = 0; rnd < NRA; ++rnd) {
    const int i = tid + NT * rnd;
    iwa[rnd] = -1;
    if (active && i < NPOS_A) {
      const uint32_t ent = entA[rnd];
      int slot = int((ent >> 10) & 63u), cb = int((ent >> 16) & 7u);
      if (fl) {
        // outflow faces: clamp the position into the domain (zero gradient)
        const int raw = int(ent >> 19);
        int sx = (raw & 7) - 2, sy = ((raw >> 3) & 7) - 2, sz = (raw >> 6) - 2;
        if ((fl & CL_LOX) && sx < 0) sx = 0;
        if ((fl & CL_HIX) && sx > 3) sx = 3;
        if ((fl & CL_LOY) && sy < 0) sy = 0;
        if ((fl & CL_HIY) && sy > 3) sy = 3;
        if ((fl & CL_LOZ) && sz < 0) sz = 0;
        if ((fl & CL_HIZ) && sz > 3) sz = 3;
        slot = ((sx >> 1) + 1) + 4 * ((sy >> 1) + 1) + 16 * ((sz >> 1) + 1);
        cb = (sx & 1) | ((sy & 1) << 1) | ((sz & 1) << 2);
      }
      const int32_t e = S.tab[slot];
      iwa[rnd] = int(ent & 1023u);
      // 32-bit cell index (octs of a level stay below 2^29).  A slot without
      // an oct is one no leaf update reads: it takes the (valid, finite)
      // state of the level's first cell instead of a branch
      const uint32_t cell = (e >= 0) ? uint32_t(e) * 8u + uint32_t(cb) : 0u;
      if (off32) {
        // planes under 4 GiB: one 32-bit byte offset serves every plane
        // (base in scalar registers + unsigned 32-bit lane offset)
        const uint32_t boff = cell << 3;
#pragma unroll
        for (int v = 0; v < NV; ++v)
          Ua[rnd][v] = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(Up[v]) + boff);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) Ua[rnd][v] = Up[v][cell];
      }
    }
  }
  const uint8_t rb = (e_tab >= 0) ? A.refined[e_tab] : uint8_t(0);
#pragma unroll
  for (int rnd = 0; rnd < NRA; ++rnd) {
    if (iwa[rnd] >= 0) {
      double Wc[NV];
      cons2prim<NS>(Ua[rnd], Wc, g, rf, pf, nfl);
#pragma unroll
      for (int v = 0; v < NV; ++v) W[v * WSIZE + iwa[rnd]] = Real(Wc[v]);
    }
  }
  if (active && tid < TILE_TAB) S.ref[tid] = rb;
  __syncthreads();

  // --- phase B1: slopes + predictor.  The core cell of a thread (first pass,
  // tid < 64) keeps W~ and its slopes in registers for its six faces; a
  // one-layer cell keeps only its state on the face toward the core.
  constexpr int st[3] = {1, WB, WBB};
  const bool core = (NT == 64) || tid < NCORE;
  const int cx = tid & 3, cy = (tid >> 2) & 3, cz = (tid >> 4) & 3;
  const Real rfr = Real(rf), pfr = Real(pf), gr = Real(g);
  Real Pw[NV], Pd[3][NV];
  Real Ls[NRB][NV];
  uint32_t Lb[NRB];
#pragma unroll
  for (int rnd = 0; rnd < NRB; ++rnd) {
    const int i = tid + NT * rnd;
    Lb[rnd] = 0u;
    if (!active || i >= NPOS_B) continue;
    if (rnd == 0 && core) {
      const int iw = (cx + 1) + WB * (cy + 1) + WBB * (cz + 1);
      Real W0[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) W0[v] = W[v * WSIZE + iw];
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int v = 0; v < NV; ++v)
          Pd[d][v] = mmod(W0[v] - W[v * WSIZE + iw - st[d]], W[v * WSIZE + iw + st[d]] - W0[v]);
      predict<Real, NS>(W0, Pd, h, gr, Pw);
    } else {
      const uint32_t e = entB[rnd];
      Lb[rnd] = e;
      const int iw = int(e & 511u), far = int((e >> 9) & 511u), dn = int((e >> 18) & 3u);
      const bool up = (e >> 20) & 1u;
      Real W0[NV], D[3][NV], Q[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) W0[v] = W[v * WSIZE + iw];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int lo = (d == dn && !up) ? far : iw - st[d];
        const int hi = (d == dn && up) ? far : iw + st[d];
#pragma unroll
        for (int v = 0; v < NV; ++v) D[d][v] = mmod(W0[v] - W[v * WSIZE + lo], W[v * WSIZE + hi] - W0[v]);
      }
      predict<Real, NS>(W0, D, h, gr, Q);
      // the face state Q +- D/2 along the normal: the weights of the two other
      // axes are zero, so their fused terms add exact zeros
      const Real sg = up ? Real(-0.5) : Real(0.5);
      const Real t0 = (dn == 0) ? sg : Real(0), t1 = (dn == 1) ? sg : Real(0), t2 = (dn == 2) ? sg : Real(0);
#pragma unroll
      for (int v = 0; v < NV; ++v) Ls[rnd][v] = fma(t2, D[2][v], fma(t1, D[1][v], fma(t0, D[0][v], Q[v])));
      floor_state<Real>(Ls[rnd], rfr, pfr, nfl);
    }
  }
  __syncthreads();

  // --- phase B2: the left states (W~ + D/2 of the lower cell) of the 240
  // faces replace the primitives in LDS
  Real* FL = S.buf;                             // [NV][NFACE]
  Real* FR = S.buf + NV * NFACE;              // [NV][NUPPER]: right states of the upper layer
#pragma unroll
  for (int rnd = 0; rnd < NRB; ++rnd) {
    const int i = tid + NT * rnd;
    if (!active || i >= NPOS_B) continue;
    if (rnd == 0 && core) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        Real s[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) s[v] = Pw[v] + Real(0.5) * Pd[d][v];
        floor_state<Real>(s, rfr, pfr, nfl);
        const int f = fidx(d, cx + (d == 0), cy + (d == 1), cz + (d == 2));
#pragma unroll
        for (int v = 0; v < NV; ++v) FL[v * NFACE + f] = s[v];
      }
    } else if (!((Lb[rnd] >> 20) & 1u)) {
      const int f = int(Lb[rnd] >> 21);
#pragma unroll
      for (int v = 0; v < NV; ++v) FL[v * NFACE + f] = Ls[rnd][v];
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) FR[v * NUPPER + (i - NCORE)] = Ls[rnd][v];
    }
  }
  __syncthreads();

  // --- phase C: HLLC on the faces whose upper cell the thread holds (a core
  // cell: its three lower faces; an upper one-layer cell: its face, read in
  // the face-normal frame straight from LDS)
  Real Fc[3][NV];
  Real Fl[NRB][NV];
#pragma unroll
  for (int rnd = 0; rnd < NRB; ++rnd) {
    const int i = tid + NT * rnd;
    if (!active || i >= NPOS_B) continue;
    if (rnd == 0 && core) {
      core_face_flux<Real, 0, NS>(FL, fidx(0, cx, cy, cz), Pw, Pd[0], rfr, pfr, gr, igm1, nfl, Fc[0]);
      core_face_flux<Real, 1, NS>(FL, fidx(1, cx, cy, cz), Pw, Pd[1], rfr, pfr, gr, igm1, nfl, Fc[1]);
      core_face_flux<Real, 2, NS>(FL, fidx(2, cx, cy, cz), Pw, Pd[2], rfr, pfr, gr, igm1, nfl, Fc[2]);
    } else if ((Lb[rnd] >> 20) & 1u) {
      const int f = int(Lb[rnd] >> 21), dn = int((Lb[rnd] >> 18) & 3u), k = i - NCORE;
      const int iu = 1 + dn, i1 = (dn == 0) ? 2 : 1, i2 = (dn == 2) ? 2 : 3;
      HllcSide<Real> side;
      hllc_n<Real>(FL[f], FL[iu * NFACE + f], FL[i1 * NFACE + f], FL[i2 * NFACE + f], FL[4 * NFACE + f], FR[k],
                   FR[iu * NUPPER + k], FR[i1 * NUPPER + k], FR[i2 * NUPPER + k], FR[4 * NUPPER + k], gr, igm1,
                   Fl[rnd], side);
#pragma unroll
      for (int v = NVAR; v < NV; ++v) Fl[rnd][v] = side.scalar_flux(FL[v * NFACE + f], FR[v * NUPPER + k]);
    }
  }
  __syncthreads();
  Real* SF = S.buf;                             // [NV][NFACE]
#pragma unroll
  for (int rnd = 0; rnd < NRB; ++rnd) {
    const int i = tid + NT * rnd;
    if (!active || i >= NPOS_B) continue;
    if (rnd == 0 && core) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int f = fidx(d, cx, cy, cz);
#pragma unroll
        for (int v = 0; v < NV; ++v) SF[v * NFACE + f] = Fc[d][v];
      }
    } else if ((Lb[rnd] >> 20) & 1u) {
      // Fl is in the face-normal frame: rotate back on the way out
      const int f = int(Lb[rnd] >> 21), dn = int((Lb[rnd] >> 18) & 3u);
      const int iu = 1 + dn, i1 = (dn == 0) ? 2 : 1, i2 = (dn == 2) ? 2 : 3;
      SF[f] = Fl[rnd][0];
      SF[iu * NFACE + f] = Fl[rnd][1];
      SF[i1 * NFACE + f] = Fl[rnd][2];
      SF[i2 * NFACE + f] = Fl[rnd][3];
      SF[4 * NFACE + f] = Fl[rnd][4];
#pragma unroll
      for (int v = NVAR; v < NV; ++v) SF[v * NFACE + f] = Fl[rnd][v];
    }
  }
  __syncthreads();

  // --- phase D: the first wavefront updates the tile's 64 cells
  if (tid < 64) {
    const int ts = ((cx >> 1) + 1) + 4 * ((cy >> 1) + 1) + 16 * ((cz >> 1) + 1);
    const int32_t e = active ? S.tab[ts] : -1;
    const int ci = (cx & 1) | ((cy & 1) << 1) | ((cz & 1) << 2);
    const bool leaf = (e >= 0) && (e < A.n_oct) && !((S.ref[ts] >> ci) & 1);
    double s = 0.0;
    if (leaf) {
      // the cell's old state is loaded first: the stores to the new state
      // below may alias it as far as the compiler knows, and a load issued
      // after a store would wait for it
      const uint32_t cell = uint32_t(e) * 8u + uint32_t(ci);
      double Uo[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Uo[v] = (A.U + v * P)[cell];
      double acc[NV];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        // the lower face's flux is the thread's own (phase C), the upper
        // one comes from the neighbouring cell's thread through LDS
        const int fp = fidx(d, cx + (d == 0), cy + (d == 1), cz + (d == 2));
        double Fm[NV], Fp[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          Fm[v] = double(Fc[d][v]);
          Fp[v] = double(SF[v * NFACE + fp]);
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
              const double* q = A.reg_fine + (int64_t(ch) * 6 + face) * NV * 2;
#pragma unroll
              for (int v = 0; v < NV; ++v) {
                const double fb = 0.125 * (q[2 * v] + q[2 * v + 1]);
                if (side) Fp[v] = fb; else Fm[v] = fb;
              }
            }
          }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = (d == 0) ? (Fm[v] - Fp[v]) : acc[v] + (Fm[v] - Fp[v]);
      }
      double Un[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Un[v] = Uo[v] + lam * acc[v];
        (A.Un + v * P)[cell] = Un[v];
      }
      if (A.tile_smax || A.smax_bits || A.err) {
        s = signal_speed(Un, g, rf, pf);
        const bool bad = !(isfinite(Un[0]) && isfinite(Un[1]) && isfinite(Un[2]) && isfinite(Un[3]) &&
                           isfinite(Un[4])) || !(Un[0] > 0.0) || !(Un[4] > 0.0) || !isfinite(s);
        if (bad) {
          atomicOr(A.err, 1);
          s = 0.0;
        }
      }
    }
    if (active && A.smax_bits) {
      // one atomic maximum per tile on one of the level's slots (a
      // non-negative double orders like its bit pattern); the maximum does
      // not depend on the order of arrival
      const double m = wave_max(s);
      if (lane == 0) atomicMax(A.smax_bits + (tile & (SMAX_SLOTS - 1)), (unsigned long long)__double_as_longlong(m));
    } else if (active && A.tile_smax) {
      // batched boxes: one partial per tile, reduced per box by the
      // segmented max kernel before the next time step
      const double m = wave_max(s);
      if (lane == 0) A.tile_smax[tile] = m;
    }
  }

  // --- fine-side registers: q_s = (f1 + f2) + (f3 + f4) on coarse-fine faces
  const int rt = (NT > 64) ? tid - 64 : tid;   // a second wavefront, when there is one
  if (active && A.record_reg && rt >= 0 && rt < 48) {
    const int b = rt / 6, face = rt - 6 * (rt / 6);
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
          fi[j] = fidx(d, ccx + (d == 0 ? up : 0), ccy + (d == 1 ? up : 0), ccz + (d == 2 ? up : 0));
        }
        double* q = A.reg_own + (int64_t(eb) * 6 + face) * NV * 2;
#pragma unroll
        for (int v = 0; v < NV; ++v)
          q[2 * v + A.substep] = (double(SF[v * NFACE + fi[0]]) + double(SF[v * NFACE + fi[1]])) +
                                 (double(SF[v * NFACE + fi[2]]) + double(SF[v * NFACE + fi[3]]));
      }
    }
  }
  // floor activations are rare: the shuffle sum runs only in a wavefront
  // that has any
  if (active && A.floors && __any(nfl != 0)) {
    const int tot = wave_sum(nfl);
    if (lane == 0 && tot) atomicAdd(A.floors, (unsigned long long)tot);
  }
  __syncthreads();
}

// Hydro variables alone: at least 3 wavefronts per SIMD (the FP64 tile's LDS
// allows no more, so the register budget of an instruction-level-parallel
// schedule stops there).  With passive scalars the LDS tile sets the limit.
template <typename Real, int TPW, int WPT, int NS>
__global__ __launch_bounds__(64 * WPT * TPW) __attribute__((amdgpu_waves_per_eu(NS == 0 ? 3 : 1))) void hydro_kernel(
    HydroArgs A) {
  constexpr int NT = 64 * WPT;
  __shared__ TileLDS<Real, NVAR + NS> S[TPW];
  if (A.skip && *A.skip) return;
  const int w = threadIdx.x / NT, tid = threadIdx.x % NT;
  const int ngroups = (A.n_tile + TPW - 1) / TPW;
  const int grp = xcd_remap(blockIdx.x, gridDim.x);
  if (grp >= ngroups) return;
  const int tile = grp * TPW + w;
  hydro_tile<Real, NT, NS>(A, tile < A.n_tile ? tile : 0, S[w], tid, tile < A.n_tile);
}

// Persistent variant: workgroups pop groups of tiles from 8 per-XCD queues
// (one contiguous slice of the Hilbert-ordered tile list per XCD; a
// workgroup whose own queue is empty takes from the next one).  Every
// workgroup exits once all 8 queues are exhausted.
template <typename Real, int TPW, int WPT>
__global__ __launch_bounds__(64 * WPT * TPW) __attribute__((amdgpu_waves_per_eu(3))) void hydro_kernel_persistent(HydroArgs A,
                                                                                                      int batch) {
  constexpr int NT = 64 * WPT;
  __shared__ TileLDS<Real, NVAR> S[TPW];
  __shared__ int s_item;
  if (A.skip && *A.skip) return;
  const int w = threadIdx.x / NT, tid = threadIdx.x % NT;
  const int ngroups = (A.n_tile + TPW - 1) / TPW;
  const int nitems = (ngroups + batch - 1) / batch;
  const int q = nitems >> 3, r = nitems & 7;
  int cur = blockIdx.x & 7;
  int exhausted = 0;
  auto qlen = [&](int c) { return q + (c < r ? 1 : 0); };
  auto item_of = [&](int c, unsigned int k) { return c * q + (c < r ? c : r) + int(k); };
  // a blocking pop (thread 0): the next item of this XCD's queue, then of
  // the others once it is exhausted; -1 when every queue is
  auto pop = [&]() {
    while (exhausted < 8) {
      const unsigned int k = atomicAdd(&A.queue[cur * QUEUE_STRIDE], 1u);
      if (int(k) < qlen(cur)) return item_of(cur, k);
      cur = (cur + 1) & 7;
      ++exhausted;
    }
    return -1;
  };
  if (threadIdx.x == 0) s_item = pop();
  __syncthreads();
  // the item is uniform: tile indices, table rows and tile flags stay in
  // scalar registers
  int item = __builtin_amdgcn_readfirstlane(s_item);
  __syncthreads();
  while (item >= 0) {
    // claim the next slot of the current queue before this item's tiles and
    // look at the answer after them: the atomic's round trip overlaps the
    // tiles' own loads
    unsigned int k = 0;
    const int kc = cur;
    if (threadIdx.x == 0 && exhausted < 8) k = atomicAdd(&A.queue[kc * QUEUE_STRIDE], 1u);
    for (int j = 0; j < batch; ++j) {
      const int grp = item * batch + j;
      if (grp >= ngroups) break;
      const int tile = grp * TPW + w;
      hydro_tile<Real, NT, 0>(A, tile < A.n_tile ? tile : 0, S[w], tid, tile < A.n_tile);
    }
    if (threadIdx.x == 0) {
      int next = -1;
      if (exhausted < 8) {
        if (int(k) < qlen(kc)) {
          next = item_of(kc, k);
        } else {
          cur = (cur + 1) & 7;
          ++exhausted;
          next = pop();
        }
      }
      s_item = next;
    }
    __syncthreads();
    item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
  }
}

// The persistent kernel exists for the hydro variables alone (NS = 0).
template <typename Real, int TPW, int WPT, int NS>
static int launch_hydro_t(const HydroArgs& a, const ry_tuning& t, int num_cu, hipStream_t s) {
  const int ngroups = (a.n_tile + TPW - 1) / TPW;
  if (ngroups == 0) return 0;
  if (NS > 0 || !t.persistent) {
    hipLaunchKernelGGL((hydro_kernel<Real, TPW, WPT, NS>), dim3(ngroups), dim3(64 * WPT * TPW), 0, s, a);
  } else if constexpr (NS == 0) {
    const int batch = t.batch > 0 ? t.batch : 1;
    const int nitems = (ngroups + batch - 1) / batch;
    int grid = num_cu * (t.waves_per_cu > 0 ? t.waves_per_cu : 4) / (TPW * WPT);
    if (grid < 8) grid = 8;
    if (grid > nitems) grid = ((nitems + 7) / 8) * 8;
    hipLaunchKernelGGL((hydro_kernel_persistent<Real, TPW, WPT>), dim3(grid), dim3(64 * WPT * TPW), 0, s, a,
                       batch);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

#pragma clang fp contract(off)

}  // namespace ry
