// Per-tile hydro update of the octree MUSCL-Hancock / MinMod / HLLC step
// (gfx950 device code; included by kernels.hip and hydro.hip).
//
// Work unit: a tile = an aligned block of K x K x K cells, K = 4 (2x2x2
// octs, the octs sharing their Hilbert key except for the lowest 3 bits) or
// K = 8 (4x4x4 octs, a "super-tile" assembled from up to 8 small tiles),
// handled by the threads of one workgroup; the tile's primitive-variable
// stencil (the positions of the (K+4)^3 box around the K^3 core that the
// scheme reads) is staged in LDS once and shared by the tile's cells, so the
// larger tile converts, predicts and solves fewer halo positions per cell
// (per cell: 4.75 / 2.5 / 3.75 primitives / predictions / faces at K = 4,
// 2.69 / 1.75 / 3.375 at K = 8).  Phases per tile:
//   A  gather U of the stencil positions through the tile's table of
//      neighbouring octs (real or ghost), convert to primitives -> LDS
//   B1 MinMod slopes and the half-step predictor for the cells that border
//      a flux face (the core cells + one layer per face), kept in registers
//      by the thread that owns the cell
//   B2 the left states W~ + D/2 of the faces replace the stencil in LDS
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
#include <type_traits>

#include "ry_internal.h"

namespace ry {

// Multiply-adds written in one expression are fused (FMA) in the per-tile
// update: the same source expression compiles to the same fused operations
// wherever it is inlined, so a face flux computed by two tiles stays
// identical.  The code after this header (in the files that include it) is
// compiled without contraction again.
#pragma clang fp contract(on)

// ---------------------------------------------------------------------------
// Tile geometry.  Stencil positions s in [-2,K+1]^3 relative to the tile's
// first cell.  The primitives that are needed sit in LDS as the (K+2)^3 box
// [-1,K]^3 (strides 1, WB, WBB) followed by the six K x K far planes at -2
// and K+1 (x-, x+, y-, y+, z-, z+); only the one-layer cells next to a far
// plane read it.
// ---------------------------------------------------------------------------
template <int K>
struct Geom {
  static_assert(K == 4 || K == 8, "tile edge of 4 or 8 cells");
  static constexpr int LK = (K == 4) ? 2 : 3;            // log2 K
  // box rows and planes, padded past their K + 2 entries to spread the
  // 8^3-cell tile's LDS accesses over the banks: a 64-bit access serves 16
  // lanes per pass, and 16 consecutive threads hold a 4x2x2-cell block
  // (oct-major order); with a row stride of 12 and a plane stride of 120 the
  // 16 cells of such a block, and of each of its shifts by one cell, fall on
  // 16 distinct bank pairs
  static constexpr int PAD_ROW = (K == 8) ? 2 : 0, PAD_PLANE = 0;
  static constexpr int WB = K + 2 + PAD_ROW, WBB = WB * (K + 2) + PAD_PLANE, NBOX = WBB * (K + 2);
  static constexpr int WSIZE = NBOX + 6 * K * K;         // primitives per variable
  static constexpr int NPOS_A = K * K * K + 12 * K * K + 12 * K;   // positions whose primitives are needed
  static constexpr int NPOS_B = K * K * K + 6 * K * K;   // positions that get a predicted state
  static constexpr int NCORE = K * K * K;                // A and B positions 0..NCORE-1: the core cells
  static constexpr int NUPPER = 3 * K * K;               // then the upper one-layer cells, then the lower ones
  // faces: 3 directions x (K+1) planes x K^2 (K = 4); K = 8 pads each
  // direction's array for the same bank spread (layouts in fidx)
  static constexpr int FD0 = (K == 8) ? 66 * (K + 1) : (K + 1) * K * K;
  static constexpr int FD1 = (K == 8) ? 68 * (K + 1) : (K + 1) * K * K;
  static constexpr int NFACE = (K == 8) ? FD0 + 2 * FD1 : 3 * (K + 1) * K * K;
  static constexpr int KO = K / 2;                       // octs per tile edge
  static constexpr int TS = KO + 2;                      // oct neighbourhood edge (one oct of halo)
  static constexpr int TAB = TS * TS * TS;               // oct neighbourhood entries per tile
  static constexpr int R = K + 4;                        // stencil positions per axis
  // table a entry: LDS index | oct slot | in-oct cell | raw position
  static constexpr int A_LB = (K == 4) ? 10 : 11, A_SB = (K == 4) ? 6 : 8;
  static constexpr int A_CS = A_LB + A_SB, A_RS = A_CS + 3;
  // table b entry (one-layer cells): cell LDS index | far-plane neighbour
  // LDS index | normal axis | upper layer | face between the cell and the core
  static constexpr int B_LB = (K == 4) ? 9 : 11;
  static constexpr int B_DS = 2 * B_LB, B_US = B_DS + 2, B_FS = B_US + 1;
  using EntA = std::conditional_t<K == 4, uint32_t, uint64_t>;
  using EntB = std::conditional_t<K == 4, uint32_t, uint64_t>;
  static_assert(WSIZE < (1 << B_LB) && WSIZE < (1 << A_LB) && TAB <= (1 << A_SB), "LDS / slot fields");
  static_assert(int64_t(R) * R * R <= (int64_t(1) << (8 * sizeof(EntA) - A_RS)), "raw position field");
  static_assert(NFACE <= (int64_t(1) << (8 * sizeof(EntB) - B_FS)), "face field");

  __host__ __device__ static constexpr int widx(int x, int y, int z) {
    return (x >= -1 && x <= K && y >= -1 && y <= K && z >= -1 && z <= K)
               ? (x + 1) + WB * (y + 1) + WBB * (z + 1)
               : (x == -2      ? NBOX + y + K * z
                  : x == K + 1 ? NBOX + K * K + y + K * z
                  : y == -2    ? NBOX + 2 * K * K + x + K * z
                  : y == K + 1 ? NBOX + 3 * K * K + x + K * z
                  : z == -2    ? NBOX + 4 * K * K + x + K * y
                               : NBOX + 5 * K * K + x + K * y);
  }
  // Face index of the face along d whose upper cell is (x, y, z) (the plane
  // coordinate runs 0..K, the transverse ones 0..K-1).  K = 4: x runs
  // fastest in every direction.  K = 8: the index of a 4x2x2-cell block's
  // faces (16 consecutive threads) covers 16 distinct residues mod 16 in
  // every direction -- y + 8 z + 66 x along x, x + 8 z + 68 y along y,
  // x + 8 y + 68 z along z -- so a 64-bit access meets no bank conflict.
  __host__ __device__ static constexpr int fidx(int d, int x, int y, int z) {
    if constexpr (K == 8)
      return d == 0 ? y + 8 * z + 66 * x : (d == 1 ? FD0 + x + 8 * z + 68 * y : FD0 + FD1 + x + 8 * y + 68 * z);
    return d == 0 ? x + (K + 1) * y + (K + 1) * K * z
                  : (d == 1 ? (K + 1) * K * K + x + K * y + K * (K + 1) * z
                            : 2 * (K + 1) * K * K + x + K * y + K * K * z);
  }
  // Core cell of thread t < NCORE, oct-major: 8 consecutive threads hold the
  // 8 cells of one oct (in-oct index t & 7) and 64 consecutive threads the
  // octs of one 2x2x2 block of octs, which lie next to each other in memory
  // (Hilbert order), so a wavefront's state loads and stores cover whole
  // octs.
  static constexpr int NBLK = K / 4;                     // 2x2x2-oct blocks per tile edge
  __host__ __device__ static constexpr int core_x(int t) {
    return 4 * ((t >> 6) % NBLK) + 2 * ((t >> 3) & 1) + (t & 1);
  }
  __host__ __device__ static constexpr int core_y(int t) {
    return 4 * (((t >> 6) / NBLK) % NBLK) + 2 * ((t >> 4) & 1) + ((t >> 1) & 1);
  }
  __host__ __device__ static constexpr int core_z(int t) {
    return 4 * ((t >> 6) / (NBLK * NBLK)) + 2 * ((t >> 5) & 1) + ((t >> 2) & 1);
  }
  // Slot of the oct at oct offset (ox, oy, oz) from the tile's first oct
  // (-1 .. KO) in the tile's oct neighbourhood table.
  __host__ __device__ static constexpr int slot(int ox, int oy, int oz) {
    return (ox + 1) + TS * (oy + 1) + TS * TS * (oz + 1);
  }
};

// Per-item constants, computed at compile time:
//  a[i]: LDS index, oct-table slot, in-oct cell and raw (x+2) + R (y+2) +
//        R^2 (z+2) of stencil position i (fields as Geom<K>::A_*)
//  b[i], i >= NCORE (one-layer cells: the upper ones at coordinate K along
//        their normal, then the lower ones at -1): LDS index of the cell, LDS
//        index of its outward neighbour (a far plane), normal axis, upper
//        layer, the face between the cell and the core (fields as
//        Geom<K>::B_*).  b[i < NCORE] = LDS index of core cell i (the
//        threads' oct-major order, Geom<K>::core_x/y/z).
template <int K>
struct StencilTables {
  typename Geom<K>::EntA a[Geom<K>::NPOS_A];
  typename Geom<K>::EntB b[Geom<K>::NPOS_B];
};

template <int K>
constexpr StencilTables<K> make_tables() {
  using G = Geom<K>;
  using EA = typename G::EntA;
  using EB = typename G::EntB;
  StencilTables<K> t{};
  int na = 0;
  auto put = [&](int x, int y, int z) {
    const int slot = G::slot(x >> 1, y >> 1, z >> 1);
    const int cb = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2);
    const int raw = (x + 2) + G::R * (y + 2) + G::R * G::R * (z + 2);
    t.a[na++] = EA(G::widx(x, y, z)) | (EA(slot) << G::A_LB) | (EA(cb) << G::A_CS) | (EA(raw) << G::A_RS);
  };
  // the core cells first, in the threads' oct-major order (a thread's first
  // gathered position is its own cell), then the halo positions oct by oct
  // (consecutive threads read the cells of one oct)
  for (int i = 0; i < G::NCORE; ++i) put(G::core_x(i), G::core_y(i), G::core_z(i));
  for (int sz = -1; sz <= G::KO; ++sz)
    for (int sy = -1; sy <= G::KO; ++sy)
      for (int sx = -1; sx <= G::KO; ++sx)
        for (int cb = 0; cb < 8; ++cb) {
          const int x = 2 * sx + (cb & 1), y = 2 * sy + ((cb >> 1) & 1), z = 2 * sz + (cb >> 2);
          const int ox = (x < 0 || x > K - 1), oy = (y < 0 || y > K - 1), oz = (z < 0 || z > K - 1);
          const int nout = ox + oy + oz;
          const bool ex = (x == -1 || x == K), ey = (y == -1 || y == K), ez = (z == -1 || z == K);
          const bool edges = (ox ? ex : true) && (oy ? ey : true) && (oz ? ez : true);
          if ((nout == 1) || (nout == 2 && edges)) put(x, y, z);
        }
  for (int i = 0; i < G::NCORE; ++i) t.b[i] = EB(G::widx(G::core_x(i), G::core_y(i), G::core_z(i)));
  int nb = G::NCORE;
  for (int up = 1; up >= 0; --up)
    for (int d = 0; d < 3; ++d)
      for (int t2 = 0; t2 < K; ++t2)
        for (int t1 = 0; t1 < K; ++t1) {
          int c[3] = {0, 0, 0};
          c[d] = up ? K : -1;
          c[d == 0 ? 1 : 0] = t1;
          c[d == 2 ? 1 : 2] = t2;
          int o[3] = {c[0], c[1], c[2]};
          o[d] += up ? 1 : -1;
          int u[3] = {c[0], c[1], c[2]};
          if (!up) u[d] += 1;
          const int face = G::fidx(d, u[0], u[1], u[2]);
          t.b[nb++] = EB(G::widx(c[0], c[1], c[2])) | (EB(G::widx(o[0], o[1], o[2])) << G::B_LB) |
                      (EB(d) << G::B_DS) | (EB(up) << G::B_US) | (EB(face) << G::B_FS);
        }
  return t;
}
static __constant__ StencilTables<4> c_st4 = make_tables<4>();
static __constant__ StencilTables<8> c_st8 = make_tables<8>();
// every table entry filled (the position counts match the enumerations)
template <int K>
constexpr bool tables_full() {
  constexpr StencilTables<K> t = make_tables<K>();
  for (int i = 0; i < Geom<K>::NPOS_A; ++i)
    if (t.a[i] == 0) return false;
  for (int i = Geom<K>::NCORE; i < Geom<K>::NPOS_B; ++i)
    if (t.b[i] == 0) return false;
  return true;
}
static_assert(tables_full<4>() && tables_full<8>(), "stencil tables");
template <int K>
__device__ __forceinline__ const StencilTables<K>& stencil_tables() {
  if constexpr (K == 4) return c_st4;
  else return c_st8;
}

// One LDS buffer serves three phases in turn: primitives [NVAR][WSIZE] (A,
// B1), then the left face states [NVAR][NFACE] and the upper one-layer
// cells' right states [NVAR][NUPPER] (B2 -> C), then the face fluxes
// [NVAR][NFACE] (C -> D).  Fluxes are stored in Real: in the mixed
// form they are FP32 results, so FP32 storage loses nothing.
template <typename Real, int NV, int K>
struct TileLDS {
  using G = Geom<K>;
  static constexpr int NW = NV * G::WSIZE, NF = NV * (G::NFACE + G::NUPPER);
  Real buf[NW > NF ? NW : NF];
  // ext oct index of the oct neighbourhood (ghost octs shifted as the
  // current state buffer needs) and the refined-cell bytes of those octs
  int32_t tab[G::TAB];
  uint8_t ref[G::TAB];
  // the threads' signal speeds (tiles of several wavefronts: one wavefront
  // reduces them after the tile's last barrier), in the upper one-layer
  // states' part of buf (unused after phase C) when it holds them
  static constexpr bool SMAX_IN_BUF = (K == 8) && sizeof(Real) * NV * G::NUPPER >= sizeof(double) * G::NCORE;
  double smx[(K == 8 && !SMAX_IN_BUF) ? G::NCORE : 1];
};

// ---------------------------------------------------------------------------
// Scalar helpers.
// ---------------------------------------------------------------------------
// MinMod: min(a,b) if both > 0, max(a,b) if both < 0, else 0 -- which is
// the median of (a, b, 0): max(min(a,b), min(max(a,b), 0)) in FP64 (four
// min/max), one v_med3 in FP32.
__device__ __forceinline__ double mmod(double a, double b) { return fmax(fmin(a, b), fmin(fmax(a, b), 0.0)); }

// max(x, f) for a wavefront-uniform floor f, as the bare hardware
// instruction with f in scalar registers: the library maximum first quiets
// each operand it cannot prove canonical (a value from memory, a kernel
// argument), one more instruction per operand and use.  Identical for every
// operand but a signalling NaN, which no state here holds.
__device__ __forceinline__ double floor_max(double x, double f) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(x), "s"(f));
  return r;
}
__device__ __forceinline__ float floor_max(float x, float f) {
  float r;
  asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(x), "s"(f));
  return r;
}
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
                                          double pf, int& nfl, double* ir_out = nullptr) {
  // floors as max(): a non-finite state never gets here unnoticed (the CFL
  // pass flags it on upload, the update flags it where it is produced)
  const bool lo_r = U[0] < rf;
  const double rho = floor_max(U[0], rf);
  const double ir = rcp(rho);
  if (ir_out) *ir_out = ir;
  const double ke = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) * ir;
  const double p0 = (g - 1.0) * (U[4] - ke);
  const bool lo_p = p0 < pf;
  nfl += int(lo_r) + int(lo_p);
  W[0] = rho;
  W[1] = U[1] * ir;
  W[2] = U[2] * ir;
  W[3] = U[3] * ir;
  W[4] = floor_max(p0, pf);
#pragma unroll
  for (int k = 0; k < NS; ++k) W[NVAR + k] = U[NVAR + k] * ir;
}

// CFL signal speed |u|+|v|+|w|+3c of a conserved state (floors as for the
// primitives), with one refined reciprocal and one refined reciprocal
// square root: within a few ulp of the definition.
__device__ __forceinline__ double signal_speed(const double U[NVAR], double g, double rf, double pf) {
  const double rho = floor_max(U[0], rf);
  const double ir = rcp(rho);
  const double ke = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) * ir;
  double p = (g - 1.0) * (U[4] - ke);
  p = floor_max(p, pf);
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
// D[axis][var] and h = lambda / 2; ir = 1 / W0[0].
template <typename Real, int NS>
__device__ __forceinline__ void predict(const Real W0[NVAR + NS], const Real D[3][NVAR + NS], Real h, Real g,
                                        Real P[NVAR + NS], Real ir) {
  const Real r = W0[0], u = W0[1], vv = W0[2], w = W0[3], p = W0[4];
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
  s[0] = floor_max(s[0], rf);
  s[4] = floor_max(s[4], pf);
}

// Flux through the lower face along axis D of a core cell: the left state
// comes from LDS (FL[var * NFACE + f]), the right one, W~ - D/2, from the
// cell's predicted state Pw and slope Pdd along D.  The HLLC runs in the
// face-normal frame; F is returned in the global frame.
template <typename Real, int D, int NS, int NFACE>
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

// Maximum over a wavefront's 64 lanes (all active), returned to every lane:
// DPP steps within each row of 16 lanes (lane pairs, quads, half-rows,
// rows), two row broadcasts that carry rows 0-2 into row 3, then lane 63
// read out.  The maximum does not depend on the order of combination.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_max_step(double x) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
  const int lo = int(uint32_t(b)), hi = int(uint32_t(b >> 32));
  const int tlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xf, false);
  const int thi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xf, false);
  const unsigned long long t = (static_cast<unsigned long long>(uint32_t(thi)) << 32) | uint32_t(tlo);
  // the bare maximum (the moved bits are a value the library maximum would
  // first quiet); the operands are never signalling NaNs
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(x), "v"(__longlong_as_double(static_cast<long long>(t))));
  return r;
}
__device__ __forceinline__ double wave_max(double v) {
  v = dpp_max_step<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
  v = dpp_max_step<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
  v = dpp_max_step<0x141, 0xf>(v);   // row_half_mirror
  v = dpp_max_step<0x140, 0xf>(v);   // row_mirror: every lane holds its row's maximum
  v = dpp_max_step<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v = dpp_max_step<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(b)), 63));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(b >> 32)), 63));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
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
// The per-tile hydro update.  NT = threads cooperating on one tile: 64, 128
// or 256 for K = 4 (8, 16 or 32 threads per oct), 512 for K = 8 (one thread
// per core cell).  `active` is uniform over the NT threads; an inactive
// group only keeps the workgroup's barrier count.
// ---------------------------------------------------------------------------
// Hides a value from the optimiser so that per-thread table loads are issued
// per tile instead of being hoisted (and held in registers) across the tile
// loop of the persistent kernel.
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Floor activations are counted once per event of the step, although a tile
// recomputes halo values that neighbouring tiles compute too: a leaf cell's
// own primitive conversion by the tile holding the cell, the face states of
// a face by the tile holding its upper cell when that is a leaf, else its
// lower cell (ghost cells are counted once per parent step by the ghost
// kernel).  The checks run only where a floor was applied.
// Kind of the cell at tile position (x, y, z), each in [-1, K]: 1 a leaf
// cell, 2 a refined cell, 0 otherwise (a ghost cell, or past an outflow face).
template <int K>
__device__ int census_kind(const int32_t* tab, const uint8_t* ref, uint32_t fl, const int hb[3], int32_t n_oct, int x,
                           int y, int z) {
  const int p[3] = {x, y, z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (p[a] < 0 && (fl & (1u << (2 * a)))) return 0;
    if (p[a] > hb[a] && (fl & (2u << (2 * a)))) return 0;
  }
  const int slot = Geom<K>::slot(x >> 1, y >> 1, z >> 1);
  const int32_t e = tab[slot];
  if (e < 0 || e >= n_oct) return 0;
  const int cb = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2);
  return ((ref[slot] >> cb) & 1) ? 2 : 1;
}
// Whether tile position (x, y, z) is one of the tile's own cells.
__device__ __forceinline__ bool census_own(const int hb[3], int x, int y, int z) {
  return x >= 0 && y >= 0 && z >= 0 && x <= hb[0] && y <= hb[1] && z <= hb[2];
}
// Whether this tile counts the floors of the face along d whose lower cell
// is at tile position (x, y, z).
template <int K>
__device__ bool census_face(const int32_t* tab, const uint8_t* ref, uint32_t fl, const int hb[3], int32_t n_oct, int x,
                            int y, int z, int d) {
  const int bx = x + (d == 0), by = y + (d == 1), bz = z + (d == 2);
  const int ka = census_kind<K>(tab, ref, fl, hb, n_oct, x, y, z), kb = census_kind<K>(tab, ref, fl, hb, n_oct, bx, by, bz);
  if (kb == 1) return ka != 2 && census_own(hb, bx, by, bz);
  return ka == 1 && kb == 0 && census_own(hb, x, y, z);
}

// Registers that carry a tile's gathered conserved states from their loads
// to their conversion (phase A).
template <int K, int NT, int NV>
struct GatherRegs {
  static constexpr int NRA = (Geom<K>::NPOS_A + NT - 1) / NT;
  double Ua[NRA][NV];
  int iwa[NRA];   // LDS index of each position, -1 when the thread has none
};

// Last in-domain cell of a tile along each axis (a tile cut by the domain's
// high side has fewer than K).
template <int K>
__device__ __forceinline__ void tile_hb(uint32_t fl, int hb[3]) {
  hb[0] = K - 1 - int((fl >> CL_CUT_SHIFT) & 7u);
  hb[1] = K - 1 - int((fl >> (CL_CUT_SHIFT + 3)) & 7u);
  hb[2] = K - 1 - int((fl >> (CL_CUT_SHIFT + 6)) & 7u);
}

// A state plane as a raw buffer resource (base in scalar registers, no
// range limit: the callers keep every byte offset below 4 GiB), so that a
// per-lane 32-bit byte offset addresses it with no 64-bit address
// arithmetic per lane.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const double* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), short(0), int(0xffffffffu), 0x00020000);
}
__device__ __forceinline__ double plane_load(__amdgpu_buffer_rsrc_t r, uint32_t boff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, 0));
}
__device__ __forceinline__ void plane_store(__amdgpu_buffer_rsrc_t r, uint32_t boff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v),
                                        r, boff, 0, 0);
}
// Whether every byte offset into a level's state planes that the tile code
// forms fits 32 bits (planes and the ghost shift under 2^29 cells).
__device__ __forceinline__ bool level_off32(const HydroArgs& A) {
  return A.plane + 8 * int64_t(A.ghost_adj) <= (int64_t(1) << 29);
}

// Phase A's loads: the conserved state at the thread's gather positions of
// a tile whose oct table is in LDS (`tab`), issued without waiting for them.
template <int K, int NT, int NV>
__device__ __forceinline__ void gather_issue(const HydroArgs& A, const int32_t* tab, uint32_t fl, const int hb[3],
                                             int tid, bool active,
                                             const typename Geom<K>::EntA (&entA)[GatherRegs<K, NT, NV>::NRA],
                                             GatherRegs<K, NT, NV>& R) {
  using G = Geom<K>;
  using EA = typename G::EntA;
  constexpr int NRA = GatherRegs<K, NT, NV>::NRA;
  const int64_t P = A.plane;
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
  const bool off32 = level_off32(A);
  __amdgpu_buffer_rsrc_t Ur[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Ur[v] = plane_rsrc(Up[v]);
#pragma unroll
  for (int rnd = 0; rnd < NRA; ++rnd) {
    const int i = tid + NT * rnd;
    R.iwa[rnd] = -1;
    if (active && i < G::NPOS_A) {
      const EA ent = entA[rnd];
      int slot = int((ent >> G::A_LB) & EA((1u << G::A_SB) - 1)), cb = int((ent >> G::A_CS) & EA(7));
      if (fl & CL_ANY) {
        // outflow faces: clamp the position into the domain (zero gradient)
        const int raw = int(ent >> G::A_RS);
        int sx = raw % G::R - 2, sy = (raw / G::R) % G::R - 2, sz = raw / (G::R * G::R) - 2;
        if ((fl & CL_LOX) && sx < 0) sx = 0;
        if ((fl & CL_HIX) && sx > hb[0]) sx = hb[0];
        if ((fl & CL_LOY) && sy < 0) sy = 0;
        if ((fl & CL_HIY) && sy > hb[1]) sy = hb[1];
        if ((fl & CL_LOZ) && sz < 0) sz = 0;
        if ((fl & CL_HIZ) && sz > hb[2]) sz = hb[2];
        slot = G::slot(sx >> 1, sy >> 1, sz >> 1);
        cb = (sx & 1) | ((sy & 1) << 1) | ((sz & 1) << 2);
      }
      int32_t e = tab[slot];
      if (!debug_in_bounds(e < A.n_oct || (e >= A.n_oct + A.ghost_adj && e < A.n_ext + A.ghost_adj), A.err))
        e = -1;
      R.iwa[rnd] = int(ent & EA((1u << G::A_LB) - 1));
      // 32-bit cell index (a level's octs, ghost octs and the ghost shift
      // stay below 2^29 octs).  A slot without an oct is one no leaf update
      // reads: it takes the (valid, finite) state of the level's first cell
      // instead of a branch
      const uint32_t cell = (e >= 0) ? uint32_t(e) * 8u + uint32_t(cb) : 0u;
      if (off32) {
        // planes under 4 GiB: one 32-bit byte offset serves every plane
        const uint32_t boff = cell << 3;
#pragma unroll
        for (int v = 0; v < NV; ++v) R.Ua[rnd][v] = plane_load(Ur[v], boff);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) R.Ua[rnd][v] = Up[v][cell];
      }
    }
  }
}

// A tile's oct table entry as LDS keeps it: a ghost oct is read from the
// second state buffer (the shifted index stays >= n_oct, so every
// real/ghost test on the table still holds).
__device__ __forceinline__ int32_t lds_tab_entry(const HydroArgs& A, int32_t e) {
  return (e >= A.n_oct) ? e + A.ghost_adj : e;
}

template <typename Real, int NT, int NS, int K>
__device__ __forceinline__ void hydro_tile(const HydroArgs& A, int tile, TileLDS<Real, NVAR + NS, K>& S, int tid_in,
                                           bool active, GatherRegs<K, NT, NVAR + NS>& R) {
  using G = Geom<K>;
  using EA = typename G::EntA;
  using EB = typename G::EntB;
  constexpr int NV = NVAR + NS;
  constexpr int WSIZE = G::WSIZE, NFACE = G::NFACE, NUPPER = G::NUPPER, NCORE = G::NCORE;
  constexpr int NPOS_A = G::NPOS_A, NPOS_B = G::NPOS_B, TAB = G::TAB;
  static_assert(NT >= TAB && (K == 4 || NT == NCORE || 2 * NT == NCORE), "threads per tile");
  // core cells per thread: one (NT >= NCORE; threads past NCORE hold none),
  // or two (8^3-cell tile on 256 threads: cells tid and tid + 256)
  constexpr int NCR = (NT >= NCORE) ? 1 : NCORE / NT;
  const int tid = opaque(tid_in);
  const int lane = tid & 63;
  const double g = A.gamma, rf = A.rho_floor, pf = A.p_floor;
  const int64_t P = A.plane;
  int nfl = 0;
  const uint32_t fl = active ? A.tflag[tile] : 0u;
  int hb[3];
  tile_hb<K>(fl, hb);
  const int box = (active && A.tile_box) ? A.tile_box[tile] : 0;
  const double lam = A.lam_dev ? A.lam_dev[box] : A.lam_host;
  const Real h = Real(0.5 * lam);
  const Real igm1 = Real(A.igm1);
  const StencilTables<K>& ST = stencil_tables<K>();
  const int32_t* tab = S.tab;
  const uint8_t* ref = S.ref;

  // The thread's stencil-table entries for phases A and B, loaded together up
  // front: a load issued inside a round would make that round wait for every
  // state load issued before it.
  constexpr int NRA = GatherRegs<K, NT, NV>::NRA;
  constexpr int NRB = (NPOS_B + NT - 1) / NT;
  // floors applied by this thread, 2 bits per site (each site applies at
  // most 2: density and pressure): the conversions of its phase-A positions,
  // its phase-B one-layer face states, its core cell's 3 left and 3 right
  // face states; which of them the tile counts is decided at the end
  constexpr int SITE_A = 0, SITE_B = NRA, SITE_L = NRA + NRB, SITE_R = SITE_L + 3 * NCR;
  static_assert(2 * (SITE_R + 3 * NCR) <= 64, "floor sites");
  using Pend = std::conditional_t<(2 * (SITE_R + 3 * NCR) <= 32), uint32_t, uint64_t>;
  Pend pending = 0;
  EB entB[NRB];
#pragma unroll
  for (int rnd = 0; rnd < NRB; ++rnd) {
    const int i = tid + NT * rnd;
    entB[rnd] = ST.b[uint32_t(i < NPOS_B ? i : 0)];
  }

  EA entA[NRA];
#pragma unroll
  for (int rnd = 0; rnd < NRA; ++rnd) {
    const int i = tid + NT * rnd;
    entA[rnd] = ST.a[uint32_t(i < NPOS_A ? i : 0)];
  }
  // --- phase 0: the tile's oct table (the refined bytes of its octs are
  // loaded in phase A behind the state loads; phase D is their first reader)
  int32_t e_tab = -1;
  if (active && tid < TAB) {
    e_tab = A.tab[size_t(tile) * TAB + tid];
    if (!debug_in_bounds(e_tab >= -1 && e_tab < A.n_ext, A.err)) e_tab = -1;
    S.tab[tid] = lds_tab_entry(A, e_tab);
  }
  __syncthreads();
  // Wait for the table entries here on every path: otherwise the gather's
  // conditional state loads leave the compiler's load counting unsure of
  // them, and each round would wait for the state loads of the rounds
  // before it.
#pragma unroll
  for (int rnd = 0; rnd < NRA; ++rnd) asm volatile("" ::"v"(entA[rnd]));
#pragma unroll
  for (int rnd = 0; rnd < NRB; ++rnd) asm volatile("" ::"v"(entB[rnd]));
  // --- phase A: gather + primitives (all loads of the thread's positions
  // are issued before any conversion)
  gather_issue<K, NT, NV>(A, tab, fl, hb, tid, active, entA, R);
  const uint8_t rb = (e_tab >= 0) ? A.refined[e_tab] : uint8_t(0);

  // --- phase A (conversion): primitives into LDS.  A core cell's first
  // gathered position is the cell itself (the tables' oct-major order): its
  // conserved state stays in registers for the update (phase D), except in
  // the FP64 8^3-cell tile, whose register budget (4 wavefronts per SIMD)
  // it would overrun: there phase D loads it again.
  constexpr bool KEEP_CORE = (K == 4) || (sizeof(Real) == 4) || (NCR > 1);
  Real* W = S.buf;                              // [NV][WSIZE]
  double Ucore[NCR][NV];
  // 1 / rho of the thread's core cells, from their conversion (the FP64
  // predictor divides by the same density)
  double irc[NCR];
#pragma unroll
  for (int r = 0; r < NCR; ++r)
#pragma unroll
    for (int v = 0; v < NV; ++v) Ucore[r][v] = KEEP_CORE ? R.Ua[r][v] : 0.0;
#pragma unroll
  for (int rnd = 0; rnd < NRA; ++rnd) {
    if (R.iwa[rnd] >= 0) {
      double Wc[NV];
      int nc = 0;
      cons2prim<NS>(R.Ua[rnd], Wc, g, rf, pf, nc, rnd < NCR ? &irc[rnd < NCR ? rnd : 0] : nullptr);
      pending |= Pend(nc) << (2 * (SITE_A + rnd));
#pragma unroll
      for (int v = 0; v < NV; ++v) W[v * WSIZE + R.iwa[rnd]] = Real(Wc[v]);
    }
  }
  if (active && tid < TAB) S.ref[tid] = rb;
  __syncthreads();

  // --- phase B1: slopes + predictor.  The core cell of a thread (first pass,
  // tid < NCORE) keeps W~ and its slopes in registers for its six faces; a
  // one-layer cell keeps only its state on the face toward the core.
  constexpr int st[3] = {1, G::WB, G::WBB};
  const bool core = (NT <= NCORE) || tid < NCORE;
  int cxs[NCR], cys[NCR], czs[NCR];
#pragma unroll
  for (int r = 0; r < NCR; ++r) {
    const int ct = (tid + NT * r) & (NCORE - 1);
    cxs[r] = G::core_x(ct);
    cys[r] = G::core_y(ct);
    czs[r] = G::core_z(ct);
  }
  const Real rfr = Real(rf), pfr = Real(pf), gr = Real(g);
  constexpr EB LMASK = EB((1u << G::B_LB) - 1);
  Real Pw[NCR][NV], Pd[NCR][3][NV];
  Real Ls[NRB][NV];
  EB Lb[NRB];
#pragma unroll
  for (int rnd = 0; rnd < NRB; ++rnd) {
    const int i = tid + NT * rnd;
    Lb[rnd] = 0u;
    if (!active || i >= NPOS_B) continue;
    if (rnd < NCR && core) {
      const int r = rnd < NCR ? rnd : 0;
      const int iw = (cxs[r] + 1) + G::WB * (cys[r] + 1) + G::WBB * (czs[r] + 1);
      Real W0[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) W0[v] = W[v * WSIZE + iw];
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int v = 0; v < NV; ++v)
          Pd[r][d][v] = mmod(W0[v] - W[v * WSIZE + iw - st[d]], W[v * WSIZE + iw + st[d]] - W0[v]);
      // FP64: the conversion's 1 / rho (the same quotient of the same density)
      const Real ir = (sizeof(Real) == 8) ? Real(irc[r]) : rcp(W0[0]);
      predict<Real, NS>(W0, Pd[r], h, gr, Pw[r], ir);
    } else {
      const EB e = entB[rnd];
      Lb[rnd] = e;
      const int iw = int(e & LMASK), far = int((e >> G::B_LB) & LMASK), dn = int((e >> G::B_DS) & EB(3));
      const bool up = (e >> G::B_US) & EB(1);
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
      predict<Real, NS>(W0, D, h, gr, Q, rcp(W0[0]));
      // the face state Q +- D/2 along the normal: the weights of the two other
      // axes are zero, so their fused terms add exact zeros
      const Real sg = up ? Real(-0.5) : Real(0.5);
      const Real t0 = (dn == 0) ? sg : Real(0), t1 = (dn == 1) ? sg : Real(0), t2 = (dn == 2) ? sg : Real(0);
#pragma unroll
      for (int v = 0; v < NV; ++v) Ls[rnd][v] = fma(t2, D[2][v], fma(t1, D[1][v], fma(t0, D[0][v], Q[v])));
      int nc = 0;
      floor_state<Real>(Ls[rnd], rfr, pfr, nc);
      pending |= Pend(nc) << (2 * (SITE_B + rnd));
    }
  }
  __syncthreads();

  // --- phase B2: the left states (W~ + D/2 of the lower cell) of the faces
  // replace the primitives in LDS
  Real* FL = S.buf;                             // [NV][NFACE]
  Real* FR = S.buf + NV * NFACE;                // [NV][NUPPER]: right states of the upper layer
#pragma unroll
  for (int rnd = 0; rnd < NRB; ++rnd) {
    const int i = tid + NT * rnd;
    if (!active || i >= NPOS_B) continue;
    if (rnd < NCR && core) {
      const int r = rnd < NCR ? rnd : 0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        Real s[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) s[v] = Pw[r][v] + Real(0.5) * Pd[r][d][v];
        int nc = 0;
        floor_state<Real>(s, rfr, pfr, nc);
        pending |= Pend(nc) << (2 * (SITE_L + 3 * r + d));
        const int f = G::fidx(d, cxs[r] + (d == 0), cys[r] + (d == 1), czs[r] + (d == 2));
#pragma unroll
        for (int v = 0; v < NV; ++v) FL[v * NFACE + f] = s[v];
      }
    } else if (!((Lb[rnd] >> G::B_US) & EB(1))) {
      const int f = int(Lb[rnd] >> G::B_FS);
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
  Real Fc[NCR][3][NV];
  Real Fl[NRB][NV];
#pragma unroll
  for (int rnd = 0; rnd < NRB; ++rnd) {
    const int i = tid + NT * rnd;
    if (!active || i >= NPOS_B) continue;
    if (rnd < NCR && core) {
      const int r = rnd < NCR ? rnd : 0;
      const int cx = cxs[r], cy = cys[r], cz = czs[r];
      int nc[3] = {0, 0, 0};
      core_face_flux<Real, 0, NS, NFACE>(FL, G::fidx(0, cx, cy, cz), Pw[r], Pd[r][0], rfr, pfr, gr, igm1, nc[0],
                                         Fc[r][0]);
      core_face_flux<Real, 1, NS, NFACE>(FL, G::fidx(1, cx, cy, cz), Pw[r], Pd[r][1], rfr, pfr, gr, igm1, nc[1],
                                         Fc[r][1]);
      core_face_flux<Real, 2, NS, NFACE>(FL, G::fidx(2, cx, cy, cz), Pw[r], Pd[r][2], rfr, pfr, gr, igm1, nc[2],
                                         Fc[r][2]);
      pending |= (Pend(nc[0]) << (2 * (SITE_R + 3 * r))) | (Pend(nc[1]) << (2 * (SITE_R + 3 * r + 1))) |
                 (Pend(nc[2]) << (2 * (SITE_R + 3 * r + 2)));
    } else if ((Lb[rnd] >> G::B_US) & EB(1)) {
      const int f = int(Lb[rnd] >> G::B_FS), dn = int((Lb[rnd] >> G::B_DS) & EB(3)), k = i - NCORE;
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
    if (rnd < NCR && core) {
      const int r = rnd < NCR ? rnd : 0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int f = G::fidx(d, cxs[r], cys[r], czs[r]);
#pragma unroll
        for (int v = 0; v < NV; ++v) SF[v * NFACE + f] = Fc[r][d][v];
      }
    } else if ((Lb[rnd] >> G::B_US) & EB(1)) {
      // Fl is in the face-normal frame: rotate back on the way out
      const int f = int(Lb[rnd] >> G::B_FS), dn = int((Lb[rnd] >> G::B_DS) & EB(3));
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

  // --- phase D: the threads of the core cells update them (the old state of
  // the cell is the one gathered in phase A, or loaded again first: the
  // stores to the new state may alias it as far as the compiler knows, and
  // a load issued after a store would wait for it)
  // the thread holds core cells (with more threads than core cells, the
  // threads past them hold none)
  const bool cthr = (NT <= NCORE) || tid < NCORE;
  using LDS = TileLDS<Real, NV, K>;
  double* smx = LDS::SMAX_IN_BUF ? reinterpret_cast<double*>(S.buf + NV * NFACE) : S.smx;
  int32_t e[NCR];
  uint32_t cell[NCR];
  bool leaf[NCR];
#pragma unroll
  for (int r = 0; r < NCR; ++r) {
    const int cx = cxs[r], cy = cys[r], cz = czs[r];
    const int ts = G::slot(cx >> 1, cy >> 1, cz >> 1);
    e[r] = (active && cthr) ? tab[ts] : -1;
    const int ci = (cx & 1) | ((cy & 1) << 1) | ((cz & 1) << 2);
    // a tile cut by the domain's high side: its slots past the cut hold the
    // periodic images of other octs, which other tiles update
    const bool inside = cx <= hb[0] && cy <= hb[1] && cz <= hb[2];
    leaf[r] = cthr && inside && (e[r] >= 0) && (e[r] < A.n_oct) && !((ref[ts] >> ci) & 1);
    cell[r] = uint32_t(e[r]) * 8u + uint32_t(ci);
  }
  // planes addressed by 32-bit byte offsets where they fit (as the gather)
  const bool off32 = level_off32(A);
  if (!KEEP_CORE) {
#pragma unroll
    for (int r = 0; r < NCR; ++r)
      if (leaf[r]) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
          Ucore[r][v] = off32 ? plane_load(plane_rsrc(A.U + v * P), cell[r] << 3) : (A.U + v * P)[cell[r]];
      }
  }
  double acc[NCR][NV];
#pragma unroll
  for (int r = 0; r < NCR; ++r) {
    if (!leaf[r]) continue;
    const int cx = cxs[r], cy = cys[r], cz = czs[r];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      // the lower face's flux is the thread's own (phase C), the upper one
      // comes from the neighbouring cell's thread through LDS
      const int fp = G::fidx(d, cx + (d == 0), cy + (d == 1), cz + (d == 2));
      double Fm[NV], Fp[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Fm[v] = double(Fc[r][d][v]);
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
          if ((n[d] < 0 && (fl & lo)) || (n[d] > hb[d] && (fl & hi))) continue;
          const int tn = G::slot(n[0] >> 1, n[1] >> 1, n[2] >> 1);
          const int32_t en = tab[tn];
          const int cn = (n[0] & 1) | ((n[1] & 1) << 1) | ((n[2] & 1) << 2);
          if (en >= 0 && en < A.n_oct && ((ref[tn] >> cn) & 1)) {
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
      for (int v = 0; v < NV; ++v) acc[r][v] = (d == 0) ? (Fm[v] - Fp[v]) : acc[r][v] + (Fm[v] - Fp[v]);
    }
  }
  if (cthr) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < NCR; ++r) {
      if (!leaf[r]) continue;
      double Un[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Un[v] = Ucore[r][v] + lam * acc[r][v];
      if (off32) {
#pragma unroll
        for (int v = 0; v < NV; ++v) plane_store(plane_rsrc(A.Un + v * P), cell[r] << 3, Un[v]);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) (A.Un + v * P)[cell[r]] = Un[v];
      }
      if (A.tile_smax || A.smax_bits || A.err) {
        const double sr = signal_speed(Un, g, rf, pf);
        const bool bad = !(isfinite(Un[0]) && isfinite(Un[1]) && isfinite(Un[2]) && isfinite(Un[3]) &&
                           isfinite(Un[4])) || !(Un[0] > 0.0) || !(Un[4] > 0.0) || !isfinite(sr);
        if (bad) atomicOr(A.err, 1);
        s = (r == 0) ? (bad ? 0.0 : sr) : fmax(s, bad ? 0.0 : sr);
      }
    }
    if constexpr (NCORE > 64) {
      // several wavefronts: the first reduces the tile's speeds after the
      // tile's last barrier
      smx[tid] = s;
    } else if (active && A.smax_bits) {
      // one atomic maximum per wavefront on one of the level's slots (a
      // non-negative double orders like its bit pattern); the maximum does
      // not depend on the order of arrival
      const double m = wave_max(s);
      const int sl = tile & (SMAX_SLOTS - 1);
      if (lane == 0) atomicMax(A.smax_bits + sl, (unsigned long long)__double_as_longlong(m));
    } else if (active && A.tile_smax) {
      // batched boxes: one partial per tile, reduced per box by the
      // segmented max kernel before the next time step
      const double m = wave_max(s);
      const int slot = A.tile_part ? A.tile_part[tile] : tile;
      if (lane == 0) A.tile_smax[slot] = m;
    }
  }

  // --- fine-side registers: q_s = (f1 + f2) + (f3 + f4) on coarse-fine faces
  constexpr int KO = G::KO, NREG = 6 * KO * KO * KO;
  const int rt0 = (K == 4 && NT > 64) ? tid - 64 : tid;   // K = 4: a second wavefront, when there is one
#pragma unroll
  for (int rr = 0; rr < (NREG + NT - 1) / NT; ++rr) {
    const int rt = rt0 + NT * rr;
    if (!(active && A.record_reg && rt >= 0 && rt < NREG)) continue;
    const int b = rt / 6, face = rt - 6 * (rt / 6);
    const int bx = b % KO, by = (b / KO) % KO, bz = b / (KO * KO);
    const int tb_ = G::slot(bx, by, bz);
    const int32_t eb = tab[tb_];
    const int d = face >> 1, up = face & 1;
    const int dd = up ? 1 : -1;
    const int rx = bx + (d == 0 ? dd : 0), ry_ = by + (d == 1 ? dd : 0), rz = bz + (d == 2 ? dd : 0);
    const int rd = (d == 0) ? rx : ((d == 1) ? ry_ : rz);
    const uint32_t lo = (d == 0) ? CL_LOX : ((d == 1) ? CL_LOY : CL_LOZ);
    const bool clamped = (rd < 0 && (fl & lo)) || (rd > (hb[d] >> 1) && (fl & (lo << 1)));
    const bool inside = bx <= (hb[0] >> 1) && by <= (hb[1] >> 1) && bz <= (hb[2] >> 1);
    if (inside && eb >= 0 && eb < A.n_oct && !clamped) {
      const int tn = G::slot(rx, ry_, rz);
      if (tab[tn] >= A.n_oct) {
        // the 4 cells of the oct on this face, ascending in-oct index: insert
        // bit `up` at position d into j = 0..3
        const int m = (1 << d) - 1;
        int fi[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = (j & m) | (up << d) | ((j & ~m) << 1);
          const int ccx = 2 * bx + (c & 1), ccy = 2 * by + ((c >> 1) & 1), ccz = 2 * bz + ((c >> 2) & 1);
          fi[j] = G::fidx(d, ccx + (d == 0 ? up : 0), ccy + (d == 1 ? up : 0), ccz + (d == 2 ? up : 0));
        }
        double* q = A.reg_own + (int64_t(eb) * 6 + face) * NV * 2;
#pragma unroll
        for (int v = 0; v < NV; ++v)
          q[2 * v + A.substep] = (double(SF[v * NFACE + fi[0]]) + double(SF[v * NFACE + fi[1]])) +
                                 (double(SF[v * NFACE + fi[2]]) + double(SF[v * NFACE + fi[3]]));
      }
    }
  }
  // the floors applied here that this tile counts (rare: evaluated only in a
  // thread that applied any); LDS still holds the tile's oct table
  if (pending) {
#pragma unroll
    for (int rnd = 0; rnd < NRA; ++rnd) {
      const int f = int(pending >> (2 * (SITE_A + rnd))) & 3;
      if (!f) continue;
      // a conversion: counted when the position is one of the tile's own leaf cells
      const int raw = int(ST.a[tid + NT * rnd] >> G::A_RS);
      const int sx = raw % G::R - 2, sy = (raw / G::R) % G::R - 2, sz = raw / (G::R * G::R) - 2;
      if (census_own(hb, sx, sy, sz) && census_kind<K>(tab, ref, fl, hb, A.n_oct, sx, sy, sz) == 1) nfl += f;
    }
#pragma unroll
    for (int rnd = 0; rnd < NRB; ++rnd) {
      const int f = int(pending >> (2 * (SITE_B + rnd))) & 3;
      if (!f) continue;
      // a one-layer face state: the face between the cell and the core, whose
      // lower cell is this cell (lower layer) or the core cell below it
      const EB e = ST.b[tid + NT * rnd];
      const int iw = int(e & LMASK), dn = int((e >> G::B_DS) & EB(3));
      const bool up = (e >> G::B_US) & EB(1);
      const int x = (iw % G::WB) - 1 - (up && dn == 0), y = (iw % G::WBB) / G::WB - 1 - (up && dn == 1),
                z = iw / G::WBB - 1 - (up && dn == 2);
      if (census_face<K>(tab, ref, fl, hb, A.n_oct, x, y, z, dn)) nfl += f;
    }
#pragma unroll
    for (int r = 0; r < NCR; ++r)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int cx = cxs[r], cy = cys[r], cz = czs[r];
        const int fl_ = int(pending >> (2 * (SITE_L + 3 * r + d))) & 3;
        const int fr = int(pending >> (2 * (SITE_R + 3 * r + d))) & 3;
        if (fl_ && census_face<K>(tab, ref, fl, hb, A.n_oct, cx, cy, cz, d)) nfl += fl_;
        if (fr && census_face<K>(tab, ref, fl, hb, A.n_oct, cx - (d == 0), cy - (d == 1), cz - (d == 2), d))
          nfl += fr;
      }
  }
  // floor activations are rare: the shuffle sum runs only in a wavefront
  // that has any
  if (active && A.floors && __any(nfl != 0)) {
    const int tot = wave_sum(nfl);
    if (lane == 0 && tot) atomicAdd(A.floors, (unsigned long long)tot);
  }
  __syncthreads();
  if constexpr (NCORE > 64) {
    if (active && tid < 64 && (A.smax_bits || A.tile_smax)) {
      double m = smx[tid];
#pragma unroll
      for (int k = 1; k < NT / 64; ++k) m = fmax(m, smx[tid + 64 * k]);
      m = wave_max(m);
      if (lane == 0) {
        if (A.smax_bits) {
          atomicMax(A.smax_bits + (tile & (SMAX_SLOTS - 1)), (unsigned long long)__double_as_longlong(m));
        } else {
          // batched boxes: the tile's partial (an atomic maximum on its bit
          // pattern into a slot cleared before the launch)
          const int slot = A.tile_part ? A.tile_part[tile] : tile;
          atomicMax(reinterpret_cast<unsigned long long*>(A.tile_smax) + slot,
                    (unsigned long long)__double_as_longlong(m));
        }
      }
    }
  }
}

// Occupancy targets.  K = 4, hydro variables alone: at least 3 wavefronts
// per SIMD (the FP64 tile's LDS allows no more, so the register budget of an
// instruction-level-parallel schedule stops there); with passive scalars the
// LDS tile sets the limit.  K = 8: two 512-thread tiles per CU (the FP64
// tile takes 81.5 KB of the 160 KB of LDS), so 4 wavefronts per SIMD; on
// 256 threads (two cells per thread) the FP64 tile keeps 2 tiles per CU, 2
// wavefronts per SIMD with up to 256 registers, the mixed tile 3 tiles per
// CU (its LDS allows them) at 3 wavefronts per SIMD.
template <typename Real, int K, int NS, int WPT>
constexpr int hydro_waves_per_eu() {
  return K == 8 ? (WPT == 8 ? 4 : (sizeof(Real) == 4 ? 3 : 2)) : (NS == 0 ? 3 : 1);
}

template <typename Real, int TPW, int WPT, int NS, int K>
__global__ __launch_bounds__(64 * WPT * TPW) __attribute__((amdgpu_waves_per_eu(hydro_waves_per_eu<Real, K, NS, WPT>())))
void hydro_kernel(HydroArgs A) {
  constexpr int NT = 64 * WPT;
  __shared__ TileLDS<Real, NVAR + NS, K> S[TPW];
  if (A.skip && *A.skip) return;
  const int w = threadIdx.x / NT, tid = threadIdx.x % NT;
  const int ngroups = (A.n_tile + TPW - 1) / TPW;
  const int grp = xcd_remap(blockIdx.x, gridDim.x);
  if (grp >= ngroups) return;
  const int tile = grp * TPW + w;
  GatherRegs<K, NT, NVAR + NS> R;
  hydro_tile<Real, NT, NS, K>(A, tile < A.n_tile ? tile : 0, S[w], tid, tile < A.n_tile, R);
}

// Persistent variant (K = 4): workgroups pop groups of tiles from 8 per-XCD
// queues (one contiguous slice of the Hilbert-ordered tile list per XCD; a
// workgroup whose own queue is empty takes from the next one).  Every
// workgroup exits once all 8 queues are exhausted.
template <typename Real, int TPW, int WPT>
__global__ __launch_bounds__(64 * WPT * TPW) __attribute__((amdgpu_waves_per_eu(3))) void hydro_kernel_persistent(HydroArgs A,
                                                                                                      int batch) {
  constexpr int NT = 64 * WPT;
  __shared__ TileLDS<Real, NVAR, 4> S[TPW];
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
      GatherRegs<4, NT, NVAR> R;
      hydro_tile<Real, NT, 0, 4>(A, tile < A.n_tile ? tile : 0, S[w], tid, tile < A.n_tile, R);
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

// The persistent kernel exists for the hydro variables alone (NS = 0) on
// small tiles (K = 4).
template <typename Real, int TPW, int WPT, int NS, int K = 4>
static int launch_hydro_t(const HydroArgs& a, const ry_tuning& t, int num_cu, hipStream_t s) {
  const int ngroups = (a.n_tile + TPW - 1) / TPW;
  if (ngroups == 0) return 0;
  if (NS > 0 || K != 4 || !t.persistent) {
    hipLaunchKernelGGL((hydro_kernel<Real, TPW, WPT, NS, K>), dim3(ngroups), dim3(64 * WPT * TPW), 0, s, a);
  } else if constexpr (NS == 0 && K == 4) {
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
