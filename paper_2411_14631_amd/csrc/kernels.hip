// HIP kernels (gfx950) around the hydro step: hydro launch dispatch (the
// kernels with passive scalars), coarse-fine ghost octs, restriction, CFL
// reductions, conserved totals, the regrid state remap, a plain copy.  The
// per-tile hydro update itself is in hydro_tile.h; its hydro-only
// instantiations are compiled in hydro.hip.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hydro_tile.h"
#include "ry_internal.h"
#include "regrid.h"

namespace ry {

int hydro_max_tiles_per_wg() { return 4; }

bool hydro_tuning_supported(int precision, int nscalar, const ry_tuning& t) {
  if (t.tile_cells == 8)
    return nscalar == 0 && !t.persistent && t.tiles_per_wg == 1 && (t.waves_per_tile == 8 || t.waves_per_tile == 4);
  if (t.tile_cells != 4) return false;
  const int key = t.tiles_per_wg * 10 + t.waves_per_tile;
  if (nscalar == 0) {
    if (precision == RY_MIXED) return key == 11 || key == 21 || key == 41 || key == 12 || key == 22 || key == 14;
    return key == 11 || key == 21 || key == 41 || key == 12 || key == 22 || key == 14;
  }
  return nscalar <= RY_MAX_SCALARS && !t.persistent && (key == 11 || key == 12 || key == 21);
}

template <typename Real, int NS>
static int launch_hydro_ns(const HydroArgs& a, const ry_tuning& t, int num_cu, hipStream_t s) {
  switch (t.tiles_per_wg * 10 + t.waves_per_tile) {
    case 11: return launch_hydro_t<Real, 1, 1, NS>(a, t, num_cu, s);
    case 12: return launch_hydro_t<Real, 1, 2, NS>(a, t, num_cu, s);
    case 21: return launch_hydro_t<Real, 2, 1, NS>(a, t, num_cu, s);
    default: return -1;
  }
}

template <typename Real>
static int launch_hydro_scalars(const HydroArgs& a, int nscalar, const ry_tuning& t, int num_cu, hipStream_t s) {
  switch (nscalar) {
    case 1: return launch_hydro_ns<Real, 1>(a, t, num_cu, s);
    case 2: return launch_hydro_ns<Real, 2>(a, t, num_cu, s);
    case 3: return launch_hydro_ns<Real, 3>(a, t, num_cu, s);
    case 4: return launch_hydro_ns<Real, 4>(a, t, num_cu, s);
    default: return -1;
  }
}

int launch_hydro(const HydroArgs& a, int precision, int nscalar, const ry_tuning& t, int num_cu, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (!hydro_tuning_supported(precision, nscalar, t)) return -1;
  if (a.n_tile == 0) return 0;   // a level whose octs are all fully refined has no tile to update
  if (nscalar > 0)
    return precision == RY_MIXED ? launch_hydro_scalars<float>(a, nscalar, t, num_cu, s)
                                 : launch_hydro_scalars<double>(a, nscalar, t, num_cu, s);
  return launch_hydro_plain(a, precision, t, num_cu, stream);
}

// ---------------------------------------------------------------------------
// Ghost octs: MinMod-limited linear interpolation of the covering coarse
// cell's conserved variables, written into the level's second state buffer
// (both hydro substeps of the parent step read them there).
// ---------------------------------------------------------------------------
// One thread per ghost oct: its 8 cells are the children of one coarse cell
// Q and share Q's 7 sources, loaded once (NV, the variable count, is a
// template parameter so that all 7 x NV loads issue before the first use);
// each variable's 8 results go out as four 16-byte stores per buffer.
template <int NV>
__global__ void ghost_kernel(GhostArgs A) {
  if (A.skip && *A.skip) return;
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi >= A.n_ghost) return;
  const double* base[7];
  int64_t cell[7], pl[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const int64_t src = A.gsrc[gi * 7 + k];
    const int up = int(src >> 48);
    cell[k] = src & ((int64_t(1) << 48) - 1);
    base[k] = A.src[up];
    pl[k] = A.src_plane[up];
    if (!debug_in_bounds(up < RY_MAX_LEVELS && cell[k] >= 0 && cell[k] < pl[k], A.err)) cell[k] = 0;
  }
  double val[NV][7];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int k = 0; k < 7; ++k) val[v][k] = base[k][v * pl[k] + cell[k]];
  int64_t dst = (A.n_oct + gi) * 8;
  if (!debug_in_bounds(dst + 8 <= A.plane, A.err)) return;
  double keep[NVAR][8];   // the hydro variables of the 8 cells, for the floor census
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double q = val[v][0];
    const double mx = mmod(q - val[v][1], val[v][2] - q);
    const double my = mmod(q - val[v][3], val[v][4] - q);
    const double mz = mmod(q - val[v][5], val[v][6] - q);
    double out[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double sx = (c & 1) ? 0.25 : -0.25, sy = (c & 2) ? 0.25 : -0.25, sz = (c & 4) ? 0.25 : -0.25;
      out[c] = q + (sx * mx + sy * my + sz * mz);
      if (v < NVAR) keep[v][c] = out[c];
    }
    double2* d = reinterpret_cast<double2*>(A.dst + v * A.plane + dst);
#pragma unroll
    for (int j = 0; j < 4; ++j) d[j] = make_double2(out[2 * j], out[2 * j + 1]);
  }
  if (A.floors && A.gread) {
    // the floors the primitive conversion of each cell applies (density,
    // then pressure from E minus the kinetic energy at the floored density),
    // counted for the cells an update reads
    const uint32_t rd = A.gread[gi];
    int n = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double r = keep[0][c] < A.rho_floor ? A.rho_floor : keep[0][c];
      const double ke = 0.5 * (keep[1][c] * keep[1][c] + keep[2][c] * keep[2][c] + keep[3][c] * keep[3][c]) / r;
      const int f = int(keep[0][c] < A.rho_floor) + int((A.gamma - 1.0) * (keep[4][c] - ke) < A.p_floor);
      if ((rd >> c) & 1u) n += f;
    }
    if (n) atomicAdd(A.floors, (unsigned long long)n);
  }
}

// One wavefront per small tile, one lane per (tile, slot) of its table: a
// slot holding a ghost oct gets the bits of its cells that lie in the
// stencil of a leaf cell of the tile's core (one or two steps along an axis,
// or one step along each of two axes).  Every leaf cell is in exactly one
// tile's core, and its stencil stays within that tile's oct neighbourhood,
// so the union over the tiles is exact.  Cells past the domain's high side
// of a cut tile are other tiles' cells and are skipped.
//
// The core's 4x4x4 cells are the wavefront's 64 lanes: a ballot gives the
// leaf set, which goes into eight 64-bit words, one per cell layer z, bit
// x + 8y, with every coordinate shifted by 2 so that the core sits at 2..5
// and its dilation by the stencil (at most 2 cells) stays inside 0..7 and
// inside each word's rows.  The read set is that dilation (the stencil's
// offsets are symmetric); each ghost lane then takes its 8 cells' bits.
__global__ void ghost_read_kernel(const int32_t* __restrict__ tab, const uint32_t* __restrict__ tflag,
                                  const uint8_t* __restrict__ refined, int32_t n_tile, int64_t n_oct,
                                  uint32_t* __restrict__ gread) {
  using G = Geom<4>;
  static_assert(G::TAB == 64 && G::TS == 4, "one lane per slot and per core cell");
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(n_tile) * G::TAB) return;   // whole wavefronts: blocks of whole wavefronts, 64 slots a tile
  const int tile = __builtin_amdgcn_readfirstlane(int(i / G::TAB));
  const int lane = int(i % G::TAB);
  const int32_t* t = tab + int64_t(tile) * G::TAB;
  const uint32_t fl = tflag[tile];
  const int hb[3] = {3 - int((fl >> CL_CUT_SHIFT) & 7u), 3 - int((fl >> (CL_CUT_SHIFT + 3)) & 7u),
                     3 - int((fl >> (CL_CUT_SHIFT + 6)) & 7u)};
  // this lane's core cell and whether it is a leaf of the tile
  const int cx = lane & 3, cy = (lane >> 2) & 3, cz = lane >> 4;
  const int32_t q = t[G::slot(cx >> 1, cy >> 1, cz >> 1)];
  const bool leaf = cx <= hb[0] && cy <= hb[1] && cz <= hb[2] && q >= 0 && q < n_oct &&
                    !((refined[q] >> ((cx & 1) | ((cy & 1) << 1) | ((cz & 1) << 2))) & 1);
  const uint64_t core = __ballot(leaf);   // bit x + 4y + 16z
  const int32_t e = t[lane];
  if (e < n_oct) return;
  uint64_t w[8];
#pragma unroll
  for (int z = 0; z < 8; ++z) {
    w[z] = 0;
    if (z >= 2 && z <= 5)
#pragma unroll
      for (int y = 0; y < 4; ++y) w[z] |= ((core >> (16 * (z - 2) + 4 * y)) & 0xFull) << (8 * (y + 2) + 2);
  }
  // this lane's ghost oct: cells at x 2sx..2sx+1 (shifted coordinates), etc.
  const int sx = 2 * (lane & 3), sy = 2 * ((lane >> 2) & 3), sz = 2 * (lane >> 4);
  uint32_t m = 0;
#pragma unroll
  for (int z = 0; z < 8; ++z) {
    const uint64_t v = w[z];
    const uint64_t a1 = (z >= 1 ? w[z - 1] : 0) | (z <= 6 ? w[z + 1] : 0);   // one step along z
    const uint64_t a2 = (z >= 2 ? w[z - 2] : 0) | (z <= 5 ? w[z + 2] : 0);   // two steps along z
    const uint64_t r = (v << 1) | (v >> 1) | (v << 2) | (v >> 2)             // x
                       | (v << 8) | (v >> 8) | (v << 16) | (v >> 16)         // y
                       | (v << 9) | (v >> 9) | (v << 7) | (v >> 7)           // x and y
                       | a1 | a2 | (a1 << 1) | (a1 >> 1) | (a1 << 8) | (a1 >> 8);   // z; x and z; y and z
    if (z == sz || z == sz + 1) {
      const int bz = z - sz;
#pragma unroll
      for (int by = 0; by < 2; ++by)
#pragma unroll
        for (int bx = 0; bx < 2; ++bx)
          if ((r >> ((sx + bx) + 8 * (sy + by))) & 1ull) m |= 1u << (bx | (by << 1) | (bz << 2));
    }
  }
  if (m) atomicOr(gread + (e - n_oct), m);
}

int launch_ghost_read(const int32_t* tab, const uint32_t* tflag, const uint8_t* refined, int32_t n_tile,
                      int64_t n_oct, uint32_t* gread, void* stream) {
  const int64_t n = int64_t(n_tile) * Geom<4>::TAB;
  if (n == 0) return 0;
  hipLaunchKernelGGL(ghost_read_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, tab,
                     tflag, refined, n_tile, n_oct, gread);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_ghost(const GhostArgs& a, void* stream) {
  if (a.n_ghost == 0) return 0;
  const dim3 grid(unsigned((a.n_ghost + 127) / 128)), block(128);
  hipStream_t s = (hipStream_t)stream;
  switch (a.nv) {
    case 5: hipLaunchKernelGGL(ghost_kernel<5>, grid, block, 0, s, a); break;
    case 6: hipLaunchKernelGGL(ghost_kernel<6>, grid, block, 0, s, a); break;
    case 7: hipLaunchKernelGGL(ghost_kernel<7>, grid, block, 0, s, a); break;
    case 8: hipLaunchKernelGGL(ghost_kernel<8>, grid, block, 0, s, a); break;
    case 9: hipLaunchKernelGGL(ghost_kernel<9>, grid, block, 0, s, a); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// Restriction: refined cell of level l = mean of its 8 children.
// ---------------------------------------------------------------------------
// The ordered mean of fine oct k's 8 cells in plane v (64 contiguous bytes,
// as four 16-byte loads).
__device__ __forceinline__ double child_mean(const double* __restrict__ Uf, int64_t pf, int v, int64_t k) {
  const double2* s = reinterpret_cast<const double2*>(Uf + v * pf + 8 * k);
  const double2 a = s[0], b = s[1], c = s[2], d = s[3];
  return 0.125 * (((a.x + a.y) + (b.x + b.y)) + ((c.x + c.y) + (d.x + d.y)));
}

__global__ void restrict_kernel(const double* __restrict__ Uf, int64_t pf, int64_t nf,
                                const int32_t* __restrict__ parent, double* __restrict__ Uc, int64_t pc, int nv,
                                const int32_t* skip, int32_t* err) {
  if (skip && *skip) return;
  // variable-major: consecutive threads read consecutive octs of one plane
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nf * nv) return;
  const int v = int(i / nf);
  const int64_t k = i - int64_t(v) * nf;
  const int32_t q = parent[k];
  if (!debug_in_bounds(q >= 0 && q < pc, err)) return;
  Uc[v * pc + q] = child_mean(Uf, pf, v, k);
}

// The same restriction for the fine octs marked in dirty_f only; each marks
// its parent oct in dirty_c (when given).
__global__ void restrict_dirty_kernel(const double* __restrict__ Uf, int64_t pf, int64_t nf,
                                      const int32_t* __restrict__ parent, double* __restrict__ Uc, int64_t pc, int nv,
                                      const uint8_t* __restrict__ dirty_f, uint8_t* __restrict__ dirty_c,
                                      int32_t* err) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nf * nv) return;
  const int v = int(i / nf);
  const int64_t k = i - int64_t(v) * nf;
  if (!dirty_f[k]) return;
  const int32_t q = parent[k];
  if (!debug_in_bounds(q >= 0 && q < pc, err)) return;
  Uc[v * pc + q] = child_mean(Uf, pf, v, k);
  if (v == 0 && dirty_c) dirty_c[q >> 3] = 1;
}

int launch_restrict_dirty(const double* Uf, int64_t pf, int64_t nf, const int32_t* parent, double* Uc, int64_t pc,
                          int nv, const uint8_t* dirty_f, uint8_t* dirty_c, int32_t* err, void* stream) {
  if (nf == 0) return 0;
  const int64_t n = nf * nv;
  hipLaunchKernelGGL(restrict_dirty_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, Uf,
                     pf, nf, parent, Uc, pc, nv, dirty_f, dirty_c, err);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_restrict(const double* Uf, int64_t pf, int64_t nf, const int32_t* parent, double* Uc, int64_t pc,
                    int nv, const int32_t* skip, int32_t* err, void* stream) {
  if (nf == 0) return 0;
  const int64_t n = nf * nv;
  hipLaunchKernelGGL(restrict_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, Uf, pf,
                     nf, parent, Uc, pc, nv, skip, err);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// CFL: max signal speed over the leaf cells of a level, one partial per
// 256-thread block (wave shuffles, then LDS across the block's 4 waves).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void cfl_kernel(const double* __restrict__ U, int64_t plane, int64_t n_oct,
                                                  const uint8_t* __restrict__ refined, double g, double rf, double pf,
                                                  double* __restrict__ part, int32_t* err) {
  __shared__ double red[4];
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
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

int launch_cfl(const double* U, int64_t plane, int64_t n_oct, const uint8_t* refined, double g, double rf, double pf,
               double* part, int64_t part_cap, int32_t* err, void* stream) {
  if (n_oct == 0) return 0;
  // one partial per block: the grid must fit the caller's segment
  const int64_t nblk = cfl_blocks(n_oct);
  if (nblk > part_cap) return LAUNCH_EXCEEDS_BUFFER;
  hipLaunchKernelGGL(cfl_kernel, dim3(unsigned(nblk)), dim3(256), 0, (hipStream_t)stream, U, plane, n_oct,
                     refined, g, rf, pf, part, err);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ __launch_bounds__(1024) void seg_max_kernel(const double* __restrict__ part,
                                                       const int64_t* __restrict__ off, double* __restrict__ out,
                                                       unsigned long long* __restrict__ slots) {
  __shared__ double red[16];
  __shared__ double seg;
  const int64_t a = off[blockIdx.x], b = off[blockIdx.x + 1];
  // four independent accumulators per thread keep four loads in flight
  double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
  int64_t i = a + threadIdx.x;
  for (; i + 3 * 1024 < b; i += 4 * 1024) {
    m0 = fmax(m0, part[i]);
    m1 = fmax(m1, part[i + 1024]);
    m2 = fmax(m2, part[i + 2 * 1024]);
    m3 = fmax(m3, part[i + 3 * 1024]);
  }
  for (; i < b; i += 1024) m0 = fmax(m0, part[i]);
  double m = wave_max(fmax(fmax(m0, m1), fmax(m2, m3)));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x < 64) {
    m = (threadIdx.x < 16) ? red[threadIdx.x] : 0.0;
    m = wave_max(m);
    if (threadIdx.x == 0) {
      out[blockIdx.x] = m;
      seg = m;
    }
  }
  __syncthreads();
  if (slots && threadIdx.x < SMAX_SLOTS)
    slots[int64_t(blockIdx.x) * SMAX_SLOTS + threadIdx.x] =
        threadIdx.x == 0 ? (unsigned long long)__double_as_longlong(seg) : 0ull;
}

int launch_seg_max(const double* part, const int64_t* off, int nseg, double* out, unsigned long long* slots,
                   void* stream) {
  if (nseg <= 0) return 0;
  hipLaunchKernelGGL(seg_max_kernel, dim3(nseg), dim3(1024), 0, (hipStream_t)stream, part, off, out, slots);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// Time step on the device: dt from the CFL slots, clipped to t_end; lambda.
// ---------------------------------------------------------------------------
// One thread: dt of the next coarse step from the per-level maxima; returns
// whether that step runs (then the slots are cleared for its own maxima).
__device__ bool finalize_dt(const FinalizeArgs& A) {
#pragma clang fp contract(off)
  if (*A.done) {
    *A.skip = 1;
    *A.lam = 0.0;
    return false;
  }
  double best = INFINITY;
  for (int k = 0; k < A.nslot; ++k) {
    const double smax = A.smax[k];
    if (!(smax > 0.0)) continue;
    const double dtl = A.cfl * A.dx[k] / smax;
    const double cand = ldexp(dtl, k);
    if (cand < best) best = cand;
  }
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
    return false;
  }
  *A.lam = dt / A.dx[0];
  *A.t = last ? A.t_end : t + dt;
  *A.skip = 0;
  *A.nstep += 1;
  if (last) *A.done = 1;
  return true;
}

__global__ void finalize_kernel(FinalizeArgs A) {
#pragma clang fp contract(off)
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (!A.batch) {
    // one block of SMAX_SLOTS threads: each level's slots -> smax, then dt
    __shared__ double red[SMAX_SLOTS / 64];
    __shared__ int runs;
    const int tid = threadIdx.x;
    for (int k = 0; k < A.nslot; ++k) {
      const double v = wave_max(__longlong_as_double((long long)A.slots[int64_t(k) * SMAX_SLOTS + tid]));
      if ((tid & 63) == 0) red[tid >> 6] = v;
      __syncthreads();
      if (tid == 0) {
        double r = red[0];
        for (int w = 1; w < SMAX_SLOTS / 64; ++w) r = fmax(r, red[w]);
        A.smax[k] = r;
      }
      __syncthreads();
    }
    if (tid == 0) runs = finalize_dt(A) ? 1 : 0;
    __syncthreads();
    if (runs)
      for (int k = 0; k < A.nslot; ++k) A.slots[int64_t(k) * SMAX_SLOTS + tid] = 0ull;
  } else {
    if (i >= A.nslot) return;
    const double smax = A.smax[i];
    const double dx = A.dx_box[i];
    const double dt = A.cfl * dx / smax;
    A.lam[i] = dt / dx;
    A.t[i] = A.t[i] + dt;
    if (i == 0) *A.nstep += 1;
  }
}

int launch_finalize(const FinalizeArgs& a, void* stream) {
  if (!a.batch) {
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(SMAX_SLOTS), 0, (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  hipLaunchKernelGGL(finalize_kernel, dim3(unsigned((a.nslot + 255) / 256)), dim3(256), 0, (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
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
                              const uint8_t* __restrict__ refined, double vol, int nv, double* __restrict__ partial) {
  __shared__ double red[256];
  const int64_t ncell = n_oct * 8;
  const int64_t per = (ncell + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = int64_t(blockIdx.x) * per;
  const int64_t i1 = (i0 + per < ncell) ? i0 + per : ncell;
  for (int v = 0; v < nv; ++v) {
    double acc = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
      if ((refined[i >> 3] >> (i & 7)) & 1) continue;
      acc += U[v * plane + i] * vol;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[v * TOT_BLOCKS + blockIdx.x] += red[0];
    __syncthreads();
  }
}

__global__ void totals_final_kernel(const double* __restrict__ partial, int nparts, int nv, double* out) {
  __shared__ double red[256];
  for (int v = 0; v < nv; ++v) {
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

int launch_totals(const double* U, int64_t plane, int64_t n_oct, const uint8_t* refined, double vol, int nv,
                  double* partial, int nblocks, void* stream) {
  if (n_oct == 0) return 0;
  hipLaunchKernelGGL(totals_kernel, dim3(nblocks), dim3(256), 0, (hipStream_t)stream, U, plane, n_oct, refined, vol,
                     nv, partial);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int launch_totals_final(const double* partial, int nparts, int nv, double* out, void* stream) {
  hipLaunchKernelGGL(totals_final_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, partial, nparts, nv, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// Regrid remap: kept octs copy their state, new octs take the MinMod-linear
// interpolation of their parent cell (the ghost formula).
// ---------------------------------------------------------------------------
__global__ void regrid_remap_kernel(const int32_t* __restrict__ src_old, const int32_t* __restrict__ src7,
                                    int64_t n_new, const double* __restrict__ Uold, int64_t pold,
                                    const double* __restrict__ Uc, int64_t pc, double* __restrict__ Unew,
                                    int64_t pnew, int nv) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_new * 8) return;
  const int64_t k = i >> 3;
  const int c = int(i & 7);
  const int32_t so = src_old[k];
  if (so >= 0) {
    for (int v = 0; v < nv; ++v) Unew[v * pnew + i] = Uold[v * pold + int64_t(so) * 8 + c];
    return;
  }
  const double sx = (c & 1) ? 0.25 : -0.25, sy = (c & 2) ? 0.25 : -0.25, sz = (c & 4) ? 0.25 : -0.25;
  int32_t src[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) src[j] = src7[7 * k + j];
  for (int v = 0; v < nv; ++v) {
    double val[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) val[j] = Uc[v * pc + src[j]];
    const double q = val[0];
    const double mx = mmod(q - val[1], val[2] - q);
    const double my = mmod(q - val[3], val[4] - q);
    const double mz = mmod(q - val[5], val[6] - q);
    Unew[v * pnew + i] = q + (sx * mx + sy * my + sz * mz);
  }
}

int launch_regrid_remap(const int32_t* src_old, const int32_t* src7, int64_t n_new, const double* Uold, int64_t pold,
                        const double* Uc, int64_t pc, double* Unew, int64_t pnew, int nv, void* stream) {
  if (n_new == 0) return 0;
  const int64_t n = n_new * 8;
  hipLaunchKernelGGL(regrid_remap_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     src_old, src7, n_new, Uold, pold, Uc, pc, Unew, pnew, nv);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// Super-tiles: the aligned 4x4x4-oct blocks (8^3 cells) of a level, each
// assembled from the level's small tiles (aligned 2x2x2-oct blocks) inside
// it.  Small tiles are in Hilbert order, and the Hilbert curve runs through
// an aligned block before leaving it, so the small tiles of one block are
// consecutive in the list.  A super-tile's 6x6x6 oct neighbourhood is the
// union of its small tiles' 4x4x4 neighbourhoods: two tables that both hold
// a position hold the same oct (or ghost oct), and a position that none
// holds is read by no cell that is updated.
// ---------------------------------------------------------------------------
constexpr int SMALL_TAB = 64, SUPER_TAB = 216;

// Block key: block coordinates (21 bits each) or, in a batch of boxes, the
// box (from bit 45) and the block coordinates in the box (15 bits each).
__device__ __forceinline__ uint64_t pack_block(int64_t x, int64_t y, int64_t z, int box) {
  if (box < 0) return uint64_t(x) | (uint64_t(y) << 21) | (uint64_t(z) << 42);
  return uint64_t(x) | (uint64_t(y) << 15) | (uint64_t(z) << 30) | (uint64_t(box) << 45);
}
__device__ __forceinline__ void unpack_block(uint64_t b, bool batch, int64_t o[3], int& box) {
  if (!batch) {
    o[0] = int64_t(b & 0x1FFFFF);
    o[1] = int64_t((b >> 21) & 0x1FFFFF);
    o[2] = int64_t(b >> 42);
    box = -1;
  } else {
    o[0] = int64_t(b & 0x7FFF);
    o[1] = int64_t((b >> 15) & 0x7FFF);
    o[2] = int64_t((b >> 30) & 0x7FFF);
    box = int(b >> 45);
  }
}

// Per small tile: the key of its 4x4x4-oct block and its position (0..7)
// inside the block, from one of its own octs (a tile holds at least one,
// and its 2x2x2 core slots of the table hold every present one).
__global__ void super_key_kernel(const int32_t* __restrict__ tab, int32_t n_tile, const int32_t* __restrict__ oc,
                                 int64_t n_oct, const int32_t* __restrict__ tile_box, uint64_t* __restrict__ skey,
                                 int32_t* __restrict__ ssub, int32_t* __restrict__ start) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_tile) return;
  int32_t e = -1;
  for (int c = 0; c < 8 && e < 0; ++c) {
    const int slot = 21 + (c & 1) + 4 * ((c >> 1) & 1) + 16 * (c >> 2);
    const int32_t v = tab[t * SMALL_TAB + slot];
    if (v >= 0 && v < n_oct) e = v;
  }
  start[t] = 0;
  if (e < 0) {
    // every tile the mesh builders make holds a real oct; a tile without one
    // would be a builder error: it gets a block of its own
    skey[t] = ~uint64_t(t);
    ssub[t] = 0;
    return;
  }
  const int64_t bx = oc[3 * int64_t(e)] & ~1, by = oc[3 * int64_t(e) + 1] & ~1, bz = oc[3 * int64_t(e) + 2] & ~1;
  skey[t] = pack_block(bx >> 2, by >> 2, bz >> 2, tile_box ? tile_box[t] : -1);
  ssub[t] = int32_t(((bx >> 1) & 1) | (((by >> 1) & 1) << 1) | (((bz >> 1) & 1) << 2));
}

__global__ void super_start_kernel(const uint64_t* __restrict__ skey, int32_t n_tile, int32_t* __restrict__ start) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n_tile) start[t] = (t == 0 || skey[t] != skey[t - 1]) ? 1 : 0;
}

// sub[s][8]: the small tile at each position of super-tile s (or -1), and
// the block key of every super-tile.
__global__ void super_sub_kernel(const uint64_t* __restrict__ skey, const int32_t* __restrict__ ssub,
                                 const int32_t* __restrict__ start, const int32_t* __restrict__ excl, int32_t n_tile,
                                 int32_t* __restrict__ sub, uint64_t* __restrict__ sblock) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_tile) return;
  const int32_t s = excl[t] + start[t] - 1;
  sub[int64_t(s) * 8 + ssub[t]] = int32_t(t);
  if (start[t]) sblock[s] = skey[t];
}

// One thread per (super-tile, slot of its 6x6x6 neighbourhood); the slot-0
// thread also writes the super-tile's flags: outflow faces it touches, and
// the cells past the domain's high side per axis.
__global__ void super_table_kernel(const int32_t* __restrict__ tab, const int32_t* __restrict__ sub,
                                   const uint64_t* __restrict__ sblock, int32_t n_super, SuperDom D,
                                   int32_t* __restrict__ stab, uint32_t* __restrict__ stflag) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(n_super) * SUPER_TAB) return;
  const int64_t s = i / SUPER_TAB;
  const int slot = int(i % SUPER_TAB);
  const int px = slot % 6 - 1, py = (slot / 6) % 6 - 1, pz = slot / 36 - 1;
  int32_t v = -1;
  for (int c = 0; c < 8; ++c) {
    const int32_t t = sub[s * 8 + c];
    if (t < 0) continue;
    const int qx = px - 2 * (c & 1), qy = py - 2 * ((c >> 1) & 1), qz = pz - 2 * (c >> 2);
    if (qx < -1 || qx > 2 || qy < -1 || qy > 2 || qz < -1 || qz > 2) continue;
    const int32_t e = tab[int64_t(t) * SMALL_TAB + (qx + 1) + 4 * (qy + 1) + 16 * (qz + 1)];
    v = e > v ? e : v;
  }
  stab[i] = v;
  if (slot == 0) {
    int64_t o[3];
    int box;
    unpack_block(sblock[s], D.box_noct != nullptr, o, box);
    uint32_t fl = 0;
    int cut[3];
    for (int a = 0; a < 3; ++a) {
      o[a] *= 4;
      const int64_t n = D.box_noct ? D.box_noct[3 * int64_t(box) + a] : D.noct[a];
      if (o[a] == 0 && D.bc[2 * a] == RY_BC_OUTFLOW) fl |= (1u << (2 * a));
      if (o[a] + 4 >= n && D.bc[2 * a + 1] == RY_BC_OUTFLOW) fl |= (2u << (2 * a));
      const int64_t past = o[a] + 4 - n;
      cut[a] = past > 0 ? int(2 * past) : 0;
    }
    stflag[s] = fl | (uint32_t(cut[0]) << CL_CUT_SHIFT) | (uint32_t(cut[1]) << (CL_CUT_SHIFT + 3)) |
                (uint32_t(cut[2]) << (CL_CUT_SHIFT + 6));
  }
}

int super_table_slots() { return SUPER_TAB; }

// Batched boxes: the first super-tile of every box (super-tiles come box by
// box), then each super-tile's box and partial slot in its box's segment.
__global__ void super_first_kernel(const uint64_t* __restrict__ sblock, int32_t n_super, int32_t* __restrict__ sfirst,
                                   int32_t* __restrict__ sbox) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n_super) return;
  const int box = int(sblock[s] >> 45);
  sbox[s] = box;
  if (s == 0 || int(sblock[s - 1] >> 45) != box) sfirst[box] = int32_t(s);
}
__global__ void super_part_kernel(const int32_t* __restrict__ sbox, int32_t n_super, const int64_t* __restrict__ seg_off,
                                  const int32_t* __restrict__ sfirst, int32_t* __restrict__ spart) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n_super) return;
  const int box = sbox[s];
  spart[s] = int32_t(seg_off[box] + (s - sfirst[box]));
}

int launch_super_boxes(const uint64_t* sblock, int32_t n_super, const int64_t* seg_off, int32_t* sfirst,
                       int32_t* sbox, int32_t* spart, void* stream) {
  if (n_super == 0) return 0;
  const dim3 g(unsigned((n_super + 255) / 256)), b(256);
  hipLaunchKernelGGL(super_first_kernel, g, b, 0, (hipStream_t)stream, sblock, n_super, sfirst, sbox);
  hipLaunchKernelGGL(super_part_kernel, g, b, 0, (hipStream_t)stream, sbox, n_super, seg_off, sfirst, spart);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_super_keys(const int32_t* tab, int32_t n_tile, const int32_t* oc, int64_t n_oct, const SuperDom& D,
                      uint64_t* skey, int32_t* ssub, int32_t* start, void* stream) {
  if (n_tile == 0) return 0;
  const dim3 g(unsigned((n_tile + 255) / 256)), b(256);
  hipLaunchKernelGGL(super_key_kernel, g, b, 0, (hipStream_t)stream, tab, n_tile, oc, n_oct, D.tile_box, skey, ssub,
                     start);
  hipLaunchKernelGGL(super_start_kernel, g, b, 0, (hipStream_t)stream, skey, n_tile, start);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_super_tables(const int32_t* tab, const uint64_t* skey, const int32_t* ssub, const int32_t* start,
                        const int32_t* excl, int32_t n_tile, int32_t n_super, const SuperDom& D, int32_t* sub,
                        uint64_t* sblock, int32_t* stab, uint32_t* stflag, void* stream) {
  if (n_tile == 0 || n_super == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  const int64_t nsub = int64_t(n_super) * 8;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(unsigned((nsub + 255) / 256)), dim3(256), 0, st, sub, nsub, -1);
  hipLaunchKernelGGL(super_sub_kernel, dim3(unsigned((n_tile + 255) / 256)), dim3(256), 0, st, skey, ssub, start,
                     excl, n_tile, sub, sblock);
  const int64_t n = int64_t(n_super) * SUPER_TAB;
  hipLaunchKernelGGL(super_table_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, tab, sub, sblock, n_super,
                     D, stab, stflag);
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
