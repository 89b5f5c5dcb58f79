// Internal declarations shared by the host side (mesh.cpp, api.cpp) and the
// HIP kernels (kernels.hip) of the octree hydro library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ry.h"

namespace ry {

constexpr int NVAR = 5;            // hydro variables; passive scalars follow them
constexpr int NVMAX = NVAR + RY_MAX_SCALARS;
constexpr int TILE_TAB = 64;       // 4x4x4 oct positions around a 2x2x2-oct tile
// Slots per level of the maximum signal speed fused into the hydro update:
// tile t takes an atomic maximum on slot t % SMAX_SLOTS, so that no single
// address takes every tile's atomic.
constexpr int SMAX_SLOTS = 256;
// persistent-kernel work queues: 8 counters (one per XCD), 128 B apart so
// that no two share a cache line
constexpr int QUEUE_STRIDE = 32;
// flux registers per oct: [face 6][variable nv][substep 2]
constexpr int reg_per_oct(int nv) { return 6 * nv * 2; }

// Tile flag bits: outflow clamping at the domain faces touched by the tile
// (bits 0-5), and per axis (3 bits each from CL_CUT_SHIFT, x then y then z)
// the number of the tile's cells that lie past the domain's high side (0 for
// a tile inside the domain; even, below the tile edge): those cells are not
// updated, and an outflow face clamps to the last cell before them.
enum : uint32_t { CL_LOX = 1, CL_HIX = 2, CL_LOY = 4, CL_HIY = 8, CL_LOZ = 16, CL_HIZ = 32, CL_ANY = 63 };
constexpr int CL_CUT_SHIFT = 8;
inline uint32_t tile_cut_bits(int cx, int cy, int cz) {
  return (uint32_t(cx) << CL_CUT_SHIFT) | (uint32_t(cy) << (CL_CUT_SHIFT + 3)) | (uint32_t(cz) << (CL_CUT_SHIFT + 6));
}

// ---------------------------------------------------------------- host mesh
struct OctIndex {
  // open addressing: packed coordinates -> oct index
  std::vector<uint64_t> slot_key;
  std::vector<int32_t> slot_val;
  uint64_t mask = 0;
  void build(const std::vector<int32_t>& x, const std::vector<int32_t>& y, const std::vector<int32_t>& z);
  int32_t find(int64_t x, int64_t y, int64_t z) const;
};

struct HostLevel {
  int64_t n = 0;                     // octs
  std::vector<uint64_t> key;         // Hilbert keys, ascending
  std::vector<int32_t> ox, oy, oz;   // oct coordinates
  std::vector<uint8_t> refined;      // bit c: cell c refined
  std::vector<double> U;             // nv planes of 8n
  OctIndex index;
};

struct DomainSpec {
  int32_t lmin = 0, lmax = 0;
  int32_t nbase[3] = {0, 0, 0};
  int32_t bc[6] = {0, 0, 0, 0, 0, 0};
  int32_t refine = 0;
  double refine_param = 0.0;
  int nv = NVAR;                     // 5 + passive scalars
  int hbits0 = 0;                    // Hilbert bits per axis at lmin
  int64_t ncell(int l, int a) const { return (int64_t)nbase[a] << (l - lmin); }
  int64_t noct(int l, int a) const { return ncell(l, a) / 2; }
};

// Hilbert key of oct coordinates with `bits` bits per axis (Skilling 2004,
// transpose form; x is the most significant axis of each 3-bit group).
__host__ __device__ inline uint64_t hilbert3(int bits, uint32_t x, uint32_t y, uint32_t z) {
  uint32_t a[3] = {x, y, z};
  if (bits <= 0) return 0;
  const uint32_t top = 1u << (bits - 1);
  for (uint32_t q = top; q > 1; q >>= 1) {
    const uint32_t low = q - 1;
    for (int i = 0; i < 3; ++i) {
      if (a[i] & q) {
        a[0] ^= low;
      } else {
        const uint32_t swap = (a[0] ^ a[i]) & low;
        a[0] ^= swap;
        a[i] ^= swap;
      }
    }
  }
  a[1] ^= a[0];
  a[2] ^= a[1];
  uint32_t flip = 0;
  for (uint32_t q = top; q > 1; q >>= 1)
    if (a[2] & q) flip ^= (q - 1);
  for (int i = 0; i < 3; ++i) a[i] ^= flip;
  uint64_t key = 0;
  for (int b = bits - 1; b >= 0; --b) {
    key = (key << 3) | (uint64_t((a[0] >> b) & 1u) << 2) | (uint64_t((a[1] >> b) & 1u) << 1) |
          uint64_t((a[2] >> b) & 1u);
  }
  return key;
}

// Device-side description of one level, produced by the host builder.
struct LevelTables {
  int64_t n_oct = 0, n_ghost = 0;
  int64_t n_leaf = 0;
  int32_t n_tile = 0;
  std::vector<int32_t> tab;          // n_tile * 64 ext indices, -1 = unused
  std::vector<uint32_t> tflag;       // n_tile
  std::vector<uint8_t> refined_ext;  // n_oct + n_ghost
  std::vector<int32_t> child;        // 8 * n_oct, child oct at l+1 or -1
  std::vector<int32_t> parent_cell;  // n_oct: cell index at l-1 (l > lmin)
  std::vector<int64_t> gsrc;         // n_ghost * 7: (level_up << 48) | cell index
  std::vector<int32_t> tile_box;     // batch only
};

// Builds the refined octree (refinement, neighbour rule, Hilbert order,
// fill, restriction). Returns an error string or empty.
std::string build_mesh(const DomainSpec& dom, const double* U_base, ry_fill_fn fill, void* user,
                       std::vector<HostLevel>& levels);
// One level of a regrid: flags of level l (densities rho, 8 per oct) by the
// build's criterion and neighbour rule replace C.refined; F_new gets the
// children of the refined cells in Hilbert order; per F_new oct, src_old is
// its index in F_old (kept) or -1 (new), and for new octs src7 holds the 7
// level-l cells (Q, -x, +x, -y, +y, -z, +z) its values are interpolated from.
std::string regrid_level(const DomainSpec& d, int l, HostLevel& C, const std::vector<double>& rho,
                         const HostLevel& F_old, HostLevel& F_new, std::vector<int32_t>& src_old,
                         std::vector<int32_t>& src7, int64_t& created, int64_t& destroyed);
// Builds tile tables, ghost lists, child/parent maps for every level.
std::string build_tables(const DomainSpec& dom, const std::vector<HostLevel>& levels,
                         std::vector<LevelTables>& out);

// ------------------------------------------------------------- kernels
struct HydroArgs {
  const double* U;            // current state (ext octs), nv planes of 8*n_ext
  double* Un;                 // next state
  int64_t plane;              // 8 * n_ext
  int32_t n_oct;              // real octs: ext index < n_oct
  int32_t n_ext;              // octs + ghost octs (debug bounds checks)
  // ghost octs live only in the level's second state buffer, which follows
  // the first one in memory (nv planes later): reading through the first,
  // a ghost oct's index is shifted by ghost_adj = nv * n_ext octs; 0 when
  // the current buffer is the second one or the level has no ghosts
  int32_t ghost_adj;
  int32_t n_tile;
  const int32_t* tab;
  const uint32_t* tflag;
  const uint8_t* refined;     // n_ext
  const int32_t* child;       // 8 n_oct (nullptr when no finer level)
  const double* reg_fine;     // registers of level l+1
  double* reg_own;            // registers of level l (written when record_reg)
  int32_t substep;
  int32_t record_reg;
  double gamma, rho_floor, p_floor;
  double igm1;                // 1 / (gamma - 1)
  const double* lam_dev;      // device lambda (per box when tile_box != nullptr)
  double lam_host;            // used when lam_dev == nullptr
  const int32_t* tile_box;
  double* tile_smax;          // CFL epilogue: max signal speed per tile, nullptr = off
  const int32_t* tile_part;   // index of each tile's partial in tile_smax (nullptr: the tile index)
  unsigned long long* smax_bits;  // CFL epilogue: the level's SMAX_SLOTS slots of the maximum
                                  // signal speed (bit patterns of non-negative doubles, one
                                  // atomic max per tile); nullptr = off (else tile_smax)
  unsigned long long* floors;
  int32_t* err;
  const int32_t* skip;        // device flag: skip this launch's work
  unsigned int* queue;        // persistent mode: 8 per-XCD counters, QUEUE_STRIDE apart
};

struct GhostArgs {
  const double* src[RY_MAX_LEVELS];   // current U of level l-1-k at index k
  int64_t src_plane[RY_MAX_LEVELS];
  const int64_t* gsrc;
  int64_t n_ghost;
  int64_t n_oct;
  double* dst;                // the level's second state buffer (ghosts live there only)
  int64_t plane;
  int32_t nv;
  const int32_t* skip;
  // floor census of the ghost cells (once per parent step): activations of
  // the primitive conversion of each interpolated cell that an update reads
  // (a leaf cell of the level in its stencil); nullptr = off
  unsigned long long* floors;
  double gamma, rho_floor, p_floor;
  const uint32_t* gread;             // per ghost oct: bit c set when an update reads its cell c
  int32_t* err;                      // error word (debug bounds checks)
};

// launchers (kernels.hip)
int launch_hydro(const HydroArgs& a, int precision, int nscalar, const ry_tuning& t, int num_cu, void* stream);
// the hydro-only (nscalar = 0) part of launch_hydro (hydro.hip)
int launch_hydro_plain(const HydroArgs& a, int precision, const ry_tuning& t, int num_cu, void* stream);
// whether a hydro kernel exists for this precision / scalar count / tuning
bool hydro_tuning_supported(int precision, int nscalar, const ry_tuning& t);
int launch_ghost(const GhostArgs& a, void* stream);
// The ghost read masks of a level from its small-tile tables: for every
// ghost oct, bit c set when a leaf cell of a tile's core has the oct's cell
// c in its stencil (gread zeroed before, n_ghost entries; OR-accumulated).
int launch_ghost_read(const int32_t* tab, const uint32_t* tflag, const uint8_t* refined, int32_t n_tile,
                      int64_t n_oct, uint32_t* gread, void* stream);
int launch_restrict(const double* Uf, int64_t plane_f, int64_t n_fine, const int32_t* parent_cell,
                    double* Uc, int64_t plane_c, int nv, const int32_t* skip, int32_t* err, void* stream);
// Blocks of the CFL pass over n_oct octs (256 cells each): the number of
// partial maxima it writes.
inline int64_t cfl_blocks(int64_t n_oct) { return (8 * n_oct + 255) / 256; }

// Device index checks of a debug build (compiled with -DRY_DEBUG): an index
// outside its buffer sets bit ERR_BOUNDS of the error word, and the caller
// redirects the access to index 0 instead of making it; the next syncing
// call reports it.  A release build compiles the checks away.
constexpr int32_t ERR_NUMERIC = 1, ERR_BOUNDS = 2;
#ifdef RY_DEBUG
constexpr bool kDebugChecks = true;
#else
constexpr bool kDebugChecks = false;
#endif
__device__ __forceinline__ bool debug_in_bounds(bool ok, int32_t* err) {
  if constexpr (kDebugChecks) {
    if (!ok) {
      if (err) atomicOr(err, ERR_BOUNDS);
      return false;
    }
  }
  return true;
}
// The hydro kernel indexes a level's cells in 32 bits: its octs and ghost
// octs (8 cells each) and, on a level with ghost octs, the shift by
// nv * (octs + ghost octs) octs that reads a ghost oct from the second state
// buffer; all of it stays below 2^29 octs.
inline bool level_index_fits(int64_t n_oct, int64_t n_ghost, int nv) {
  const int64_t n_ext = n_oct + n_ghost;
  return (n_ghost > 0 ? (1 + int64_t(nv)) * n_ext : n_ext) < (int64_t(1) << 29);
}
// Launch failures that the launchers detect before any device call.
constexpr int LAUNCH_EXCEEDS_BUFFER = -2;
// per-block maxima of the signal speed over leaf cells -> part[0 ..
// cfl_blocks(n_oct)); part holds part_cap values: a grid that would write
// past them is refused (LAUNCH_EXCEEDS_BUFFER) before anything is launched
int launch_cfl(const double* U, int64_t plane, int64_t n_oct, const uint8_t* refined, double gamma,
               double rho_floor, double p_floor, double* part, int64_t part_cap, int32_t* err, void* stream);
// out[s] = max of part[off[s] .. off[s+1])
// per-segment maxima of part; with slots != nullptr also slot 0 of each
// segment's SMAX_SLOTS slots = the maximum, the others 0
int launch_seg_max(const double* part, const int64_t* off, int nseg, double* out, unsigned long long* slots,
                   void* stream);
struct FinalizeArgs {
  unsigned long long* slots;       // AMR: nslot x SMAX_SLOTS maxima, reduced into smax, then cleared
  double* smax;                    // per level (AMR) or per box (batch)
  int32_t nslot;
  double cfl;
  double dx[RY_MAX_LEVELS];        // AMR: dx of each level; batch: unused
  const double* dx_box;            // batch: dx per box
  double t_end;
  double* t;                       // AMR: 1 value; batch: per box
  double* lam;                     // AMR: 1 value; batch: per box
  int32_t* skip;
  int32_t* done;
  int32_t* nstep;
  int32_t batch;
};
int launch_finalize(const FinalizeArgs& a, void* stream);
int launch_zero_u32(unsigned int* p, int64_t n, void* stream);
int launch_zero_u64(unsigned long long* p, int64_t n, void* stream);
int launch_totals(const double* U, int64_t plane, int64_t n_oct, const uint8_t* refined, double vol, int nv,
                  double* partial, int nblocks, void* stream);
int launch_totals_final(const double* partial, int nparts, int nv, double* out, void* stream);
int launch_copy(const double* src, double* dst, int64_t n, void* stream);
// ---- super-tiles (kernels.hip): 4x4x4-oct blocks for the 8^3-cell tile ----
struct SuperDom {
  int64_t noct[3];                   // octs per axis of the level
  int32_t bc[6];
  // batched boxes: the box of every small tile and the octs per axis of
  // every box (3 per box); nullptr for a level of one domain
  const int32_t* tile_box;
  const int64_t* box_noct;
};
int super_table_slots();             // 6^3 oct neighbourhood entries per super-tile
// per small tile: its block key, its position in the block, block starts
// (start[t] = 1 where a new block begins; scan it for the block numbers)
int launch_super_keys(const int32_t* tab, int32_t n_tile, const int32_t* oc, int64_t n_oct, const SuperDom& D,
                      uint64_t* skey, int32_t* ssub, int32_t* start, void* stream);
// the super-tiles' tables and flags (excl = exclusive scan of start; sub:
// n_super * 8 scratch ints; sblock: n_super scratch keys)
int launch_super_tables(const int32_t* tab, const uint64_t* skey, const int32_t* ssub, const int32_t* start,
                        const int32_t* excl, int32_t n_tile, int32_t n_super, const SuperDom& D, int32_t* sub,
                        uint64_t* sblock, int32_t* stab, uint32_t* stflag, void* stream);
// batched boxes: the box of every super-tile and the index of its CFL
// partial inside its box's segment (seg_off: the boxes' segment offsets;
// sfirst: nbox scratch ints)
int launch_super_boxes(const uint64_t* sblock, int32_t n_super, const int64_t* seg_off, int32_t* sfirst,
                       int32_t* sbox, int32_t* spart, void* stream);

}  // namespace ry
