// Declarations of the device regrid (regrid.hip; the state remap in
// kernels.hip), used by the context's regrid driver (api.cpp).
#pragma once

#include <cstdint>

#include "ry_internal.h"

namespace ry {

// ---- device regrid (regrid.hip) ----
// What the device regrid reads of one level: sorted Hilbert keys, oct
// coordinates (x, y, z interleaved), counts.
struct LevelView {
  const uint64_t* key;
  const int32_t* oc;
  int64_t n;
  int32_t bits;                      // Hilbert bits per axis at this level
  int32_t noct[3];                   // octs per axis at this level
  // optional position hash of the level's octs (launch_pos_hash); null:
  // octs are found by binary search of their key
  const unsigned long long* hash;
  uint64_t hmask;                    // hash entries - 1 (a power of two minus one)
};
// Hash entries (64 bytes each, one per aligned 2x2x2 block of oct positions
// holding an oct) for n_blocks such blocks: a power of two >= 2 n_blocks, so
// that at most half the entries are used.
uint64_t pos_hash_entries(int64_t n_blocks);
// Position hash of a level's n octs (key: their sorted Hilbert keys; oc: 3
// int32 per oct): tab holds pos_hash_entries(blocks) entries of 8 unsigned
// long long; cleared and filled on the stream.  A table too small for the
// level's blocks sets bit 4 of *err.
int launch_pos_hash(const uint64_t* key, const int32_t* oc, int64_t n, unsigned long long* tab, uint64_t entries,
                    int32_t* err, void* stream);
struct RegridDom {
  int32_t bc[6];
  int32_t lmin;
  int32_t refine;
  double refine_param;
};
// Refinement flags of level l (rho: the density plane), their counts (cnt)
// and has = 1 where an oct has a flagged cell.  The neighbour rule reads the
// level's tile presence masks when given (pres; tile_of: each oct's tile),
// else takes every position as holding an oct when complete != 0, else
// looks the octs up; the gradient criterion takes the face neighbours from
// the tile tables (tab, n_oct) when given, else looks them up.
struct FlagTiles {
  const int32_t* tile_of;
  const unsigned long long* pres;
  const int32_t* tab;
  int64_t n_oct;
  int32_t complete;
};
int launch_regrid_flags(const LevelView& L, const RegridDom& D, int l, const double* rho, const FlagTiles& T,
                        uint8_t* flag, int32_t* cnt, int32_t* has, void* stream);
// exclusive scan of n int32 (tmp: scan_tmp_ints(n) ints; the total lands in
// tmp[scan_tmp_ints(n) - 1])
int scan_tmp_ints(int64_t n);
int launch_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, void* stream);
// The old tree around level C: old_of[o] the index in the old level of C's
// oct o, or -1 when it is new (null: C's octs are the old ones, unchanged);
// old_child the old level's child map (8 per oct: the child oct or -1; null
// when the old level had no children).
struct OldTree {
  const int32_t* old_of;
  const int32_t* old_child;
};
// The child level's tiles (one per parent oct with children): toff the
// exclusive scan of the flag kernel's has (a parent's tile), n_tile their
// number; written: tile_of (the tile of each child oct), tfirst (each
// tile's first child oct, n_tile + 1 entries) and fresh (1 for a child oct
// not in the old level, else 0).
struct ChildTiles {
  const int32_t* toff;
  int32_t n_tile;
  int32_t* tile_of;
  int32_t* tfirst;
  uint8_t* fresh;
};
// Children of level C's flagged cells (one thread per oct of C); kept gets
// the number of children found in the old child level added.
int launch_regrid_children(const LevelView& C, const OldTree& T, const RegridDom& D, int fbits,
                           const uint8_t* flag, const int32_t* off, const ChildTiles& CT, uint64_t* nkey,
                           int32_t* noc, int32_t* parent, int32_t* child, int32_t* src_old, int32_t* src7,
                           int32_t* err, unsigned long long* kept, void* stream);
// pres: per tile, bit slot set when the slot's position holds an oct or lies
// outside an outflow face
int launch_tile_table(const LevelView& L, const RegridDom& D, const int32_t* first, int32_t n_tile, int32_t* tab,
                      uint32_t* tflag, int32_t* miss, unsigned long long* pres, void* stream);
int launch_missing_list(const LevelView& L, const int32_t* first, int32_t n_tile, const int32_t* miss,
                        const int32_t* midx, uint64_t* mpos, int32_t* mentry, void* stream);
int launch_ghost_numbering(const uint64_t* mpos, const int32_t* mentry, int64_t nm, unsigned long long* hkey,
                           int32_t* hval, uint64_t hsize, int32_t* owner, int32_t* gidx, int32_t* scan_tmp,
                           int64_t n_oct, int32_t* tab, int32_t* gpos, void* stream);
int launch_ghost_sources(const LevelView* coarse_dev, int ncoarse, const RegridDom& D, const int32_t* gpos,
                         int64_t n_ghost, int64_t* gsrc, int32_t* err, void* stream);
int launch_refined_ext(const uint8_t* flag, int64_t n, int64_t n_ext, uint8_t* out, void* stream);

// Restriction after a regrid of the fine octs marked in dirty_f only (the
// same ordered 8-child means as launch_restrict); each marks its parent oct
// in dirty_c when given.  A refined cell whose children neither are new nor
// had a cell restricted again keeps the mean it already holds.
int launch_restrict_dirty(const double* Uf, int64_t pf, int64_t nf, const int32_t* parent, double* Uc, int64_t pc,
                          int nv, const uint8_t* dirty_f, uint8_t* dirty_c, int32_t* err, void* stream);
// Regrid state remap of one level: for new oct k, cell c, variable v: a kept
// oct copies Uold[v*pold + 8*src_old[k] + c]; a new one takes the MinMod-
// linear interpolation of the level-l cells src7[7k..7k+6] of Uc (plane pc).
int launch_regrid_remap(const int32_t* src_old, const int32_t* src7, int64_t n_new, const double* Uold, int64_t pold,
                        const double* Uc, int64_t pc, double* Unew, int64_t pnew, int nv, void* stream);
int totals_blocks();
int hydro_max_tiles_per_wg();

}  // namespace ry
