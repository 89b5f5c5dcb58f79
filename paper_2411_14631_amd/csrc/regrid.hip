// Device-side mesh work of the regrid between coarse steps: refinement
// flags, the child level in Hilbert order with its kept / new mapping and
// interpolation sources, and the per-level device tables (tiles, the 4x4x4
// oct neighbourhood of each tile, ghost octs and their sources).
//
// Octs of a level are looked up in a hash of their positions built at the
// start of the level's turn (binary search of the sorted Hilbert keys when a
// level has no hash); the refinement flags read most of what they need from
// the tile tables instead.  Children of a level-l oct occupy a contiguous,
// ordered run of level-l+1 keys (key_{l+1} >> 3 == key_l), so the child level
// comes out sorted from a scan over the parent octs: no global sort, and each
// parent's children are one tile of the child level.  Surviving children are
// read from the old tree (the old parent's child map).  Ghost octs are
// numbered in the order the host builder numbers them (first use over tiles
// and slots), found with a device hash of positions.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ry_internal.h"
#include "regrid.h"

namespace ry {

namespace {

__device__ __forceinline__ int64_t find_key(const uint64_t* __restrict__ key, int64_t n, uint64_t k) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return (lo < n && key[lo] == k) ? lo : -1;
}

// Packed oct position, 21 bits per axis.
__device__ __forceinline__ uint64_t pack_pos(int64_t x, int64_t y, int64_t z) {
  return uint64_t(x) | (uint64_t(y) << 21) | (uint64_t(z) << 42);
}

// MurmurHash3's 64-bit finaliser (xor-shift / multiply, two rounds).
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// Position hash of a level: one 64-byte entry per aligned 2x2x2 block of
// oct positions that holds an oct, {packed block position, the indices of
// the 8 octs at child position (x & 1) + 2 (y & 1) + 4 (z & 1), -1 where
// absent}; an empty entry is all ones (no packed position has bit 63 set).
// Open addressing with linear probing; at most half the entries are used,
// so a probe sequence ends at the block or at an empty entry (the loops
// also stop after visiting every entry, and report a full table).
constexpr unsigned long long kEmptyPos = ~0ull;
constexpr int kBlockWords = 8;   // unsigned long long per entry

struct alignas(64) BlockEntry {
  unsigned long long key;
  int32_t oct[8];
  unsigned long long pad[3];
};
static_assert(sizeof(BlockEntry) == kBlockWords * 8, "one 64-byte entry per block");

__device__ __forceinline__ const BlockEntry* block_entry(const unsigned long long* tab, uint64_t s) {
  return reinterpret_cast<const BlockEntry*>(tab) + s;
}

// The rest of a probe sequence for block key k, child position c, whose
// entry at slot s held key ek and oct eo.
__device__ __forceinline__ int64_t hash_probe_on(const unsigned long long* tab, uint64_t mask, uint64_t k, int c,
                                                 uint64_t s, unsigned long long ek, int32_t eo) {
  for (uint64_t p = 0; ek != k && ek != kEmptyPos && p <= mask; ++p) {
    s = (s + 1) & mask;
    ek = block_entry(tab, s)->key;
    eo = block_entry(tab, s)->oct[c];
  }
  return ek == k ? int64_t(eo) : -1;
}

__device__ __forceinline__ uint64_t block_key(int64_t x, int64_t y, int64_t z) {
  return pack_pos(x >> 1, y >> 1, z >> 1);
}
__device__ __forceinline__ int child_pos(int64_t x, int64_t y, int64_t z) {
  return int((x & 1) | ((y & 1) << 1) | ((z & 1) << 2));
}

__device__ __forceinline__ int64_t hash_lookup(const unsigned long long* tab, uint64_t mask, int64_t x, int64_t y,
                                               int64_t z) {
  const uint64_t k = block_key(x, y, z);
  const int c = child_pos(x, y, z);
  const uint64_t s = fmix64(k) & mask;
  return hash_probe_on(tab, mask, k, c, s, block_entry(tab, s)->key, block_entry(tab, s)->oct[c]);
}

// Build, first pass: the first oct of each block (in key order; siblings
// share key >> 3) enters the block's key.
__global__ void pos_hash_key_kernel(const uint64_t* __restrict__ key, const int32_t* __restrict__ oc, int64_t n,
                                    unsigned long long* tab, uint64_t mask, int32_t* __restrict__ err) {
  const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (o >= n || (o > 0 && (key[o] >> 3) == (key[o - 1] >> 3))) return;
  const unsigned long long k = block_key(oc[3 * o], oc[3 * o + 1], oc[3 * o + 2]);
  uint64_t s = fmix64(k) & mask;
  for (uint64_t p = 0; p <= mask; ++p) {
    const unsigned long long prev = atomicCAS(&tab[kBlockWords * s], kEmptyPos, k);
    if (prev == kEmptyPos || prev == k) return;
    s = (s + 1) & mask;
  }
  atomicOr(err, 4);   // table full
}

// Build, second pass: every oct writes its index into its block's entry
// (read by later launches only).
__global__ void pos_hash_oct_kernel(const int32_t* __restrict__ oc, int64_t n, unsigned long long* tab,
                                    uint64_t mask, int32_t* __restrict__ err) {
  const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const int64_t x = oc[3 * o], y = oc[3 * o + 1], z = oc[3 * o + 2];
  const unsigned long long k = block_key(x, y, z);
  uint64_t s = fmix64(k) & mask;
  for (uint64_t p = 0; p <= mask; ++p) {
    const unsigned long long e = tab[kBlockWords * s];
    if (e == k) {
      reinterpret_cast<BlockEntry*>(tab)[s].oct[child_pos(x, y, z)] = int32_t(o);
      return;
    }
    if (e == kEmptyPos) break;
    s = (s + 1) & mask;
  }
  atomicOr(err, 4);   // block not entered
}

// Integer oct position q of a level after the boundary rule (periodic
// wrap); false when q lies outside an outflow face.
__device__ __forceinline__ bool wrap_oct(const LevelView& L, const int32_t* bc, int64_t q[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t n = L.noct[a];
    if (q[a] < 0) {
      if (bc[2 * a] != RY_BC_PERIODIC) return false;
      q[a] = ((q[a] % n) + n) % n;
    } else if (q[a] >= n) {
      if (bc[2 * a + 1] != RY_BC_PERIODIC) return false;
      q[a] = q[a] % n;
    }
  }
  return true;
}

// Index of the oct at an in-domain position, -1 when there is none.
__device__ __forceinline__ int64_t find_oct(const LevelView& L, int64_t x, int64_t y, int64_t z) {
  if (L.hash) return hash_lookup(L.hash, L.hmask, x, y, z);
  return find_key(L.key, L.n, hilbert3(L.bits, uint32_t(x), uint32_t(y), uint32_t(z)));
}

// Oct at integer oct position q of a level after the boundary rule: returns
// its index, -1 when it does not exist, or -2 when q lies outside an
// outflow face (such positions count as existing; the caller clamps).
__device__ __forceinline__ int64_t oct_at(const LevelView& L, const int32_t* bc, int64_t qx, int64_t qy, int64_t qz) {
  int64_t q[3] = {qx, qy, qz};
  if (!wrap_oct(L, bc, q)) return -2;
  return find_oct(L, q[0], q[1], q[2]);
}

__device__ __forceinline__ int cell_bits(int64_t x, int64_t y, int64_t z) {
  return int((x & 1) | ((y & 1) << 1) | ((z & 1) << 2));
}

// Level-l cell index (8*oct + cell) of cell position p after the boundary
// rule (periodic wrap, outflow clamp); -1 when its oct does not exist.
__device__ __forceinline__ int64_t cell_at(const LevelView& L, const int32_t* bc, int64_t x, int64_t y, int64_t z) {
  int64_t p[3] = {x, y, z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t n = 2 * int64_t(L.noct[a]);
    if (p[a] < 0) p[a] = (bc[2 * a] == RY_BC_PERIODIC) ? ((p[a] % n) + n) % n : 0;
    else if (p[a] >= n) p[a] = (bc[2 * a + 1] == RY_BC_PERIODIC) ? p[a] % n : n - 1;
  }
  const int64_t o = find_oct(L, p[0] >> 1, p[1] >> 1, p[2] >> 1);
  return o < 0 ? -1 : o * 8 + cell_bits(p[0], p[1], p[2]);
}

// The six face-neighbour octs of oct o (-x, +x, -y, +y, -z, +z), as oct_at:
// index, -1 absent, -2 outside an outflow face.  With a hash, the six first
// probes are issued together.
__device__ __forceinline__ void face_neighbours(const LevelView& L, const int32_t* bc, int64_t ox, int64_t oy,
                                                int64_t oz, int32_t nb[6]) {
  if (!L.hash) {
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const int64_t st = (m & 1) ? 1 : -1;
      nb[m] = int32_t(oct_at(L, bc, ox + (m >> 1 == 0 ? st : 0), oy + (m >> 1 == 1 ? st : 0),
                             oz + (m >> 1 == 2 ? st : 0)));
    }
    return;
  }
  uint64_t key[6], slot[6];
  int cp[6];
  unsigned long long ek[6];
  int32_t eo[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int64_t st = (m & 1) ? 1 : -1;
    int64_t q[3] = {ox + (m >> 1 == 0 ? st : 0), oy + (m >> 1 == 1 ? st : 0), oz + (m >> 1 == 2 ? st : 0)};
    const bool in = wrap_oct(L, bc, q);
    key[m] = in ? block_key(q[0], q[1], q[2]) : kEmptyPos;   // all ones: outside
    cp[m] = child_pos(q[0], q[1], q[2]);
    slot[m] = fmix64(key[m]) & L.hmask;
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    ek[m] = block_entry(L.hash, slot[m])->key;
    eo[m] = block_entry(L.hash, slot[m])->oct[cp[m]];
  }
#pragma unroll
  for (int m = 0; m < 6; ++m)
    nb[m] = key[m] == kEmptyPos ? -2
                                : int32_t(hash_probe_on(L.hash, L.hmask, key[m], cp[m], slot[m], ek[m], eo[m]));
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Flags: the build's criterion under the 26-neighbour rule.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void regrid_flag_kernel(LevelView L, RegridDom D, int l,
                                                          const double* __restrict__ rho, FlagTiles T,
                                                          uint8_t* __restrict__ flag, int32_t* __restrict__ cnt,
                                                          int32_t* __restrict__ has) {
  const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (o >= L.n) return;
  const double mass_thr = D.refine_param * ldexp(1.0, 3 * (l - D.lmin));
  double rc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) rc[c] = rho[8 * o + c];
  uint32_t cand = 0;   // cells the criterion looks at further
#pragma unroll
  for (int c = 0; c < 8; ++c)
    if (D.refine == RY_REFINE_MASS ? rc[c] > mass_thr : D.refine == RY_REFINE_GRAD) cand |= 1u << c;
  uint8_t f = 0;
  if (cand) {
    const int64_t ox = L.oc[3 * o], oy = L.oc[3 * o + 1], oz = L.oc[3 * o + 2];
    const bool grad = D.refine == RY_REFINE_GRAD;
    // have: bit (dx+1) + 3(dy+1) + 9(dz+1) when the oct position at that
    // offset holds an oct or lies outside an outflow face; nb6: the face
    // neighbours (-x, +x, -y, +y, -z, +z) as oct_at, for the gradient
    uint32_t have = 0;
    int32_t nb6[6] = {-1, -1, -1, -1, -1, -1};
    if (T.pres) {
      // the oct sits at (1 + (ox & 1), ...) in its tile's 4x4x4 table
      const int32_t t = T.tile_of[o];
      const int px = 1 + int(ox & 1), py = 1 + int(oy & 1), pz = 1 + int(oz & 1);
      const unsigned long long q = T.pres[t] >> ((px - 1) + 4 * (py - 1) + 16 * (pz - 1));
#pragma unroll
      for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) have |= uint32_t((q >> (4 * dy + 16 * dz)) & 7u) << (3 * dy + 9 * dz);
      if (grad) {
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          const int st = (m & 1) ? 1 : -1, a = m >> 1;
          const int32_t v = T.tab[int64_t(t) * TILE_TAB + (px + (a == 0 ? st : 0)) + 4 * (py + (a == 1 ? st : 0)) +
                                  16 * (pz + (a == 2 ? st : 0))];
          // a present oct's face neighbours are all in the table: the oct,
          // a ghost / missing entry, or -1 outside an outflow face
          nb6[m] = (v >= 0 && v < T.n_oct) ? v : (v == -1 ? -2 : -1);
        }
      }
    } else if (T.complete) {
      have = (1u << 27) - 1;
      if (grad) face_neighbours(L, D.bc, ox, oy, oz, nb6);
    } else {   // a base level that does not hold every position: one lookup after another
      for (int j = 0; j < 27; ++j)
        if (j == 13 || oct_at(L, D.bc, ox + j % 3 - 1, oy + (j / 3) % 3 - 1, oz + j / 9 - 1) != -1) have |= 1u << j;
      if (grad) face_neighbours(L, D.bc, ox, oy, oz, nb6);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (!((cand >> c) & 1u)) continue;
      const int bx = c & 1, by = (c >> 1) & 1, bz = c >> 2;
      // the rule: the 2x2x2 octs at the cell's outer corner all exist
      uint32_t need = 0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int dx = (k & 1) ? (bx ? 1 : -1) : 0, dy = (k & 2) ? (by ? 1 : -1) : 0,
                  dz = (k & 4) ? (bz ? 1 : -1) : 0;
        need |= 1u << ((dx + 1) + 3 * (dy + 1) + 9 * (dz + 1));
      }
      if ((have & need) != need) continue;
      bool want = true;
      if (grad) {
#pragma clang fp contract(off)
        // the six face-neighbour cells (-1 and +1 along x, y, z): the other
        // cell of the oct along that axis, or a cell of the face-neighbour
        // oct on the cell's side (the cell itself past an outflow face)
        int64_t nc[6];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const int b = (c >> a) & 1;
            if (b != s) {
              nc[2 * a + s] = 8 * o + (c ^ (1 << a));
            } else {
              const int32_t e = nb6[2 * a + s];
              nc[2 * a + s] = e >= 0 ? 8 * int64_t(e) + (c ^ (1 << a)) : (e == -2 ? 8 * o + c : -1);
            }
          }
        if ((nc[0] | nc[1] | nc[2] | nc[3] | nc[4] | nc[5]) < 0) continue;
        const double gx = 0.5 * (rho[nc[1]] - rho[nc[0]]);
        const double gy = 0.5 * (rho[nc[3]] - rho[nc[2]]);
        const double gz = 0.5 * (rho[nc[5]] - rho[nc[4]]);
        const double th = D.refine_param;
        want = gx * gx + gy * gy + gz * gz > (th * rc[c]) * (th * rc[c]);
      }
      if (want) f |= uint8_t(1u << c);
    }
  }
  flag[o] = f;
  cnt[o] = __popc(uint32_t(f));
  has[o] = f != 0;
}

// ---------------------------------------------------------------------------
// Children of the refined cells (level l+1) in Hilbert order, their
// mapping to the old level l+1 and the interpolation sources of new octs.
// ---------------------------------------------------------------------------
// Last key digits of the 8 children of the oct at (px, py, pz), bits 3c..3c+2
// for child c (x + 2y + 4z), for a child level of `bits` bits per axis.  A
// child's key is its parent's key followed by one digit, so only the digit
// is missing.  In the transpose algorithm every decision (which axes swap,
// which flip) reads bits above the lowest one, and the lowest bit only
// moves between the axes or flips; so one pass over the parent's bits, with
// the lowest bit of each axis replaced by an 8-bit mask of its value in the
// 8 children (x: 0xAA, y: 0xCC, z: 0xF0) and the parent's bits shifted
// above it, carries all 8 children at once.  Needs bits + 7 <= 32.
__device__ __forceinline__ uint32_t child_digits(int bits, uint32_t px, uint32_t py, uint32_t pz) {
  uint32_t a[3] = {(px << 8) | 0xAAu, (py << 8) | 0xCCu, (pz << 8) | 0xF0u};
  const uint32_t top = 1u << (bits + 6);   // the parent's top bit
  for (uint32_t q = top; q > 0x80u; q >>= 1) {
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
  for (uint32_t q = top; q > 0x80u; q >>= 1)
    if (a[2] & q) flip ^= q - 1;
  uint32_t d = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c)
    d |= (((((a[0] ^ flip) >> c) & 1u) << 2) | ((((a[1] ^ flip) >> c) & 1u) << 1) | (((a[2] ^ flip) >> c) & 1u))
         << (3 * c);
  return d;
}

// Children of oct o; returns how many were found in the old level.
__device__ __forceinline__ int children_of(int64_t o, const LevelView& C, const OldTree& T, const RegridDom& D,
                                           int fbits, const uint8_t* __restrict__ flag,
                                           const int32_t* __restrict__ off, const ChildTiles& CT,
                                           uint64_t* __restrict__ nkey,
                                           int32_t* __restrict__ noc, int32_t* __restrict__ parent,
                                           int32_t* __restrict__ child, int32_t* __restrict__ src_old,
                                           int32_t* __restrict__ src7, int32_t* __restrict__ err) {
  const uint8_t f = flag[o];
  for (int c = 0; c < 8; ++c) child[8 * o + c] = -1;
  if (!f) return 0;
  const int64_t ox = C.oc[3 * o], oy = C.oc[3 * o + 1], oz = C.oc[3 * o + 2];
  const uint64_t pkey = C.key[o];
  const uint32_t dg = child_digits(fbits, uint32_t(ox), uint32_t(oy), uint32_t(oz));
  uint32_t fd = 0;   // digits of the flagged children: a child's rank among them is its output slot
#pragma unroll
  for (int c = 0; c < 8; ++c)
    if ((f >> c) & 1) fd |= 1u << ((dg >> (3 * c)) & 7u);
  // the flagged children in the old level (-1: new): an old child at this
  // position has an old parent at the parent's position, and is that old
  // parent's child at the same cell
  int32_t so8[8];
  const int64_t op = T.old_of ? T.old_of[o] : o;
  if (op >= 0 && T.old_child) {
    const int4 a = *reinterpret_cast<const int4*>(T.old_child + 8 * op);
    const int4 b = *reinterpret_cast<const int4*>(T.old_child + 8 * op + 4);
    so8[0] = a.x; so8[1] = a.y; so8[2] = a.z; so8[3] = a.w;
    so8[4] = b.x; so8[5] = b.y; so8[6] = b.z; so8[7] = b.w;
  } else {
#pragma unroll
    for (int c = 0; c < 8; ++c) so8[c] = -1;
  }
  const int64_t base = off[o];
  // the children are one tile of the child level: its first oct, and the
  // tile of each
  const int32_t tile = CT.toff[o];
  CT.tfirst[tile] = int32_t(base);
  if (tile + 1 == CT.n_tile) CT.tfirst[tile + 1] = int32_t(base + __popc(uint32_t(f)));
  int kept = 0;
  uint32_t fresh = 0;   // children not in the old level
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    if (!((f >> c) & 1)) continue;
    const uint32_t d = (dg >> (3 * c)) & 7u;
    const int64_t k = base + __popc(fd & ((1u << d) - 1u));
    const int64_t x = 2 * ox + (c & 1), y = 2 * oy + ((c >> 1) & 1), z = 2 * oz + ((c >> 2) & 1);
    nkey[k] = (pkey << 3) | uint64_t(d);
    CT.tile_of[k] = tile;
    noc[3 * k] = int32_t(x);
    noc[3 * k + 1] = int32_t(y);
    noc[3 * k + 2] = int32_t(z);
    parent[k] = int32_t(o * 8 + c);
    child[8 * o + c] = int32_t(k);
    src_old[k] = so8[c];
    CT.fresh[k] = so8[c] < 0;
    if (so8[c] >= 0) ++kept;
    else fresh |= 1u << c;
  }
  // interpolation sources of the new children: the parent cell Q and its
  // six face neighbours (cell_at's rule), each the other cell of the oct
  // along that axis or a cell of the face-neighbour oct on Q's side (Q
  // itself past an outflow face)
  if (fresh) {
    int32_t nb[6];
    face_neighbours(C, D.bc, ox, oy, oz, nb);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (!((fresh >> c) & 1)) continue;
      const int64_t k = base + __popc(fd & ((1u << ((dg >> (3 * c)) & 7u)) - 1u));
      const int64_t q = o * 8 + c;
      src7[7 * k] = int32_t(q);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          int64_t r;
          if (((c >> a) & 1) != s) {
            r = o * 8 + (c ^ (1 << a));
          } else {
            const int32_t e = nb[2 * a + s];
            r = e >= 0 ? 8 * int64_t(e) + (c ^ (1 << a)) : (e == -2 ? q : -1);
          }
          if (r < 0) {   // excluded by the neighbour rule; reported, read kept in bounds
            atomicOr(err, 1);
            r = q;
          }
          src7[7 * k + 1 + 2 * a + s] = int32_t(r);
        }
    }
  }
  return kept;
}

__global__ __launch_bounds__(256) void regrid_children_kernel(LevelView C, OldTree T, RegridDom D, int fbits,
                                       const uint8_t* __restrict__ flag, const int32_t* __restrict__ off,
                                       ChildTiles CT,
                                       uint64_t* __restrict__ nkey, int32_t* __restrict__ noc,
                                       int32_t* __restrict__ parent, int32_t* __restrict__ child,
                                       int32_t* __restrict__ src_old, int32_t* __restrict__ src7,
                                       int32_t* __restrict__ err, unsigned long long* __restrict__ kept) {
  const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int n = 0;
  if (o < C.n) n = children_of(o, C, T, D, fbits, flag, off, CT, nkey, noc, parent, child, src_old, src7, err);
  n = wave_sum(n);   // every lane of the wavefront takes part (blocks of whole wavefronts)
  if ((threadIdx.x & 63) == 0 && n) atomicAdd(kept, (unsigned long long)n);
}

// ---------------------------------------------------------------------------
// Exclusive scan of int32 counts (three passes: block scans, a scan of the
// block sums, block offsets).  tmp holds nblocks + 1 ints; *total gets the
// sum.
// ---------------------------------------------------------------------------
constexpr int SCAN_BLOCK = 1024;

__device__ __forceinline__ int32_t wave_incl_scan(int32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t* total) {
  __shared__ int32_t ws[SCAN_BLOCK / 64];
  const int32_t incl = wave_incl_scan(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) ws[w] = incl;
  __syncthreads();
  if (w == 0) {
    const int32_t s = (lane < SCAN_BLOCK / 64) ? ws[lane] : 0;
    const int32_t si = wave_incl_scan(s);
    if (lane < SCAN_BLOCK / 64) ws[lane] = si - s;
    if (lane == SCAN_BLOCK / 64 - 1) *total = si;
  }
  __syncthreads();
  return incl - v + ws[w];
}

__global__ __launch_bounds__(SCAN_BLOCK) void scan_blocks_kernel(const int32_t* __restrict__ in,
                                                                 int32_t* __restrict__ out, int64_t n,
                                                                 int32_t* __restrict__ bsum) {
  __shared__ int32_t tot;
  const int64_t i = int64_t(blockIdx.x) * SCAN_BLOCK + threadIdx.x;
  const int32_t v = (i < n) ? in[i] : 0;
  const int32_t e = block_excl_scan(v, &tot);
  if (i < n) out[i] = e;
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_BLOCK) void scan_sums_kernel(int32_t* __restrict__ bsum, int nb,
                                                               int32_t* __restrict__ total) {
  __shared__ int32_t tot;
  int32_t carry = 0;
  for (int b0 = 0; b0 < nb; b0 += SCAN_BLOCK) {
    const int i = b0 + threadIdx.x;
    const int32_t v = (i < nb) ? bsum[i] : 0;
    const int32_t e = block_excl_scan(v, &tot);
    __syncthreads();
    if (i < nb) bsum[i] = e + carry;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(SCAN_BLOCK) void scan_add_kernel(int32_t* __restrict__ out, int64_t n,
                                                              const int32_t* __restrict__ bsum) {
  const int64_t i = int64_t(blockIdx.x) * SCAN_BLOCK + threadIdx.x;
  if (i < n) out[i] += bsum[blockIdx.x];
}

// ---------------------------------------------------------------------------
// Tiles: octs sharing key >> 3 (on a refined level, the children of one
// parent oct: the children kernel lists them).
// ---------------------------------------------------------------------------
// One wavefront per tile, one lane per slot: the tile's 4x4x4 oct
// neighbourhood.  tab gets the oct index, -1 (not needed, or outside an
// outflow face) or -2 (missing: a ghost oct, numbered later); miss = 1 for
// missing entries; pres gets bit slot set when the position holds an oct or
// lies outside an outflow face (every slot looked up, needed or not: the
// refinement flags' neighbour rule reads the corners too).
__global__ void tile_table_kernel(LevelView L, RegridDom D, const int32_t* __restrict__ first, int32_t n_tile,
                                  int32_t* __restrict__ tab, uint32_t* __restrict__ tflag,
                                  int32_t* __restrict__ miss, unsigned long long* __restrict__ pres) {
  static_assert(TILE_TAB == 64, "one wavefront per tile");
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(n_tile) * TILE_TAB) return;   // whole wavefronts: blocks of whole wavefronts, 64 slots a tile
  const int t = int(i / TILE_TAB), slot = int(i % TILE_TAB);
  const int rx = slot % 4 - 1, ry_ = (slot / 4) % 4 - 1, rz = slot / 16 - 1;
  const int64_t o0 = first[t], o1 = first[t + 1];
  const int64_t bx = L.oc[3 * o0] & ~1, by = L.oc[3 * o0 + 1] & ~1, bz = L.oc[3 * o0 + 2] & ~1;
  bool needed = false;
  for (int64_t o = o0; o < o1 && !needed; ++o) {
    const int px = int(L.oc[3 * o] - bx), py = int(L.oc[3 * o + 1] - by), pz = int(L.oc[3 * o + 2] - bz);
    // a face or edge neighbour of a present oct (no stencil reads across an
    // oct's corner)
    const int ax = abs(rx - px), ay = abs(ry_ - py), az = abs(rz - pz);
    needed = ax <= 1 && ay <= 1 && az <= 1 && ax + ay + az <= 2;
  }
  if (slot == 0) {
    uint32_t fl = 0;
    if (bx == 0 && D.bc[0] == RY_BC_OUTFLOW) fl |= CL_LOX;
    if (bx + 2 == L.noct[0] && D.bc[1] == RY_BC_OUTFLOW) fl |= CL_HIX;
    if (by == 0 && D.bc[2] == RY_BC_OUTFLOW) fl |= CL_LOY;
    if (by + 2 == L.noct[1] && D.bc[3] == RY_BC_OUTFLOW) fl |= CL_HIY;
    if (bz == 0 && D.bc[4] == RY_BC_OUTFLOW) fl |= CL_LOZ;
    if (bz + 2 == L.noct[2] && D.bc[5] == RY_BC_OUTFLOW) fl |= CL_HIZ;
    tflag[t] = fl;
  }
  const int64_t e = oct_at(L, D.bc, bx + rx, by + ry_, bz + rz);
  const unsigned long long p = __ballot(e != -1);
  if (slot == 0) pres[t] = p;
  int32_t v = -1, m = 0;
  if (needed) {
    if (e >= 0) v = int32_t(e);
    else if (e == -1) {
      v = -2;
      m = 1;
    }
  }
  tab[i] = v;
  miss[i] = m;
}

// Missing entries in (tile, slot) order: their wrapped oct positions.

__global__ void missing_list_kernel(LevelView L, const int32_t* __restrict__ first, int32_t n_tile,
                                    const int32_t* __restrict__ miss, const int32_t* __restrict__ midx,
                                    uint64_t* __restrict__ mpos, int32_t* __restrict__ mentry) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(n_tile) * TILE_TAB || !miss[i]) return;
  const int t = int(i / TILE_TAB), slot = int(i % TILE_TAB);
  const int64_t o0 = first[t];
  int64_t q[3] = {(L.oc[3 * o0] & ~1) + slot % 4 - 1, (L.oc[3 * o0 + 1] & ~1) + (slot / 4) % 4 - 1,
                  (L.oc[3 * o0 + 2] & ~1) + slot / 16 - 1};
  for (int a = 0; a < 3; ++a) q[a] = ((q[a] % L.noct[a]) + L.noct[a]) % L.noct[a];
  mpos[midx[i]] = pack_pos(q[0], q[1], q[2]);
  mentry[midx[i]] = int32_t(i);
}

// Open-addressing hash of positions -> the first (smallest) list index
// (the same mixer as the oct position hash).
__global__ void hash_insert_kernel(const uint64_t* __restrict__ mpos, int64_t nm, unsigned long long* hkey,
                                   int32_t* hval, uint64_t mask) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nm) return;
  const unsigned long long k = mpos[i];
  uint64_t s = fmix64(k) & mask;
  while (true) {
    const unsigned long long prev = atomicCAS(&hkey[s], ~0ull, k);
    if (prev == ~0ull || prev == k) {
      atomicMin(&hval[s], int32_t(i));
      return;
    }
    s = (s + 1) & mask;
  }
}

__device__ __forceinline__ int64_t hash_find(const unsigned long long* hkey, uint64_t mask, uint64_t k) {
  uint64_t s = fmix64(k) & mask;
  while (hkey[s] != k) s = (s + 1) & mask;
  return int64_t(s);
}

__global__ void owner_kernel(const uint64_t* __restrict__ mpos, int64_t nm, const unsigned long long* hkey,
                             const int32_t* hval, uint64_t mask, int32_t* __restrict__ owner) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nm) return;
  owner[i] = (hval[hash_find(hkey, mask, mpos[i])] == int32_t(i)) ? 1 : 0;
}

__global__ void ghost_assign_kernel(const uint64_t* __restrict__ mpos, const int32_t* __restrict__ mentry,
                                    int64_t nm, const unsigned long long* hkey, const int32_t* hval, uint64_t mask,
                                    const int32_t* __restrict__ owner, const int32_t* __restrict__ gidx,
                                    int64_t n_oct, int32_t* __restrict__ tab, int32_t* __restrict__ gpos) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nm) return;
  const int32_t first = hval[hash_find(hkey, mask, mpos[i])];
  const int32_t g = gidx[first];
  tab[mentry[i]] = int32_t(n_oct + g);
  if (owner[i]) {
    const uint64_t p = mpos[i];
    gpos[3 * g] = int32_t(p & 0x1FFFFF);
    gpos[3 * g + 1] = int32_t((p >> 21) & 0x1FFFFF);
    gpos[3 * g + 2] = int32_t((p >> 42) & 0x1FFFFF);
  }
}

// Ghost sources: the covering level l-1 cell Q and, per face, the cell of the
// finest level <= l-1 covering Q's neighbour: (levels up << 48) | cell.
// Sources that cannot exist under the neighbour rule are reported in err and
// replaced by cell 0 of level l-1, so that later reads stay in bounds.
__global__ void ghost_source_kernel(const LevelView* __restrict__ coarse, int ncoarse, RegridDom D,
                                    const int32_t* __restrict__ gpos, int64_t n_ghost, int64_t* __restrict__ gsrc,
                                    int32_t* __restrict__ err) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= n_ghost) return;
  const int64_t qx = gpos[3 * g], qy = gpos[3 * g + 1], qz = gpos[3 * g + 2];   // a cell of level l-1
  const int64_t q = cell_at(coarse[0], D.bc, qx, qy, qz);
  if (q < 0) atomicOr(err, 2);
  gsrc[7 * g] = q < 0 ? 0 : q;
  for (int a = 0; a < 3; ++a)
    for (int s = 0; s < 2; ++s) {
      int64_t p[3] = {qx, qy, qz};
      p[a] += s ? 1 : -1;
      int64_t r = -1;
      int up = 0;
      for (; up < ncoarse; ++up) {
        r = cell_at(coarse[up], D.bc, p[0], p[1], p[2]);
        if (r >= 0) break;
        p[0] >>= 1;
        p[1] >>= 1;
        p[2] >>= 1;
      }
      if (r < 0) {
        atomicOr(err, 2);
        r = 0;
        up = 0;
      }
      gsrc[7 * g + 1 + 2 * a + s] = (int64_t(up) << 48) | r;
    }
}

__global__ void refined_ext_kernel(const uint8_t* __restrict__ flag, int64_t n, int64_t n_ext,
                                   uint8_t* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n_ext) out[i] = (i < n) ? flag[i] : uint8_t(0);
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void fill_u64_kernel(unsigned long long* p, int64_t n, unsigned long long v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned blocks(int64_t n, int b = 256) { return unsigned((n + b - 1) / b); }

}  // namespace

// ------------------------------------------------------------- launchers
int launch_regrid_flags(const LevelView& L, const RegridDom& D, int l, const double* rho, const FlagTiles& T,
                        uint8_t* flag, int32_t* cnt, int32_t* has, void* stream) {
  if (L.n == 0) return 0;
  if (T.pres && (!T.tile_of || !T.tab)) return -1;
  hipLaunchKernelGGL(regrid_flag_kernel, dim3(blocks(L.n)), dim3(256), 0, (hipStream_t)stream, L, D, l, rho, T, flag,
                     cnt, has);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

uint64_t pos_hash_entries(int64_t n_blocks) {
  uint64_t e = 64;
  while (e < 2 * uint64_t(n_blocks)) e <<= 1;
  return e;
}

int launch_pos_hash(const uint64_t* key, const int32_t* oc, int64_t n, unsigned long long* tab, uint64_t entries,
                    int32_t* err, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks(int64_t(kBlockWords * entries))), dim3(256), 0, s, tab,
                     int64_t(kBlockWords * entries), kEmptyPos);
  if (n > 0) {
    hipLaunchKernelGGL(pos_hash_key_kernel, dim3(blocks(n)), dim3(256), 0, s, key, oc, n, tab, entries - 1, err);
    hipLaunchKernelGGL(pos_hash_oct_kernel, dim3(blocks(n)), dim3(256), 0, s, oc, n, tab, entries - 1, err);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int scan_tmp_ints(int64_t n) { return int((n + SCAN_BLOCK - 1) / SCAN_BLOCK) + 2; }

int launch_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const int nb = int((n + SCAN_BLOCK - 1) / SCAN_BLOCK);
  int32_t* total = tmp + nb + 1;
  if (n == 0) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(1), 0, s, total, int64_t(1), int32_t(0));
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(nb), dim3(SCAN_BLOCK), 0, s, in, out, n, tmp);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(SCAN_BLOCK), 0, s, tmp, nb, total);
  hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(SCAN_BLOCK), 0, s, out, n, tmp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_regrid_children(const LevelView& C, const OldTree& T, const RegridDom& D, int fbits,
                           const uint8_t* flag, const int32_t* off, const ChildTiles& CT, uint64_t* nkey,
                           int32_t* noc, int32_t* parent, int32_t* child, int32_t* src_old, int32_t* src7,
                           int32_t* err, unsigned long long* kept, void* stream) {
  if (C.n == 0) return 0;
  if (fbits < 1 || fbits > 25) return -1;   // child_digits' range
  if (!CT.toff || !CT.tile_of || !CT.tfirst || !CT.fresh) return -1;
  hipLaunchKernelGGL(regrid_children_kernel, dim3(blocks(C.n)), dim3(256), 0, (hipStream_t)stream, C, T, D, fbits,
                     flag, off, CT, nkey, noc, parent, child, src_old, src7, err, kept);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_tile_table(const LevelView& L, const RegridDom& D, const int32_t* first, int32_t n_tile, int32_t* tab,
                      uint32_t* tflag, int32_t* miss, unsigned long long* pres, void* stream) {
  if (n_tile == 0) return 0;
  hipLaunchKernelGGL(tile_table_kernel, dim3(blocks(int64_t(n_tile) * TILE_TAB)), dim3(256), 0, (hipStream_t)stream,
                     L, D, first, n_tile, tab, tflag, miss, pres);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_missing_list(const LevelView& L, const int32_t* first, int32_t n_tile, const int32_t* miss,
                        const int32_t* midx, uint64_t* mpos, int32_t* mentry, void* stream) {
  if (n_tile == 0) return 0;
  hipLaunchKernelGGL(missing_list_kernel, dim3(blocks(int64_t(n_tile) * TILE_TAB)), dim3(256), 0,
                     (hipStream_t)stream, L, first, n_tile, miss, midx, mpos, mentry);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_ghost_numbering(const uint64_t* mpos, const int32_t* mentry, int64_t nm, unsigned long long* hkey,
                           int32_t* hval, uint64_t hsize, int32_t* owner, int32_t* gidx, int32_t* scan_tmp,
                           int64_t n_oct, int32_t* tab, int32_t* gpos, void* stream) {
  if (nm == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  const uint64_t mask = hsize - 1;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks(int64_t(hsize))), dim3(256), 0, s, hkey, int64_t(hsize), ~0ull);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks(int64_t(hsize))), dim3(256), 0, s, hval, int64_t(hsize),
                     int32_t(0x7fffffff));
  hipLaunchKernelGGL(hash_insert_kernel, dim3(blocks(nm)), dim3(256), 0, s, mpos, nm, hkey, hval, mask);
  hipLaunchKernelGGL(owner_kernel, dim3(blocks(nm)), dim3(256), 0, s, mpos, nm, hkey, hval, mask, owner);
  if (launch_scan(owner, gidx, nm, scan_tmp, stream)) return -1;
  hipLaunchKernelGGL(ghost_assign_kernel, dim3(blocks(nm)), dim3(256), 0, s, mpos, mentry, nm, hkey, hval, mask,
                     owner, gidx, n_oct, tab, gpos);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_ghost_sources(const LevelView* coarse_dev, int ncoarse, const RegridDom& D, const int32_t* gpos,
                         int64_t n_ghost, int64_t* gsrc, int32_t* err, void* stream) {
  if (n_ghost == 0) return 0;
  hipLaunchKernelGGL(ghost_source_kernel, dim3(blocks(n_ghost)), dim3(256), 0, (hipStream_t)stream, coarse_dev,
                     ncoarse, D, gpos, n_ghost, gsrc, err);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_refined_ext(const uint8_t* flag, int64_t n, int64_t n_ext, uint8_t* out, void* stream) {
  if (n_ext == 0) return 0;
  hipLaunchKernelGGL(refined_ext_kernel, dim3(blocks(n_ext)), dim3(256), 0, (hipStream_t)stream, flag, n, n_ext, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ry
