// Host-side octree builder of the GPU library: Hilbert ordering, refinement
// flags, the neighbour rule, fill, restriction, and the per-level tables the
// kernels read (2x2x2-oct tiles with their 4x4x4 neighbourhoods, ghost octs
// on coarse-fine interfaces, child / parent maps).
//
// Compiled with -ffp-contract=off: the refinement criterion and the initial
// restriction are evaluated in plain IEEE double in the order written, so the
// refinement map is a pure function of the input bytes.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <unordered_map>

#include "ry_internal.h"

namespace ry {

// ---------------------------------------------------------------------------
// Peano-Hilbert key of oct coordinates, Skilling (2004, AIP Conf. Proc. 707):
// the axes are converted to the "transposed" Hilbert index by undoing the
// excess rotations/reflections from the top bit down and Gray-coding, then
// the transposed form is read out bit-plane by bit-plane, x first.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
static inline uint64_t packc(int64_t x, int64_t y, int64_t z) {
  return uint64_t(x) | (uint64_t(y) << 22) | (uint64_t(z) << 44);
}
static inline uint64_t fib_hash(uint64_t k) { return (k * 0x9E3779B97F4A7C15ull) ^ (k >> 29); }

void OctIndex::build(const std::vector<int32_t>& x, const std::vector<int32_t>& y,
                     const std::vector<int32_t>& z) {
  size_t n = x.size();
  uint64_t cap = 64;
  while (cap < 2 * n + 64) cap <<= 1;
  slot_key.assign(cap, ~0ull);
  slot_val.assign(cap, -1);
  mask = cap - 1;
  for (size_t i = 0; i < n; ++i) {
    uint64_t k = packc(x[i], y[i], z[i]);
    uint64_t s = fib_hash(k) & mask;
    while (slot_key[s] != ~0ull) s = (s + 1) & mask;
    slot_key[s] = k;
    slot_val[s] = int32_t(i);
  }
}

int32_t OctIndex::find(int64_t x, int64_t y, int64_t z) const {
  if (slot_key.empty()) return -1;
  uint64_t k = packc(x, y, z);
  uint64_t s = fib_hash(k) & mask;
  while (slot_key[s] != ~0ull) {
    if (slot_key[s] == k) return slot_val[s];
    s = (s + 1) & mask;
  }
  return -1;
}

// ---------------------------------------------------------------------------
// Boundary handling on cell positions of level l.
// ---------------------------------------------------------------------------
struct Geo {
  const DomainSpec& d;
  explicit Geo(const DomainSpec& dd) : d(dd) {}
  // periodic wrap / outflow clamp, in place
  void apply(int l, int64_t& x, int64_t& y, int64_t& z) const {
    int64_t* p[3] = {&x, &y, &z};
    for (int a = 0; a < 3; ++a) {
      const int64_t n = d.ncell(l, a);
      int64_t& v = *p[a];
      if (v < 0) v = (d.bc[2 * a] == RY_BC_PERIODIC) ? ((v % n) + n) % n : 0;
      else if (v >= n) v = (d.bc[2 * a + 1] == RY_BC_PERIODIC) ? v % n : n - 1;
    }
  }
  bool outside_outflow(int l, int64_t x, int64_t y, int64_t z) const {
    const int64_t v[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) {
      if (v[a] < 0 && d.bc[2 * a] != RY_BC_PERIODIC) return true;
      if (v[a] >= d.ncell(l, a) && d.bc[2 * a + 1] != RY_BC_PERIODIC) return true;
    }
    return false;
  }
};

static inline int cidx(int64_t x, int64_t y, int64_t z) {
  return int((x & 1) | ((y & 1) << 1) | ((z & 1) << 2));
}

// cell of the finest existing level <= l covering position (x,y,z) of l
struct CellRef {
  int level;
  int64_t cell;
};
static CellRef covering(const DomainSpec& d, const std::vector<HostLevel>& L, int l, int64_t x, int64_t y,
                        int64_t z) {
  Geo g(d);
  g.apply(l, x, y, z);
  while (true) {
    const HostLevel& H = L[l - d.lmin];
    int32_t o = H.index.find(x >> 1, y >> 1, z >> 1);
    if (o >= 0) return {l, int64_t(o) * 8 + cidx(x, y, z)};
    x >>= 1;
    y >>= 1;
    z >>= 1;
    --l;
  }
}

static void sort_level(const DomainSpec& d, int l, HostLevel& H, bool with_state = true) {
  const int bits = d.hbits0 + (l - d.lmin);
  std::vector<uint64_t> k(H.n);
  for (int64_t i = 0; i < H.n; ++i) k[i] = hilbert3(bits, uint32_t(H.ox[i]), uint32_t(H.oy[i]), uint32_t(H.oz[i]));
  std::vector<int64_t> ord(H.n);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return k[a] < k[b]; });
  std::vector<int32_t> x(H.n), y(H.n), z(H.n);
  H.key.resize(H.n);
  for (int64_t i = 0; i < H.n; ++i) {
    H.key[i] = k[ord[i]];
    x[i] = H.ox[ord[i]];
    y[i] = H.oy[ord[i]];
    z[i] = H.oz[ord[i]];
  }
  H.ox.swap(x);
  H.oy.swap(y);
  H.oz.swap(z);
  H.index.build(H.ox, H.oy, H.oz);
  H.refined.assign(H.n, 0);
  if (with_state) H.U.assign(size_t(H.n) * 8 * d.nv, 0.0);
}

static void restrict_into(const HostLevel& F, HostLevel& C, int nv) {
  for (int64_t k = 0; k < F.n; ++k) {
    const int64_t px = F.ox[k], py = F.oy[k], pz = F.oz[k];
    int32_t o = C.index.find(px >> 1, py >> 1, pz >> 1);
    const int64_t cell = int64_t(o) * 8 + cidx(px, py, pz);
    for (int v = 0; v < nv; ++v) {
      const double* s = &F.U[size_t(v) * 8 * F.n + 8 * k];
      C.U[size_t(v) * 8 * C.n + cell] =
          0.125 * (((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])));
    }
  }
}

// Refinement flags of level l (bit c of flag[o] for cell c of oct o): a cell
// is refined when its 26 neighbour cells exist at level l (outside an
// outflow face counts as existing) and the criterion holds on its density
// rho(o, c) -- GRAD with the central differences of its face neighbours
// (which exist at level l once the neighbour rule holds), MASS against
// rho_thr 8^(l - lmin).  Returns the number of refined cells.
template <typename RhoFn>
static int64_t flag_level(const DomainSpec& d, const HostLevel& H, int l, RhoFn rho, std::vector<uint8_t>& flag) {
  Geo g(d);
  flag.assign(H.n, 0);
  int64_t nnew = 0;
  const double mass_thr = d.refine_param * std::ldexp(1.0, 3 * (l - d.lmin));
  auto rho_at = [&](int64_t x, int64_t y, int64_t z) {
    g.apply(l, x, y, z);
    return rho(H.index.find(x >> 1, y >> 1, z >> 1), cidx(x, y, z));
  };
  for (int64_t o = 0; o < H.n; ++o) {
    // which of the 27 octs around o exist at this level (outside an outflow
    // face counts as existing); bit (dx+1) + 3 (dy+1) + 9 (dz+1)
    uint32_t have = 0;
    bool known = false;
    auto neighbour_octs = [&]() {
      if (known) return;
      known = true;
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            // a representative cell of the neighbouring oct
            int64_t qx = 2 * int64_t(H.ox[o]) + 2 * dx, qy = 2 * int64_t(H.oy[o]) + 2 * dy,
                    qz = 2 * int64_t(H.oz[o]) + 2 * dz;
            bool ex;
            if (g.outside_outflow(l, qx, qy, qz)) {
              ex = true;
            } else {
              g.apply(l, qx, qy, qz);
              ex = H.index.find(qx >> 1, qy >> 1, qz >> 1) >= 0;
            }
            if (ex) have |= 1u << ((dx + 1) + 3 * (dy + 1) + 9 * (dz + 1));
          }
    };
    for (int c = 0; c < 8; ++c) {
      const int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
      const int64_t x = 2 * int64_t(H.ox[o]) + bx, y = 2 * int64_t(H.oy[o]) + by, z = 2 * int64_t(H.oz[o]) + bz;
      const double rc = rho(o, c);
      // the mass criterion needs nothing else: test it before the rule
      if (d.refine == RY_REFINE_MASS && !(rc > mass_thr)) continue;
      if (d.refine != RY_REFINE_MASS && d.refine != RY_REFINE_GRAD) continue;
      // neighbour rule: the 26 neighbour cells lie in the 7 octs of the
      // cell's corner of the 3x3x3 oct block (and in o itself)
      neighbour_octs();
      const int sx = bx ? 1 : -1, sy = by ? 1 : -1, sz = bz ? 1 : -1;
      bool ok = true;
      for (int k = 1; k < 8 && ok; ++k) {
        const int dx = (k & 1) ? sx : 0, dy = (k & 2) ? sy : 0, dz = (k & 4) ? sz : 0;
        if (!((have >> ((dx + 1) + 3 * (dy + 1) + 9 * (dz + 1))) & 1u)) ok = false;
      }
      if (!ok) continue;
      bool want = true;
      if (d.refine == RY_REFINE_GRAD) {
        const double gx = 0.5 * (rho_at(x + 1, y, z) - rho_at(x - 1, y, z));
        const double gy = 0.5 * (rho_at(x, y + 1, z) - rho_at(x, y - 1, z));
        const double gz = 0.5 * (rho_at(x, y, z + 1) - rho_at(x, y, z - 1));
        const double th = d.refine_param;
        want = gx * gx + gy * gy + gz * gz > (th * rc) * (th * rc);
      }
      if (want) {
        flag[o] |= uint8_t(1u << c);
        ++nnew;
      }
    }
  }
  return nnew;
}

std::string build_mesh(const DomainSpec& d, const double* U_base, ry_fill_fn fill, void* user,
                       std::vector<HostLevel>& L) {
  L.assign(d.lmax - d.lmin + 1, HostLevel());
  Geo g(d);
  // --- base level: every oct of the box
  {
    HostLevel& H = L[0];
    const int64_t nx = d.noct(d.lmin, 0), ny = d.noct(d.lmin, 1), nz = d.noct(d.lmin, 2);
    H.n = nx * ny * nz;
    H.ox.reserve(H.n);
    H.oy.reserve(H.n);
    H.oz.reserve(H.n);
    for (int64_t z = 0; z < nz; ++z)
      for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x) {
          H.ox.push_back(int32_t(x));
          H.oy.push_back(int32_t(y));
          H.oz.push_back(int32_t(z));
        }
    sort_level(d, d.lmin, H);
    const int64_t cx = d.nbase[0], cy = d.nbase[1], ncell = int64_t(d.nbase[0]) * d.nbase[1] * d.nbase[2];
    for (int64_t o = 0; o < H.n; ++o)
      for (int c = 0; c < 8; ++c) {
        const int64_t x = 2 * int64_t(H.ox[o]) + (c & 1), y = 2 * int64_t(H.oy[o]) + ((c >> 1) & 1),
                      z = 2 * int64_t(H.oz[o]) + ((c >> 2) & 1);
        for (int v = 0; v < d.nv; ++v)
          H.U[size_t(v) * 8 * H.n + 8 * o + c] = U_base[size_t(v) * ncell + x + cx * (y + cy * z)];
      }
  }
  // --- refine level by level
  for (int l = d.lmin; l < d.lmax; ++l) {
    HostLevel& H = L[l - d.lmin];
    if (H.n == 0 || d.refine == RY_REFINE_NONE) break;
    std::vector<uint8_t> flag;
    const int64_t nnew = flag_level(d, H, l, [&](int64_t o, int c) { return H.U[8 * o + c]; }, flag);
    if (nnew == 0) break;
    HostLevel& F = L[l + 1 - d.lmin];
    F.n = nnew;
    for (int64_t o = 0; o < H.n; ++o) {
      H.refined[o] = flag[o];
      for (int c = 0; c < 8; ++c)
        if (flag[o] & (1u << c)) {
          F.ox.push_back(2 * H.ox[o] + (c & 1));
          F.oy.push_back(2 * H.oy[o] + ((c >> 1) & 1));
          F.oz.push_back(2 * H.oz[o] + ((c >> 2) & 1));
        }
    }
    sort_level(d, l + 1, F);
    if (!fill) return "fill callback required for refined levels";
    std::vector<int32_t> ijk(size_t(F.n) * 24);
    for (int64_t o = 0; o < F.n; ++o)
      for (int c = 0; c < 8; ++c) {
        ijk[(8 * o + c) * 3 + 0] = 2 * F.ox[o] + (c & 1);
        ijk[(8 * o + c) * 3 + 1] = 2 * F.oy[o] + ((c >> 1) & 1);
        ijk[(8 * o + c) * 3 + 2] = 2 * F.oz[o] + ((c >> 2) & 1);
      }
    fill(user, l + 1, F.n * 8, ijk.data(), F.U.data());
  }
  for (int l = d.lmax - 1; l >= d.lmin; --l)
    if (L[l + 1 - d.lmin].n > 0) restrict_into(L[l + 1 - d.lmin], L[l - d.lmin], d.nv);
  return "";
}

// ---------------------------------------------------------------------------
// One level of a regrid between coarse steps.
// ---------------------------------------------------------------------------
std::string regrid_level(const DomainSpec& d, int l, HostLevel& C, const std::vector<double>& rho,
                         const HostLevel& F_old, HostLevel& F_new, std::vector<int32_t>& src_old,
                         std::vector<int32_t>& src7, int64_t& created, int64_t& destroyed) {
  if (int64_t(rho.size()) < 8 * C.n) return "regrid: density array too short";
  std::vector<uint8_t> flag;
  const int64_t nnew = (C.n == 0 || d.refine == RY_REFINE_NONE)
                           ? (flag.assign(C.n, 0), 0)
                           : flag_level(d, C, l, [&](int64_t o, int c) { return rho[8 * o + c]; }, flag);
  C.refined = flag;
  F_new = HostLevel();
  F_new.n = nnew;
  for (int64_t o = 0; o < C.n; ++o)
    for (int c = 0; c < 8; ++c)
      if (flag[o] & (1u << c)) {
        F_new.ox.push_back(2 * C.ox[o] + (c & 1));
        F_new.oy.push_back(2 * C.oy[o] + ((c >> 1) & 1));
        F_new.oz.push_back(2 * C.oz[o] + ((c >> 2) & 1));
      }
  sort_level(d, l + 1, F_new, false);
  src_old.assign(F_new.n, -1);
  src7.assign(size_t(F_new.n) * 7, -1);
  Geo g(d);
  for (int64_t k = 0; k < F_new.n; ++k) {
    const int32_t o = F_old.index.find(F_new.ox[k], F_new.oy[k], F_new.oz[k]);
    if (o >= 0) {
      src_old[k] = o;
      continue;
    }
    ++created;
    // the parent cell Q (level l) and its six face neighbours, which exist
    // at level l by the neighbour rule (or are clamped to Q at an outflow face)
    const int64_t q[3] = {F_new.ox[k], F_new.oy[k], F_new.oz[k]};
    for (int j = 0; j < 7; ++j) {
      int64_t p[3] = {q[0], q[1], q[2]};
      if (j > 0) p[(j - 1) >> 1] += ((j - 1) & 1) ? 1 : -1;
      g.apply(l, p[0], p[1], p[2]);
      const int32_t po = C.index.find(p[0] >> 1, p[1] >> 1, p[2] >> 1);
      if (po < 0) return "regrid: interpolation source missing";
      src7[7 * k + j] = po * 8 + cidx(p[0], p[1], p[2]);
    }
  }
  for (int64_t o = 0; o < F_old.n; ++o)
    if (F_new.index.find(F_old.ox[o], F_old.oy[o], F_old.oz[o]) < 0) ++destroyed;
  return "";
}

// ---------------------------------------------------------------------------
// Device tables.
// ---------------------------------------------------------------------------
// Tables of level k (reads the host levels only; levels are independent).
static std::string build_level_tables(const DomainSpec& d, const std::vector<HostLevel>& L, int k,
                                      LevelTables& T) {
  const int nl = int(L.size());
  {
    const int l = d.lmin + k;
    const HostLevel& H = L[k];
    T.n_oct = H.n;
    if (H.n == 0) return "";
    for (int64_t o = 0; o < H.n; ++o) T.n_leaf += 8 - __builtin_popcount(H.refined[o]);
    // tiles: groups of octs sharing key >> 3 (an aligned 2x2x2 block of
    // octs).  On refined levels a tile is kept only when one of its cells is
    // a leaf: a tile of fully refined octs updates nothing (the restriction
    // overwrites its cells) and records no flux register (a refined cell
    // never borders a coarser leaf).  The base level keeps every tile: the
    // device regrid keeps its tables while its refinement changes
    std::vector<int64_t> tile_start, tile_end;
    for (int64_t o0 = 0; o0 < H.n;) {
      int64_t o1 = o0 + 1;
      while (o1 < H.n && (H.key[o1] >> 3) == (H.key[o0] >> 3)) ++o1;
      bool leaf = (k == 0);
      for (int64_t o = o0; o < o1 && !leaf; ++o) leaf = H.refined[o] != 0xFF;
      if (leaf) {
        tile_start.push_back(o0);
        tile_end.push_back(o1);
      }
      o0 = o1;
    }
    T.n_tile = int32_t(tile_start.size());
    T.tab.assign(size_t(T.n_tile) * TILE_TAB, -1);
    T.tflag.assign(T.n_tile, 0);
    std::unordered_map<uint64_t, int64_t> ghost_of;  // packed oct position -> ghost number
    std::vector<std::array<int64_t, 3>> ghost_pos;
    const int64_t nox = d.noct(l, 0), noy = d.noct(l, 1), noz = d.noct(l, 2);
    for (int32_t t = 0; t < T.n_tile; ++t) {
      const int64_t o0 = tile_start[t], o1 = tile_end[t];
      const int64_t bx = H.ox[o0] & ~1, by = H.oy[o0] & ~1, bz = H.oz[o0] & ~1;
      bool present[8] = {false, false, false, false, false, false, false, false};
      for (int64_t o = o0; o < o1; ++o)
        present[(H.ox[o] - bx) + 2 * (H.oy[o] - by) + 4 * (H.oz[o] - bz)] = true;
      // a base side of 2 mod 4 cells ends halfway through its last tiles:
      // their second oct row lies past the domain (cut, never updated)
      uint32_t fl = tile_cut_bits(bx + 2 > nox ? 2 : 0, by + 2 > noy ? 2 : 0, bz + 2 > noz ? 2 : 0);
      if (bx == 0 && d.bc[0] == RY_BC_OUTFLOW) fl |= CL_LOX;
      if (bx + 2 >= nox && d.bc[1] == RY_BC_OUTFLOW) fl |= CL_HIX;
      if (by == 0 && d.bc[2] == RY_BC_OUTFLOW) fl |= CL_LOY;
      if (by + 2 >= noy && d.bc[3] == RY_BC_OUTFLOW) fl |= CL_HIY;
      if (bz == 0 && d.bc[4] == RY_BC_OUTFLOW) fl |= CL_LOZ;
      if (bz + 2 >= noz && d.bc[5] == RY_BC_OUTFLOW) fl |= CL_HIZ;
      T.tflag[t] = fl;
      for (int rz = -1; rz <= 2; ++rz)
        for (int ry_ = -1; ry_ <= 2; ++ry_)
          for (int rx = -1; rx <= 2; ++rx) {
            const int slot = (rx + 1) + 4 * (ry_ + 1) + 16 * (rz + 1);
            bool needed = false;
            for (int b = 0; b < 8 && !needed; ++b) {
              if (!present[b]) continue;
              const int px = b & 1, py = (b >> 1) & 1, pz = b >> 2;
              // a face or edge neighbour of a present oct (the stencil reads
              // no cell diagonally across a corner of an oct)
              const int ax = std::abs(rx - px), ay = std::abs(ry_ - py), az = std::abs(rz - pz);
              needed = ax <= 1 && ay <= 1 && az <= 1 && ax + ay + az <= 2;
            }
            if (!needed) continue;
            int64_t qx = bx + rx, qy = by + ry_, qz = bz + rz;
            // oct positions outside an outflow face are never read (the kernel clamps)
            bool out = false;
            const int64_t q[3] = {qx, qy, qz}, nq[3] = {nox, noy, noz};
            for (int a = 0; a < 3; ++a) {
              if (q[a] < 0 && d.bc[2 * a] != RY_BC_PERIODIC) out = true;
              if (q[a] >= nq[a] && d.bc[2 * a + 1] != RY_BC_PERIODIC) out = true;
            }
            if (out) continue;
            qx = ((qx % nox) + nox) % nox;
            qy = ((qy % noy) + noy) % noy;
            qz = ((qz % noz) + noz) % noz;
            int32_t o = H.index.find(qx, qy, qz);
            if (o >= 0) {
              T.tab[size_t(t) * TILE_TAB + slot] = o;
              continue;
            }
            if (l == d.lmin) return "internal: missing oct on the base level";
            const uint64_t pk = packc(qx, qy, qz);
            auto it = ghost_of.find(pk);
            int64_t gnum;
            if (it == ghost_of.end()) {
              gnum = int64_t(ghost_pos.size());
              ghost_of.emplace(pk, gnum);
              ghost_pos.push_back({qx, qy, qz});
            } else {
              gnum = it->second;
            }
            T.tab[size_t(t) * TILE_TAB + slot] = int32_t(H.n + gnum);
          }
    }
    T.n_ghost = int64_t(ghost_pos.size());
    T.refined_ext.assign(H.n + T.n_ghost, 0);
    std::copy(H.refined.begin(), H.refined.end(), T.refined_ext.begin());
    // ghost sources: the covering coarse cell Q and its 6 neighbours
    T.gsrc.assign(size_t(T.n_ghost) * 7, 0);
    for (int64_t gi = 0; gi < T.n_ghost; ++gi) {
      const int64_t qx = ghost_pos[gi][0], qy = ghost_pos[gi][1], qz = ghost_pos[gi][2];  // cell of l-1
      const HostLevel& C = L[k - 1];
      const int32_t oq = C.index.find(qx >> 1, qy >> 1, qz >> 1);
      if (oq < 0) return "internal: coarse cell of a ghost oct does not exist (neighbour rule)";
      T.gsrc[gi * 7 + 0] = int64_t(oq) * 8 + cidx(qx, qy, qz);   // level_up = 0
      for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s) {
          int64_t p[3] = {qx, qy, qz};
          p[a] += s ? 1 : -1;
          CellRef r = covering(d, L, l - 1, p[0], p[1], p[2]);
          const int64_t up = (l - 1) - r.level;
          T.gsrc[gi * 7 + 1 + 2 * a + s] = (up << 48) | r.cell;
        }
    }
    // child map
    if (k + 1 < nl && L[k + 1].n > 0) {
      const HostLevel& F = L[k + 1];
      T.child.assign(size_t(H.n) * 8, -1);
      for (int64_t o = 0; o < H.n; ++o)
        for (int c = 0; c < 8; ++c)
          if (H.refined[o] & (1u << c)) {
            const int64_t cx = 2 * int64_t(H.ox[o]) + (c & 1), cy = 2 * int64_t(H.oy[o]) + ((c >> 1) & 1),
                          cz = 2 * int64_t(H.oz[o]) + ((c >> 2) & 1);
            const int32_t f = F.index.find(cx, cy, cz);
            if (f < 0) return "internal: child oct missing";
            T.child[8 * o + c] = f;
          }
    }
    // parent cell of every oct (restriction target on level l-1)
    if (k > 0) {
      const HostLevel& C = L[k - 1];
      T.parent_cell.assign(H.n, -1);
      for (int64_t o = 0; o < H.n; ++o) {
        const int32_t p = C.index.find(H.ox[o] >> 1, H.oy[o] >> 1, H.oz[o] >> 1);
        if (p < 0) return "internal: parent oct missing";
        T.parent_cell[o] = p * 8 + cidx(H.ox[o], H.oy[o], H.oz[o]);
      }
    }
  }
  return "";
}

std::string build_tables(const DomainSpec& d, const std::vector<HostLevel>& L,
                         std::vector<LevelTables>& out) {
  const int nl = int(L.size());
  out.assign(nl, LevelTables());
  std::vector<std::string> err(nl);
  std::vector<std::thread> pool;
  for (int k = 0; k < nl; ++k)
    pool.emplace_back([&, k]() { err[k] = build_level_tables(d, L, k, out[k]); });
  for (auto& t : pool) t.join();
  for (auto& e : err)
    if (!e.empty()) return e;
  for (int k = 0; k < nl; ++k)
    if (!level_index_fits(out[k].n_oct, out[k].n_ghost, d.nv))
      return "level " + std::to_string(d.lmin + k) + ": " + std::to_string(out[k].n_oct) + " octs + " +
             std::to_string(out[k].n_ghost) + " ghost octs reach the 32-bit cell index (2^29 octs, " +
             "(1 + nv) times the octs + ghost octs on a level with ghosts)";
  return "";
}

}  // namespace ry
