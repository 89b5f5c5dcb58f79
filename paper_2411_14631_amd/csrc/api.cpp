// C ABI of the octree hydro library: context lifetime, device buffers,
// subcycling driver, graph capture, batched boxes, autotuning, diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "ry_internal.h"
#include "regrid.h"

using namespace ry;

namespace {

struct DevLevel {
  int64_t n_oct = 0, n_ghost = 0, n_ext = 0, n_leaf = 0;
  int32_t n_tile = 0;
  double* U[2] = {nullptr, nullptr};
  int cur = 0;
  int32_t* tab = nullptr;
  uint32_t* tflag = nullptr;
  uint8_t* refined = nullptr;
  int32_t* child = nullptr;
  double* reg = nullptr;
  int64_t* gsrc = nullptr;
  uint32_t* gread = nullptr;         // per ghost oct: the cells an update reads (floor census)
  int32_t* parent_cell = nullptr;
  int32_t* tile_box = nullptr;
  int32_t* oct_box = nullptr;
  uint64_t* dkey = nullptr;          // sorted Hilbert keys (device regrid lookups)
  int32_t* doc = nullptr;            // oct coordinates, x y z interleaved
  // super-tiles (4x4x4-oct blocks) for the 8^3-cell tile, built on demand
  // from the small-tile tables of the current mesh
  bool super_ok = false;
  int32_t n_super = 0;
  int32_t* stab = nullptr;
  uint32_t* stflag = nullptr;
  int32_t* sbox = nullptr;           // batched boxes: box of each super-tile
  int32_t* spart = nullptr;          // batched boxes: its CFL partial's index
  int64_t plane() const { return 8 * n_ext; }
};

struct TimedLaunch {
  std::string name;
  hipEvent_t a, b;
};

}  // namespace

struct ry_ctx {
  ry_config cfg{};
  DomainSpec dom;
  int nlev = 0;
  bool built = false;
  bool batch = false;
  std::vector<DevLevel> lev;
  std::vector<HostLevel> host;            // topology of the current mesh (no state)
  bool host_valid = true;                 // false after a device-side regrid
  bool regrid_device = true;              // build regrid flags / tables on the device
  bool means_valid = true;                // every refined cell holds its children's ordered mean
                                          // (the builder and every step restrict; an upload may not)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int num_cu = 256;
  // launch tuning of the hydro kernel, per level (index level - level_min)
  ry_tuning tune[RY_MAX_LEVELS];
  // device scalars
  double* d_smax = nullptr;               // max signal speed per level / per box
  unsigned long long* d_slots = nullptr;  // per level: SMAX_SLOTS partial maxima of the fused CFL
  double* d_part = nullptr;               // per-tile (or per-block) partial maxima
  int64_t* d_segoff = nullptr;            // tile offsets of levels / boxes in d_part
  std::vector<int64_t> seg_off;           // host copy
  double* d_lam = nullptr;                // 1 / per box
  double* d_t = nullptr;                  // 1 / per box
  int32_t* d_flags = nullptr;             // [0]=skip [1]=done [2]=nstep [3]=err
  // pinned host copy of the flags and the time read back after ry_advance
  // (one round trip for both), allocated on first use
  struct Readback {
    int32_t flags[4];
    double t;
  };
  Readback* h_rb = nullptr;
  unsigned long long* d_floors = nullptr;
  unsigned int* d_queue = nullptr;        // 8 counters, QUEUE_STRIDE apart
  double* d_partial = nullptr;
  double* d_tot = nullptr;
  double* d_dx_box = nullptr;
  int64_t* d_box_noct = nullptr;          // batch: octs per axis of each box (3 per box)
  bool slots_valid = false;
  // subcycling order state for ry_hydro_step
  int count[RY_MAX_LEVELS] = {0};
  double dt_of[RY_MAX_LEVELS] = {0};
  // graphs of 1, 2, 4, 8 and 16 coarse steps: [log2 of the step count]
  // [parity of the base level buffer]
  hipGraphExec_t graph[5][2] = {};
  std::vector<int> graph_par[5][2];
  double graph_tend[5][2] = {};
  // batch
  int nbox = 0;
  std::vector<int64_t> box_off, box_noct;
  std::vector<double> box_dx;
  hipGraphExec_t bgraph = nullptr;
  int bgraph_steps = -1, bgraph_par = -1;
  // timing
  bool timing = false;
  std::vector<TimedLaunch> pending;
  std::map<std::string, std::pair<int64_t, double>> ktime;
  // memory
  std::vector<void*> allocs;
  std::string err;
};

namespace {

ry_status fail(ry_ctx* c, ry_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

#define HIPCHK(c, call)                                                                     \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail((c), RY_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// Default launch: small tiles, one 64-thread wavefront per tile, one tile
// per workgroup, the hardware dispatcher as the queue.
constexpr ry_tuning kDefaultTuning{1, 0, 4, 1, 1, 4};

void* dalloc(ry_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (c->cfg.dev_alloc) {
    p = c->cfg.dev_alloc(bytes, c->cfg.alloc_user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) c->allocs.push_back(p);
  return p;
}

// Release one allocation made by dalloc (the stream must be idle).
void dfree(ry_ctx* c, void* p) {
  if (!p) return;
  auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
  if (it == c->allocs.end()) return;
  c->allocs.erase(it);
  if (c->cfg.dev_free) c->cfg.dev_free(p, c->cfg.alloc_user);
  else if (!c->cfg.dev_alloc) (void)hipFree(p);
}

void free_all(ry_ctx* c) {
  if (c->stream) hipStreamSynchronize(c->stream);
  for (void* p : c->allocs) {
    if (c->cfg.dev_free) c->cfg.dev_free(p, c->cfg.alloc_user);
    else if (!c->cfg.dev_alloc) hipFree(p);
  }
  c->allocs.clear();
  for (auto& gs : c->graph)
    for (auto& g : gs)
      if (g) {
        hipGraphExecDestroy(g);
        g = nullptr;
      }
  if (c->bgraph) {
    hipGraphExecDestroy(c->bgraph);
    c->bgraph = nullptr;
  }
  c->lev.clear();
}

// A level's two state buffers in one allocation, the second nv planes after
// the first: ghost octs live in the second only and are read through the
// first with a fixed index shift (HydroArgs::ghost_adj).  Freed through U[0].
bool alloc_state_pair(ry_ctx* c, double* U[2], int64_t n_ext, int nv) {
  const size_t n = size_t(nv) * 8 * size_t(n_ext);
  U[0] = static_cast<double*>(dalloc(c, sizeof(double) * 2 * n));
  U[1] = U[0] ? U[0] + n : nullptr;
  return U[0] != nullptr;
}

template <typename T>
T* upload_vec(ry_ctx* c, const std::vector<T>& v, bool& ok) {
  T* p = static_cast<T*>(dalloc(c, v.size() * sizeof(T)));
  if (!p) {
    ok = false;
    return nullptr;
  }
  if (!v.empty() && hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream) != hipSuccess)
    ok = false;
  return p;
}

ry_status validate(const ry_config* cfg, bool single_level) {
  if (!cfg) return RY_EINVAL;
  if (cfg->level_min < 0 || cfg->level_max < cfg->level_min ||
      cfg->level_max - cfg->level_min + 1 > RY_MAX_LEVELS || cfg->level_max > 20)
    return RY_EINVAL;
  if (single_level && cfg->level_max != cfg->level_min) return RY_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (cfg->nbase[a] < 2 || (cfg->nbase[a] % 2) != 0) return RY_EINVAL;
  for (int a = 0; a < 3; ++a) {
    const int lo = cfg->bc[2 * a], hi = cfg->bc[2 * a + 1];
    if (lo != RY_BC_PERIODIC && lo != RY_BC_OUTFLOW) return RY_EINVAL;
    if (hi != RY_BC_PERIODIC && hi != RY_BC_OUTFLOW) return RY_EINVAL;
    if ((lo == RY_BC_PERIODIC) != (hi == RY_BC_PERIODIC)) return RY_EINVAL;
  }
  if (!(cfg->gamma > 1.0) || !(cfg->cfl > 0.0) || !(cfg->boxlen > 0.0)) return RY_EINVAL;
  if (!(cfg->rho_floor > 0.0) || !(cfg->p_floor > 0.0)) return RY_EINVAL;
  if (cfg->precision != RY_FP64 && cfg->precision != RY_MIXED) return RY_EINVAL;
  if (cfg->refine < RY_REFINE_NONE || cfg->refine > RY_REFINE_MASS) return RY_EINVAL;
  if ((cfg->dev_alloc == nullptr) != (cfg->dev_free == nullptr)) return RY_EINVAL;
  if (cfg->nscalar < 0 || cfg->nscalar > RY_MAX_SCALARS) return RY_EINVAL;
  for (int a = 0; a < 3; ++a)
    if ((int64_t(cfg->nbase[a] / 2) << (cfg->level_max - cfg->level_min)) >= (int64_t(1) << 21)) return RY_EINVAL;
  return RY_OK;
}

DomainSpec make_dom(const ry_config& cfg) {
  DomainSpec d;
  d.lmin = cfg.level_min;
  d.lmax = cfg.level_max;
  for (int a = 0; a < 3; ++a) d.nbase[a] = cfg.nbase[a];
  for (int i = 0; i < 6; ++i) d.bc[i] = cfg.bc[i];
  d.refine = cfg.refine;
  d.refine_param = cfg.refine_param;
  d.nv = NVAR + cfg.nscalar;
  int m = std::max(cfg.nbase[0], std::max(cfg.nbase[1], cfg.nbase[2])) / 2, bits = 0;
  while ((1 << bits) < m) ++bits;
  d.hbits0 = bits;
  return d;
}

double level_dx(const ry_ctx* c, int l) {
  return c->cfg.boxlen / double(int64_t(c->cfg.nbase[0]) << (l - c->cfg.level_min));
}

ry_status init_common(ry_ctx* c) {
  if (c->cfg.stream) {
    c->stream = (hipStream_t)c->cfg.stream;
  } else {
    HIPCHK(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  int dev = 0;
  HIPCHK(c, hipGetDevice(&dev));
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
    c->num_cu = ncu;
  return RY_OK;
}

ry_status alloc_scalars(ry_ctx* c, int nslot) {
  c->d_smax = static_cast<double*>(dalloc(c, sizeof(double) * nslot));
  c->d_slots = static_cast<unsigned long long*>(dalloc(c, sizeof(unsigned long long) * nslot * SMAX_SLOTS));
  const int64_t npart = std::max<int64_t>(c->seg_off.back(), 1);
  c->d_part = static_cast<double*>(dalloc(c, sizeof(double) * npart));
  c->d_segoff = static_cast<int64_t*>(dalloc(c, sizeof(int64_t) * c->seg_off.size()));
  c->d_lam = static_cast<double*>(dalloc(c, sizeof(double) * nslot));
  c->d_t = static_cast<double*>(dalloc(c, sizeof(double) * nslot));
  c->d_flags = static_cast<int32_t*>(dalloc(c, sizeof(int32_t) * 8));
  c->d_floors = static_cast<unsigned long long*>(dalloc(c, sizeof(unsigned long long)));
  c->d_queue = static_cast<unsigned int*>(dalloc(c, sizeof(unsigned int) * 8 * QUEUE_STRIDE));
  c->d_partial = static_cast<double*>(dalloc(c, sizeof(double) * NVMAX * totals_blocks()));
  c->d_tot = static_cast<double*>(dalloc(c, sizeof(double) * NVMAX));
  if (!c->d_smax || !c->d_slots || !c->d_lam || !c->d_t || !c->d_flags || !c->d_floors || !c->d_queue || !c->d_partial ||
      !c->d_tot || !c->d_part || !c->d_segoff)
    return RY_ENOMEM;
  HIPCHK(c, hipMemcpyAsync(c->d_segoff, c->seg_off.data(), sizeof(int64_t) * c->seg_off.size(),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_smax, 0, sizeof(double) * nslot, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_slots, 0, sizeof(unsigned long long) * nslot * SMAX_SLOTS, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_lam, 0, sizeof(double) * nslot, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_t, 0, sizeof(double) * nslot, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_flags, 0, sizeof(int32_t) * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_floors, 0, sizeof(unsigned long long), c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_queue, 0, sizeof(unsigned int) * 8 * QUEUE_STRIDE, c->stream));
  return RY_OK;
}

int32_t* skip_ptr(ry_ctx* c) { return c->d_flags + 0; }
int32_t* done_ptr(ry_ctx* c) { return c->d_flags + 1; }
int32_t* nstep_ptr(ry_ctx* c) { return c->d_flags + 2; }
int32_t* err_ptr(ry_ctx* c) { return c->d_flags + 3; }

bool level_nonempty(const ry_ctx* c, int l) {
  return l >= c->cfg.level_min && l <= c->cfg.level_max && c->lev[l - c->cfg.level_min].n_oct > 0;
}

// --- timing helpers -------------------------------------------------------
void time_begin(ry_ctx* c, const char* name, TimedLaunch& tl) {
  tl.name = name;
  // timing-only events: without the system-scope fence on recording, which
  // would write back and invalidate caches around every timed launch
  hipEventCreateWithFlags(&tl.a, hipEventDisableSystemFence);
  hipEventCreateWithFlags(&tl.b, hipEventDisableSystemFence);
  hipEventRecord(tl.a, c->stream);
}
void time_end(ry_ctx* c, TimedLaunch& tl) {
  hipEventRecord(tl.b, c->stream);
  c->pending.push_back(tl);
}
void time_collect(ry_ctx* c) {
  for (auto& tl : c->pending) {
    float ms = 0.f;
    hipEventSynchronize(tl.b);
    hipEventElapsedTime(&ms, tl.a, tl.b);
    auto& e = c->ktime[tl.name];
    e.first += 1;
    e.second += ms;
    hipEventDestroy(tl.a);
    hipEventDestroy(tl.b);
  }
  c->pending.clear();
}

// --- kernel enqueue helpers -------------------------------------------------
ry_status enqueue_seg_max(ry_ctx* c) {
  const int nseg = int(c->seg_off.size()) - 1;
  if (launch_seg_max(c->d_part, c->d_segoff, nseg, c->d_smax, c->batch ? nullptr : c->d_slots, c->stream))
    return fail(c, RY_EHIP, "seg_max kernel");
  return RY_OK;
}

// Maximum signal speed of every level (box) from the current state.
// CFL partials of a level: one per tile (batched boxes: the hydro epilogue)
// and one per 256-thread block of `cfl_kernel` (32 octs); a level whose
// tiles skip fully refined octs can have fewer tiles than blocks
int64_t part_slots(const DevLevel& L) { return std::max<int64_t>(L.n_tile, cfl_blocks(L.n_oct)); }

ry_status cfl_launch_status(ry_ctx* c, int rc, int seg) {
  if (rc == LAUNCH_EXCEEDS_BUFFER)
    return fail(c, RY_EINVAL, "cfl kernel: grid exceeds its partial-maximum segment %d", seg);
  return rc ? fail(c, RY_EHIP, "cfl kernel") : RY_OK;
}

ry_status enqueue_cfl_all(ry_ctx* c) {
  if (launch_zero_u64(reinterpret_cast<unsigned long long*>(c->d_part), c->seg_off.back(), c->stream))
    return fail(c, RY_EHIP, "zero kernel");
  for (int k = 0; k < c->nlev; ++k) {
    DevLevel& L = c->lev[k];
    if (L.n_oct == 0) continue;
    if (c->batch) {
      for (int b = 0; b < c->nbox; ++b) {
        const int64_t off = c->box_off[b] * 8;
        const int rc = launch_cfl(L.U[L.cur] + off, L.plane(), c->box_noct[b], L.refined + c->box_off[b],
                                  c->cfg.gamma, c->cfg.rho_floor, c->cfg.p_floor, c->d_part + c->seg_off[b],
                                  c->seg_off[b + 1] - c->seg_off[b], err_ptr(c), c->stream);
        if (ry_status s = cfl_launch_status(c, rc, b)) return s;
      }
    } else {
      const int rc = launch_cfl(L.U[L.cur], L.plane(), L.n_oct, L.refined, c->cfg.gamma, c->cfg.rho_floor,
                                c->cfg.p_floor, c->d_part + c->seg_off[k], c->seg_off[k + 1] - c->seg_off[k],
                                err_ptr(c), c->stream);
      if (ry_status s = cfl_launch_status(c, rc, k)) return s;
    }
  }
  ry_status s = enqueue_seg_max(c);
  if (s) return s;
  c->slots_valid = true;
  return RY_OK;
}

ry_status enqueue_ghost(ry_ctx* c, int l, const int32_t* skip) {
  DevLevel& L = c->lev[l - c->cfg.level_min];
  if (L.n_ghost == 0) return RY_OK;
  GhostArgs g{};
  for (int k = 0; k < RY_MAX_LEVELS; ++k) {
    const int lc = l - 1 - k;
    if (lc < c->cfg.level_min) break;
    DevLevel& C = c->lev[lc - c->cfg.level_min];
    g.src[k] = C.U[C.cur];
    g.src_plane[k] = C.plane();
  }
  g.gsrc = L.gsrc;
  g.n_ghost = L.n_ghost;
  g.n_oct = L.n_oct;
  g.dst = L.U[1];
  g.plane = L.plane();
  g.nv = c->dom.nv;
  g.skip = skip;
  g.floors = c->d_floors;
  g.gamma = c->cfg.gamma;
  g.rho_floor = c->cfg.rho_floor;
  g.p_floor = c->cfg.p_floor;
  g.gread = L.gread;
  g.err = err_ptr(c);
  TimedLaunch tl;
  if (c->timing) time_begin(c, "ghost", tl);
  if (launch_ghost(g, c->stream)) return fail(c, RY_EHIP, "ghost kernel");
  if (c->timing) time_end(c, tl);
  return RY_OK;
}

HydroArgs hydro_args(ry_ctx* c, int l, int substep) {
  DevLevel& L = c->lev[l - c->cfg.level_min];
  HydroArgs a{};
  a.U = L.U[L.cur];
  a.Un = L.U[L.cur ^ 1];
  a.plane = L.plane();
  a.n_oct = int32_t(L.n_oct);
  a.n_ext = int32_t(L.n_ext);
  a.ghost_adj = (L.n_ghost > 0 && L.cur == 0) ? int32_t(int64_t(c->dom.nv) * L.n_ext) : 0;
  a.n_tile = L.n_tile;
  a.tab = L.tab;
  a.tflag = L.tflag;
  a.refined = L.refined;
  const bool fine = level_nonempty(c, l + 1);
  a.child = fine ? L.child : nullptr;
  a.reg_fine = fine ? c->lev[l + 1 - c->cfg.level_min].reg : nullptr;
  a.reg_own = L.reg;
  a.substep = substep;
  a.record_reg = (l > c->cfg.level_min) ? 1 : 0;
  a.gamma = c->cfg.gamma;
  a.igm1 = 1.0 / (c->cfg.gamma - 1.0);
  a.rho_floor = c->cfg.rho_floor;
  a.p_floor = c->cfg.p_floor;
  a.floors = c->d_floors;
  a.err = err_ptr(c);
  a.queue = c->d_queue;
  a.tile_box = L.tile_box;
  return a;
}

// Super-tile tables of level k (the 8^3-cell tile's work list): block keys
// of the small tiles, a scan of the block starts, then each super-tile's
// 6x6x6 oct neighbourhood assembled from its small tiles' tables.  Syncs
// once (the super-tile count).  Not inside a graph capture.
void free_super(ry_ctx* c, DevLevel& L) {
  for (void* p : {(void*)L.stab, (void*)L.stflag, (void*)L.sbox, (void*)L.spart}) dfree(c, p);
  L.stab = nullptr;
  L.stflag = nullptr;
  L.sbox = nullptr;
  L.spart = nullptr;
  L.n_super = 0;
  L.super_ok = false;
}

ry_status build_super(ry_ctx* c, int k) {
  DevLevel& L = c->lev[k];
  free_super(c, L);
  if (L.n_tile > 0) {
    const int32_t nt = L.n_tile;
    std::vector<void*> tmp;
    auto A = [&](size_t bytes) {
      void* p = dalloc(c, bytes);
      if (p) tmp.push_back(p);
      return p;
    };
    auto release = [&]() {
      for (void* p : tmp) dfree(c, p);
    };
    auto* skey = static_cast<uint64_t*>(A(sizeof(uint64_t) * nt));
    auto* ssub = static_cast<int32_t*>(A(sizeof(int32_t) * nt));
    auto* start = static_cast<int32_t*>(A(sizeof(int32_t) * nt));
    auto* excl = static_cast<int32_t*>(A(sizeof(int32_t) * nt));
    const int ntmp = scan_tmp_ints(nt);
    auto* stmp = static_cast<int32_t*>(A(sizeof(int32_t) * ntmp));
    if (!skey || !ssub || !start || !excl || !stmp) {
      release();
      return fail(c, RY_ENOMEM, "super-tile tables: allocation failed");
    }
    SuperDom D{};
    const int l = c->cfg.level_min + k;
    for (int a = 0; a < 3; ++a) D.noct[a] = c->dom.noct(l, a);
    for (int i = 0; i < 6; ++i) D.bc[i] = c->dom.bc[i];
    if (c->batch) {
      D.tile_box = L.tile_box;
      D.box_noct = c->d_box_noct;
    }
    int32_t ns = 0;
    if (launch_super_keys(L.tab, nt, L.doc, L.n_oct, D, skey, ssub, start, c->stream) ||
        launch_scan(start, excl, nt, stmp, c->stream) ||
        hipMemcpyAsync(&ns, stmp + ntmp - 1, sizeof ns, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
      release();
      return fail(c, RY_EHIP, "super-tile key kernels");
    }
    auto* sub = static_cast<int32_t*>(A(sizeof(int32_t) * 8 * std::max(ns, 1)));
    auto* sblock = static_cast<uint64_t*>(A(sizeof(uint64_t) * std::max(ns, 1)));
    L.stab = static_cast<int32_t*>(dalloc(c, sizeof(int32_t) * super_table_slots() * std::max(ns, 1)));
    L.stflag = static_cast<uint32_t*>(dalloc(c, sizeof(uint32_t) * std::max(ns, 1)));
    if (!sub || !sblock || !L.stab || !L.stflag) {
      release();
      return fail(c, RY_ENOMEM, "super-tile tables: allocation failed");
    }
    if (launch_super_tables(L.tab, skey, ssub, start, excl, nt, ns, D, sub, sblock, L.stab, L.stflag, c->stream)) {
      release();
      return fail(c, RY_EHIP, "super-tile table kernels");
    }
    if (c->batch) {
      // each super-tile's box (lambda) and CFL partial slot in its box's segment
      auto* sfirst = static_cast<int32_t*>(A(sizeof(int32_t) * std::max(c->nbox, 1)));
      L.sbox = static_cast<int32_t*>(dalloc(c, sizeof(int32_t) * std::max(ns, 1)));
      L.spart = static_cast<int32_t*>(dalloc(c, sizeof(int32_t) * std::max(ns, 1)));
      if (!sfirst || !L.sbox || !L.spart) {
        release();
        return fail(c, RY_ENOMEM, "super-tile tables: allocation failed");
      }
      if (launch_super_boxes(sblock, ns, c->d_segoff, sfirst, L.sbox, L.spart, c->stream)) {
        release();
        return fail(c, RY_EHIP, "super-tile box kernels");
      }
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
      release();
      return fail(c, RY_EHIP, "super-tile table kernels");
    }
    release();
    L.n_super = ns;
  }
  L.super_ok = true;
  return RY_OK;
}

// The ghost read masks of every refined level (after a mesh change): for
// each ghost oct, which of its cells a leaf update reads.
ry_status build_ghost_read(ry_ctx* c) {
  for (int k = 0; k < c->nlev; ++k) {
    DevLevel& L = c->lev[k];
    if (L.gread) {
      dfree(c, L.gread);
      L.gread = nullptr;
    }
    if (k == 0 || L.n_ghost == 0 || L.n_tile == 0) continue;
    L.gread = static_cast<uint32_t*>(dalloc(c, sizeof(uint32_t) * L.n_ghost));
    if (!L.gread) return fail(c, RY_ENOMEM, "ghost read masks: allocation failed");
    if (launch_zero_u32(L.gread, L.n_ghost, c->stream) ||
        launch_ghost_read(L.tab, L.tflag, L.refined, L.n_tile, L.n_oct, L.gread, c->stream))
      return fail(c, RY_EHIP, "ghost read-mask kernel");
  }
  return RY_OK;
}

// Super-tile tables for every level whose tuning uses the 8^3-cell tile
// (after a mesh change, or a tuning change).
ry_status ensure_super(ry_ctx* c) {
  for (int k = 0; k < c->nlev; ++k) {
    DevLevel& L = c->lev[k];
    if (c->tune[k].tile_cells == 8 && !L.super_ok && L.n_oct > 0) {
      ry_status s = build_super(c, k);
      if (s) return s;
    }
  }
  return RY_OK;
}

// Super-tile tables of every level are stale (the mesh changed).
void drop_super(ry_ctx* c) {
  for (auto& L : c->lev) free_super(c, L);
}

// One hydro launch of level k with the level's tuning (or `t`): on the small
// tiles or, for the 8^3-cell tile, on the level's super-tiles.
ry_status enqueue_hydro(ry_ctx* c, const HydroArgs& a, int k, const ry_tuning* t = nullptr) {
  const ry_tuning& tu = t ? *t : c->tune[k];
  HydroArgs b = a;
  if (tu.tile_cells == 8) {
    const DevLevel& L = c->lev[k];
    if (!L.super_ok) return fail(c, RY_ESTATE, "level %d: super-tile tables not built", c->cfg.level_min + k);
    b.tab = L.stab;
    b.tflag = L.stflag;
    b.n_tile = L.n_super;
    if (c->batch) {
      b.tile_box = L.sbox;
      b.tile_part = L.spart;
    }
    // the 8^3-cell tile's wavefronts take an atomic maximum of the batch's
    // per-tile CFL partials: clear them (the segmented maximum of the
    // previous partials has been taken by now)
    if (b.tile_smax && launch_zero_u64(reinterpret_cast<unsigned long long*>(c->d_part), c->seg_off.back(), c->stream))
      return fail(c, RY_EHIP, "zero kernel");
  }
  if (tu.persistent && launch_zero_u32(c->d_queue, 8 * QUEUE_STRIDE, c->stream)) return fail(c, RY_EHIP, "zero kernel");
  TimedLaunch tl;
  if (c->timing) time_begin(c, "hydro", tl);
  if (launch_hydro(b, c->cfg.precision, c->cfg.nscalar, tu, c->num_cu, c->stream))
    return fail(c, RY_EHIP, "hydro kernel");
  if (c->timing) time_end(c, tl);
  return RY_OK;
}

ry_status enqueue_restrict(ry_ctx* c, int l, const int32_t* skip) {
  DevLevel& L = c->lev[l - c->cfg.level_min];
  DevLevel& F = c->lev[l + 1 - c->cfg.level_min];
  if (launch_restrict(F.U[F.cur], F.plane(), F.n_oct, F.parent_cell, L.U[L.cur ^ 1], L.plane(), c->dom.nv, skip,
                      err_ptr(c), c->stream))
    return fail(c, RY_EHIP, "restrict kernel");
  return RY_OK;
}

// Fine-first recursion of one parent step of level l (device lambda).
ry_status enqueue_level(ry_ctx* c, int l, int substep, bool last) {
  ry_status s;
  const bool fine = level_nonempty(c, l + 1);
  if (fine) {
    if ((s = enqueue_ghost(c, l + 1, skip_ptr(c)))) return s;
    if ((s = enqueue_level(c, l + 1, 0, false))) return s;
    if ((s = enqueue_level(c, l + 1, 1, last))) return s;
  }
  HydroArgs a = hydro_args(c, l, substep);
  a.lam_dev = c->d_lam;
  a.skip = skip_ptr(c);
  a.tile_smax = nullptr;
  a.smax_bits = last ? c->d_slots + int64_t(l - c->cfg.level_min) * SMAX_SLOTS : nullptr;
  if ((s = enqueue_hydro(c, a, l - c->cfg.level_min))) return s;
  if (fine && (s = enqueue_restrict(c, l, skip_ptr(c)))) return s;
  DevLevel& L = c->lev[l - c->cfg.level_min];
  L.cur ^= 1;
  return RY_OK;
}

ry_status enqueue_coarse_step(ry_ctx* c, double t_end) {
  FinalizeArgs f{};
  f.slots = c->d_slots;
  f.smax = c->d_smax;
  f.nslot = c->nlev;
  f.cfl = c->cfg.cfl;
  for (int k = 0; k < c->nlev; ++k) f.dx[k] = level_dx(c, c->cfg.level_min + k);
  f.t_end = t_end;
  f.t = c->d_t;
  f.lam = c->d_lam;
  f.skip = skip_ptr(c);
  f.done = done_ptr(c);
  f.nstep = nstep_ptr(c);
  f.batch = 0;
  if (launch_finalize(f, c->stream)) return fail(c, RY_EHIP, "finalize kernel");
  return enqueue_level(c, c->cfg.level_min, 0, true);
}

ry_status sync_and_check(ry_ctx* c) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->timing) time_collect(c);
  int32_t e = 0;
  HIPCHK(c, hipMemcpy(&e, err_ptr(c), sizeof e, hipMemcpyDeviceToHost));
  if (e & ERR_BOUNDS) return fail(c, RY_EHIP, "device index outside its buffer (debug build bounds check)");
  if (e) return fail(c, RY_ENUMERIC, "non-finite or non-positive density/energy latched on the device");
  return RY_OK;
}

// Device tables of one level (tiles, flags, refined bytes, child / parent
// maps, ghost sources, zeroed flux registers on refined levels).
void upload_level_tables(ry_ctx* c, DevLevel& D, const LevelTables& t, int k, bool& ok) {
  D.tab = upload_vec(c, t.tab, ok);
  D.tflag = upload_vec(c, t.tflag, ok);
  D.refined = upload_vec(c, t.refined_ext, ok);
  D.child = t.child.empty() ? nullptr : upload_vec(c, t.child, ok);
  D.parent_cell = t.parent_cell.empty() ? nullptr : upload_vec(c, t.parent_cell, ok);
  D.gsrc = t.gsrc.empty() ? nullptr : upload_vec(c, t.gsrc, ok);
  std::vector<double> zeros(size_t(D.n_oct) * reg_per_oct(c->dom.nv), 0.0);
  D.reg = (k > 0) ? upload_vec(c, zeros, ok) : nullptr;
}

// Sorted keys and interleaved oct coordinates of one level (device copies).
void upload_level_topology(ry_ctx* c, DevLevel& D, const HostLevel& H, bool& ok) {
  std::vector<int32_t> oc(size_t(3 * H.n));
  for (int64_t o = 0; o < H.n; ++o) {
    oc[3 * o] = H.ox[o];
    oc[3 * o + 1] = H.oy[o];
    oc[3 * o + 2] = H.oz[o];
  }
  D.dkey = upload_vec(c, H.key, ok);
  D.doc = upload_vec(c, oc, ok);
}

ry_status upload_level_state(ry_ctx* c, DevLevel& D, const double* U_host) {
  for (int b = 0; b < 2; ++b)
    for (int v = 0; v < c->dom.nv; ++v)
      HIPCHK(c, hipMemcpyAsync(D.U[b] + v * D.plane(), U_host + size_t(v) * 8 * D.n_oct,
                               sizeof(double) * 8 * D.n_oct, hipMemcpyHostToDevice, c->stream));
  return RY_OK;
}

void drop_graphs(ry_ctx* c) {
  for (auto& gs : c->graph)
    for (auto& g : gs)
      if (g) {
        hipGraphExecDestroy(g);
        g = nullptr;
      }
}

}  // namespace

// No C++ exception crosses the C ABI: a failed host allocation inside an
// entry point becomes RY_ENOMEM, any other exception RY_EINVAL.
#define RY_ABI_TRY try {
#define RY_ABI_CATCH                    \
  }                                     \
  catch (const std::bad_alloc&) {       \
    return RY_ENOMEM;                   \
  }                                     \
  catch (...) {                         \
    return RY_EINVAL;                   \
  }

extern "C" {

ry_status ry_create(const ry_config* cfg, ry_ctx** out) {
  RY_ABI_TRY
  if (!out) return RY_EINVAL;
  *out = nullptr;
  ry_status s = validate(cfg, false);
  if (s) return s;
  ry_ctx* c = new (std::nothrow) ry_ctx();
  if (!c) return RY_ENOMEM;
  c->cfg = *cfg;
  c->dom = make_dom(*cfg);
  c->nlev = cfg->level_max - cfg->level_min + 1;
  std::fill(std::begin(c->tune), std::end(c->tune), kDefaultTuning);
  if ((s = init_common(c))) {
    delete c;
    return s;
  }
  *out = c;
  return RY_OK;
  RY_ABI_CATCH
}

void ry_destroy(ry_ctx* c) {
  if (!c) return;
  free_all(c);
  if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
  if (c->h_rb) hipHostFree(c->h_rb);
  for (auto& tl : c->pending) {
    hipEventDestroy(tl.a);
    hipEventDestroy(tl.b);
  }
  delete c;
}

const char* ry_last_error(const ry_ctx* c) { return c ? c->err.c_str() : "null context"; }

ry_status ry_amr_build(ry_ctx* c, const double* U_base, ry_fill_fn fill, void* user) {
  RY_ABI_TRY
  if (!c || !U_base || c->batch) return RY_EINVAL;
  if (c->cfg.level_max > c->cfg.level_min && c->cfg.refine != RY_REFINE_NONE && !fill)
    return fail(c, RY_EINVAL, "fill callback required when level_max > level_min");
  free_all(c);
  c->built = false;
  std::vector<HostLevel> H;
  std::string e = build_mesh(c->dom, U_base, fill, user, H);
  if (!e.empty()) return fail(c, RY_EINVAL, "%s", e.c_str());
  std::vector<LevelTables> T;
  e = build_tables(c->dom, H, T);
  if (!e.empty()) return fail(c, RY_EINVAL, "%s", e.c_str());
  c->lev.assign(c->nlev, DevLevel());
  bool ok = true;
  for (int k = 0; k < c->nlev && ok; ++k) {
    DevLevel& D = c->lev[k];
    LevelTables& t = T[k];
    D.n_oct = t.n_oct;
    D.n_ghost = t.n_ghost;
    D.n_ext = t.n_oct + t.n_ghost;
    D.n_leaf = t.n_leaf;
    D.n_tile = t.n_tile;
    if (D.n_oct == 0) continue;
    if (!alloc_state_pair(c, D.U, D.n_ext, c->dom.nv)) ok = false;
    if (!ok) break;
    if (upload_level_state(c, D, H[k].U.data())) return c->err.empty() ? RY_EHIP : RY_EHIP;
    upload_level_tables(c, D, t, k, ok);
    upload_level_topology(c, D, H[k], ok);
  }
  if (!ok) {
    free_all(c);
    return fail(c, RY_ENOMEM, "device allocation failed");
  }
  c->seg_off.assign(1, 0);
  for (int k = 0; k < c->nlev; ++k) c->seg_off.push_back(c->seg_off.back() + part_slots(c->lev[k]));
  ry_status s = alloc_scalars(c, std::max(c->nlev, 1));
  if (s) {
    free_all(c);
    return fail(c, s, "device allocation failed");
  }
  std::fill(std::begin(c->count), std::end(c->count), 0);
  if ((s = enqueue_cfl_all(c))) return s;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if ((s = build_ghost_read(c))) return s;
  if ((s = ensure_super(c))) return s;
  for (auto& h : H) std::vector<double>().swap(h.U);
  c->host = std::move(H);
  c->host_valid = true;
  c->means_valid = true;   // the builder restricts every refined cell
  c->built = true;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_set_refine_param(ry_ctx* c, double value) {
  RY_ABI_TRY
  if (!c || c->batch || std::isnan(value)) return RY_EINVAL;
  c->cfg.refine_param = value;
  c->dom.refine_param = value;
  return RY_OK;
  RY_ABI_CATCH
}

}  // extern "C"

namespace {

// Host copy of the mesh topology from the device mirrors (after a device
// regrid the host copy is stale).
ry_status refresh_host_topology(ry_ctx* c) {
  if (c->host_valid) return RY_OK;
  c->host.assign(c->nlev, HostLevel());
  for (int k = 0; k < c->nlev; ++k) {
    DevLevel& D = c->lev[k];
    HostLevel& H = c->host[k];
    H.n = D.n_oct;
    H.key.resize(H.n);
    H.refined.resize(H.n);
    std::vector<int32_t> oc(size_t(3 * H.n));
    if (H.n) {
      HIPCHK(c, hipMemcpy(H.key.data(), D.dkey, sizeof(uint64_t) * H.n, hipMemcpyDeviceToHost));
      HIPCHK(c, hipMemcpy(H.refined.data(), D.refined, H.n, hipMemcpyDeviceToHost));
      HIPCHK(c, hipMemcpy(oc.data(), D.doc, sizeof(int32_t) * oc.size(), hipMemcpyDeviceToHost));
    }
    H.ox.resize(H.n);
    H.oy.resize(H.n);
    H.oz.resize(H.n);
    for (int64_t o = 0; o < H.n; ++o) {
      H.ox[o] = oc[3 * o];
      H.oy[o] = oc[3 * o + 1];
      H.oz[o] = oc[3 * o + 2];
    }
    H.index.build(H.ox, H.oy, H.oz);
  }
  c->host_valid = true;
  return RY_OK;
}

ry_status finish_regrid(ry_ctx* c, const std::vector<uint8_t*>* dirty = nullptr);

// Regrid with flags and tables built on the host (the state stays on the
// device).
ry_status regrid_host(ry_ctx* c, int64_t* n_created, int64_t* n_destroyed) {
  ry_status s = refresh_host_topology(c);
  if (s) return s;
  const int nl = c->nlev, nv = c->dom.nv;
  std::vector<HostLevel>& H = c->host;
  // new state of levels 1.. (level 0 keeps its octs and its buffers)
  std::vector<double*> tmp(nl, nullptr);
  int64_t created = 0, destroyed = 0;
  for (int k = 0; k + 1 < nl; ++k) {
    const int l = c->cfg.level_min + k;
    DevLevel& Lk = c->lev[k];
    const double* Uk = (k == 0) ? Lk.U[Lk.cur] : tmp[k];
    const int64_t pk = (k == 0) ? Lk.plane() : 8 * H[k].n;
    std::vector<double> rho(size_t(8 * H[k].n));
    if (H[k].n) HIPCHK(c, hipMemcpy(rho.data(), Uk, sizeof(double) * rho.size(), hipMemcpyDeviceToHost));
    HostLevel Fnew;
    std::vector<int32_t> src_old, src7;
    std::string e = regrid_level(c->dom, l, H[k], rho, H[k + 1], Fnew, src_old, src7, created, destroyed);
    if (!e.empty()) return fail(c, RY_EINVAL, "%s", e.c_str());
    if (Fnew.n > 0) {
      bool ok = true;
      tmp[k + 1] = static_cast<double*>(dalloc(c, sizeof(double) * nv * 8 * Fnew.n));
      int32_t* d_old = upload_vec(c, src_old, ok);
      int32_t* d_src = upload_vec(c, src7, ok);
      if (!tmp[k + 1] || !ok) {
        for (double* p : tmp) dfree(c, p);
        dfree(c, d_old);
        dfree(c, d_src);
        return fail(c, RY_ENOMEM, "regrid allocation failed (mesh unchanged on the device, host topology stale)");
      }
      const DevLevel& Fo = c->lev[k + 1];
      if (launch_regrid_remap(d_old, d_src, Fnew.n, Fo.n_oct ? Fo.U[Fo.cur] : nullptr, Fo.plane(), Uk, pk,
                              tmp[k + 1], 8 * Fnew.n, nv, c->stream))
        return fail(c, RY_EHIP, "regrid remap kernel");
      HIPCHK(c, hipStreamSynchronize(c->stream));
      dfree(c, d_old);
      dfree(c, d_src);
    }
    H[k + 1] = std::move(Fnew);
  }
  // tables of the new mesh
  std::vector<LevelTables> T;
  std::string e = build_tables(c->dom, H, T);
  if (!e.empty()) return fail(c, RY_EINVAL, "%s", e.c_str());
  // release the old per-level arrays (level 0 keeps its state buffers)
  for (int k = 0; k < nl; ++k) {
    DevLevel& D = c->lev[k];
    for (void* p : {(void*)D.tab, (void*)D.tflag, (void*)D.refined, (void*)D.child, (void*)D.parent_cell,
                    (void*)D.gsrc, (void*)D.reg, (void*)D.dkey, (void*)D.doc})
      dfree(c, p);
    D.dkey = nullptr;
    D.doc = nullptr;
    if (k > 0) {
      dfree(c, D.U[0]);   // both buffers
      D.U[0] = D.U[1] = nullptr;
    }
    D.tab = nullptr;
    D.tflag = nullptr;
    D.refined = nullptr;
    D.child = nullptr;
    D.parent_cell = nullptr;
    D.gsrc = nullptr;
    D.reg = nullptr;
  }
  bool ok = true;
  for (int k = 0; k < nl && ok; ++k) {
    DevLevel& D = c->lev[k];
    const LevelTables& t = T[k];
    D.n_oct = t.n_oct;
    D.n_ghost = t.n_ghost;
    D.n_ext = t.n_oct + t.n_ghost;
    D.n_leaf = t.n_leaf;
    D.n_tile = t.n_tile;
    if (D.n_oct == 0) continue;
    if (k > 0) {
      D.cur = 0;
      if (!alloc_state_pair(c, D.U, D.n_ext, nv)) ok = false;
      if (!ok) break;
      for (int v = 0; v < nv; ++v)
        HIPCHK(c, hipMemcpyAsync(D.U[0] + v * D.plane(), tmp[k] + v * 8 * D.n_oct, sizeof(double) * 8 * D.n_oct,
                                 hipMemcpyDeviceToDevice, c->stream));
    }
    upload_level_tables(c, D, t, k, ok);
    upload_level_topology(c, D, H[k], ok);
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (double* p : tmp) dfree(c, p);
  if (!ok) {
    free_all(c);
    c->built = false;
    return fail(c, RY_ENOMEM, "regrid allocation failed; the context must be rebuilt");
  }
  if ((s = finish_regrid(c))) return s;
  if (n_created) *n_created = created;
  if (n_destroyed) *n_destroyed = destroyed;
  return RY_OK;
}

// Common tail of both regrid paths: CFL partial slots for the new tile
// counts, restriction bottom-up, CFL data; graphs and subcycle counters reset.
// dirty (device regrid): per level, the octs whose state changed (new, or a
// cell restricted again), filled bottom-up by the restriction; null: every
// refined cell is restricted.
ry_status finish_regrid(ry_ctx* c, const std::vector<uint8_t*>* dirty) {
  const int nl = c->nlev, nv = c->dom.nv;
  ry_status s;
  dfree(c, c->d_part);
  dfree(c, c->d_segoff);
  c->seg_off.assign(1, 0);
  for (int k = 0; k < nl; ++k) c->seg_off.push_back(c->seg_off.back() + part_slots(c->lev[k]));
  c->d_part = static_cast<double*>(dalloc(c, sizeof(double) * std::max<int64_t>(c->seg_off.back(), 1)));
  c->d_segoff = static_cast<int64_t*>(dalloc(c, sizeof(int64_t) * c->seg_off.size()));
  if (!c->d_part || !c->d_segoff) {
    free_all(c);
    c->built = false;
    return fail(c, RY_ENOMEM, "regrid allocation failed; the context must be rebuilt");
  }
  HIPCHK(c, hipMemcpyAsync(c->d_segoff, c->seg_off.data(), sizeof(int64_t) * c->seg_off.size(),
                           hipMemcpyHostToDevice, c->stream));
  // refined cells = ordered 8-child means, bottom-up (after a device
  // regrid only those above changed octs: the others hold these means)
  for (int k = nl - 2; k >= 0; --k) {
    DevLevel& L = c->lev[k];
    DevLevel& F = c->lev[k + 1];
    if (F.n_oct == 0) continue;
    const int rc = dirty ? launch_restrict_dirty(F.U[F.cur], F.plane(), F.n_oct, F.parent_cell, L.U[L.cur],
                                                 L.plane(), nv, (*dirty)[k + 1], k > 0 ? (*dirty)[k] : nullptr,
                                                 err_ptr(c), c->stream)
                         : launch_restrict(F.U[F.cur], F.plane(), F.n_oct, F.parent_cell, L.U[L.cur], L.plane(),
                                           nv, nullptr, err_ptr(c), c->stream);
    if (rc) return fail(c, RY_EHIP, "restrict kernel");
  }
  drop_graphs(c);
  drop_super(c);
  std::fill(std::begin(c->count), std::end(c->count), 0);
  c->slots_valid = false;
  if ((s = build_ghost_read(c))) return s;
  if ((s = ensure_super(c))) return s;
  if ((s = enqueue_cfl_all(c))) return s;
  if ((s = sync_and_check(c))) return s;
  c->means_valid = true;
  return RY_OK;
}

// Regrid with the mesh work on the device: per level, refinement flags from
// the new state, the child level in Hilbert order (kept octs copied, new octs
// interpolated), then its tiles, 4x4x4 tables, ghost octs and their sources.
// The host only reads back counts.  Level lmin keeps its octs, state and
// tile tables.
ry_status regrid_device(ry_ctx* c, int64_t* n_created, int64_t* n_destroyed) {
  const int nl = c->nlev, nv = c->dom.nv, lmin = c->cfg.level_min;
  hipStream_t st = c->stream;
  RegridDom RD{};
  for (int i = 0; i < 6; ++i) RD.bc[i] = c->dom.bc[i];
  RD.lmin = lmin;
  RD.refine = c->dom.refine;
  RD.refine_param = c->dom.refine_param;

  struct NewLevel {
    int64_t n = 0, n_ghost = 0, n_leaf = 0;
    int32_t n_tile = 0;
    uint64_t* key = nullptr;
    int32_t* oc = nullptr;
    int32_t* parent = nullptr;
    uint8_t* flag = nullptr;
    int32_t* child = nullptr;
    int32_t* tab = nullptr;
    uint32_t* tflag = nullptr;
    int32_t* tile_of = nullptr;        // refined levels: each oct's tile and each tile's
    int32_t* tfirst = nullptr;         // first oct (from the parent level's children kernel)
    uint8_t* fresh = nullptr;          // refined levels: 1 for octs not in the old level
    uint8_t* refined = nullptr;
    int64_t* gsrc = nullptr;
    double* reg = nullptr;
    double* U[2] = {nullptr, nullptr};
  };
  std::vector<NewLevel> N(nl);
  std::vector<unsigned long long*> H(nl, nullptr);   // position hash of each new level
  std::vector<std::vector<LevelView>> coarse_views;   // host sources of async copies, kept to the end
  std::vector<uint64_t> HE(nl, 0);                    // its entries
  std::vector<void*> fresh, temps;   // new level arrays / scratch of this call
  bool ok = true;
  // new level arrays: one allocation each (they outlive the call); scratch:
  // 256-byte-aligned pieces of a few large chunks (64 MiB, then doubling),
  // all released at the end
  struct Chunk {
    char* base;
    size_t size, used;
  };
  std::vector<Chunk> chunks;
  auto A = [&](size_t bytes, bool temp) -> void* {
    if (!temp) {
      void* p = dalloc(c, bytes);
      if (!p) ok = false;
      else fresh.push_back(p);
      return p;
    }
    bytes = std::max<size_t>(256, (bytes + 255) & ~size_t(255));
    if (chunks.empty() || chunks.back().used + bytes > chunks.back().size) {
      const size_t sz = std::max(bytes, chunks.empty() ? size_t(64) << 20 : 2 * chunks.back().size);
      void* p = dalloc(c, sz);
      if (!p) {
        ok = false;
        return nullptr;
      }
      temps.push_back(p);
      chunks.push_back({static_cast<char*>(p), sz, 0});
    }
    Chunk& ch = chunks.back();
    void* p = ch.base + ch.used;
    ch.used += bytes;
    return p;
  };
  auto release = [&](std::vector<void*>& v) {
    for (void* p : v) dfree(c, p);
    v.clear();
  };
  // failure before the new mesh is installed: the old mesh stays as it was
  auto abandon = [&](ry_status s, const char* what) {
    (void)hipStreamSynchronize(st);
    release(temps);
    release(fresh);
    return fail(c, s, "regrid: %s (mesh unchanged)", what);
  };
#define RG_TRY(cond, status, what) \
  do {                              \
    if (!(cond)) return abandon(status, what); \
  } while (0)
  auto view = [&](int k) {
    LevelView v{};
    v.key = N[k].key;
    v.oc = N[k].oc;
    v.n = N[k].n;
    v.bits = c->dom.hbits0 + k;
    for (int a = 0; a < 3; ++a) v.noct[a] = int32_t(c->dom.noct(lmin + k, a));
    v.hash = H[k];
    v.hmask = HE[k] ? HE[k] - 1 : 0;
    return v;
  };
  // exclusive scan of n counts; returns the total (stream synchronised)
  auto scan_total = [&](const int32_t* in, int32_t* out, int64_t n, int64_t& total) -> bool {
    const int nt = scan_tmp_ints(n);
    int32_t* tmp = static_cast<int32_t*>(A(sizeof(int32_t) * nt, true));
    if (!tmp || launch_scan(in, out, n, tmp, st)) return false;
    int32_t h = 0;
    if (hipMemcpyAsync(&h, tmp + nt - 1, sizeof h, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return false;
    total = h;
    return true;
  };
  // two exclusive scans of n counts and both totals in one round trip
  auto scan_totals = [&](const int32_t* in1, int32_t* out1, const int32_t* in2, int32_t* out2, int64_t n,
                         int64_t& total1, int64_t& total2) -> bool {
    const int nt = scan_tmp_ints(n);
    int32_t* tmp1 = static_cast<int32_t*>(A(sizeof(int32_t) * nt, true));
    int32_t* tmp2 = static_cast<int32_t*>(A(sizeof(int32_t) * nt, true));
    if (!tmp1 || !tmp2 || launch_scan(in1, out1, n, tmp1, st) || launch_scan(in2, out2, n, tmp2, st)) return false;
    int32_t h[2] = {0, 0};
    if (hipMemcpyAsync(&h[0], tmp1 + nt - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&h[1], tmp2 + nt - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return false;
    total1 = h[0];
    total2 = h[1];
    return true;
  };
  int32_t* d_err = static_cast<int32_t*>(A(sizeof(int32_t), true));
  // per level: children of the new level found in the old one
  auto* d_kept = static_cast<unsigned long long*>(A(sizeof(unsigned long long) * nl, true));
  RG_TRY(ok && hipMemsetAsync(d_err, 0, sizeof(int32_t), st) == hipSuccess &&
             hipMemsetAsync(d_kept, 0, sizeof(unsigned long long) * nl, st) == hipSuccess,
         RY_ENOMEM, "allocation failed");
  std::vector<int64_t> n_new(nl, 0), n_prev(nl, 0);   // child level sizes, new and old

  {  // level lmin keeps its octs and tile tables (a complete level: no ghost octs)
    const DevLevel& D = c->lev[0];
    RG_TRY(D.n_ghost == 0, RY_EINVAL, "base level with ghost octs");
    N[0].n = D.n_oct;
    N[0].key = D.dkey;
    N[0].oc = D.doc;
    N[0].n_tile = D.n_tile;
    N[0].tab = D.tab;
    N[0].tflag = D.tflag;
    N[0].U[0] = D.U[D.cur];
  }
  int64_t created = 0, destroyed = 0;
  int32_t* src_old = nullptr;   // remap sources of the level built last
  int32_t* src7 = nullptr;
  for (int k = 0; k < nl; ++k) {
    NewLevel& L = N[k];
    const int l = lmin + k;
    if (L.n == 0) {
      if (k + 1 < nl) destroyed += c->lev[k + 1].n_oct;
      continue;
    }
    // the device regrid counts cells (8 per oct) and tile slots (64 per tile)
    // in 32-bit integers
    RG_TRY(L.n < (int64_t(1) << 28), RY_EINVAL, "level too large for the device regrid (use the host path)");
    // the level's aligned 2x2x2 blocks of octs are its tiles
    HE[k] = pos_hash_entries(std::max<int64_t>(L.n_tile, (L.n + 7) / 8));
    H[k] = static_cast<unsigned long long*>(A(64 * HE[k], true));
    RG_TRY(ok, RY_ENOMEM, "allocation failed");
    RG_TRY(!launch_pos_hash(L.key, L.oc, L.n, H[k], HE[k], d_err, st), RY_EHIP, "position hash kernel");
    const LevelView V = view(k);
    // what the flag kernel reads of the tiles (refined levels) or of a
    // complete level (the base level, when it holds every position)
    FlagTiles FT{};
    FT.n_oct = L.n;
    FT.complete = k == 0 && L.n == c->dom.noct(l, 0) * c->dom.noct(l, 1) * c->dom.noct(l, 2);
    if (k > 0) {
      // tiles: octs sharing key >> 3, the children of one parent oct (listed
      // by the parent level's children kernel)
      const int64_t nt = L.n_tile;
      int32_t* first = L.tfirst;
      const int64_t nslot = nt * TILE_TAB;
      L.tab = static_cast<int32_t*>(A(sizeof(int32_t) * nslot, false));
      L.tflag = static_cast<uint32_t*>(A(sizeof(uint32_t) * nt, false));
      int32_t* miss = static_cast<int32_t*>(A(sizeof(int32_t) * nslot, true));
      int32_t* midx = static_cast<int32_t*>(A(sizeof(int32_t) * nslot, true));
      auto* pres = static_cast<unsigned long long*>(A(sizeof(unsigned long long) * nt, true));
      RG_TRY(ok, RY_ENOMEM, "allocation failed");
      FT.tile_of = L.tile_of;
      FT.pres = pres;
      FT.tab = L.tab;
      int64_t nm = 0;
      RG_TRY(!launch_tile_table(V, RD, first, L.n_tile, L.tab, L.tflag, miss, pres, st) &&
                 scan_total(miss, midx, nslot, nm),
             RY_EHIP, "tile table kernels");
      // ghost octs: numbered by first use over (tile, slot)
      int32_t* gpos = nullptr;
      if (nm > 0) {
        uint64_t hsize = 64;
        while (hsize < 2 * uint64_t(nm)) hsize <<= 1;
        uint64_t* mpos = static_cast<uint64_t*>(A(sizeof(uint64_t) * nm, true));
        int32_t* mentry = static_cast<int32_t*>(A(sizeof(int32_t) * nm, true));
        auto* hkey = static_cast<unsigned long long*>(A(sizeof(unsigned long long) * hsize, true));
        int32_t* hval = static_cast<int32_t*>(A(sizeof(int32_t) * hsize, true));
        int32_t* owner = static_cast<int32_t*>(A(sizeof(int32_t) * nm, true));
        int32_t* gidx = static_cast<int32_t*>(A(sizeof(int32_t) * nm, true));
        const int ntmp = scan_tmp_ints(nm);
        int32_t* gtmp = static_cast<int32_t*>(A(sizeof(int32_t) * ntmp, true));
        gpos = static_cast<int32_t*>(A(sizeof(int32_t) * 3 * nm, true));
        RG_TRY(ok, RY_ENOMEM, "allocation failed");
        RG_TRY(!launch_missing_list(V, first, L.n_tile, miss, midx, mpos, mentry, st) &&
                   !launch_ghost_numbering(mpos, mentry, nm, hkey, hval, hsize, owner, gidx, gtmp, L.n, L.tab, gpos,
                                           st),
               RY_EHIP, "ghost numbering kernels");
        int32_t h = 0;
        RG_TRY(hipMemcpyAsync(&h, gtmp + ntmp - 1, sizeof h, hipMemcpyDeviceToHost, st) == hipSuccess &&
                   hipStreamSynchronize(st) == hipSuccess,
               RY_EHIP, "ghost count");
        L.n_ghost = h;
      }
      if (L.n_ghost > 0) {
        coarse_views.emplace_back(k);
        std::vector<LevelView>& cv = coarse_views.back();
        for (int j = 0; j < k; ++j) cv[j] = view(k - 1 - j);
        LevelView* d_cv = static_cast<LevelView*>(A(sizeof(LevelView) * k, true));
        L.gsrc = static_cast<int64_t*>(A(sizeof(int64_t) * 7 * L.n_ghost, false));
        RG_TRY(ok, RY_ENOMEM, "allocation failed");
        RG_TRY(hipMemcpyAsync(d_cv, cv.data(), sizeof(LevelView) * k, hipMemcpyHostToDevice, st) == hipSuccess &&
                   !launch_ghost_sources(d_cv, k, RD, gpos, L.n_ghost, L.gsrc, d_err, st),
               RY_EHIP, "ghost source kernel");
      }
      // state: kept octs copied, new octs interpolated from level l-1
      const int64_t n_ext = L.n + L.n_ghost;
      RG_TRY(level_index_fits(L.n, L.n_ghost, nv), RY_EINVAL,
             "level octs + ghost octs reach the 32-bit cell index (2^29 octs; (1 + nv) times the octs + ghost octs "
             "with ghosts)");
      // both state buffers in one allocation (ghosts in the second, read
      // through the first with a fixed index shift)
      L.U[0] = static_cast<double*>(A(sizeof(double) * 2 * nv * 8 * n_ext, false));
      L.U[1] = L.U[0] ? L.U[0] + size_t(nv) * 8 * n_ext : nullptr;
      L.reg = static_cast<double*>(A(sizeof(double) * L.n * reg_per_oct(nv), false));
      RG_TRY(ok, RY_ENOMEM, "allocation failed");
      const DevLevel& Fo = c->lev[k];
      const double* Uc = N[k - 1].U[0];
      const int64_t pc = (k == 1) ? c->lev[0].plane() : 8 * (N[k - 1].n + N[k - 1].n_ghost);
      RG_TRY(!launch_regrid_remap(src_old, src7, L.n, Fo.n_oct ? Fo.U[Fo.cur] : nullptr, Fo.plane(), Uc, pc, L.U[0],
                                  8 * n_ext, nv, st) &&
                 !launch_zero_u64(reinterpret_cast<unsigned long long*>(L.reg), L.n * reg_per_oct(nv), st),
             RY_EHIP, "regrid remap kernel");
    }
    // flags of level l from its new state, the child level, its remap sources
    int64_t n_fine = 0;
    L.flag = static_cast<uint8_t*>(A(L.n, true));
    RG_TRY(ok, RY_ENOMEM, "allocation failed");
    if (k + 1 < nl) {
      int32_t* cnt = static_cast<int32_t*>(A(sizeof(int32_t) * L.n, true));
      int32_t* off = static_cast<int32_t*>(A(sizeof(int32_t) * L.n, true));
      int32_t* has = static_cast<int32_t*>(A(sizeof(int32_t) * L.n, true));
      int32_t* toff = static_cast<int32_t*>(A(sizeof(int32_t) * L.n, true));
      RG_TRY(ok, RY_ENOMEM, "allocation failed");
      // child octs and child tiles (parents with children): both counts in
      // one round trip
      int64_t n_ctile = 0;
      RG_TRY(!launch_regrid_flags(V, RD, l, L.U[0], FT, L.flag, cnt, has, st) &&
                 scan_totals(cnt, off, has, toff, L.n, n_fine, n_ctile),
             RY_EHIP, "regrid flag kernel");
      RG_TRY(n_ctile * TILE_TAB < (int64_t(1) << 31), RY_EINVAL,
             "level too large for the device regrid (use the host path)");
      NewLevel& F = N[k + 1];
      F.n = n_fine;
      F.n_tile = int32_t(n_ctile);
      const int64_t n_old = c->lev[k + 1].n_oct;
      n_new[k + 1] = n_fine;
      n_prev[k + 1] = n_old;
      if (n_fine > 0) {
        F.key = static_cast<uint64_t*>(A(sizeof(uint64_t) * n_fine, false));
        F.oc = static_cast<int32_t*>(A(sizeof(int32_t) * 3 * n_fine, false));
        F.parent = static_cast<int32_t*>(A(sizeof(int32_t) * n_fine, false));
        L.child = static_cast<int32_t*>(A(sizeof(int32_t) * 8 * L.n, false));
        // the old tree: level l's octs in the old level (its remap sources;
        // the base level is unchanged) and the old level l's child map
        OldTree OT{};
        OT.old_of = k == 0 ? nullptr : src_old;
        OT.old_child = n_old > 0 ? c->lev[k].child : nullptr;
        RG_TRY(n_old == 0 || OT.old_child, RY_EINVAL, "old level without a child map");
        src_old = static_cast<int32_t*>(A(sizeof(int32_t) * n_fine, true));
        src7 = static_cast<int32_t*>(A(sizeof(int32_t) * 7 * n_fine, true));
        F.tile_of = static_cast<int32_t*>(A(sizeof(int32_t) * n_fine, true));
        F.tfirst = static_cast<int32_t*>(A(sizeof(int32_t) * (n_ctile + 1), true));
        F.fresh = static_cast<uint8_t*>(A(n_fine, true));
        RG_TRY(ok, RY_ENOMEM, "allocation failed");
        const ChildTiles CT{toff, int32_t(n_ctile), F.tile_of, F.tfirst, F.fresh};
        RG_TRY(!launch_regrid_children(V, OT, RD, c->dom.hbits0 + k + 1, L.flag, off, CT, F.key, F.oc, F.parent,
                                       L.child, src_old, src7, d_err, d_kept + k + 1, st),
               RY_EHIP, "regrid children kernel");
      }
    } else {
      RG_TRY(hipMemsetAsync(L.flag, 0, L.n, st) == hipSuccess, RY_EHIP, "flag clear");
    }
    L.n_leaf = 8 * L.n - n_fine;
    L.refined = static_cast<uint8_t*>(A(L.n + L.n_ghost, false));
    RG_TRY(ok, RY_ENOMEM, "allocation failed");
    RG_TRY(!launch_refined_ext(L.flag, L.n, L.n + L.n_ghost, L.refined, st), RY_EHIP, "refined kernel");
  }
  int32_t herr = 0;
  std::vector<unsigned long long> kept(nl, 0);
  RG_TRY(hipMemcpyAsync(&herr, d_err, sizeof herr, hipMemcpyDeviceToHost, st) == hipSuccess &&
             hipMemcpyAsync(kept.data(), d_kept, sizeof(unsigned long long) * nl, hipMemcpyDeviceToHost, st) ==
                 hipSuccess &&
             hipStreamSynchronize(st) == hipSuccess,
         RY_EHIP, "regrid kernels");
  for (int k = 1; k < nl; ++k) {
    created += n_new[k] - int64_t(kept[k]);
    destroyed += n_prev[k] - int64_t(kept[k]);
  }
  RG_TRY(herr == 0, RY_EINVAL,
         herr & 4 ? "position hash full" : herr & 1 ? "interpolation source missing" : "ghost source missing");
#undef RG_TRY
  // install: release the old arrays (level lmin keeps state, keys, tables)
  for (int k = 0; k < nl; ++k) {
    DevLevel& D = c->lev[k];
    for (void* p : {(void*)D.refined, (void*)D.child, (void*)D.parent_cell, (void*)D.gsrc, (void*)D.reg})
      dfree(c, p);
    if (k > 0) {
      for (void* p : {(void*)D.tab, (void*)D.tflag, (void*)D.dkey, (void*)D.doc, (void*)D.U[0]})
        dfree(c, p);
      D.tab = nullptr;
      D.tflag = nullptr;
      D.dkey = nullptr;
      D.doc = nullptr;
      D.U[0] = D.U[1] = nullptr;
      D.cur = 0;
    }
    const NewLevel& L = N[k];
    D.n_oct = L.n;
    D.n_ghost = L.n_ghost;
    D.n_ext = L.n + L.n_ghost;
    D.n_leaf = L.n_leaf;
    D.refined = L.n ? L.refined : nullptr;
    D.child = (k + 1 < nl && N[k + 1].n > 0) ? L.child : nullptr;
    D.parent_cell = L.parent;
    D.gsrc = L.gsrc;
    D.reg = L.reg;
    if (k > 0) {
      D.n_tile = L.n_tile;
      D.tab = L.tab;
      D.tflag = L.tflag;
      D.dkey = L.key;
      D.doc = L.oc;
      D.U[0] = L.U[0];
      D.U[1] = L.U[1];
    }
  }
  fresh.clear();
  c->host_valid = false;
  // the restriction reads the new-oct marks (scratch): released after it;
  // all refined cells are restricted when an upload may have left means
  // out of date
  std::vector<uint8_t*> dirty(nl, nullptr);
  for (int k = 1; k < nl; ++k) dirty[k] = N[k].fresh;
  ry_status s = finish_regrid(c, c->means_valid ? &dirty : nullptr);
  release(temps);
  if (s) return s;
  if (n_created) *n_created = created;
  if (n_destroyed) *n_destroyed = destroyed;
  return RY_OK;
}

}  // namespace

extern "C" {

ry_status ry_set_regrid_device(ry_ctx* c, int32_t on) {
  RY_ABI_TRY
  if (!c || c->batch) return RY_EINVAL;
  c->regrid_device = on != 0;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_regrid(ry_ctx* c, int64_t* n_created, int64_t* n_destroyed) {
  RY_ABI_TRY
  if (!c || c->batch) return RY_EINVAL;
  if (!c->built) return fail(c, RY_ESTATE, "not built");
  for (int k = 0; k < c->nlev; ++k)
    if (c->count[k]) return fail(c, RY_ESTATE, "regrid inside a coarse step");
  ry_status s = sync_and_check(c);
  if (s) return s;
  return c->regrid_device ? regrid_device(c, n_created, n_destroyed) : regrid_host(c, n_created, n_destroyed);
  RY_ABI_CATCH
}

ry_status ry_level_info(const ry_ctx* c, int32_t level, int64_t* n_oct, int64_t* n_leaf) {
  RY_ABI_TRY
  if (!c || !c->built || c->batch || level < c->cfg.level_min || level > c->cfg.level_max) return RY_EINVAL;
  const DevLevel& D = c->lev[level - c->cfg.level_min];
  if (n_oct) *n_oct = D.n_oct;
  if (n_leaf) *n_leaf = D.n_leaf;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_get_mesh(const ry_ctx* c, int32_t level, uint64_t* keys, uint8_t* refined) {
  RY_ABI_TRY
  if (!c || !c->built || c->batch || level < c->cfg.level_min || level > c->cfg.level_max) return RY_EINVAL;
  const DevLevel& D = c->lev[level - c->cfg.level_min];
  if (!D.n_oct) return RY_OK;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return RY_EHIP;
  if (keys && hipMemcpy(keys, D.dkey, sizeof(uint64_t) * D.n_oct, hipMemcpyDeviceToHost) != hipSuccess) return RY_EHIP;
  if (refined && hipMemcpy(refined, D.refined, D.n_oct, hipMemcpyDeviceToHost) != hipSuccess) return RY_EHIP;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_cfl_dt(ry_ctx* c, double* dt) {
  RY_ABI_TRY
  if (!c || !dt || !c->built || c->batch) return RY_EINVAL;
  ry_status s = enqueue_cfl_all(c);
  if (s) return s;
  if ((s = sync_and_check(c))) return s;
  std::vector<double> sm(c->nlev);
  HIPCHK(c, hipMemcpy(sm.data(), c->d_smax, sizeof(double) * c->nlev, hipMemcpyDeviceToHost));
  double best = INFINITY;
  for (int k = 0; k < c->nlev; ++k) {
    const double smax = sm[k];
    if (!(smax > 0.0)) continue;
    const double dtl = c->cfg.cfl * level_dx(c, c->cfg.level_min + k) / smax;
    const double cand = std::ldexp(dtl, k);
    if (cand < best) best = cand;
  }
  *dt = best;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_hydro_step(ry_ctx* c, int32_t level, double dt) {
  RY_ABI_TRY
  if (!c || c->batch) return RY_EINVAL;
  if (!c->built) return fail(c, RY_ESTATE, "not built");
  if (!(dt > 0.0) || !std::isfinite(dt) || !level_nonempty(c, level)) return fail(c, RY_EINVAL, "bad level or dt");
  const int lmin = c->cfg.level_min;
  const int k = level - lmin;
  const bool fine = level_nonempty(c, level + 1);
  if (fine) {
    if (c->count[k + 1] != 2) return fail(c, RY_ESTATE, "level %d needs two steps of level %d first", level, level + 1);
    if (dt != 2.0 * c->dt_of[k + 1]) return fail(c, RY_EINVAL, "dt must be twice the finer level's dt");
  }
  if (level > lmin) {
    if (c->count[k] >= 2) return fail(c, RY_ESTATE, "level %d already took two substeps", level);
    if (c->count[k] == 1 && dt != c->dt_of[k]) return fail(c, RY_EINVAL, "both substeps need the same dt");
  }
  ry_status s;
  if (level > lmin && c->count[k] == 0 && (s = enqueue_ghost(c, level, nullptr))) return s;
  HydroArgs a = hydro_args(c, level, level > lmin ? c->count[k] : 0);
  a.lam_dev = nullptr;
  a.lam_host = dt / level_dx(c, level);
  a.skip = nullptr;
  a.tile_smax = nullptr;
  if ((s = enqueue_hydro(c, a, k))) return s;
  if (fine && (s = enqueue_restrict(c, level, nullptr))) return s;
  c->lev[k].cur ^= 1;
  c->dt_of[k] = dt;
  if (level > lmin) c->count[k] += 1;
  if (fine) c->count[k + 1] = 0;
  c->slots_valid = false;
  drop_graphs(c);
  return RY_OK;
  RY_ABI_CATCH
}

// Coarse steps per captured graph: 2^g for g = 0..4.  A run of n steps
// launches the largest graphs that fit (20 steps: 16 + 4), so that the gap of
// a few microseconds each graph launch costs is paid about once per 16
// steps; every graph but the 1-step one has an even step count, so every
// level's buffer parity is back where it started after it.
constexpr int kGraphLevels = 5;

static ry_status capture_step(ry_ctx* c, int gi, int par, double t_end) {
  hipGraphExec_t& ge = c->graph[gi][par];
  if (ge) {
    hipGraphExecDestroy(ge);
    ge = nullptr;
  }
  std::vector<int> saved;
  for (auto& L : c->lev) saved.push_back(L.cur);
  hipGraph_t g = nullptr;
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  ry_status s = RY_OK;
  for (int k = 0; k < (1 << gi) && !s; ++k) s = enqueue_coarse_step(c, t_end);
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  for (size_t i = 0; i < c->lev.size(); ++i) c->lev[i].cur = saved[i];
  if (s) {
    if (g) hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(c, RY_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) return fail(c, RY_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  c->graph_par[gi][par] = saved;
  c->graph_tend[gi][par] = t_end;
  return RY_OK;
}

ry_status ry_advance(ry_ctx* c, int32_t n_coarse, double t_end, double* t_io) {
  RY_ABI_TRY
  if (!c || !t_io || c->batch || n_coarse < 0) return RY_EINVAL;
  if (!c->built) return fail(c, RY_ESTATE, "not built");
  for (int k = 1; k < c->nlev; ++k)
    if (c->count[k] != 0) return fail(c, RY_ESTATE, "ry_advance called inside a coarse step");
  ry_status s;
  if (!c->slots_valid && (s = enqueue_cfl_all(c))) return s;
  // the time goes up and comes back through a pinned buffer (asynchronous
  // copies; the ones from pageable memory are staged)
  if (!c->h_rb && hipHostMalloc(reinterpret_cast<void**>(&c->h_rb), sizeof(ry_ctx::Readback)) != hipSuccess) {
    c->h_rb = nullptr;
    return fail(c, RY_ENOMEM, "pinned readback buffer");
  }
  c->h_rb->t = *t_io;
  HIPCHK(c, hipMemcpyAsync(c->d_t, &c->h_rb->t, sizeof(double), hipMemcpyHostToDevice, c->stream));
  if (launch_zero_u32(reinterpret_cast<unsigned int*>(c->d_flags), 3, c->stream))
    return fail(c, RY_EHIP, "zero kernel");
  const bool use_graph = !c->timing;
  // Buffer parity of the base level before the steps: each executed coarse
  // step flips it once (finer levels take two substeps per coarse step, so
  // theirs come back).  Steps enqueued after t_end is reached are skipped on
  // the device and write nothing, so the parity is set from the device's
  // count of executed steps afterwards, not from the number enqueued.
  const int cur0 = c->lev[0].cur;
  for (int32_t i = 0; i < n_coarse;) {
    if (use_graph) {
      const int par = c->lev[0].cur;
      int gi = kGraphLevels - 1;
      while ((1 << gi) > n_coarse - i) --gi;
      std::vector<int> now;
      for (auto& L : c->lev) now.push_back(L.cur);
      if (!c->graph[gi][par] || c->graph_par[gi][par] != now || c->graph_tend[gi][par] != t_end)
        if ((s = capture_step(c, gi, par, t_end))) return s;
      HIPCHK(c, hipGraphLaunch(c->graph[gi][par], c->stream));
      i += 1 << gi;
      if (gi == 0) c->lev[0].cur ^= 1;   // the other graphs take an even number of steps
    } else {
      if ((s = enqueue_coarse_step(c, t_end))) return s;
      ++i;
    }
  }
  c->slots_valid = true;
  // one round trip for the error word, the device's step count and the time
  HIPCHK(c, hipMemcpyAsync(c->h_rb->flags, c->d_flags, sizeof c->h_rb->flags, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&c->h_rb->t, c->d_t, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->timing) time_collect(c);
  const int32_t e = c->h_rb->flags[3];
  if (e & ERR_BOUNDS) return fail(c, RY_EHIP, "device index outside its buffer (debug build bounds check)");
  if (e) return fail(c, RY_ENUMERIC, "non-finite or non-positive density/energy latched on the device");
  const int32_t nrun = c->h_rb->flags[2];
  if (nrun < 0 || nrun > n_coarse) return fail(c, RY_EHIP, "device step count %d out of range", nrun);
  c->lev[0].cur = cur0 ^ (nrun & 1);
  *t_io = c->h_rb->t;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_conserved_totals(ry_ctx* c, double* tot) {
  RY_ABI_TRY
  if (!c || !tot || !c->built || c->batch) return RY_EINVAL;
  const int nb = totals_blocks();
  const int nv = c->dom.nv;
  if (launch_zero_u64(reinterpret_cast<unsigned long long*>(c->d_partial), int64_t(nv) * nb, c->stream))
    return fail(c, RY_EHIP, "zero kernel");
  for (int k = 0; k < c->nlev; ++k) {
    DevLevel& L = c->lev[k];
    if (!L.n_oct) continue;
    const double dx = level_dx(c, c->cfg.level_min + k);
    if (launch_totals(L.U[L.cur], L.plane(), L.n_oct, L.refined, dx * dx * dx, nv, c->d_partial, nb, c->stream))
      return fail(c, RY_EHIP, "totals kernel");
  }
  if (launch_totals_final(c->d_partial, nb, nv, c->d_tot, c->stream)) return fail(c, RY_EHIP, "totals kernel");
  ry_status s = sync_and_check(c);
  if (s) return s;
  HIPCHK(c, hipMemcpy(tot, c->d_tot, sizeof(double) * nv, hipMemcpyDeviceToHost));
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_download(ry_ctx* c, int32_t level, double* U) {
  RY_ABI_TRY
  if (!c || !U || !c->built || c->batch || level < c->cfg.level_min || level > c->cfg.level_max) return RY_EINVAL;
  DevLevel& D = c->lev[level - c->cfg.level_min];
  for (int v = 0; v < c->dom.nv && D.n_oct; ++v)
    HIPCHK(c, hipMemcpyAsync(U + size_t(v) * 8 * D.n_oct, D.U[D.cur] + v * D.plane(), sizeof(double) * 8 * D.n_oct,
                             hipMemcpyDeviceToHost, c->stream));
  return sync_and_check(c);
  RY_ABI_CATCH
}

ry_status ry_upload(ry_ctx* c, int32_t level, const double* U) {
  RY_ABI_TRY
  if (!c || !U || !c->built || c->batch || level < c->cfg.level_min || level > c->cfg.level_max) return RY_EINVAL;
  DevLevel& D = c->lev[level - c->cfg.level_min];
  if (!D.n_oct) return RY_OK;
  ry_status s = upload_level_state(c, D, U);
  if (s) return s;
  c->means_valid = false;
  HIPCHK(c, hipMemsetAsync(err_ptr(c), 0, sizeof(int32_t), c->stream));
  if ((s = enqueue_cfl_all(c))) return s;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RY_OK;
  RY_ABI_CATCH
}

// --------------------------------------------------------------- batching
ry_status ry_batch_create(const ry_config* cfgs, int32_t nbox, const double* const* U0, ry_ctx** out) {
  RY_ABI_TRY
  if (!out || !cfgs || !U0 || nbox <= 0) return RY_EINVAL;
  *out = nullptr;
  for (int b = 0; b < nbox; ++b) {
    ry_status s = validate(&cfgs[b], true);
    if (s) return s;
    if (!U0[b]) return RY_EINVAL;
    if (cfgs[b].gamma != cfgs[0].gamma || cfgs[b].cfl != cfgs[0].cfl || cfgs[b].rho_floor != cfgs[0].rho_floor ||
        cfgs[b].p_floor != cfgs[0].p_floor || cfgs[b].precision != cfgs[0].precision || cfgs[b].nscalar != 0)
      return RY_EINVAL;
  }
  ry_ctx* c = new (std::nothrow) ry_ctx();
  if (!c) return RY_ENOMEM;
  c->cfg = cfgs[0];
  c->batch = true;
  c->nlev = 1;
  c->nbox = nbox;
  // the plain launch (one wavefront per tile, the hardware dispatcher as the
  // queue) measures fastest for batches too; the queue-fed persistent
  // kernel stays an autotuner candidate
  std::fill(std::begin(c->tune), std::end(c->tune), kDefaultTuning);
  ry_status s = init_common(c);
  if (s) {
    delete c;
    return s;
  }
  LevelTables all;
  std::vector<double> Uall;
  std::vector<int32_t> oct_box;
  std::vector<int32_t> oc;                  // oct coordinates in each box, x y z interleaved
  std::vector<int64_t> box_noct;            // octs per axis of each box
  std::vector<std::vector<double>> Ubox(nbox);
  int64_t off = 0;
  for (int b = 0; b < nbox; ++b) {
    DomainSpec d = make_dom(cfgs[b]);
    std::vector<HostLevel> H;
    std::string e = build_mesh(d, U0[b], nullptr, nullptr, H);
    std::vector<LevelTables> T;
    if (e.empty()) e = build_tables(d, H, T);
    if (!e.empty()) {
      ry_destroy(c);
      return RY_EINVAL;
    }
    const LevelTables& t = T[0];
    if (b == 0) c->seg_off.assign(1, 0);
    c->seg_off.push_back(c->seg_off.back() + t.n_tile);
    c->box_off.push_back(off);
    c->box_noct.push_back(t.n_oct);
    c->box_dx.push_back(cfgs[b].boxlen / double(cfgs[b].nbase[0]));
    for (int32_t i = 0; i < t.n_tile; ++i) {
      for (int j = 0; j < TILE_TAB; ++j) {
        const int32_t v = t.tab[size_t(i) * TILE_TAB + j];
        all.tab.push_back(v >= 0 ? int32_t(v + off) : -1);
      }
      all.tflag.push_back(t.tflag[i]);
      all.tile_box.push_back(b);
    }
    for (int64_t o = 0; o < t.n_oct; ++o) {
      oct_box.push_back(b);
      oc.push_back(H[0].ox[o]);
      oc.push_back(H[0].oy[o]);
      oc.push_back(H[0].oz[o]);
    }
    for (int a = 0; a < 3; ++a) box_noct.push_back(cfgs[b].nbase[a] / 2);
    Ubox[b] = H[0].U;
    off += t.n_oct;
  }
  all.n_oct = off;
  all.n_tile = int32_t(all.tflag.size());
  if (off >= (int64_t(1) << 29)) {
    ry_destroy(c);
    return RY_EINVAL;                  // cells are indexed in 32 bits
  }
  all.refined_ext.assign(off, 0);
  c->lev.assign(1, DevLevel());
  DevLevel& D = c->lev[0];
  D.n_oct = off;
  D.n_ext = off;
  D.n_leaf = off * 8;
  D.n_tile = all.n_tile;
  bool ok = true;
  for (int b = 0; b < 2; ++b) {
    D.U[b] = static_cast<double*>(dalloc(c, sizeof(double) * NVAR * 8 * D.n_ext));
    if (!D.U[b]) ok = false;
  }
  if (ok) {
    for (int b = 0; b < nbox; ++b)
      for (int buf = 0; buf < 2; ++buf)
        for (int v = 0; v < NVAR; ++v)
          if (hipMemcpyAsync(D.U[buf] + v * D.plane() + c->box_off[b] * 8, Ubox[b].data() + size_t(v) * 8 * c->box_noct[b],
                             sizeof(double) * 8 * c->box_noct[b], hipMemcpyHostToDevice, c->stream) != hipSuccess)
            ok = false;
    D.tab = upload_vec(c, all.tab, ok);
    D.tflag = upload_vec(c, all.tflag, ok);
    D.refined = upload_vec(c, all.refined_ext, ok);
    D.tile_box = upload_vec(c, all.tile_box, ok);
    D.oct_box = upload_vec(c, oct_box, ok);
    D.doc = upload_vec(c, oc, ok);
    c->d_dx_box = upload_vec(c, c->box_dx, ok);
    c->d_box_noct = upload_vec(c, box_noct, ok);
  }
  if (!ok || alloc_scalars(c, nbox)) {
    ry_destroy(c);
    return RY_ENOMEM;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    ry_destroy(c);
    return RY_EHIP;
  }
  c->built = true;
  *out = c;
  return RY_OK;
  RY_ABI_CATCH
}

static ry_status enqueue_batch_step(ry_ctx* c) {
  DevLevel& L = c->lev[0];
  FinalizeArgs f{};
  f.smax = c->d_smax;
  f.nslot = c->nbox;
  f.cfl = c->cfg.cfl;
  f.dx_box = c->d_dx_box;
  f.t = c->d_t;
  f.lam = c->d_lam;
  f.nstep = nstep_ptr(c);
  f.batch = 1;
  ry_status s0 = enqueue_seg_max(c);
  if (s0) return s0;
  if (launch_finalize(f, c->stream)) return fail(c, RY_EHIP, "finalize kernel");
  HydroArgs a = hydro_args(c, c->cfg.level_min, 0);
  a.child = nullptr;
  a.reg_fine = nullptr;
  a.reg_own = nullptr;
  a.record_reg = 0;
  a.lam_dev = c->d_lam;
  a.tile_box = L.tile_box;
  a.tile_smax = c->d_part;
  a.skip = nullptr;
  ry_status s = enqueue_hydro(c, a, 0);
  if (s) return s;
  L.cur ^= 1;
  return RY_OK;
}

ry_status ry_batch_run(ry_ctx* c, int32_t nsteps) {
  RY_ABI_TRY
  if (!c || !c->batch || !c->built || nsteps < 0) return RY_EINVAL;
  ry_status s;
  if (!c->slots_valid && (s = enqueue_cfl_all(c))) return s;
  DevLevel& L = c->lev[0];
  if (c->timing) {
    for (int i = 0; i < nsteps; ++i)
      if ((s = enqueue_batch_step(c))) return s;
  } else if (nsteps > 0) {
    if (!c->bgraph || c->bgraph_steps != nsteps || c->bgraph_par != L.cur) {
      if (c->bgraph) {
        hipGraphExecDestroy(c->bgraph);
        c->bgraph = nullptr;
      }
      const int saved = L.cur;
      hipGraph_t g = nullptr;
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      for (int i = 0; i < nsteps && !s; ++i) s = enqueue_batch_step(c);
      hipError_t e = hipStreamEndCapture(c->stream, &g);
      L.cur = saved;
      if (s) {
        if (g) hipGraphDestroy(g);
        return s;
      }
      if (e != hipSuccess) return fail(c, RY_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
      e = hipGraphInstantiate(&c->bgraph, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e != hipSuccess) return fail(c, RY_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
      c->bgraph_steps = nsteps;
      c->bgraph_par = saved;
    }
    HIPCHK(c, hipGraphLaunch(c->bgraph, c->stream));
    if (nsteps & 1) L.cur ^= 1;
  }
  c->slots_valid = true;
  return sync_and_check(c);
  RY_ABI_CATCH
}

ry_status ry_batch_box_info(const ry_ctx* c, int32_t box, int64_t* n_oct, double* t) {
  RY_ABI_TRY
  if (!c || !c->batch || box < 0 || box >= c->nbox) return RY_EINVAL;
  if (n_oct) *n_oct = c->box_noct[box];
  if (t && hipMemcpy(t, c->d_t + box, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return RY_EHIP;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_batch_download(ry_ctx* c, int32_t box, double* U) {
  RY_ABI_TRY
  if (!c || !c->batch || !U || box < 0 || box >= c->nbox) return RY_EINVAL;
  DevLevel& D = c->lev[0];
  const int64_t n = c->box_noct[box];
  for (int v = 0; v < NVAR; ++v)
    HIPCHK(c, hipMemcpyAsync(U + size_t(v) * 8 * n, D.U[D.cur] + v * D.plane() + c->box_off[box] * 8,
                             sizeof(double) * 8 * n, hipMemcpyDeviceToHost, c->stream));
  return sync_and_check(c);
  RY_ABI_CATCH
}

// ---------------------------------------------------------------- tuning
namespace {

bool same_tuning(const ry_tuning& a, const ry_tuning& b) {
  return a.tiles_per_wg == b.tiles_per_wg && a.persistent == b.persistent && a.waves_per_cu == b.waves_per_cu &&
         a.batch == b.batch && a.waves_per_tile == b.waves_per_tile && a.tile_cells == b.tile_cells;
}

// Whether the context can run a tuning (RY_OK) or not (RY_EINVAL, with the
// reason).
ry_status check_tuning(ry_ctx* c, const ry_tuning& t) {
  if (t.persistent < 0 || t.persistent > 1) return fail(c, RY_EINVAL, "persistent must be 0 or 1");
  if (t.tile_cells == 8) {
    if (t.tiles_per_wg != 1 || (t.waves_per_tile != 8 && t.waves_per_tile != 4) || t.persistent)
      return fail(c, RY_EINVAL, "tile_cells 8 needs tiles_per_wg 1, waves_per_tile 8 or 4, persistent 0");
  } else if (t.tile_cells == 4) {
    if (t.tiles_per_wg != 1 && t.tiles_per_wg != 2 && t.tiles_per_wg != 4) return fail(c, RY_EINVAL, "tiles_per_wg");
    if (t.waves_per_tile != 1 && t.waves_per_tile != 2 && t.waves_per_tile != 4)
      return fail(c, RY_EINVAL, "waves_per_tile");
    if (t.tiles_per_wg * t.waves_per_tile > 4) return fail(c, RY_EINVAL, "tiles_per_wg * waves_per_tile > 4");
  } else {
    return fail(c, RY_EINVAL, "tile_cells must be 4 or 8");
  }
  if (!hydro_tuning_supported(c->cfg.precision, c->cfg.nscalar, t))
    return fail(c, RY_EINVAL, "no hydro kernel for this tuning (precision / passive scalars)");
  if (t.persistent && (t.waves_per_cu < 1 || t.waves_per_cu > 32 || t.batch < 1 || t.batch > 64))
    return fail(c, RY_EINVAL, "persistent launch: waves_per_cu 1..32, batch 1..64");
  return RY_OK;
}

void drop_all_graphs(ry_ctx* c) {
  drop_graphs(c);
  if (c->bgraph) {
    hipGraphExecDestroy(c->bgraph);
    c->bgraph = nullptr;
  }
}

}  // namespace

ry_status ry_set_tuning(ry_ctx* c, const ry_tuning* t) {
  RY_ABI_TRY
  if (!c || !t) return RY_EINVAL;
  ry_status s = check_tuning(c, *t);
  if (s) return s;
  std::fill(std::begin(c->tune), std::end(c->tune), *t);
  drop_all_graphs(c);
  if (c->built && (s = ensure_super(c))) return s;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_get_tuning(const ry_ctx* c, ry_tuning* t) {
  RY_ABI_TRY
  if (!c || !t) return RY_EINVAL;
  *t = c->tune[0];
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_set_level_tuning(ry_ctx* c, int32_t level, const ry_tuning* t) {
  RY_ABI_TRY
  if (!c || !t || level < c->cfg.level_min || level > c->cfg.level_max) return RY_EINVAL;
  ry_status s = check_tuning(c, *t);
  if (s) return s;
  c->tune[level - c->cfg.level_min] = *t;
  drop_all_graphs(c);
  if (c->built && (s = ensure_super(c))) return s;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_get_level_tuning(const ry_ctx* c, int32_t level, ry_tuning* t) {
  RY_ABI_TRY
  if (!c || !t || level < c->cfg.level_min || level > c->cfg.level_max) return RY_EINVAL;
  *t = c->tune[level - c->cfg.level_min];
  return RY_OK;
  RY_ABI_CATCH
}

// Time level k's hydro launch under tuning t (four launches, the best of the
// last three), writing only the level's other state buffer.
static ry_status time_level(ry_ctx* c, int k, const ry_tuning& t, double* ms_out) {
  hipEvent_t a, b;
  hipEventCreateWithFlags(&a, hipEventDisableSystemFence);
  hipEventCreateWithFlags(&b, hipEventDisableSystemFence);
  double best = INFINITY;
  ry_status s = RY_OK;
  const int l = c->cfg.level_min + k;
  HydroArgs h = hydro_args(c, l, 0);
  h.lam_dev = c->batch ? c->d_lam : nullptr;
  h.lam_host = 0.1;
  h.record_reg = 0;
  h.reg_own = nullptr;
  h.tile_smax = nullptr;
  h.floors = nullptr;
  h.err = nullptr;
  h.skip = nullptr;
  for (int rep = 0; rep < 4 && !s; ++rep) {
    hipEventRecord(a, c->stream);
    s = enqueue_hydro(c, h, k, &t);
    hipEventRecord(b, c->stream);
    hipEventSynchronize(b);
    float ms = 0.f;
    hipEventElapsedTime(&ms, a, b);
    if (rep > 0) best = std::min(best, double(ms));
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  *ms_out = best;
  return s;
}

ry_status ry_autotune(ry_ctx* c, ry_tuning* best, double* times_ms, int32_t max_cand, int32_t* n_cand) {
  RY_ABI_TRY
  if (!c || !c->built) return RY_EINVAL;
  if (c->batch) {
    // the batched launch reads per-box lambda: make sure it holds values
    ry_status s0 = enqueue_cfl_all(c);
    if (s0) return s0;
  }
  std::vector<ry_tuning> cand;
  for (int wpt : {1, 2, 4})
    for (int tpw : {1, 2, 4})
      if (tpw * wpt <= 4) cand.push_back({tpw, 0, 4, 1, wpt, 4});
  for (int wpt : {1, 2, 4})
    for (int w : {8, 14, 20})
      for (int bt : {1, 4}) cand.push_back({1, 1, w, bt, wpt, 4});
  cand.push_back({1, 0, 4, 1, 8, 8});
  cand.push_back({1, 0, 4, 1, 4, 8});
  {
    std::string keep = c->err;
    cand.erase(std::remove_if(cand.begin(), cand.end(), [&](const ry_tuning& t) { return check_tuning(c, t) != RY_OK; }),
               cand.end());
    c->err = keep;
  }
  const int n = int(cand.size());
  if (n_cand) *n_cand = n;
  // the 8^3-cell tile's tables of every level
  ry_tuning saved[RY_MAX_LEVELS];
  std::copy(std::begin(c->tune), std::end(c->tune), saved);
  const ry_tuning* t8 = nullptr;
  for (const auto& t : cand)
    if (t.tile_cells == 8 && !t8) t8 = &t;
  if (t8) {
    std::fill(std::begin(c->tune), std::end(c->tune), *t8);
    ry_status s = ensure_super(c);
    std::copy(std::begin(saved), std::end(saved), c->tune);
    if (s) return s;
  }
  // per level: stage 1 times every candidate once (best of three launches);
  // stage 2 times the three fastest and the default launch again in six
  // interleaved rounds (drift and noise hit all alike); the median decides,
  // and a candidate must beat the default by more than 2% to replace it
  // (isolated launches and the production sequence differ by a few percent)
  std::vector<double> coarse(n, 0.0);   // per candidate: the coarse step's hydro time if used on every level
  ry_tuning chosen[RY_MAX_LEVELS];
  std::copy(std::begin(saved), std::end(saved), chosen);
  for (int k = 0; k < c->nlev; ++k) {
    if (c->lev[k].n_tile == 0) continue;
    std::vector<double> t1(n);
    for (int i = 0; i < n; ++i) {
      ry_status s = time_level(c, k, cand[i], &t1[i]);
      if (s) return s;
      coarse[i] += std::ldexp(t1[i], k);
    }
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return t1[a] < t1[b]; });
    std::vector<ry_tuning> fin;
    for (int i = 0; i < n && i < 3; ++i) fin.push_back(cand[order[i]]);
    int idef = -1;
    for (size_t i = 0; i < fin.size(); ++i)
      if (same_tuning(fin[i], kDefaultTuning)) idef = int(i);
    if (idef < 0 && hydro_tuning_supported(c->cfg.precision, c->cfg.nscalar, kDefaultTuning)) {
      fin.push_back(kDefaultTuning);
      idef = int(fin.size()) - 1;
    }
    std::vector<std::vector<double>> t2(fin.size());
    for (int round = 0; round < 6; ++round)
      for (size_t i = 0; i < fin.size(); ++i) {
        double ms = 0;
        ry_status s = time_level(c, k, fin[i], &ms);
        if (s) return s;
        t2[i].push_back(ms);
      }
    std::vector<double> med(fin.size());
    for (size_t i = 0; i < fin.size(); ++i) {
      std::sort(t2[i].begin(), t2[i].end());
      med[i] = 0.5 * (t2[i][2] + t2[i][3]);
    }
    int ib = 0;
    for (size_t i = 1; i < fin.size(); ++i)
      if (med[i] < med[ib]) ib = int(i);
    if (idef >= 0 && ib != idef && med[idef] <= 1.02 * med[ib]) ib = idef;
    chosen[k] = fin[ib];
  }
  if (times_ms)
    for (int i = 0; i < n && i < max_cand; ++i) times_ms[i] = coarse[i];
  std::copy(std::begin(chosen), std::end(chosen), c->tune);
  drop_all_graphs(c);
  // tables of levels left without the 8^3-cell tile are not needed any more
  for (int k = 0; k < c->nlev; ++k)
    if (c->tune[k].tile_cells != 8 && c->lev[k].super_ok) free_super(c, c->lev[k]);
  ry_status s = ensure_super(c);
  if (s) return s;
  if (best) *best = c->tune[0];
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RY_OK;
  RY_ABI_CATCH
}

// ----------------------------------------------------------- diagnostics
int64_t ry_floor_count(ry_ctx* c) {
  if (!c || !c->built) return -1;
  unsigned long long v = 0;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return -1;
  if (hipMemcpy(&v, c->d_floors, sizeof v, hipMemcpyDeviceToHost) != hipSuccess) return -1;
  return int64_t(v);
}

ry_status ry_set_timing(ry_ctx* c, int32_t on) {
  RY_ABI_TRY
  if (!c) return RY_EINVAL;
  c->timing = on != 0;
  if (!c->timing) c->ktime.clear();
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_kernel_time(ry_ctx* c, const char* kernel, int64_t* launches, double* total_ms) {
  RY_ABI_TRY
  if (!c || !kernel) return RY_EINVAL;
  if (!c->pending.empty()) {
    if (hipStreamSynchronize(c->stream) != hipSuccess) return RY_EHIP;
    time_collect(c);
  }
  auto it = c->ktime.find(kernel);
  if (launches) *launches = it == c->ktime.end() ? 0 : it->second.first;
  if (total_ms) *total_ms = it == c->ktime.end() ? 0.0 : it->second.second;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_copy_probe(ry_ctx* c, size_t bytes, int32_t reps, double* ms) {
  RY_ABI_TRY
  if (!c || !ms || bytes < 1024 || reps < 1) return RY_EINVAL;
  double *a = nullptr, *b = nullptr;
  HIPCHK(c, hipMalloc(&a, bytes));
  if (hipMalloc(&b, bytes) != hipSuccess) {
    hipFree(a);
    return fail(c, RY_ENOMEM, "probe allocation");
  }
  hipMemsetAsync(a, 0, bytes, c->stream);
  const int64_t n = int64_t(bytes / sizeof(double));
  launch_copy(a, b, n, c->stream);
  hipEvent_t e0, e1;
  hipEventCreateWithFlags(&e0, hipEventDisableSystemFence);
  hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
  hipEventRecord(e0, c->stream);
  for (int i = 0; i < reps; ++i) launch_copy(a, b, n, c->stream);
  hipEventRecord(e1, c->stream);
  hipEventSynchronize(e1);
  float t = 0.f;
  hipEventElapsedTime(&t, e0, e1);
  *ms = double(t) / reps;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(a);
  hipFree(b);
  return RY_OK;
  RY_ABI_CATCH
}

// ------------------------------------------------------- host-only mesh
struct ry_mesh {
  ry_config cfg;
  std::vector<HostLevel> levels;
  std::vector<LevelTables> tables;
};

ry_status ry_mesh_build(const ry_config* cfg, const double* U_base, ry_fill_fn fill, void* user, ry_mesh** out) {
  RY_ABI_TRY
  if (!out || !U_base) return RY_EINVAL;
  *out = nullptr;
  ry_status s = validate(cfg, false);
  if (s) return s;
  ry_mesh* m = new (std::nothrow) ry_mesh();
  if (!m) return RY_ENOMEM;
  m->cfg = *cfg;
  DomainSpec d = make_dom(*cfg);
  std::string e = build_mesh(d, U_base, fill, user, m->levels);
  if (e.empty()) e = build_tables(d, m->levels, m->tables);
  if (!e.empty()) {
    delete m;
    return RY_EINVAL;
  }
  *out = m;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_mesh_level(const ry_mesh* m, int32_t level, int64_t* n_oct, uint64_t* keys, uint8_t* refined,
                        int64_t* n_ghost) {
  RY_ABI_TRY
  if (!m || level < m->cfg.level_min || level > m->cfg.level_max) return RY_EINVAL;
  const HostLevel& H = m->levels[level - m->cfg.level_min];
  if (n_oct) *n_oct = H.n;
  if (keys && H.n) std::memcpy(keys, H.key.data(), sizeof(uint64_t) * H.n);
  if (refined && H.n) std::memcpy(refined, H.refined.data(), H.n);
  if (n_ghost) *n_ghost = m->tables[level - m->cfg.level_min].n_ghost;
  return RY_OK;
  RY_ABI_CATCH
}

void ry_mesh_free(ry_mesh* m) { delete m; }

uint64_t ry_hilbert_key(int32_t bits, uint32_t x, uint32_t y, uint32_t z) { return hilbert3(bits, x, y, z); }

}  // extern "C"
