// Uniform-level Poisson solver on gfx950: the preconditioned pipelined
// conjugate-gradient method (PPCG; Ghysels & Vanroose 2014, Algorithm 4)
// with the seven-point preconditioner 13/12 (centre), 1/6 (face neighbours).
//
// One iteration i is two launches on the solver's stream:
//   finalize  sums the per-workgroup partials of gamma_i = r_i.u_i and
//             delta_i = w_i.u_i in a fixed order, records eps_i, tests
//             convergence and forms alpha_i, beta_i on the device;
//   iterate   a z-marching stencil sweep that, per cell, forms
//             m_i = M^-1 w_i and n_i = A m_i from w_i staged in LDS, updates
//             the eight recurrence vectors (z, q, s, p, then x, r, u, w) and
//             accumulates the partials of gamma_{i+1}, delta_{i+1}.
// So each iteration reads and writes every recurrence vector once (8 + 8
// FP64 values per cell), with one device-wide reduction, which is the
// single synchronisation per iteration the pipelined method is built for.
// w is double-buffered (neighbouring workgroups read w_i while w_{i+1} is
// written); every other vector is updated in place.
//
// Iteration kernel geometry: a workgroup owns a TX x TY column of cells and
// a chunk of z planes; it keeps five w planes (2-cell halo in x, y) and
// three m planes (1-cell halo) in LDS as a rolling window.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ry_poisson.h"

namespace ryp {


constexpr int TX = 32, TY = 8, NTH = TX * TY;
constexpr int WX = TX + 4, WY = TY + 4, WPL = WX * WY;   // w plane, 2-cell halo
constexpr int MX = TX + 2, MY = TY + 2, MPL = MX * MY;   // m plane, 1-cell halo
constexpr int BATCH = 16;                                // iterations per captured graph
constexpr int NVEC = 9;                                  // x r u w0 w1 z q s p

struct Grid {
  int32_t n0, n1, n2, bc;
};

// Scalars carried between launches, device-resident.
struct Scalars {
  double gamma0, alpha, beta, alpha_prev, gamma_prev, eps_target;
  int32_t iter;      // index i of the next finalize
  int32_t max_iter;  // stop when i reaches it
  int32_t done;
  int32_t src;       // buffer holding w_i for the iteration kernel
};

struct IterArgs {
  Grid g;
  double* w[2];
  double *x, *r, *u, *z, *q, *s, *p;
  Scalars* sc;
  double* part;   // [2][gridDim.x]
  int32_t cz;     // z planes per workgroup
};

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Value of v at (X, Y, Z) under the boundary rule (zero Dirichlet: 0 off the grid).
__device__ __forceinline__ double grid_val(const double* __restrict__ v, const Grid& g, int X, int Y, int Z) {
  if (g.bc == RY_PBC_PERIODIC) {
    if (unsigned(X) >= unsigned(g.n0)) X = wrap(X, g.n0);
    if (unsigned(Y) >= unsigned(g.n1)) Y = wrap(Y, g.n1);
    if (unsigned(Z) >= unsigned(g.n2)) Z = wrap(Z, g.n2);
  } else if (X < 0 || X >= g.n0 || Y < 0 || Y >= g.n1 || Z < 0 || Z >= g.n2) {
    return 0.0;
  }
  return v[int64_t(X) + int64_t(g.n0) * (int64_t(Y) + int64_t(g.n1) * Z)];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
// contiguous slab of columns so that halo rows stay in one L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int x = bid & 7, j = bid >> 3;
  const int q = nblocks >> 3, r = nblocks & 7;
  return x * q + (x < r ? x : r) + j;
}

// Block-wide sums of (a, b) -> part[blockIdx.x], part[gridDim.x + blockIdx.x],
// in a fixed order.
__device__ __forceinline__ void block_partials(double a, double b, double* part) {
  __shared__ double red[2][NTH / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = a;
    red[1][wv] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int k = 0; k < NTH / 64; ++k) {
      sa += red[0][k];
      sb += red[1][k];
    }
    part[blockIdx.x] = sa;
    part[gridDim.x + blockIdx.x] = sb;
  }
}

// ---------------------------------------------------------------------------
// The iteration kernel.
// ---------------------------------------------------------------------------
template <int PC>
__global__ __launch_bounds__(NTH) void ppcg_iterate_kernel(IterArgs A) {
  const Scalars* sc = A.sc;
  if (sc->done) return;
  __shared__ double Wp[5][WPL];
  __shared__ double Mp[3][MPL];
  const Grid g = A.g;
  const bool periodic = g.bc == RY_PBC_PERIODIC;
  const int gx = (g.n0 + TX - 1) / TX, gy = (g.n1 + TY - 1) / TY;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int bx = b % gx, by = (b / gx) % gy, bz = b / (gx * gy);
  const int x0 = bx * TX, y0 = by * TY, z0 = bz * A.cz;
  const int z1 = min(z0 + A.cz, g.n2);
  const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
  const double alpha = sc->alpha, beta = sc->beta;
  const int src = sc->src;
  const double* __restrict__ win = A.w[src];
  double* __restrict__ wout = A.w[src ^ 1];

  // plane slots: w at z in slot (z - z0 + 2) mod 5, m at z in (z - z0 + 1) mod 3
  auto wslot = [&](int z) { return (z - z0 + 2) % 5; };
  auto mslot = [&](int z) { return (z - z0 + 1) % 3; };
  auto load_w = [&](int z) {
    double* dst = Wp[wslot(z)];
    for (int k = tid; k < WPL; k += NTH) {
      const int lx = k % WX, ly = k / WX;
      dst[k] = grid_val(win, g, x0 - 2 + lx, y0 - 2 + ly, z);
    }
  };
  // m = M^-1 w on the plane z (1-cell halo); 0 off the grid under Dirichlet
  auto comp_m = [&](int z) {
    const double* wm = Wp[wslot(z - 1)];
    const double* w0 = Wp[wslot(z)];
    const double* wp = Wp[wslot(z + 1)];
    double* dst = Mp[mslot(z)];
    for (int k = tid; k < MPL; k += NTH) {
      const int lx = k % MX, ly = k / MX;
      const int X = x0 - 1 + lx, Y = y0 - 1 + ly;
      const bool in = periodic || (X >= 0 && X < g.n0 && Y >= 0 && Y < g.n1 && z >= 0 && z < g.n2);
      const int c = (lx + 1) + WX * (ly + 1);
      double v = 0.0;
      if (in) {
        if (PC == RY_PC_STENCIL7) {
          double s = w0[c - 1];
          s += w0[c + 1];
          s += w0[c - WX];
          s += w0[c + WX];
          s += wm[c];
          s += wp[c];
          v = (13.0 / 12.0) * w0[c] + (1.0 / 6.0) * s;
        } else {
          v = w0[c];
        }
      }
      dst[k] = v;
    }
  };

  load_w(z0 - 2);
  load_w(z0 - 1);
  load_w(z0);
  load_w(z0 + 1);
  __syncthreads();
  comp_m(z0 - 1);
  comp_m(z0);
  double acc_g = 0.0, acc_d = 0.0;
  const int X = x0 + tx, Y = y0 + ty;
  const bool own = X < g.n0 && Y < g.n1;
  const int64_t plane = int64_t(g.n0) * g.n1;
  const int64_t col = int64_t(X) + int64_t(g.n0) * Y;
  // The eight recurrence vectors are touched once per iteration: stream
  // them with non-temporal loads and stores so that L2 keeps the w planes
  // the neighbouring workgroups read as halo.
  constexpr int NW = (WPL + NTH - 1) / NTH;
  for (int z = z0; z < z1; ++z) {
    double wr[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const int k = tid + j * NTH;
      if (k < WPL) wr[j] = grid_val(win, g, x0 - 2 + k % WX, y0 - 2 + k / WX, z + 2);
    }
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const int k = tid + j * NTH;
      if (k < WPL) Wp[wslot(z + 2)][k] = wr[j];
    }
    __syncthreads();
    comp_m(z + 1);
    __syncthreads();
    if (own) {
      const int64_t i = col + plane * z;
      const double z_old = __builtin_nontemporal_load(A.z + i);
      const double q_old = __builtin_nontemporal_load(A.q + i);
      const double s_old = __builtin_nontemporal_load(A.s + i);
      const double p_old = __builtin_nontemporal_load(A.p + i);
      const double u_old = __builtin_nontemporal_load(A.u + i);
      const double x_old = __builtin_nontemporal_load(A.x + i);
      const double r_old = __builtin_nontemporal_load(A.r + i);
      const double* mm = Mp[mslot(z - 1)];
      const double* m0 = Mp[mslot(z)];
      const double* mp = Mp[mslot(z + 1)];
      const int c = (tx + 1) + MX * (ty + 1);
      double s = m0[c - 1];
      s += m0[c + 1];
      s += m0[c - MX];
      s += m0[c + MX];
      s += mm[c];
      s += mp[c];
      const double mv = m0[c];
      const double nv = 6.0 * mv - s;                         // n_i = A m_i
      const double wv = Wp[wslot(z)][(tx + 2) + WX * (ty + 2)];
      const double zz = nv + beta * z_old;
      const double qq = mv + beta * q_old;
      const double ss = wv + beta * s_old;
      const double pp = u_old + beta * p_old;
      const double xx = x_old + alpha * pp;
      const double rr = r_old - alpha * ss;
      const double uu = u_old - alpha * qq;
      const double ww = wv - alpha * zz;
      __builtin_nontemporal_store(zz, A.z + i);
      __builtin_nontemporal_store(qq, A.q + i);
      __builtin_nontemporal_store(ss, A.s + i);
      __builtin_nontemporal_store(pp, A.p + i);
      __builtin_nontemporal_store(xx, A.x + i);
      __builtin_nontemporal_store(rr, A.r + i);
      __builtin_nontemporal_store(uu, A.u + i);
      __builtin_nontemporal_store(ww, wout + i);
      acc_g += rr * uu;
      acc_d += ww * uu;
    }
  }
  block_partials(acc_g, acc_d, A.part);
}

// ---------------------------------------------------------------------------
// Scalar step: gamma_i, delta_i from the partials; eps_i; alpha_i, beta_i.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void ppcg_finalize_kernel(Scalars* sc, const double* __restrict__ part,
                                                             int npart, double* hist) {
  if (sc->done) return;
  __shared__ double sg[1024], sd[1024];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < npart; k += 1024) {
    a += part[k];
    b += part[npart + k];
  }
  sg[threadIdx.x] = a;
  sd[threadIdx.x] = b;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) {
      sg[threadIdx.x] += sg[threadIdx.x + h];
      sd[threadIdx.x] += sd[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double gamma = sg[0], delta = sd[0];
  const int i = sc->iter;
  if (i == 0) sc->gamma0 = gamma;
  const double g0 = (i == 0) ? gamma : sc->gamma0;
  const double eps = (g0 > 0.0 && gamma > 0.0) ? sqrt(gamma / g0) : 0.0;
  hist[i] = eps;
  if (eps <= sc->eps_target || i >= sc->max_iter || i >= RY_POISSON_HIST - 1) {
    sc->done = 1;
    return;
  }
  double alpha, beta;
  if (i > 0) {
    beta = gamma / sc->gamma_prev;
    alpha = gamma / (delta - beta * gamma / sc->alpha_prev);
  } else {
    beta = 0.0;
    alpha = gamma / delta;
  }
  sc->alpha = alpha;
  sc->beta = beta;
  sc->alpha_prev = alpha;
  sc->gamma_prev = gamma;
  sc->src = i & 1;
  sc->iter = i + 1;
}

// (Re)arm the stopping rule: absolute max_iter, or relative to the current i.
__global__ void ppcg_arm_kernel(Scalars* sc, double eps, int32_t max_iter, int32_t relative) {
  sc->done = 0;
  sc->eps_target = eps;
  sc->max_iter = relative ? sc->iter + max_iter : max_iter;
}

__global__ void ppcg_reset_kernel(Scalars* sc) {
  sc->gamma0 = sc->alpha = sc->beta = sc->alpha_prev = sc->gamma_prev = 0.0;
  sc->eps_target = -1.0;
  sc->iter = 0;
  sc->max_iter = 0;
  sc->done = 1;
  sc->src = 0;
}

// ---------------------------------------------------------------------------
// Start-up sweeps (once per solve): r = b - A x, u = M^-1 r, w = A u with the
// partials of r.u and w.u laid out like the iteration kernel's.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double nb_sum(const double* v, const Grid& g, int X, int Y, int Z) {
  double s = grid_val(v, g, X - 1, Y, Z);
  s += grid_val(v, g, X + 1, Y, Z);
  s += grid_val(v, g, X, Y - 1, Z);
  s += grid_val(v, g, X, Y + 1, Z);
  s += grid_val(v, g, X, Y, Z - 1);
  s += grid_val(v, g, X, Y, Z + 1);
  return s;
}

__global__ __launch_bounds__(256) void residual_kernel(Grid g, const double* __restrict__ b,
                                                       const double* __restrict__ x, double* __restrict__ r) {
  const int64_t N = int64_t(g.n0) * g.n1 * g.n2;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x) {
    const int X = int(i % g.n0), Y = int((i / g.n0) % g.n1), Z = int(i / (int64_t(g.n0) * g.n1));
    r[i] = b[i] - (6.0 * x[i] - nb_sum(x, g, X, Y, Z));
  }
}

__global__ __launch_bounds__(256) void minv_kernel(Grid g, int pc, const double* __restrict__ r,
                                                   double* __restrict__ u) {
  const int64_t N = int64_t(g.n0) * g.n1 * g.n2;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x) {
    const int X = int(i % g.n0), Y = int((i / g.n0) % g.n1), Z = int(i / (int64_t(g.n0) * g.n1));
    u[i] = (pc == RY_PC_STENCIL7) ? (13.0 / 12.0) * r[i] + (1.0 / 6.0) * nb_sum(r, g, X, Y, Z) : r[i];
  }
}

__global__ __launch_bounds__(NTH) void apply_a_dots_kernel(Grid g, const double* __restrict__ r,
                                                           const double* __restrict__ u, double* __restrict__ w,
                                                           double* part) {
  const int64_t N = int64_t(g.n0) * g.n1 * g.n2;
  double a = 0.0, b = 0.0;
  for (int64_t i = blockIdx.x * int64_t(NTH) + threadIdx.x; i < N; i += int64_t(gridDim.x) * NTH) {
    const int X = int(i % g.n0), Y = int((i / g.n0) % g.n1), Z = int(i / (int64_t(g.n0) * g.n1));
    const double wv = 6.0 * u[i] - nb_sum(u, g, X, Y, Z);
    w[i] = wv;
    a += r[i] * u[i];
    b += wv * u[i];
  }
  block_partials(a, b, part);
}

}  // namespace ryp

// ===========================================================================
// Host side.
// ===========================================================================
using namespace ryp;

struct ry_poisson {
  ry_poisson_config cfg{};
  Grid g{};
  int64_t N = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<void*> allocs;
  double* v[NVEC] = {};        // x r u w0 w1 z q s p
  double* part = nullptr;
  double* hist = nullptr;
  Scalars* sc = nullptr;
  int32_t* h_done = nullptr;   // pinned
  int nblk = 0, cz = 0;
  bool ready = false;          // set_rhs done
  int64_t iter_hi = 0;         // upper bound of the device iteration index
  hipGraphExec_t graph = nullptr;
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  int64_t t_launches = 0;
  double t_ms = 0.0;
  std::string err;
};

namespace {

ry_status pfail(ry_poisson* p, ry_status s, const char* fmt, ...) {
  if (p) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    p->err = buf;
  }
  return s;
}

#define PCHK(p, call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return pfail((p), RY_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

void* palloc(ry_poisson* p, size_t bytes) {
  void* a = nullptr;
  if (p->cfg.dev_alloc) a = p->cfg.dev_alloc(bytes, p->cfg.alloc_user);
  else if (hipMalloc(&a, bytes) != hipSuccess) a = nullptr;
  if (a) p->allocs.push_back(a);
  return a;
}

void pfree_all(ry_poisson* p) {
  if (p->stream) hipStreamSynchronize(p->stream);
  for (void* a : p->allocs) {
    if (p->cfg.dev_free) p->cfg.dev_free(a, p->cfg.alloc_user);
    else if (!p->cfg.dev_alloc) hipFree(a);
  }
  p->allocs.clear();
  if (p->graph) hipGraphExecDestroy(p->graph);
  p->graph = nullptr;
  for (auto& e : p->ev) {
    hipEventDestroy(e.first);
    hipEventDestroy(e.second);
  }
  p->ev.clear();
  if (p->h_done) hipHostFree(p->h_done);
  p->h_done = nullptr;
}

IterArgs iter_args(ry_poisson* p) {
  IterArgs a;
  a.g = p->g;
  a.x = p->v[0];
  a.r = p->v[1];
  a.u = p->v[2];
  a.w[0] = p->v[3];
  a.w[1] = p->v[4];
  a.z = p->v[5];
  a.q = p->v[6];
  a.s = p->v[7];
  a.p = p->v[8];
  a.sc = p->sc;
  a.part = p->part;
  a.cz = p->cz;
  return a;
}

// One finalize (+ the iteration kernel unless `finalize_only`).
ry_status launch_iteration(ry_poisson* p, bool finalize_only = false) {
  hipLaunchKernelGGL(ppcg_finalize_kernel, dim3(1), dim3(1024), 0, p->stream, p->sc, p->part, p->nblk, p->hist);
  if (finalize_only) {
    PCHK(p, hipGetLastError());
    return RY_OK;
  }
  if (p->timing) {
    hipEvent_t a, b;
    // timing-only events: no system-scope fence (cache write-back) on recording
    PCHK(p, hipEventCreateWithFlags(&a, hipEventDisableSystemFence));
    PCHK(p, hipEventCreateWithFlags(&b, hipEventDisableSystemFence));
    PCHK(p, hipEventRecord(a, p->stream));
    p->ev.push_back({a, b});
  }
  if (p->cfg.precond == RY_PC_STENCIL7)
    hipLaunchKernelGGL(ppcg_iterate_kernel<RY_PC_STENCIL7>, dim3(p->nblk), dim3(NTH), 0, p->stream, iter_args(p));
  else
    hipLaunchKernelGGL(ppcg_iterate_kernel<RY_PC_NONE>, dim3(p->nblk), dim3(NTH), 0, p->stream, iter_args(p));
  if (p->timing) PCHK(p, hipEventRecord(p->ev.back().second, p->stream));
  PCHK(p, hipGetLastError());
  return RY_OK;
}

ry_status ensure_graph(ry_poisson* p) {
  if (p->graph) return RY_OK;
  PCHK(p, hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
  ry_status s = RY_OK;
  for (int k = 0; k < BATCH && s == RY_OK; ++k) s = launch_iteration(p);
  hipGraph_t gr = nullptr;
  const hipError_t e = hipStreamEndCapture(p->stream, &gr);
  if (s) {
    if (gr) hipGraphDestroy(gr);
    return s;
  }
  if (e != hipSuccess) return pfail(p, RY_EHIP, "graph capture: %s", hipGetErrorString(e));
  const hipError_t e2 = hipGraphInstantiate(&p->graph, gr, nullptr, nullptr, 0);
  hipGraphDestroy(gr);
  if (e2 != hipSuccess) return pfail(p, RY_EHIP, "graph instantiate: %s", hipGetErrorString(e2));
  return RY_OK;
}

void collect_times(ry_poisson* p) {
  for (auto& e : p->ev) {
    float ms = 0.f;
    hipEventSynchronize(e.second);
    hipEventElapsedTime(&ms, e.first, e.second);
    p->t_ms += ms;
    ++p->t_launches;
    hipEventDestroy(e.first);
    hipEventDestroy(e.second);
  }
  p->ev.clear();
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

ry_status ry_poisson_create(const ry_poisson_config* cfg, ry_poisson** out) {
  RY_ABI_TRY
  if (!cfg || !out) return RY_EINVAL;
  *out = nullptr;
  for (int a = 0; a < 3; ++a)
    if (cfg->n[a] < 1) return RY_EINVAL;
  const int64_t N = int64_t(cfg->n[0]) * cfg->n[1] * cfg->n[2];
  if (N >= (int64_t(1) << 31)) return RY_EINVAL;
  if (cfg->bc != RY_PBC_PERIODIC && cfg->bc != RY_PBC_DIRICHLET) return RY_EINVAL;
  if (cfg->precond != RY_PC_NONE && cfg->precond != RY_PC_STENCIL7) return RY_EINVAL;
  if ((cfg->dev_alloc == nullptr) != (cfg->dev_free == nullptr)) return RY_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RY_EHIP;
  ry_poisson* p = new (std::nothrow) ry_poisson();
  if (!p) return RY_ENOMEM;
  p->cfg = *cfg;
  p->g = {cfg->n[0], cfg->n[1], cfg->n[2], cfg->bc};
  p->N = N;
  if (cfg->stream) {
    p->stream = (hipStream_t)cfg->stream;
  } else {
    if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess) {
      delete p;
      return RY_EHIP;
    }
    p->own_stream = true;
  }
  // z chunks: enough workgroups to fill 256 CUs several times over
  const int gx = (cfg->n[0] + TX - 1) / TX, gy = (cfg->n[1] + TY - 1) / TY;
  int nch = (2048 + gx * gy - 1) / (gx * gy);
  if (nch > cfg->n[2]) nch = cfg->n[2];
  if (nch < 1) nch = 1;
  p->cz = (cfg->n[2] + nch - 1) / nch;
  nch = (cfg->n[2] + p->cz - 1) / p->cz;
  p->nblk = gx * gy * nch;
  bool ok = true;
  for (int k = 0; k < NVEC && ok; ++k) ok = (p->v[k] = static_cast<double*>(palloc(p, sizeof(double) * N))) != nullptr;
  ok = ok && (p->part = static_cast<double*>(palloc(p, sizeof(double) * 2 * p->nblk))) != nullptr;
  ok = ok && (p->hist = static_cast<double*>(palloc(p, sizeof(double) * RY_POISSON_HIST))) != nullptr;
  ok = ok && (p->sc = static_cast<Scalars*>(palloc(p, sizeof(Scalars)))) != nullptr;
  if (ok && hipHostMalloc((void**)&p->h_done, sizeof(int32_t)) != hipSuccess) {
    p->h_done = nullptr;
    ok = false;
  }
  if (!ok) {
    pfree_all(p);
    if (p->own_stream) hipStreamDestroy(p->stream);
    delete p;
    return RY_ENOMEM;
  }
  hipLaunchKernelGGL(ppcg_reset_kernel, dim3(1), dim3(1), 0, p->stream, p->sc);
  if (hipGetLastError() != hipSuccess) {
    pfree_all(p);
    if (p->own_stream) hipStreamDestroy(p->stream);
    delete p;
    return RY_EHIP;
  }
  *out = p;
  return RY_OK;
  RY_ABI_CATCH
}

void ry_poisson_destroy(ry_poisson* p) {
  if (!p) return;
  pfree_all(p);
  if (p->own_stream && p->stream) hipStreamDestroy(p->stream);
  delete p;
}

ry_status ry_poisson_set_rhs(ry_poisson* p, const double* b, const double* x0) {
  RY_ABI_TRY
  if (!p || !b) return RY_EINVAL;
  const size_t bytes = sizeof(double) * size_t(p->N);
  double *x = p->v[0], *r = p->v[1], *u = p->v[2], *w0 = p->v[3], *z = p->v[5];
  // b is staged in z, which is cleared once r has been formed
  PCHK(p, hipMemcpyAsync(z, b, bytes, hipMemcpyHostToDevice, p->stream));
  if (x0) PCHK(p, hipMemcpyAsync(x, x0, bytes, hipMemcpyHostToDevice, p->stream));
  else PCHK(p, hipMemsetAsync(x, 0, bytes, p->stream));
  const int blocks = int(std::min<int64_t>((p->N + 255) / 256, 8192));
  hipLaunchKernelGGL(residual_kernel, dim3(blocks), dim3(256), 0, p->stream, p->g, z, x, r);
  hipLaunchKernelGGL(minv_kernel, dim3(blocks), dim3(256), 0, p->stream, p->g, p->cfg.precond, r, u);
  hipLaunchKernelGGL(apply_a_dots_kernel, dim3(p->nblk), dim3(NTH), 0, p->stream, p->g, r, u, w0, p->part);
  PCHK(p, hipGetLastError());
  for (int k = 5; k < NVEC; ++k) PCHK(p, hipMemsetAsync(p->v[k], 0, bytes, p->stream));
  hipLaunchKernelGGL(ppcg_reset_kernel, dim3(1), dim3(1), 0, p->stream, p->sc);
  PCHK(p, hipGetLastError());
  p->ready = true;
  p->iter_hi = 0;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_poisson_solve(ry_poisson* p, double eps, int32_t max_iter, int32_t* n_iter) {
  RY_ABI_TRY
  if (!p) return RY_EINVAL;
  if (!p->ready) return pfail(p, RY_ESTATE, "ry_poisson_solve before ry_poisson_set_rhs");
  if (max_iter < 0 || max_iter > RY_POISSON_HIST - 1 || std::isnan(eps)) return RY_EINVAL;
  hipLaunchKernelGGL(ppcg_arm_kernel, dim3(1), dim3(1), 0, p->stream, p->sc, eps, max_iter, 0);
  PCHK(p, hipGetLastError());
  if (!p->timing) {
    ry_status s = ensure_graph(p);
    if (s) return s;
  }
  const int64_t batches = int64_t(max_iter) / BATCH + 2;
  for (int64_t k = 0; k < batches; ++k) {
    if (p->timing) {
      for (int j = 0; j < BATCH; ++j) {
        ry_status s = launch_iteration(p);
        if (s) return s;
      }
    } else {
      PCHK(p, hipGraphLaunch(p->graph, p->stream));
    }
    PCHK(p, hipMemcpyAsync(p->h_done, &p->sc->done, sizeof(int32_t), hipMemcpyDeviceToHost, p->stream));
    PCHK(p, hipStreamSynchronize(p->stream));
    if (*p->h_done) break;
  }
  Scalars s{};
  PCHK(p, hipMemcpy(&s, p->sc, sizeof s, hipMemcpyDeviceToHost));
  if (!s.done) return pfail(p, RY_ESTATE, "solver did not stop");
  p->iter_hi = s.iter;
  if (n_iter) *n_iter = s.iter;
  if (p->timing) collect_times(p);
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_poisson_iterate(ry_poisson* p, int32_t n) {
  RY_ABI_TRY
  if (!p || n < 0) return RY_EINVAL;
  if (!p->ready) return pfail(p, RY_ESTATE, "ry_poisson_iterate before ry_poisson_set_rhs");
  if (p->iter_hi + n > RY_POISSON_HIST - 1) return pfail(p, RY_EINVAL, "iteration history full");
  if (n == 0) return RY_OK;
  hipLaunchKernelGGL(ppcg_arm_kernel, dim3(1), dim3(1), 0, p->stream, p->sc, -1.0, n, 1);
  PCHK(p, hipGetLastError());
  // n iterations plus the finalize that records eps of the last iterate
  if (p->timing) {
    for (int j = 0; j <= n; ++j) {
      ry_status s = launch_iteration(p, j == n);
      if (s) return s;
    }
  } else {
    ry_status s = ensure_graph(p);
    if (s) return s;
    for (int j = 0; j <= n; j += BATCH) PCHK(p, hipGraphLaunch(p->graph, p->stream));
  }
  p->iter_hi += n;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_poisson_eps_history(ry_poisson* p, double* eps, int32_t cap, int32_t* n) {
  RY_ABI_TRY
  if (!p || !eps || cap < 0) return RY_EINVAL;
  Scalars s{};
  PCHK(p, hipStreamSynchronize(p->stream));
  PCHK(p, hipMemcpy(&s, p->sc, sizeof s, hipMemcpyDeviceToHost));
  const int32_t k = std::min<int32_t>(s.iter + 1, cap);
  if (k > 0) PCHK(p, hipMemcpy(eps, p->hist, sizeof(double) * k, hipMemcpyDeviceToHost));
  if (n) *n = k;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_poisson_download(ry_poisson* p, int32_t which, double* host) {
  RY_ABI_TRY
  if (!p || !host || which < 0 || which >= RY_PV_COUNT) return RY_EINVAL;
  Scalars s{};
  PCHK(p, hipStreamSynchronize(p->stream));
  PCHK(p, hipMemcpy(&s, p->sc, sizeof s, hipMemcpyDeviceToHost));
  // x r u w z q s p; w_i lives in buffer (i & 1)... after iteration i-1 wrote it
  int slot;
  switch (which) {
    case RY_PV_X: slot = 0; break;
    case RY_PV_R: slot = 1; break;
    case RY_PV_U: slot = 2; break;
    case RY_PV_W: slot = 3 + (s.iter & 1); break;
    default: slot = which + 1; break;   // z q s p -> 5..8
  }
  PCHK(p, hipMemcpy(host, p->v[slot], sizeof(double) * size_t(p->N), hipMemcpyDeviceToHost));
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_poisson_scalars(ry_poisson* p, double* alpha_prev, double* gamma_prev, int32_t* iter) {
  RY_ABI_TRY
  if (!p) return RY_EINVAL;
  Scalars s{};
  PCHK(p, hipStreamSynchronize(p->stream));
  PCHK(p, hipMemcpy(&s, p->sc, sizeof s, hipMemcpyDeviceToHost));
  if (alpha_prev) *alpha_prev = s.alpha_prev;
  if (gamma_prev) *gamma_prev = s.gamma_prev;
  if (iter) *iter = s.iter;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_poisson_set_timing(ry_poisson* p, int32_t on) {
  RY_ABI_TRY
  if (!p) return RY_EINVAL;
  PCHK(p, hipStreamSynchronize(p->stream));
  collect_times(p);
  p->timing = on != 0;
  p->t_launches = 0;
  p->t_ms = 0.0;
  return RY_OK;
  RY_ABI_CATCH
}

ry_status ry_poisson_kernel_time(ry_poisson* p, int32_t* launches, double* total_ms) {
  RY_ABI_TRY
  if (!p) return RY_EINVAL;
  PCHK(p, hipStreamSynchronize(p->stream));
  collect_times(p);
  if (launches) *launches = int32_t(p->t_launches);
  if (total_ms) *total_ms = p->t_ms;
  return RY_OK;
  RY_ABI_CATCH
}

const char* ry_poisson_last_error(const ry_poisson* p) { return p ? p->err.c_str() : "null solver"; }

}  // extern "C"
