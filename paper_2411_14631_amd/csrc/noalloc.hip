// ry_cfl_dt_noalloc: the CFL time step of one level held in the caller's
// device memory, for callers that cannot allocate device memory.  Its
// partial maxima, error word and result live in a file-scope device array
// (one copy per GPU, held until the process ends) instead of buffers a
// context allocates; the kernels are the CFL pass of ry_cfl_dt.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "ry_internal.h"

namespace ry {
namespace {

// Scratch layout (doubles): [0, kMaxBlocks) per-block maxima of the signal
// speed, then the error word (as an int32 in the first half of a double),
// then the maximum.  kMaxBlocks partials cover kMaxOcts octs (256 cells per
// block): 2M octs (16M cells, a 256^3 level), 512 KiB of scratch.
constexpr int64_t kMaxBlocks = 1 << 16;
constexpr int64_t kMaxOcts = kMaxBlocks * 256 / 8;
constexpr int64_t kScratch = kMaxBlocks + 2;
static __device__ __align__(256) double scratch[kScratch];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
double* g_ptr[kMaxDevices] = {nullptr};

// Device address of this GPU's copy of `scratch`, looked up once per device
// (the array's name is not a device address in host code).
hipError_t scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_lock);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

// One block: the maximum of n partials (non-negative) into *out.
__global__ __launch_bounds__(1024) void max_partials_kernel(const double* __restrict__ part, int64_t n,
                                                            double* __restrict__ out) {
  __shared__ double red[16];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) m = fmax(m, part[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < 16; ++w) r = fmax(r, red[w]);
    *out = r;
  }
}

}  // namespace
}  // namespace ry

extern "C" ry_status ry_cfl_dt_noalloc(const double* U, int64_t plane, int64_t n_oct, const uint8_t* refined,
                                       double gamma, double cfl, double dx, double rho_floor, double p_floor,
                                       double* dt, void* stream) {
  using namespace ry;
  if (!U || !refined || !dt || n_oct <= 0 || plane < 8 * n_oct) return RY_EINVAL;
  if (n_oct > kMaxOcts) return RY_EINVAL;                // beyond the scratch array
  if (!(gamma > 1.0) || !(cfl > 0.0) || !(dx > 0.0) || !(rho_floor > 0.0) || !(p_floor > 0.0)) return RY_EINVAL;
  double* ptr = nullptr;
  if (scratch_ptr(&ptr) != hipSuccess) return RY_EHIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* part = ptr;
  int32_t* err = reinterpret_cast<int32_t*>(ptr + kMaxBlocks);
  double* smax = ptr + kMaxBlocks + 1;
  // the error word starts at zero (a kernel, not a memset: callers may
  // capture this sequence into a graph)
  if (launch_zero_u32(reinterpret_cast<unsigned int*>(err), 1, st)) return RY_EHIP;
  const int rc = launch_cfl(U, plane, n_oct, refined, gamma, rho_floor, p_floor, part, kMaxBlocks, err, st);
  if (rc) return rc == LAUNCH_EXCEEDS_BUFFER ? RY_EINVAL : RY_EHIP;
  const int64_t nblk = cfl_blocks(n_oct);
  hipLaunchKernelGGL(max_partials_kernel, dim3(1), dim3(1024), 0, st, part, nblk, smax);
  if (hipGetLastError() != hipSuccess) return RY_EHIP;
  double host[2] = {0.0, 0.0};
  if (hipMemcpyAsync(host, ptr + kMaxBlocks, sizeof host, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return RY_EHIP;
  int32_t e = 0;
  __builtin_memcpy(&e, &host[0], sizeof e);
  if (e) return RY_ENUMERIC;
  const double s = host[1];
  *dt = (s > 0.0) ? cfl * dx / s : INFINITY;
  return RY_OK;
}
