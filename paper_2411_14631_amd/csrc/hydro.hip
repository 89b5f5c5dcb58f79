// Hydro-only (no passive scalar) instantiations of the per-tile hydro
// kernel, FP64 and mixed, every supported launch shape and both tile sizes
// (4^3 and 8^3 cells).  Compiled on its own
// so that its scheduling options do not apply to the other kernels.
#include <hip/hip_runtime.h>

#include "hydro_tile.h"
#include "ry_internal.h"

namespace ry {

int launch_hydro_plain(const HydroArgs& a, int precision, const ry_tuning& t, int num_cu, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (t.tile_cells == 8) {
    if (t.tiles_per_wg != 1 || t.persistent) return -1;
    if (t.waves_per_tile == 8)
      return precision == RY_MIXED ? launch_hydro_t<float, 1, 8, 0, 8>(a, t, num_cu, s)
                                   : launch_hydro_t<double, 1, 8, 0, 8>(a, t, num_cu, s);
    if (t.waves_per_tile == 4)
      return precision == RY_MIXED ? launch_hydro_t<float, 1, 4, 0, 8>(a, t, num_cu, s)
                                   : launch_hydro_t<double, 1, 4, 0, 8>(a, t, num_cu, s);
    return -1;
  }
  const int key = t.tiles_per_wg * 10 + t.waves_per_tile;
  if (precision == RY_MIXED) {
    switch (key) {
      case 11: return launch_hydro_t<float, 1, 1, 0>(a, t, num_cu, s);
      case 21: return launch_hydro_t<float, 2, 1, 0>(a, t, num_cu, s);
      case 41: return launch_hydro_t<float, 4, 1, 0>(a, t, num_cu, s);
      case 12: return launch_hydro_t<float, 1, 2, 0>(a, t, num_cu, s);
      case 22: return launch_hydro_t<float, 2, 2, 0>(a, t, num_cu, s);
      case 14: return launch_hydro_t<float, 1, 4, 0>(a, t, num_cu, s);
      default: return -1;
    }
  }
  switch (key) {
    case 11: return launch_hydro_t<double, 1, 1, 0>(a, t, num_cu, s);
    case 21: return launch_hydro_t<double, 2, 1, 0>(a, t, num_cu, s);
    case 41: return launch_hydro_t<double, 4, 1, 0>(a, t, num_cu, s);
    case 12: return launch_hydro_t<double, 1, 2, 0>(a, t, num_cu, s);
    case 22: return launch_hydro_t<double, 2, 2, 0>(a, t, num_cu, s);
    case 14: return launch_hydro_t<double, 1, 4, 0>(a, t, num_cu, s);
    default: return -1;
  }
}

}  // namespace ry
