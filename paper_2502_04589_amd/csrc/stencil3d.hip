// Fine-level 3D Q1 operator: launch configuration and dispatch (float64
// instances; the float32 instances are in stencil3d_f32.hip).
#include "stencil3d_impl.hpp"

namespace pase {

void launch_fine3_f32(const Fine3Args& a, Epi epi, hipStream_t s);

int fine3_spatial_blocks(int m, int nzc, int k, bool fp32) {
  // the column-sum partial rows are per (x-tile, y-tile, z-run); column chunks share a row.  Tiles
  // are 8 x 4 nodes or 8 x 8 by fine3_wide_tile (the rule of launchv_tile)
  const int by = fine3_wide_tile(k, fp32) ? 4 : 8;
  return ((m + 7) / 8) * ((m + by - 1) / by) * nzc;
}

int fine3_max_spatial_blocks(int m) {
  // bound over every tile and z-run length (8 x 4 tiles, runs of at least 4 planes)
  return ((m + 7) / 8) * ((m + 3) / 4) * ((m + 3) / 4);
}

int fine3_default_nzc(int m) {
  // Every block marches its z-run sequentially, so short runs give the grid more
  // parallelism; each run re-reads two halo planes.  Coarse levels (m < 48) take runs of 4:
  // their grids are small and their vectors stay in L2.
  const int zl = m >= 48 ? 16 : 4;
  return (m + zl - 1) / zl;
}

void launch_fine3(const Fine3Args& a, Epi epi, hipStream_t s) {
  if (a.fp32) {
    launch_fine3_f32(a, epi, s);
    return;
  }
  switch (epi) {
    case EPI_AM:
      if (a.out1 && a.out2) launchv<double, EPI_AM>(a, s);
      else if (a.out1) launchv<double, EPI_A>(a, s);
      else if (a.out2) launchv<double, EPI_M>(a, s);
      break;
    case EPI_RESID: launchv<double, EPI_RESID>(a, s); break;
    case EPI_SWEEP: launchv<double, EPI_SWEEP>(a, s); break;
    case EPI_EIGRES: launchv<double, EPI_EIGRES>(a, s); break;
    case EPI_AMDOT: launchv<double, EPI_AMDOT>(a, s); break;
    case EPI_SWEEPDOT: launchv<double, EPI_SWEEPDOT>(a, s); break;
    case EPI_SWEEP2: launchv<double, EPI_SWEEP2>(a, s); break;
    case EPI_SWEEP2V: launchv<double, EPI_SWEEP2V>(a, s); break;
    case EPI_RESID1V: launchv<double, EPI_RESID1V>(a, s); break;
    case EPI_A: launchv<double, EPI_A>(a, s); break;
    case EPI_M: launchv<double, EPI_M>(a, s); break;
  }
}

}  // namespace pase
