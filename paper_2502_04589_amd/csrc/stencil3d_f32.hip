// Fine-level 3D Q1 operator: float32 instances (the mixed form's CG and V-cycle).
#include "stencil3d_impl.hpp"

namespace pase {

void launch_fine3_f32(const Fine3Args& a, Epi epi, hipStream_t s) {
  switch (epi) {
    case EPI_AM:
      if (a.out1 && a.out2) launchv<float, EPI_AM>(a, s);
      else if (a.out1) launchv<float, EPI_A>(a, s);
      else if (a.out2) launchv<float, EPI_M>(a, s);
      break;
    case EPI_RESID: launchv<float, EPI_RESID>(a, s); break;
    case EPI_SWEEP: launchv<float, EPI_SWEEP>(a, s); break;
    case EPI_EIGRES: launchv<float, EPI_EIGRES>(a, s); break;
    case EPI_AMDOT: launchv<float, EPI_AMDOT>(a, s); break;
    case EPI_SWEEPDOT: launchv<float, EPI_SWEEPDOT>(a, s); break;
    case EPI_SWEEP2: launchv<float, EPI_SWEEP2>(a, s); break;
    case EPI_SWEEP2V: launchv<float, EPI_SWEEP2V>(a, s); break;
    case EPI_RESID1V: launchv<float, EPI_RESID1V>(a, s); break;
    case EPI_A: launchv<float, EPI_A>(a, s); break;
    case EPI_M: launchv<float, EPI_M>(a, s); break;
  }
}

}  // namespace pase
