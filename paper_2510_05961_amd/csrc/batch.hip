// batch.hip -- batched evaluation of many independent systems.
#include "msm.h"
extern "C" msm_status msm_batch_plan_create(msm_plan* out, int, const double*, const int*, int,
                                            double, double, int, int, int) {
  if (out) *out = nullptr;
  return MSM_ERR_UNSUPPORTED;
}
extern "C" msm_status msm_batch_energy_forces(msm_plan, const int*, const void*, const void*,
                                              double*, void*, void*, void*) {
  return MSM_ERR_UNSUPPORTED;
}
