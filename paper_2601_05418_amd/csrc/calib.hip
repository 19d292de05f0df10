// Calibration of the compression bank (Eqs. 6-12).
#include <hip/hip_runtime.h>

#include "plan.h"

namespace gpjc {

int run_calibrate(Plan& pl, const uint8_t* roi, const float2* noise_cov, double* h_eig, double2* A_out) {
  (void)pl; (void)roi; (void)noise_cov; (void)h_eig; (void)A_out;
  return fail(GPJC_E_UNSUPPORTED, "calibration not built");
}

}  // namespace gpjc
