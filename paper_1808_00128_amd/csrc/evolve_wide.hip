// Evolution kernels with 16 or 32 lanes per term (4 or 2 terms per wave); one
// term per wave has its own kernel (evolve_w64.hip).
#include "evolve_kernel.hpp"

namespace chsim {

hipError_t launch_evolve_wide(int lanes, int rows, const EvolveJob& J, const DGate* gates,
                              uint32_t n_gates, bool from_zero, uint32_t* err, hipStream_t st) {
#define CHSIM_CASE(LN, R)                                                              \
  if (lanes == LN && rows == R)                                                        \
    return launch_evolve_t<LN, R>(J, gates, n_gates, from_zero, err, st);
  CHSIM_CASE(16, 1) CHSIM_CASE(16, 2) CHSIM_CASE(16, 3) CHSIM_CASE(16, 4)
  CHSIM_CASE(32, 1) CHSIM_CASE(32, 2)
#undef CHSIM_CASE
  return hipErrorInvalidValue;
}

}  // namespace chsim
