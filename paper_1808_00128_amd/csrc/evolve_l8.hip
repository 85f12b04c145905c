// Evolution kernels with 8 lanes per term (8 terms per wave), 1..8 rows per lane.
#include "evolve_kernel.hpp"

namespace chsim {

hipError_t launch_evolve_l8(int rows, const EvolveJob& J, const DGate* gates, uint32_t n_gates,
                            bool from_zero, uint32_t* err, hipStream_t st) {
  switch (rows) {
#define CHSIM_CASE(R) \
  case R: return launch_evolve_t<8, R>(J, gates, n_gates, from_zero, err, st);
    CHSIM_CASE(1) CHSIM_CASE(2) CHSIM_CASE(3) CHSIM_CASE(4) CHSIM_CASE(5) CHSIM_CASE(6)
    CHSIM_CASE(7) CHSIM_CASE(8)
#undef CHSIM_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace chsim
