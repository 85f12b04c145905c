// Proposal network state on the device and the learned-chain view.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace chsim {

// Packed FP32 parameters in the public order W1 [H][n], b1 [H], W2 [H][H],
// b2 [H], W3 [n][H], b3 [n]; BF16 copies of W1, W2, W3 back to back.
struct MLPLayout {
  uint32_t n, H;
  __host__ __device__ uint64_t off_W1() const { return 0; }
  __host__ __device__ uint64_t off_b1() const { return (uint64_t)H * n; }
  __host__ __device__ uint64_t off_W2() const { return off_b1() + H; }
  __host__ __device__ uint64_t off_b2() const { return off_W2() + (uint64_t)H * H; }
  __host__ __device__ uint64_t off_W3() const { return off_b2() + H; }
  __host__ __device__ uint64_t off_b3() const { return off_W3() + (uint64_t)n * H; }
  __host__ __device__ uint64_t count() const { return off_b3() + n; }
  __host__ __device__ uint64_t wb_W1() const { return 0; }
  __host__ __device__ uint64_t wb_W2() const { return (uint64_t)H * n; }
  __host__ __device__ uint64_t wb_W3() const { return wb_W2() + (uint64_t)H * H; }
  __host__ __device__ uint64_t wb_count() const { return wb_W3() + (uint64_t)n * H; }
  // Index into the BF16 weight copies, or -1 for a bias.
  __host__ __device__ int64_t weight_index(uint64_t i) const {
    if (i < off_b1()) return (int64_t)(wb_W1() + i);
    if (i >= off_W2() && i < off_b2()) return (int64_t)(wb_W2() + (i - off_W2()));
    if (i >= off_W3() && i < off_b3()) return (int64_t)(wb_W3() + (i - off_W3()));
    return -1;
  }
};

struct MLPDev {
  MLPLayout L{};
  uint32_t cap = 0;  // largest batch the activation buffers hold
  uint64_t step = 0; // Adam step count
  float* p = nullptr;
  float* grad = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  uint16_t* wb = nullptr;
  // activations [cap][.]
  uint16_t *a0 = nullptr, *a1 = nullptr, *a2 = nullptr;
  float *z1 = nullptr, *z2 = nullptr, *logits = nullptr;
  float *gf = nullptr, *dz1 = nullptr, *dz2 = nullptr;
  uint16_t *gb = nullptr, *gz1 = nullptr, *gz2 = nullptr;
  // FP32 partial sums of K-split products and column sums
  float* part = nullptr;
  uint64_t part_cap = 0;
};

struct LearnedView {
  uint32_t n, n_chain, n_steps;
  float eps, pi_min, pi_max;
  const double* u_mix;   // [chains][steps]
  const uint32_t* j;     // [chains][steps]
  const double* u_bits;  // [chains][steps][n]
  const double* u;       // [chains][steps]
  uint64_t* x;           // chain states (shared with the MetroView)
  uint64_t* y;           // proposals
  uint64_t* mask;        // flip masks
  float* logit_x;        // [chains][n], network output at x
  float* logit_y;        // [chains][n], at y
  uint32_t* n_flips;     // [chains][steps] or null
};

hipError_t mlp_refresh(MLPDev& d, hipStream_t st);
hipError_t mlp_forward(MLPDev& d, const uint64_t* x, uint32_t B, float* logits, hipStream_t st);
hipError_t mlp_loss_grad(MLPDev& d, const uint64_t* x, const uint64_t* t, uint32_t B,
                         double* loss_acc, hipStream_t st);
hipError_t mlp_adam(MLPDev& d, float lr, hipStream_t st);
hipError_t launch_learned_steps(const TermsView& T, MetroView& Mv, LearnedView& Lv, MLPDev& d,
                                uint32_t n_steps, hipStream_t st);

}  // namespace chsim
