// Term generation and CH-form evolution (step (a) of the hot path).
//
// Branch choice: exact enumeration (Eq. (Vphi)) or the i.i.d. draws of the
// Sparsification Lemma.  Evolution: the CH-form update rules of the
// Clifford-simulator section (L[S], L[CZ], L[CX]; the Hadamard update of
// Eqs. (H1)-(H7) with Prop. H, whose C-layer V_C acts through the right rules
// R[CX], R[CZ], R[S]).
//
// Mapping: a term is a group of LPT lanes (a sub-wave; 64 / LPT terms per
// wave) and each lane holds RPL tableau rows (F_p, G_p, M_p as uint64,
// gamma_p).  A left rule touches one or two rows: it costs a few in-group
// broadcasts (ds_bpermute, readlane for a whole-wave group) and a masked XOR,
// shared by all the terms of the wave.  The Hadamard update broadcasts row p,
// computes t, u, alpha, beta once per lane, and applies V_C to every row at
// once: each batch of commuting right rules (CX_{q,i} for i in a set W,
// CZ_{q,i} for i in V_1) collapses to a parity and a masked XOR per row.
#include "device_common.hpp"
#include "internal.hpp"

namespace chsim {

// ---------------------------------------------------------------------------
// Branch choice and coefficients, one thread per term.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_choose(TermsView T, const SlotTable* __restrict__ slots,
                                                uint32_t mode, uint64_t seed, double scale) {
  const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= T.chi) return;
  double br = 1.0, bi = 0.0;
  if (mode == CHSIM_EXACT) {
    uint64_t rem = a;
    for (uint32_t p = 0; p < T.n_slot; ++p) {
      const uint32_t nb = slots[p].n_branch;
      const uint32_t j = (uint32_t)(rem % nb);
      rem /= nb;
      T.branch[(uint64_t)p * T.chi + a] = (uint8_t)j;
      const double cr = slots[p].coef_re[j], ci = slots[p].coef_im[j];
      const double nr = br * cr - bi * ci;
      bi = br * ci + bi * cr;
      br = nr;
    }
  } else {
    for (uint32_t p = 0; p < T.n_slot; ++p) {
      const SlotTable& st = slots[p];
      const double u = philox_uniform53(seed, a, p, kStreamSparsify);
      const double uw = u * st.total;
      uint32_t j = st.n_branch - 1;
      for (uint32_t i = 0; i + 1 < st.n_branch; ++i)
        if (uw < st.cum[i]) {
          j = i;
          break;
        }
      T.branch[(uint64_t)p * T.chi + a] = (uint8_t)j;
      const double cr = st.unit_re[j], ci = st.unit_im[j];
      const double nr = br * cr - bi * ci;
      bi = br * ci + bi * cr;
      br = nr;
    }
    br *= scale;
    bi *= scale;
  }
  T.b[a] = make_double2(br, bi);
}

hipError_t launch_choose(const TermsView& T, const SlotTable* slots, uint32_t mode, uint64_t seed,
                         double scale, hipStream_t st) {
  const uint32_t blocks = (uint32_t)((T.chi + 255) / 256);
  hipLaunchKernelGGL(k_choose, dim3(blocks), dim3(256), 0, st, T, slots, mode, seed, scale);
  return hipGetLastError();
}

EvolveShape evolve_shape_for(uint32_t n, int lanes) {
  EvolveShape s;
  s.lanes = lanes;
  s.rows = lanes > 0 ? (int)((n + (uint32_t)lanes - 1) / (uint32_t)lanes) : 0;
  if (s.rows < 1) s.rows = 1;
  return s;
}

// Default: rows in LDS, 8 lanes per term (4 for n <= 16).
EvolveShape evolve_default_shape(uint32_t n) {
  EvolveShape s = evolve_shape_for(n, n <= 16 ? 4 : 8);
  s.lds = true;
  return s;
}

uint64_t evolve_capacity(EvolveShape s, uint32_t n) {
  return s.lds ? evolve_lds_capacity(s.lanes, n) : 0u;
}

// Instantiated shapes: lanes in {4, 8, 16, 32, 64} with rows = ceil(n / lanes)
// and lanes * rows <= 64; rows in LDS: lanes in {4, 8, 16} (gamma of a lane's
// rows packed in 16 bits).
bool evolve_shape_supported(EvolveShape s, uint32_t n) {
  if (s.lds)
    return (s.lanes == 4 || s.lanes == 8 || s.lanes == 16) && n >= 1 && n <= 64 &&
           (uint32_t)s.lanes * 16u >= n;
  const bool lanes_ok = s.lanes == 4 || s.lanes == 8 || s.lanes == 16 || s.lanes == 32 || s.lanes == 64;
  return lanes_ok && s.rows >= 1 && (uint32_t)(s.lanes * s.rows) >= n && s.lanes * s.rows <= 64;
}

hipError_t launch_evolve_job(const EvolveJob& J, const DGate* gates, uint32_t n_gates, bool from_zero,
                             uint32_t* err, EvolveShape shape, hipStream_t st) {
  const uint32_t n = J.dst.n;
  if (shape.lanes == 0) shape = evolve_default_shape(n);
  if (!evolve_shape_supported(shape, n)) return hipErrorInvalidValue;
  if (shape.lds) return launch_evolve_lds(shape.lanes, J, gates, n_gates, from_zero, err, st);
  if (shape.lanes == 4) return launch_evolve_l4(shape.rows, J, gates, n_gates, from_zero, err, st);
  if (shape.lanes == 8) return launch_evolve_l8(shape.rows, J, gates, n_gates, from_zero, err, st);
  if (shape.lanes == 64) return launch_evolve_w64(J, gates, n_gates, from_zero, err, st);
  return launch_evolve_wide(shape.lanes, shape.rows, J, gates, n_gates, from_zero, err, st);
}

hipError_t launch_evolve(const TermsView& T, const DGate* gates, uint32_t n_gates,
                         const uint32_t* slot_seq, uint32_t n_occ, bool from_zero, uint32_t* err,
                         EvolveShape shape, hipStream_t st) {
  EvolveJob J;
  J.src = T;
  J.dst = T;
  J.src_rs = J.dst_rs = T.chi;
  J.src_is = J.dst_is = 1;
  J.src_idx = nullptr;
  J.br_idx = nullptr;
  J.branch = T.branch;
  J.chi_br = T.chi;
  J.count_dev = nullptr;
  J.count = T.chi;
  J.slot_seq = slot_seq;
  J.n_occ = n_occ;
  return launch_evolve_job(J, gates, n_gates, from_zero, err, shape, st);
}

// Materialise |0^n> for every term (used when terms are read before any gate).
__global__ __launch_bounds__(256) void k_set_zero(TermsView T) {
  const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= T.chi) return;
  for (uint32_t p = 0; p < T.n; ++p) {
    const uint64_t off = (uint64_t)p * T.chi + a;
    T.F[off] = 1ull << p;
    T.G[off] = 1ull << p;
    T.M[off] = 0ull;
    T.gamma[off] = 0;
  }
  T.v[a] = 0ull;
  T.s[a] = 0ull;
  T.omega[a] = 0;
}

hipError_t launch_set_zero(const TermsView& T, hipStream_t st) {
  const uint32_t blocks = (uint32_t)((T.chi + 255) / 256);
  hipLaunchKernelGGL(k_set_zero, dim3(blocks), dim3(256), 0, st, T);
  return hipGetLastError();
}

// Three-step sampler: w = s with bits flipped where v and flips agree; x = w G^T.
__global__ __launch_bounds__(256) void k_sample(TermsView T, const uint64_t* __restrict__ alpha,
                                                const uint64_t* __restrict__ flips,
                                                uint64_t* __restrict__ x_out, uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t a = alpha[i];
  const uint64_t w = T.s[a] ^ (T.v[a] & flips[i]);
  uint64_t x = 0;
  for (uint32_t r = 0; r < T.n; ++r) x |= (uint64_t)par64(w & T.G[(uint64_t)r * T.chi + a]) << r;
  x_out[i] = x;
}

hipError_t launch_sample(const TermsView& T, const uint64_t* alpha, const uint64_t* flips,
                         uint64_t* x_out, uint32_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_sample, dim3((count + 255) / 256), dim3(256), 0, st, T, alpha, flips, x_out,
                     count);
  return hipGetLastError();
}

}  // namespace chsim
