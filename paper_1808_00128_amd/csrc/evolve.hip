// Term generation and CH-form evolution (step (a) of the hot path).
//
// Branch choice: exact enumeration (Eq. (Vphi)) or the i.i.d. draws of the
// Sparsification Lemma.  Evolution: the CH-form update rules of the
// Clifford-simulator section (L[S], L[CZ], L[CX]; the Hadamard update of
// Eqs. (H1)-(H7) with Prop. H, whose C-layer V_C acts through the right rules
// R[CX], R[CZ], R[S]).
//
// Mapping: one wavefront per term, lane p holds tableau row p (F_p, G_p, M_p
// as uint64, gamma_p).  The per-term words v, s, omega are wave-uniform and
// live in scalar registers.  A left rule touches one or two rows and costs a
// few readlanes; the Hadamard update reads row p by readlane, computes t, u,
// alpha, beta on the scalar unit and applies V_C to every row at once: each
// batch of commuting right rules (CX_{q,i} for i in a set W, CZ_{q,i} for i in
// V_1) collapses to a parity and a masked XOR per lane.
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

// ---------------------------------------------------------------------------
// Per-wave CH-form state.
// ---------------------------------------------------------------------------
struct WaveCH {
  uint64_t F, G, M;  // this lane's rows
  uint32_t g;        // gamma of this lane's row
  uint64_t v, s;     // wave-uniform
  uint32_t w;        // omega exponent in Z_8, wave-uniform
  uint32_t err;
};

// L[S_q]^pw: M_q ^= G_q (pw times), gamma_q -= pw.
__device__ __forceinline__ void gate_spow(WaveCH& c, uint32_t lane, uint32_t q, uint32_t pw) {
  if (lane == q) {
    if (pw & 1u) c.M ^= c.G;
    c.g = (c.g - pw) & 3u;
  }
}

// L[CZ_{q,r}]: M_q ^= G_r, M_r ^= G_q.
__device__ __forceinline__ void gate_cz(WaveCH& c, uint32_t lane, uint32_t q, uint32_t r) {
  const uint64_t Gq = rl64(c.G, q), Gr = rl64(c.G, r);
  if (lane == q) c.M ^= Gr;
  if (lane == r) c.M ^= Gq;
}

// L[CX_{q,r}]: gamma_q += gamma_r + 2 (M_q . F_r) with M_q before its update;
// G_r ^= G_q; F_q ^= F_r; M_q ^= M_r.
__device__ __forceinline__ void gate_cx(WaveCH& c, uint32_t lane, uint32_t q, uint32_t r) {
  const uint64_t Fr = rl64(c.F, r), Mr = rl64(c.M, r), Gq = rl64(c.G, q);
  const uint32_t gr = rl32(c.g, r);
  if (lane == q) {
    c.g = (c.g + gr + 2u * par64(c.M & Fr)) & 3u;
    c.F ^= Fr;
    c.M ^= Mr;
  }
  if (lane == r) c.G ^= Gq;
}

// Hadamard on qubit p.
__device__ __forceinline__ void gate_h(WaveCH& c, uint32_t lane, uint32_t p) {
  const uint64_t Fp = rl64(c.F, p), Gp = rl64(c.G, p), Mp = rl64(c.M, p);
  const uint32_t gp = rl32(c.g, p);
  const uint64_t v = c.v, s = c.s, nv = ~v;
  // Eqs. (H2), (H4).
  const uint64_t t = s ^ (Gp & v);
  const uint64_t u = s ^ (Fp & nv) ^ (Mp & v);
  const uint32_t alpha = par64(Gp & nv & s);
  const uint32_t beta = par64(Mp & nv & s) ^ par64(Fp & v & (Mp ^ s));
  const uint32_t delta = (gp + 2u * (alpha + beta)) & 3u;
  if (t == u) {
    // omega' = 2^{-1/2} (-1)^alpha (1 + i^delta), delta odd: (-1)^alpha e^{+-i pi/4}.
    if (!(delta & 1u)) c.err = 1u;
    c.w = (c.w + 4u * alpha + (delta == 1u ? 1u : 7u)) & 7u;
    c.s = t;
    return;
  }
  // Prop. H: V_0, V_1 and the C-type circuit V_C, applied on the right.
  const uint64_t d = t ^ u, V0 = d & nv, V1 = d & v;
  uint32_t q;
  if (V0) {
    q = (uint32_t)__builtin_ctzll(V0);
    const uint64_t W = V0 & ~(1ull << q);
    const uint64_t fq = (c.F >> q) & 1ull;
    // R[CX_{q,i}] for all i in W: G_{.,q} ^= G_{.,i}; F_{.,i} ^= F_{.,q}; M_{.,q} ^= M_{.,i}.
    c.G ^= (uint64_t)par64(c.G & W) << q;
    c.F ^= W & (0ull - fq);
    c.M ^= (uint64_t)par64(c.M & W) << q;
    // R[CZ_{q,i}] for all i in V_1: M_{.,q} ^= F_{.,i}; M_{.,i} ^= F_{.,q}; gamma += 2 F_{.,q} F_{.,i}.
    const uint32_t pv1 = par64(c.F & V1);
    c.M ^= (uint64_t)pv1 << q;
    c.M ^= V1 & (0ull - fq);
    c.g = (c.g + 2u * ((uint32_t)fq & pv1)) & 3u;
  } else {
    q = (uint32_t)__builtin_ctzll(V1);
    const uint64_t W = V1 & ~(1ull << q);
    // R[CX_{i,q}] for all i in W: G_{.,i} ^= G_{.,q}; F_{.,q} ^= F_{.,i}; M_{.,i} ^= M_{.,q}.
    const uint64_t gq = (c.G >> q) & 1ull, mq = (c.M >> q) & 1ull;
    c.G ^= W & (0ull - gq);
    c.F ^= (uint64_t)par64(c.F & W) << q;
    c.M ^= W & (0ull - mq);
  }
  const uint64_t qb = 1ull << q;
  const uint32_t tq = (uint32_t)((t >> q) & 1ull);
  const uint64_t y = tq ? (u ^ qb) : t;  // y, z differ only in bit q; y_q = t_q
  const uint32_t vq = (uint32_t)((v >> q) & 1ull);
  // H^{v_q}(|y_q> + i^delta |1-y_q>) = 2^{1/2} e^{i pi dw/4} S^a H^b |c>.
  // For y_q = 1 factor out i^delta: |0> + i^{-delta}|1>.
  const uint32_t dp = tq ? ((4u - delta) & 3u) : delta;
  const uint32_t ph = (2u * delta * tq) & 7u;
  uint32_t a, b, cc, dw;
  if (!vq) {
    // |0> + i^d |1> = 2^{1/2} S^{d & 1} H |d >> 1>.
    b = 1u;
    a = dp & 1u;
    cc = dp >> 1;
    dw = ph;
  } else {
    // H(|0> + i^d |1>): d = 0 -> |0>, 2 -> |1>, 1 -> e^{i pi/4} S H |1>, 3 -> e^{-i pi/4} S H |0>.
    b = dp & 1u;
    a = dp & 1u;
    cc = (dp == 2u || dp == 1u) ? 1u : 0u;
    dw = ph + (dp == 1u ? 1u : (dp == 3u ? 7u : 0u));
  }
  if (a) {
    // R[S_q]: M_{.,q} ^= F_{.,q}; gamma -= F_{.,q}.
    const uint64_t fq = (c.F >> q) & 1ull;
    c.M ^= fq << q;
    c.g = (c.g - (uint32_t)fq) & 3u;
  }
  c.s = (y & ~qb) | ((uint64_t)cc << q);
  c.v = (v & ~qb) | ((uint64_t)b << q);
  c.w = (c.w + 4u * alpha + dw) & 7u;
}

__device__ __forceinline__ void apply_gate(WaveCH& c, uint32_t lane, DGate gt) {
  switch (gt.op) {
    case OP_H: gate_h(c, lane, gt.q); break;
    case OP_S: gate_spow(c, lane, gt.q, 1u); break;
    case OP_SPOW: gate_spow(c, lane, gt.q, gt.arg); break;
    case OP_CX: gate_cx(c, lane, gt.q, gt.r); break;
    case OP_CZ: gate_cz(c, lane, gt.q, gt.r); break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// Evolution: one wave per term, 4 terms per workgroup.
// ---------------------------------------------------------------------------
template <bool kFromZero>
__global__ __launch_bounds__(256) void k_evolve(TermsView T, const DGate* __restrict__ gates,
                                                uint32_t n_gates,
                                                const SlotTable* __restrict__ slots,
                                                const DGate* __restrict__ bgates,
                                                uint32_t* __restrict__ err) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = uniform32(threadIdx.x >> 6);
  const uint64_t term = (uint64_t)blockIdx.x * 4u + wave;
  if (term >= T.chi) return;
  const uint32_t n = T.n;
  const bool act = lane < n;
  const uint64_t chi = T.chi;
  WaveCH c;
  if (kFromZero) {
    c.F = act ? (1ull << lane) : 0ull;
    c.G = c.F;
    c.M = 0ull;
    c.g = 0u;
    c.v = 0ull;
    c.s = 0ull;
    c.w = 0u;
  } else {
    const uint64_t off = (uint64_t)lane * chi + term;
    c.F = act ? T.F[off] : 0ull;
    c.G = act ? T.G[off] : 0ull;
    c.M = act ? T.M[off] : 0ull;
    c.g = act ? T.gamma[off] : 0u;
    c.v = T.v[term];
    c.s = T.s[term];
    c.w = T.omega[term];
  }
  c.err = 0u;
  for (uint32_t i = 0; i < n_gates; ++i) {
    const DGate gt = gates[i];
    if (gt.op == OP_SLOT) {
      const uint32_t j = T.branch[(uint64_t)gt.slot * chi + term];
      const uint32_t k0 = slots[gt.slot].goff[j], k1 = slots[gt.slot].goff[j + 1];
      for (uint32_t k = k0; k < k1; ++k) apply_gate(c, lane, bgates[k]);
    } else {
      apply_gate(c, lane, gt);
    }
  }
  if (act) {
    const uint64_t off = (uint64_t)lane * chi + term;
    T.F[off] = c.F;
    T.G[off] = c.G;
    T.M[off] = c.M;
    T.gamma[off] = (uint8_t)c.g;
  }
  if (lane == 0) {
    T.v[term] = c.v;
    T.s[term] = c.s;
    T.omega[term] = (uint8_t)c.w;
    if (c.err) atomicOr(err, 1u);
  }
}

hipError_t launch_evolve(const TermsView& T, const DGate* gates, uint32_t n_gates,
                         const SlotTable* slots, const DGate* bgates, bool from_zero,
                         uint32_t* err, hipStream_t st) {
  const uint32_t blocks = (uint32_t)((T.chi + 3) / 4);
  if (from_zero)
    hipLaunchKernelGGL(k_evolve<true>, dim3(blocks), dim3(256), 0, st, T, gates, n_gates, slots,
                       bgates, err);
  else
    hipLaunchKernelGGL(k_evolve<false>, dim3(blocks), dim3(256), 0, st, T, gates, n_gates, slots,
                       bgates, err);
  return hipGetLastError();
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
