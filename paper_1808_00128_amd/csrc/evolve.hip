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

// ---------------------------------------------------------------------------
// Sub-wave CH-form state.  A term owns LPT consecutive lanes (its group) and
// each lane holds RPL tableau rows: row p lives in lane p % LPT of the group,
// register p / LPT.  The per-term words v, s, omega are replicated in the
// group's lanes.  Rows p >= n are zero and stay zero under every rule.
// ---------------------------------------------------------------------------
template <int LPT, int RPL>
struct SubCH {
  uint64_t F[RPL], G[RPL], M[RPL];
  uint32_t g[RPL];
  uint64_t v, s;
  uint32_t w, err;
};

// Row registers are selected with all-ones / zero masks (k is wave-uniform),
// never by an index, so the row arrays stay in registers.
template <int RPL, typename T>
__device__ __forceinline__ T pick(const T (&a)[RPL], uint32_t k) {
  T r = 0;
#pragma unroll
  for (int j = 0; j < RPL; ++j) r |= a[j] & ((T)0 - (T)(k == (uint32_t)j));
  return r;
}
__device__ __forceinline__ uint64_t sel64(uint32_t k, int j) { return 0ull - (uint64_t)(k == (uint32_t)j); }
__device__ __forceinline__ uint32_t sel32(uint32_t k, int j) { return 0u - (uint32_t)(k == (uint32_t)j); }

// Value held by lane `src` of the caller's group (src wave-uniform).
template <int LPT>
__device__ __forceinline__ uint32_t gb32(uint32_t x, uint32_t src, uint32_t base) {
  if (LPT == 64) return rl32(x, src);
  return (uint32_t)__builtin_amdgcn_ds_bpermute((int)((base + src) << 2), (int)x);
}
template <int LPT>
__device__ __forceinline__ uint64_t gb64(uint64_t x, uint32_t src, uint32_t base) {
  if (LPT == 64) return rl64(x, src);
  const int addr = (int)((base + src) << 2);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

struct Lane {
  uint32_t li, base;  // lane index in the group, first lane of the group
};

// L[S_q]^pw (pw may differ between groups): M_q ^= G_q pw times, gamma_q -= pw.
template <int LPT, int RPL>
__device__ __forceinline__ void sw_spow(SubCH<LPT, RPL>& c, Lane L, uint32_t q, uint32_t pw) {
  const uint32_t k = q / LPT;
  if (L.li == q % LPT) {
    const uint64_t odd = 0ull - (uint64_t)(pw & 1u);
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      c.M[j] ^= c.G[j] & odd & sel64(k, j);
      c.g[j] = (c.g[j] - (pw & sel32(k, j))) & 3u;
    }
  }
}

// L[CZ_{q,r}]: M_q ^= G_r, M_r ^= G_q.
template <int LPT, int RPL>
__device__ __forceinline__ void sw_cz(SubCH<LPT, RPL>& c, Lane L, uint32_t q, uint32_t r) {
  const uint32_t kq = q / LPT, kr = r / LPT;
  const uint64_t Gq = gb64<LPT>(pick<RPL>(c.G, kq), q % LPT, L.base);
  const uint64_t Gr = gb64<LPT>(pick<RPL>(c.G, kr), r % LPT, L.base);
  const uint64_t oq = 0ull - (uint64_t)(L.li == q % LPT);
  const uint64_t orr = 0ull - (uint64_t)(L.li == r % LPT);
#pragma unroll
  for (int j = 0; j < RPL; ++j) c.M[j] ^= (Gr & oq & sel64(kq, j)) ^ (Gq & orr & sel64(kr, j));
}

// L[CX_{q,r}]: gamma_q += gamma_r + 2 (M_q . F_r) with M_q before its update;
// G_r ^= G_q; F_q ^= F_r; M_q ^= M_r.
template <int LPT, int RPL>
__device__ __forceinline__ void sw_cx(SubCH<LPT, RPL>& c, Lane L, uint32_t q, uint32_t r) {
  const uint32_t kq = q / LPT, kr = r / LPT;
  const uint64_t Fr = gb64<LPT>(pick<RPL>(c.F, kr), r % LPT, L.base);
  const uint64_t Mr = gb64<LPT>(pick<RPL>(c.M, kr), r % LPT, L.base);
  const uint32_t gr = gb32<LPT>(pick<RPL>(c.g, kr), r % LPT, L.base);
  const uint64_t Gq = gb64<LPT>(pick<RPL>(c.G, kq), q % LPT, L.base);
  const uint64_t oq = 0ull - (uint64_t)(L.li == q % LPT);
  const uint64_t orr = 0ull - (uint64_t)(L.li == r % LPT);
  const uint32_t Mq_dot_Fr = par64(pick<RPL>(c.M, kq) & Fr);
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    const uint64_t mq = oq & sel64(kq, j);
    c.g[j] = (c.g[j] + ((gr + 2u * Mq_dot_Fr) & (uint32_t)mq)) & 3u;
    c.F[j] ^= Fr & mq;
    c.M[j] ^= Mr & mq;
    c.G[j] ^= Gq & orr & sel64(kr, j);
  }
}

// Hadamard on qubit p: Eqs. (H2), (H4), the t = u case, and Prop. H with
// V_C applied to every row by batches of commuting right rules.
template <int LPT, int RPL>
__device__ __forceinline__ void sw_h(SubCH<LPT, RPL>& c, Lane L, uint32_t p) {
  const uint32_t kp = p / LPT, sp = p % LPT;
  const uint64_t Fp = gb64<LPT>(pick<RPL>(c.F, kp), sp, L.base);
  const uint64_t Gp = gb64<LPT>(pick<RPL>(c.G, kp), sp, L.base);
  const uint64_t Mp = gb64<LPT>(pick<RPL>(c.M, kp), sp, L.base);
  const uint32_t gp = gb32<LPT>(pick<RPL>(c.g, kp), sp, L.base);
  const uint64_t v = c.v, s = c.s, nv = ~v;
  const uint64_t t = s ^ (Gp & v);
  const uint64_t u = s ^ (Fp & nv) ^ (Mp & v);
  const uint32_t alpha = par64(Gp & nv & s);
  const uint32_t beta = par64(Mp & nv & s) ^ par64(Fp & v & (Mp ^ s));
  const uint32_t delta = (gp + 2u * (alpha + beta)) & 3u;
  if (t == u) {
    // omega' = 2^{-1/2} (-1)^alpha (1 + i^delta) with delta odd: (-1)^alpha e^{+-i pi/4}.
    if (!(delta & 1u)) c.err = 1u;
    c.w = (c.w + 4u * alpha + (delta == 1u ? 1u : 7u)) & 7u;
    c.s = t;
    return;
  }
  const uint64_t d = t ^ u, V0 = d & nv, V1 = d & v;
  uint32_t q;
  if (V0) {
    q = (uint32_t)__builtin_ctzll(V0);
    const uint64_t W = V0 & ~(1ull << q);
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      const uint64_t fq = (c.F[j] >> q) & 1ull;
      // R[CX_{q,i}], i in W: G_{.,q} ^= G_{.,i}; F_{.,i} ^= F_{.,q}; M_{.,q} ^= M_{.,i}.
      c.G[j] ^= (uint64_t)par64(c.G[j] & W) << q;
      c.F[j] ^= W & (0ull - fq);
      c.M[j] ^= (uint64_t)par64(c.M[j] & W) << q;
      // R[CZ_{q,i}], i in V_1: M_{.,q} ^= F_{.,i}; M_{.,i} ^= F_{.,q}; gamma += 2 F_{.,q} F_{.,i}.
      const uint32_t pv1 = par64(c.F[j] & V1);
      c.M[j] ^= ((uint64_t)pv1 << q) ^ (V1 & (0ull - fq));
      c.g[j] = (c.g[j] + 2u * ((uint32_t)fq & pv1)) & 3u;
    }
  } else {
    q = (uint32_t)__builtin_ctzll(V1);
    const uint64_t W = V1 & ~(1ull << q);
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      // R[CX_{i,q}], i in W: G_{.,i} ^= G_{.,q}; F_{.,q} ^= F_{.,i}; M_{.,i} ^= M_{.,q}.
      const uint64_t gq = (c.G[j] >> q) & 1ull, mq = (c.M[j] >> q) & 1ull;
      c.G[j] ^= W & (0ull - gq);
      c.F[j] ^= (uint64_t)par64(c.F[j] & W) << q;
      c.M[j] ^= W & (0ull - mq);
    }
  }
  const uint64_t qb = 1ull << q;
  const uint32_t tq = (uint32_t)((t >> q) & 1ull);
  const uint64_t y = tq ? (u ^ qb) : t;  // y and z differ only in bit q; y_q = t_q
  const uint32_t vq = (uint32_t)((v >> q) & 1ull);
  // H^{v_q}(|y_q> + i^delta |1 - y_q>) = 2^{1/2} e^{i pi dw/4} S^a H^b |c>; for
  // y_q = 1 factor out i^delta and use |0> + i^{-delta} |1>.
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
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      // R[S_q]: M_{.,q} ^= F_{.,q}; gamma -= F_{.,q}.
      const uint64_t fq = (c.F[j] >> q) & 1ull;
      c.M[j] ^= fq << q;
      c.g[j] = (c.g[j] - (uint32_t)fq) & 3u;
    }
  }
  c.s = (y & ~qb) | ((uint64_t)cc << q);
  c.v = (v & ~qb) | ((uint64_t)b << q);
  c.w = (c.w + 4u * alpha + dw) & 7u;
}

template <int LPT, int RPL>
__device__ __forceinline__ void sw_apply(SubCH<LPT, RPL>& c, Lane L, DGate gt) {
  switch (gt.op) {
    case OP_H: sw_h(c, L, gt.q); break;
    case OP_S: sw_spow(c, L, gt.q, 1u); break;
    case OP_SPOW: sw_spow(c, L, gt.q, gt.arg); break;
    case OP_CX: sw_cx(c, L, gt.q, gt.r); break;
    case OP_CZ: sw_cz(c, L, gt.q, gt.r); break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// Evolution kernel: 256 threads = 4 waves = 256 / LPT terms.
// ---------------------------------------------------------------------------
template <int LPT, int RPL, bool kFromZero>
__global__ __launch_bounds__(256) void k_evolve(TermsView T, const DGate* __restrict__ gates,
                                                uint32_t n_gates,
                                                const SlotTable* __restrict__ slots,
                                                uint32_t* __restrict__ err) {
  constexpr int kTermsPerBlock = 256 / LPT;
  const uint32_t lane = threadIdx.x & 63u;
  Lane L;
  L.li = lane & (LPT - 1);
  L.base = lane & ~(uint32_t)(LPT - 1);
  // A whole-wave group has a wave-uniform term index: keep it (and v, s,
  // omega, and the Hadamard's t, u, alpha, beta) on the scalar unit.
  const uint32_t group = (LPT == 64) ? uniform32(threadIdx.x >> 6) : threadIdx.x / LPT;
  const uint64_t term = (uint64_t)blockIdx.x * kTermsPerBlock + group;
  const uint64_t chi = T.chi;
  const bool live = term < chi;
  // Dead groups (ragged last block) evolve a copy of term 0 (or |0^n>) and
  // store nothing; no early return, so every group of a wave stays in step.
  const uint64_t tm = live ? term : 0;
  const uint32_t n = T.n;
  SubCH<LPT, RPL> c;
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    const uint32_t p = L.li + (uint32_t)j * LPT;
    const bool act = p < n;
    if (kFromZero) {
      c.F[j] = act ? (1ull << p) : 0ull;
      c.G[j] = c.F[j];
      c.M[j] = 0ull;
      c.g[j] = 0u;
    } else {
      const uint64_t off = (uint64_t)p * chi + tm;
      c.F[j] = act ? T.F[off] : 0ull;
      c.G[j] = act ? T.G[off] : 0ull;
      c.M[j] = act ? T.M[off] : 0ull;
      c.g[j] = act ? T.gamma[off] : 0u;
    }
  }
  if (kFromZero) {
    c.v = 0ull;
    c.s = 0ull;
    c.w = 0u;
  } else {
    c.v = T.v[tm];
    c.s = T.s[tm];
    c.w = T.omega[tm];
  }
  c.err = 0u;
  // One flat gate list: slot gates are SLOT_SPOW (a per-term power of S) or
  // conditional gates of a general branch; a single dispatch site keeps the
  // row registers in one live range.
  for (uint32_t i = 0; i < n_gates; ++i) {
    DGate gt = gates[i];
    bool on = true;
    if (gt.op == OP_SLOT_SPOW) {
      const uint32_t j = T.branch[(uint64_t)gt.slot * chi + tm];
      gt.op = OP_SPOW;
      gt.arg = slots[gt.slot].spow[j];
    } else if (gt.cond) {
      on = T.branch[(uint64_t)gt.slot * chi + tm] == gt.arg2;
    }
    if (on) sw_apply(c, L, gt);
  }
  if (live) {
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      const uint32_t p = L.li + (uint32_t)j * LPT;
      if (p < n) {
        const uint64_t off = (uint64_t)p * chi + term;
        T.F[off] = c.F[j];
        T.G[off] = c.G[j];
        T.M[off] = c.M[j];
        T.gamma[off] = (uint8_t)c.g[j];
      }
    }
    if (L.li == 0) {
      T.v[term] = c.v;
      T.s[term] = c.s;
      T.omega[term] = (uint8_t)c.w;
      if (c.err) atomicOr(err, 1u);
    }
  }
}

template <int LPT, int RPL>
hipError_t launch_evolve_t(const TermsView& T, const DGate* gates, uint32_t n_gates,
                           const SlotTable* slots, bool from_zero, uint32_t* err, hipStream_t st) {
  constexpr int kTermsPerBlock = 256 / LPT;
  const uint32_t blocks = (uint32_t)((T.chi + kTermsPerBlock - 1) / kTermsPerBlock);
  if (from_zero)
    hipLaunchKernelGGL((k_evolve<LPT, RPL, true>), dim3(blocks), dim3(256), 0, st, T, gates, n_gates,
                       slots, err);
  else
    hipLaunchKernelGGL((k_evolve<LPT, RPL, false>), dim3(blocks), dim3(256), 0, st, T, gates,
                       n_gates, slots, err);
  return hipGetLastError();
}

EvolveShape evolve_default_shape(uint32_t n) {
  EvolveShape s;
  if (n <= 8) { s.lanes = 8; s.rows = 1; }
  else if (n <= 16) { s.lanes = 16; s.rows = 1; }
  else if (n <= 32) { s.lanes = 16; s.rows = 2; }
  else { s.lanes = 16; s.rows = 4; }
  return s;
}

// Instantiated shapes: lanes in {8, 16, 32, 64}, rows in {1, 2, 4, 8}.
bool evolve_shape_supported(EvolveShape s, uint32_t n) {
  const bool lanes_ok = s.lanes == 8 || s.lanes == 16 || s.lanes == 32 || s.lanes == 64;
  const bool rows_ok = s.rows == 1 || s.rows == 2 || s.rows == 4 || s.rows == 8;
  return lanes_ok && rows_ok && (uint32_t)(s.lanes * s.rows) >= n && s.lanes * s.rows <= 128;
}

hipError_t launch_evolve(const TermsView& T, const DGate* gates, uint32_t n_gates,
                         const SlotTable* slots, bool from_zero, uint32_t* err, EvolveShape shape,
                         hipStream_t st) {
  if (shape.lanes == 0) shape = evolve_default_shape(T.n);
  if (!evolve_shape_supported(shape, T.n)) return hipErrorInvalidValue;
#define CHSIM_EVOLVE_CASE(LN, RW)                                                            \
  if (shape.lanes == LN && shape.rows == RW)                                                 \
    return launch_evolve_t<LN, RW>(T, gates, n_gates, slots, from_zero, err, st);
  CHSIM_EVOLVE_CASE(8, 1) CHSIM_EVOLVE_CASE(8, 2) CHSIM_EVOLVE_CASE(8, 4) CHSIM_EVOLVE_CASE(8, 8)
  CHSIM_EVOLVE_CASE(16, 1) CHSIM_EVOLVE_CASE(16, 2) CHSIM_EVOLVE_CASE(16, 4) CHSIM_EVOLVE_CASE(16, 8)
  CHSIM_EVOLVE_CASE(32, 1) CHSIM_EVOLVE_CASE(32, 2) CHSIM_EVOLVE_CASE(32, 4)
  CHSIM_EVOLVE_CASE(64, 1) CHSIM_EVOLVE_CASE(64, 2)
#undef CHSIM_EVOLVE_CASE
  return hipErrorInvalidValue;
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
