// CH-form evolution kernel (step (a) of the hot path), templated on the
// sub-wave mapping; instantiated by the evolve_l*.hip files.
//
// Mapping: a term is a group of LPT lanes (a sub-wave; 64 / LPT terms per
// wave) and each lane holds RPL tableau rows (F_p, G_p, M_p as uint64,
// gamma_p): row p lives in lane p % LPT of the group, register p / LPT.  The
// per-term words v, s, omega are replicated in the group's lanes.  Rows
// p >= n are zero and stay zero under every rule.
//
// Left rules L[S], L[CZ], L[CX] of the Clifford-simulator section touch one
// or two rows.  The row's register index is the same for every term of the
// wave (the gate is), so a scalar branch picks it and only that register is
// read or written; the row travels inside the group by ds_bpermute (readlane
// for a whole-wave group).  The Hadamard update of
// Eqs. (H1)-(H7) with Prop. H broadcasts row p, computes t, u, alpha, beta
// once per lane, and applies V_C to every row at once: each batch of
// commuting right rules (CX_{q,i} for i in a set W, CZ_{q,i} for i in V_1)
// collapses to a parity and a masked XOR per row.
#pragma once

#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"

namespace chsim {

// The row arrays are separate local arrays (not members of one aggregate):
// indexed with a wave-uniform register index they stay in VGPRs and the
// compiler reaches register k through M0-relative moves (s_set_gpr_idx),
// one VALU move per 32-bit word, instead of selecting over every register.
template <int LPT, int RPL>
struct SubCH {
  uint64_t (&F)[RPL];
  uint64_t (&G)[RPL];
  uint64_t (&M)[RPL];
  uint32_t (&g)[RPL];
  uint64_t& v;
  uint64_t& s;
  uint32_t& w;
  uint32_t& err;
};

// Value held by lane `src` of the caller's group (src wave-uniform).
template <int LPT>
__device__ __forceinline__ uint32_t gb32(uint32_t x, uint32_t src, uint32_t base) {
  if constexpr (LPT == 64) return rl32(x, src);
  else return (uint32_t)__builtin_amdgcn_ds_bpermute((int)((base + src) << 2), (int)x);
}
template <int LPT>
__device__ __forceinline__ uint64_t gb64(uint64_t x, uint32_t src, uint32_t base) {
  if constexpr (LPT == 64) {
    return rl64(x, src);
  } else {
    const int addr = (int)((base + src) << 2);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
  }
}

struct Lane {
  uint32_t li, base;  // lane index in the group, first lane of the group
};

// Runs fn(j) with the compile-time register index j == k (k wave-uniform)
// behind a chain of scalar branches.  Every row-array access is static, so
// the arrays stay individual registers; the empty asm keeps each case a
// branch target instead of a select over every register.
template <int J, int RPL, typename Fn>
__device__ __forceinline__ void at_row_from(uint32_t k, Fn& fn) {
  if constexpr (J < RPL) {
    if (k == (uint32_t)J) {
      asm volatile("");
      fn(std::integral_constant<int, J>{});
    } else {
      at_row_from<J + 1, RPL>(k, fn);
    }
  }
}
template <int RPL, typename Fn>
__device__ __forceinline__ void at_row(uint32_t k, Fn&& fn) {
  at_row_from<0, RPL>(k, fn);
}

// Left rules L[S]^pw, L[CZ], L[CX]: rows q and r are read at their register
// index, broadcast in the group, and the lanes holding q or r update them.
//   S^pw on q:   M_q ^= G_q pw times, gamma_q -= pw
//   CZ_{q,r}:    M_q ^= G_r, M_r ^= G_q
//   CX_{q,r}:    gamma_q += gamma_r + 2 (M_q . F_r) (M_q before the update),
//                G_r ^= G_q, F_q ^= F_r, M_q ^= M_r
// `on` is false for terms that skip the gate (a branch of another choice).
template <int LPT, int RPL>
__device__ __forceinline__ void sw_left(SubCH<LPT, RPL>& c, Lane L, uint32_t op, uint32_t q,
                                        uint32_t r, uint32_t pw, bool on) {
  const uint32_t kq = uniform32(q / LPT), kr = uniform32(r / LPT);
  const uint64_t oq = 0ull - (uint64_t)(on && L.li == q % LPT);
  const uint64_t orr = 0ull - (uint64_t)(on && L.li == r % LPT);
  if (op == OP_CX) {
    uint64_t Fr = 0, Mr = 0, Gq = 0, Mq = 0;
    uint32_t gr = 0;
    at_row<RPL>(kr, [&](auto j) {
      Fr = c.F[j];
      Mr = c.M[j];
      gr = c.g[j];
    });
    at_row<RPL>(kq, [&](auto j) {
      Gq = c.G[j];
      Mq = c.M[j];
    });
    Fr = gb64<LPT>(Fr, r % LPT, L.base);
    Mr = gb64<LPT>(Mr, r % LPT, L.base);
    gr = gb32<LPT>(gr, r % LPT, L.base);
    Gq = gb64<LPT>(Gq, q % LPT, L.base);
    const uint32_t dg = (gr + 2u * par64(Mq & Fr)) & (uint32_t)oq;
    at_row<RPL>(kq, [&](auto j) {
      c.F[j] ^= Fr & oq;
      c.M[j] ^= Mr & oq;
      c.g[j] = (c.g[j] + dg) & 3u;
    });
    at_row<RPL>(kr, [&](auto j) { c.G[j] ^= Gq & orr; });
  } else if (op == OP_CZ) {
    uint64_t Gq = 0, Gr = 0;
    at_row<RPL>(kq, [&](auto j) { Gq = c.G[j]; });
    at_row<RPL>(kr, [&](auto j) { Gr = c.G[j]; });
    Gq = gb64<LPT>(Gq, q % LPT, L.base);
    Gr = gb64<LPT>(Gr, r % LPT, L.base);
    at_row<RPL>(kq, [&](auto j) { c.M[j] ^= Gr & oq; });
    at_row<RPL>(kr, [&](auto j) { c.M[j] ^= Gq & orr; });
  } else {
    const uint64_t odd = oq & (0ull - (uint64_t)(pw & 1u));
    const uint32_t dg = (0u - pw) & (uint32_t)oq;
    at_row<RPL>(kq, [&](auto j) {
      c.M[j] ^= c.G[j] & odd;
      c.g[j] = (c.g[j] + dg) & 3u;
    });
  }
}

// Hadamard on qubit p: Eqs. (H2), (H4), the t = u case, and Prop. H with
// V_C applied to every row by batches of commuting right rules.
template <int LPT, int RPL>
__device__ __forceinline__ void sw_h(SubCH<LPT, RPL>& c, Lane L, uint32_t p) {
  const uint32_t sp = p % LPT, kp = uniform32(p / LPT);
  uint64_t Fp = 0, Gp = 0, Mp = 0;
  uint32_t gp = 0;
  at_row<RPL>(kp, [&](auto j) {
    Fp = c.F[j];
    Gp = c.G[j];
    Mp = c.M[j];
    gp = c.g[j];
  });
  Fp = gb64<LPT>(Fp, sp, L.base);
  Gp = gb64<LPT>(Gp, sp, L.base);
  Mp = gb64<LPT>(Mp, sp, L.base);
  gp = gb32<LPT>(gp, sp, L.base);
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
      // R[CZ_{q,i}], i in V_1: M_{.,q} ^= F_{.,i}; M_{.,i} ^= F_{.,q}; gamma += 2 F_{.,q} F_{.,i}.
      const uint32_t pv1 = par64(c.F[j] & V1);
      c.M[j] ^= ((uint64_t)(par64(c.M[j] & W) ^ pv1) << q) ^ (V1 & (0ull - fq));
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

// ---------------------------------------------------------------------------
// Evolution kernel: 256 threads = 4 waves = 256 / LPT work items.  Item i
// starts from |0^n> or from state src_idx[i] of J.src, reads its branch
// choices from term br_idx[i] of the term store, and leaves its result in
// state i of J.dst (see EvolveJob).
// ---------------------------------------------------------------------------
constexpr uint32_t kGateChunk = 2048;  // gates staged in LDS at a time (16 KiB)

template <int LPT, int RPL, bool kFromZero>
__global__ __launch_bounds__(256) void k_evolve(EvolveJob J, const DGate* __restrict__ gates,
                                                uint32_t n_gates, uint32_t* __restrict__ err) {
  constexpr int kTermsPerBlock = 256 / LPT;
  const uint64_t count = J.count_dev ? (uint64_t)*J.count_dev : J.count;
  if ((uint64_t)blockIdx.x * kTermsPerBlock >= count) return;  // whole block: no barrier skipped
  const uint32_t lane = threadIdx.x & 63u;
  Lane L;
  L.li = lane & (LPT - 1);
  L.base = lane & ~(uint32_t)(LPT - 1);
  // A whole-wave group has a wave-uniform item index: keep it (and v, s,
  // omega, and the Hadamard's t, u, alpha, beta) on the scalar unit.
  const uint32_t group = (LPT == 64) ? uniform32(threadIdx.x >> 6) : threadIdx.x / LPT;
  const uint64_t item = (uint64_t)blockIdx.x * kTermsPerBlock + group;
  const bool live = item < count;
  // Dead groups (ragged last block) evolve a copy of item 0 and store
  // nothing; no early return, so every group of a wave stays in step.
  const uint64_t it = live ? item : 0;
  const uint64_t sa = J.src_idx ? (uint64_t)J.src_idx[it] : it;   // input state
  const uint64_t ba = J.br_idx ? (uint64_t)J.br_idx[it] : it;     // branch choices
  const uint64_t srs = J.src_rs, sis = J.src_is, chb = J.chi_br;
  const uint8_t* __restrict__ branch = J.branch;
  const uint32_t n = J.dst.n;
  uint64_t F[RPL], G[RPL], M[RPL];
  uint32_t g[RPL];
  uint64_t v, s;
  uint32_t w, e;
  SubCH<LPT, RPL> c{F, G, M, g, v, s, w, e};
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
      const uint64_t off = (uint64_t)p * srs + sa * sis;
      c.F[j] = act ? J.src.F[off] : 0ull;
      c.G[j] = act ? J.src.G[off] : 0ull;
      c.M[j] = act ? J.src.M[off] : 0ull;
      c.g[j] = act ? J.src.gamma[off] : 0u;
    }
  }
  if (kFromZero) {
    c.v = 0ull;
    c.s = 0ull;
    c.w = 0u;
  } else {
    c.v = J.src.v[sa];
    c.s = J.src.s[sa];
    c.w = J.src.omega[sa];
  }
  c.err = 0u;
  // One flat gate list: slot gates are SLOT_SPOW (a per-term power of S) or
  // conditional gates of a general branch.  A gate is two 32-bit words read
  // on the scalar unit (wave-uniform); the term's branch choice for the next
  // slot occurrence is loaded one occurrence ahead.
  const uint2* __restrict__ g2 = reinterpret_cast<const uint2*>(gates);
  const uint32_t* __restrict__ seq = J.slot_seq;
  const uint32_t n_occ = J.n_occ;
  uint32_t next_b = n_occ ? (uint32_t)branch[(uint64_t)seq[0] * chb + ba] : 0u;
  uint32_t cur_b = 0u, occ = 1u;
  // The gate list goes through LDS in chunks (one barrier pair per chunk);
  // every wave reads gate i + 1 while it applies gate i.
  __shared__ uint2 sg[kGateChunk];
  for (uint32_t c0 = 0; c0 < n_gates; c0 += kGateChunk) {
    const uint32_t cn = min((uint32_t)kGateChunk, n_gates - c0);
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < cn; t += 256u) sg[t] = g2[c0 + t];
    __syncthreads();
    uint2 nxt = sg[0];
    for (uint32_t i = 0; i < cn; ++i) {
      const uint32_t w0 = uniform32(nxt.x), w1 = uniform32(nxt.y);
      nxt = sg[i + 1 < cn ? i + 1 : i];
      const uint32_t op = w0 & 0xffu, q = (w0 >> 8) & 0xffu, r = (w0 >> 16) & 0xffu;
      const uint32_t cond = (w1 >> 16) & 0xffu;
      if (cond & kSlotStart) {
        cur_b = next_b;
        if (occ < n_occ) next_b = (uint32_t)branch[(uint64_t)seq[occ] * chb + ba];
        ++occ;
      }
      uint32_t pw = 1u;
      if (op == OP_SLOT_SPOW) pw = ((w0 >> 16) >> (2u * cur_b)) & 3u;
      else if (op == OP_SPOW) pw = w0 >> 24;
      const bool on = !(cond & kCondApply) || ((w1 >> 24) >> cur_b & 1u);
      if (op == OP_H) {
        if (on) sw_h(c, L, q);
      } else {
        sw_left(c, L, op, q, op == OP_CX || op == OP_CZ ? r : q, pw, on);
      }
    }
  }
  if (live) {
    const uint64_t drs = J.dst_rs, dis = J.dst_is;
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      const uint32_t p = L.li + (uint32_t)j * LPT;
      if (p < n) {
        const uint64_t off = (uint64_t)p * drs + item * dis;
        J.dst.F[off] = c.F[j];
        J.dst.G[off] = c.G[j];
        J.dst.M[off] = c.M[j];
        J.dst.gamma[off] = (uint8_t)c.g[j];
      }
    }
    if (L.li == 0) {
      J.dst.v[item] = c.v;
      J.dst.s[item] = c.s;
      J.dst.omega[item] = (uint8_t)c.w;
      if (c.err) atomicOr(err, 1u);
    }
  }
}

template <int LPT, int RPL>
hipError_t launch_evolve_t(const EvolveJob& J, const DGate* gates, uint32_t n_gates, bool from_zero,
                           uint32_t* err, hipStream_t st) {
  constexpr int kTermsPerBlock = 256 / LPT;
  const uint32_t blocks = (uint32_t)((J.count + kTermsPerBlock - 1) / kTermsPerBlock);
  if (blocks == 0) return hipSuccess;
  if (from_zero)
    hipLaunchKernelGGL((k_evolve<LPT, RPL, true>), dim3(blocks), dim3(256), 0, st, J, gates, n_gates,
                       err);
  else
    hipLaunchKernelGGL((k_evolve<LPT, RPL, false>), dim3(blocks), dim3(256), 0, st, J, gates,
                       n_gates, err);
  return hipGetLastError();
}

}  // namespace chsim
