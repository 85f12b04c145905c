// One tableau row under the batch of right rules V_C that the Hadamard update
// applies (Prop. H), shared by the evolution kernels that keep rows in LDS
// and in registers.
//
// With d = t + u, V_0 = d & ~v, V_1 = d & v and q the lowest bit of V_0 if
// V_0 != 0, else of V_1 (W = the rest of that set), V_C is, per row p:
//   V_1 case, R[CX_{i,q}] for i in W:  G ^= W G_pq; F ^= e_q par(F & W); M ^= W M_pq.
//   V_0 case, R[CX_{q,i}] for i in W, then R[CZ_{q,i}] for i in V_1:
//     G ^= e_q par(G & W); F ^= W F_pq; M ^= e_q par((F & V_1) + (M & W)) + V_1 F_pq;
//     gamma_p += 2 F_pq par(F & V_1)   (W and V_1 are disjoint, so F & V_1 is
//     the same before and after F's update).
//   Then R[S_q] if a: M ^= e_q F'_pq, gamma_p -= F'_pq, with F'_pq = F_pq
//   plus, in the V_1 case, par(F & W).
// One branch-free update serves both cases with per-term masks (a wave's
// terms usually take both): P1 = par(F & X1) with X1 = W (V_1 case) or V_1
// (V_0 case) is the parity of either case, and M's two column terms merge into
// X1 times bit q of F (V_0 case) or of M (V_1 case).  Rows are 32-bit halves;
// a mask is all ones or zero (a sign-extending one-bit field extract).
#pragma once

#include "device_common.hpp"

namespace chsim {

// All ones if bit b (< 32) of x is set, else zero.
__device__ __forceinline__ uint32_t bit_mask(uint32_t x, uint32_t b) {
  return (uint32_t)__builtin_amdgcn_sbfe((int)x, b, 1u);
}

// Three-input bitwise operations by truth table (operands A, B, C; the table
// is the function's value on A = 0xF0, B = 0xCC, C = 0xAA).  On gfx950 these
// issue at twice the rate of selects, bit-field extracts and and-or, which
// the compiler would otherwise pick for masks derived from booleans.
enum : uint32_t {
  kSel = 0xCA,     // A ? B : C (bitwise)
  kAndXor = 0x6A,  // (A & B) ^ C
  kAnd3 = 0x80,    // A & B & C
  kAndOr = 0xEA,   // (A & B) | C
  kNandXor = 0xA6  // (~A & B) ^ C
};
template <uint32_t TT>
__device__ __forceinline__ uint32_t bop3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
}

// A lane's gamma values (Z_4) packed in one word: bit j is the low bit of
// the lane's j-th row, bit 16 + j its high bit (at most 16 rows per lane).
__device__ __forceinline__ uint32_t gam_get(uint32_t gw, uint32_t j) {
  return ((gw >> j) & 1u) | (((gw >> (16u + j)) & 1u) << 1);
}
// gamma_j += a (mod 4).
__device__ __forceinline__ uint32_t gam_add(uint32_t gw, uint32_t j, uint32_t a) {
  const uint32_t lo = (gw >> j) & 1u, a0 = a & 1u, a1 = (a >> 1) & 1u;
  return gw ^ (a0 << j) ^ ((a1 ^ (lo & a0)) << (16u + j));
}
// gamma += 2 on the rows in g2, then -= 1 on the rows in f1 (bit j = row j):
// the low bit flips, the high bit borrows.
__device__ __forceinline__ uint32_t gam_apply(uint32_t gw, uint32_t g2, uint32_t f1) {
  gw ^= g2 << 16;
  return gw ^ f1 ^ ((f1 & ~gw) << 16);
}

// The per-term constants of V_C.
struct HRowMasks {
  uint32_t X1l, X1h;    // W (V_1 case) or V_1 (V_0 case)
  uint32_t W1l, W1h;    // W in the V_1 case, else 0
  uint32_t W0l, W0h;    // W in the V_0 case, else 0
  uint32_t qb0l, qb0h;  // e_q in the V_0 case, else 0
  uint32_t qb1l, qb1h;  // e_q in the V_1 case, else 0
  uint32_t qbl, qbh;    // e_q
  uint32_t qs;          // q mod 32
  uint32_t u0;          // all ones in the V_0 case
  uint32_t am;          // all ones if R[S_q] follows
  uint32_t hqm;         // all ones if q >= 32
};

__device__ __forceinline__ HRowMasks h_row_masks(uint64_t W, uint64_t V1, uint32_t q, bool use0, uint32_t a) {
  HRowMasks k;
  const uint64_t u1m = use0 ? 0ull : ~0ull, u0m = ~u1m, qb = 1ull << q;
  const uint64_t X1 = use0 ? V1 : W, W1 = W & u1m, W0 = W & u0m, qb0 = qb & u0m, qb1 = qb & u1m;
  k.X1l = (uint32_t)X1;
  k.X1h = (uint32_t)(X1 >> 32);
  k.W1l = (uint32_t)W1;
  k.W1h = (uint32_t)(W1 >> 32);
  k.W0l = (uint32_t)W0;
  k.W0h = (uint32_t)(W0 >> 32);
  k.qb0l = (uint32_t)qb0;
  k.qb0h = (uint32_t)(qb0 >> 32);
  k.qb1l = (uint32_t)qb1;
  k.qb1h = (uint32_t)(qb1 >> 32);
  k.qbl = (uint32_t)qb;
  k.qbh = (uint32_t)(qb >> 32);
  k.qs = q & 31u;
  k.hqm = q >= 32u ? ~0u : 0u;
  k.u0 = use0 ? ~0u : 0u;
  k.am = a ? ~0u : 0u;
  return k;
}

// The same from 32-bit halves: W and V_1, e_q (zero for a term that takes
// no V_C) and its position (qs, hq).
__device__ __forceinline__ HRowMasks h_row_masks32(uint32_t Wl, uint32_t Wh, uint32_t V1l, uint32_t V1h,
                                                   uint32_t qbl, uint32_t qbh, uint32_t qs, bool hq, bool use0,
                                                   uint32_t a) {
  HRowMasks k;
  const uint32_t u0 = use0 ? ~0u : 0u, u1 = ~u0;
  k.X1l = use0 ? V1l : Wl;
  k.X1h = use0 ? V1h : Wh;
  k.W1l = Wl & u1;
  k.W1h = Wh & u1;
  k.W0l = Wl & u0;
  k.W0h = Wh & u0;
  k.qb0l = qbl & u0;
  k.qb0h = qbh & u0;
  k.qb1l = qbl & u1;
  k.qb1h = qbh & u1;
  k.qbl = qbl;
  k.qbh = qbh;
  k.qs = qs;
  k.hqm = hq ? ~0u : 0u;
  k.u0 = u0;
  k.am = a ? ~0u : 0u;
  return k;
}

// Updates one row in place.  g2: all ones if gamma_p gains 2; f1: all ones if
// gamma_p loses 1 (R[S_q]).  kGeneral = false drops the terms in W of the
// V_0 case (valid when W is empty for every V_0-case term of the wave).
template <bool kGeneral>
__device__ __forceinline__ void h_row(const HRowMasks& k, uint32_t& Fl, uint32_t& Fh, uint32_t& Gl, uint32_t& Gh,
                                      uint32_t& Ml, uint32_t& Mh, uint32_t& g2, uint32_t& f1) {
  // The halves holding bit q, then bit q of F, of G, and of F (V_0) or M (V_1).
  const uint32_t fx = bop3<kSel>(k.hqm, Fh, Fl), gx = bop3<kSel>(k.hqm, Gh, Gl), mx = bop3<kSel>(k.hqm, Mh, Ml);
  const uint32_t fqm = bit_mask(fx, k.qs);
  const uint32_t gqm = bit_mask(gx, k.qs);
  const uint32_t sel = bit_mask(bop3<kSel>(k.u0, fx, mx), k.qs);
  // par(a) + par(b) = par(a ^ b): one population count per parity.
  const uint32_t fx1 = bop3<kAndXor>(Fl, k.X1l, Fh & k.X1h);
  const uint32_t p1 = bit_mask(__popc(fx1), 0u);
  uint32_t pm = p1;
  if constexpr (kGeneral) {
    const uint32_t pg = bit_mask(__popc(bop3<kAndXor>(Gl, k.W0l, Gh & k.W0h)), 0u);
    pm = bit_mask(__popc(fx1 ^ bop3<kAndXor>(Ml, k.W0l, Mh & k.W0h)), 0u);
    Fl = bop3<kAndXor>(k.W0l, fqm, Fl);
    Fh = bop3<kAndXor>(k.W0h, fqm, Fh);
    Gl = bop3<kAndXor>(k.qb0l, pg, Gl);
    Gh = bop3<kAndXor>(k.qb0h, pg, Gh);
  }
  Gl = bop3<kAndXor>(k.W1l, gqm, Gl);
  Gh = bop3<kAndXor>(k.W1h, gqm, Gh);
  Fl = bop3<kAndXor>(k.qb1l, p1, Fl);
  Fh = bop3<kAndXor>(k.qb1h, p1, Fh);
  const uint32_t fq2 = bop3<kNandXor>(k.u0, p1, fqm);  // F_pq after V_C
  f1 = k.am & fq2;
  const uint32_t z = bop3<kAndXor>(k.u0, pm, f1);  // bit q of M flips
  Ml = bop3<kAndXor>(k.qbl, z, bop3<kAndXor>(k.X1l, sel, Ml));
  Mh = bop3<kAndXor>(k.qbh, z, bop3<kAndXor>(k.X1h, sel, Mh));
  g2 = bop3<kAnd3>(k.u0, fqm, p1);
}

}  // namespace chsim
