// CH-form evolution with the tableau rows resident in LDS (step (a) of the
// hot path; the same gates and rules as evolve_kernel.hpp, another mapping).
//
// A term is a group of LPT lanes (T = 64 / LPT terms per wave); lane
// li T + tw is lane li of term tw.  Each wave keeps the F, G, M rows of its
// terms in its own LDS region, laid out [matrix][row][term]: row p of one
// matrix for all terms of the wave is one contiguous run of T words, so when
// every lane touches its j-th row (p = li + j LPT) the wave reads or writes
// 512 contiguous bytes, lane by lane (no bank conflicts), and a left rule
// that reads row q of every term reads T contiguous words, each broadcast to
// the lanes of its term.  The left rules L[S], L[CZ], L[CX]
// read rows q and r at a computed LDS address and the lane that owns the row
// (lane p % LPT) writes it back, so no register is ever indexed by the gate.
// The Hadamard update (Eqs. (H1)-(H7), Prop. H) runs over the lane's rows
// p = li, li + LPT, ...: load, apply the batch of commuting right rules of
// V_C, store.  gamma stays in a register: bit j of one word is the low bit of
// gamma of row li + LPT j and bit 16 + j its high bit.
#include <type_traits>

#include "device_common.hpp"
#include "hrow.hpp"
#include "internal.hpp"

namespace chsim {
namespace {

constexpr uint32_t kLdsWaves = 4;    // waves per workgroup

// Value held by lane `src` of the caller's term (lane src T + tw).
template <uint32_t T>
__device__ __forceinline__ uint32_t grp32(uint32_t x, uint32_t src, uint32_t tw) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute((int)((src * T + tw) << 2), (int)x);
}

template <int LPT, bool kFromZero>
__global__ __launch_bounds__(256) void k_evolve_lds(EvolveJob J, const DGate* __restrict__ gates,
                                                    uint32_t n_gates, uint32_t* __restrict__ err) {
  constexpr uint32_t T = 64 / LPT;                // terms per wave
  constexpr uint32_t kTermsPerBlock = kLdsWaves * T;
  const uint64_t count = J.count_dev ? (uint64_t)*J.count_dev : J.count;
  if ((uint64_t)blockIdx.x * kTermsPerBlock >= count) return;  // whole block: no barrier skipped
  extern __shared__ __align__(16) uint64_t lds_words[];
  const uint32_t n = J.dst.n;
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t tw = lane % T, li = lane / T;
  // Row p of matrix m of this lane's term: region[(m n + p) T + tw].
  uint64_t* const RF = lds_words + (size_t)wave * 3u * n * T + tw;
  uint64_t* const RG = RF + (size_t)n * T;
  uint64_t* const RM = RG + (size_t)n * T;
  const uint32_t rpl = (n + LPT - 1) / LPT;
  const uint32_t nfull = n / LPT, ntail = n % LPT;
  // This lane's rows p = li + j LPT: word j * 64 from these.
  uint64_t* const LF = RF + (size_t)li * T;
  uint64_t* const LG = RG + (size_t)li * T;
  uint64_t* const LM = RM + (size_t)li * T;

  const uint64_t item = (uint64_t)blockIdx.x * kTermsPerBlock + wave * T + tw;
  const bool live = item < count;
  // Dead groups (ragged last block) evolve a copy of item 0 and store nothing.
  const uint64_t it = live ? item : 0;
  const uint64_t sa = J.src_idx ? (uint64_t)J.src_idx[it] : it;  // input state
  const uint64_t ba = J.br_idx ? (uint64_t)J.br_idx[it] : it;    // branch choices
  const uint64_t chb = J.chi_br;
  const uint8_t* __restrict__ branch = J.branch;

  uint32_t gw = 0u;
  for (uint32_t j = 0; j < rpl; ++j) {
    const uint32_t p = li + j * LPT;
    if (p >= n) break;
    uint64_t f, g, m;
    uint32_t ga;
    if (kFromZero) {
      f = 1ull << p;
      g = f;
      m = 0ull;
      ga = 0u;
    } else {
      const uint64_t off = (uint64_t)p * J.src_rs + sa * J.src_is;
      f = J.src.F[off];
      g = J.src.G[off];
      m = J.src.M[off];
      ga = J.src.gamma[off];
    }
    LF[j * 64u] = f;
    LG[j * 64u] = g;
    LM[j * 64u] = m;
    gw |= ((ga & 1u) << j) | (((ga >> 1) & 1u) << (16u + j));
  }
  const uint64_t v0 = kFromZero ? 0ull : J.src.v[sa], s0 = kFromZero ? 0ull : J.src.s[sa];
  uint32_t vl = (uint32_t)v0, vh = (uint32_t)(v0 >> 32), sl = (uint32_t)s0, sh = (uint32_t)(s0 >> 32);
  uint32_t w = kFromZero ? 0u : (uint32_t)J.src.omega[sa];
  uint32_t e = 0u;

  const uint2* __restrict__ g2 = reinterpret_cast<const uint2*>(gates);
  const uint32_t* __restrict__ seq = J.slot_seq;
  const uint32_t n_occ = J.n_occ;
  uint32_t next_b = n_occ ? (uint32_t)branch[(uint64_t)seq[0] * chb + ba] : 0u;
  uint32_t cur_b = 0u, occ = 1u;
  // Gates are two 32-bit words read on the scalar unit, the next one in
  // flight while the current one is applied (the device list has one
  // padding entry past its last gate, so the read past a span's end is in
  // bounds).
  uint2 nxt = n_gates ? g2[0] : make_uint2(0u, 0u);
  for (uint32_t i = 0; i < n_gates; ++i) {
    const uint32_t w0 = uniform32(nxt.x), w1 = uniform32(nxt.y);
    nxt = g2[i + 1];  // the device list holds one entry past its end
    const uint32_t op = w0 & 0xffu, q = (w0 >> 8) & 0xffu;
    const uint32_t cond = (w1 >> 16) & 0xffu;
    if (cond & kSlotStart) {
      cur_b = next_b;
      if (occ < n_occ) next_b = (uint32_t)branch[(uint64_t)seq[occ] * chb + ba];
      ++occ;
    }
    bool on = true;  // per lane: the term's branch choice decides a conditional gate
    if (cond & kCondApply) on = ((w1 >> 24) >> cur_b & 1u) != 0u;
    const uint32_t kq = q / LPT, lq = q % LPT;
    if (op == OP_H) {
      if (!on) continue;
      // Hadamard on qubit q (the gate's p): Eqs. (H2), (H4), the t = u case,
      // Prop. H with V_C applied to the lane's rows.  On 32-bit halves, and
      // branch-free over the two outcomes of (H4): a term with t = u gets
      // e_q = 0 and no R[S_q], which makes V_C the identity on its rows.
      const uint64_t Fp = RF[q * T], Gp = RG[q * T], Mp = RM[q * T];
      const uint32_t gp = gam_get(grp32<T>(gw, lq, tw), kq);
      const uint32_t Fl = (uint32_t)Fp, Fh = (uint32_t)(Fp >> 32), Gl = (uint32_t)Gp, Gh = (uint32_t)(Gp >> 32);
      const uint32_t Ml = (uint32_t)Mp, Mh = (uint32_t)(Mp >> 32);
      // t = s + G_q v, u = s + F_q ~v + M_q v: d = t + u is F_q on ~v (V_0)
      // and G_q + M_q on v (V_1).
      const uint32_t GMl = Gl ^ Ml, GMh = Gh ^ Mh;
      const uint32_t V0l = Fl & ~vl, V0h = Fh & ~vh, V1l = GMl & vl, V1h = GMh & vh;
      const uint32_t tl = sl ^ (Gl & vl), th = sh ^ (Gh & vh);
      // alpha = G_q ~v s; alpha + beta = (G_q + M_q) ~v s + F_q v (M_q + s)
      // (mod 2), each one population count of the halves' XOR.
      const uint32_t alpha = (uint32_t)__popc((Gl & ~vl & sl) ^ (Gh & ~vh & sh)) & 1u;
      const uint32_t ab = (uint32_t)__popc((GMl & ~vl & sl) ^ (GMh & ~vh & sh) ^ (Fl & vl & (Ml ^ sl)) ^
                                           (Fh & vh & (Mh ^ sh))) & 1u;
      const uint32_t delta = (gp + 2u * ab) & 3u;
      const uint32_t dl = V0l | V1l, dh = V0h | V1h;
      const bool same = (dl | dh) == 0u;  // t = u
      const bool use0 = (V0l | V0h) != 0u;
      const uint32_t Xl = use0 ? V0l : V1l, Xh = use0 ? V0h : V1h;
      // q = lowest bit of X (ffbl of zero is all ones, so a zero low half
      // defers to the high one; t = u leaves q = 31, masked below).
      const uint32_t qh = Xl ? (uint32_t)__builtin_ctz(Xl) : 32u + (uint32_t)__builtin_ctz(Xh | 0x80000000u);
      const uint32_t qs = qh & 31u;
      const bool hq = qh >= 32u;
      const uint32_t qm = same ? 0u : (1u << qs);  // e_q, zero when t = u
      const uint32_t qbl = hq ? 0u : qm, qbh = hq ? qm : 0u;
      const uint32_t Wl = Xl & ~qbl, Wh = Xh & ~qbh;
      const uint32_t tq = ((hq ? th : tl) >> qs) & 1u;
      const uint32_t vq = ((hq ? vh : vl) >> qs) & 1u;
      // H^{v_q}(|y_q> + i^delta |1 - y_q>) = 2^{1/2} e^{i pi dw/4} S^a H^b |c>; for
      // y_q = 1 factor out i^delta and use |0> + i^{-delta} |1>.
      const uint32_t dp = tq ? ((4u - delta) & 3u) : delta;
      const uint32_t ph = (2u * delta * tq) & 7u;
      uint32_t a, b, cc, dw;
      if (!vq) {
        b = 1u;
        a = dp & 1u;
        cc = dp >> 1;
        dw = ph;
      } else {
        b = dp & 1u;
        a = dp & 1u;
        cc = (dp == 2u || dp == 1u) ? 1u : 0u;
        dw = ph + (dp == 1u ? 1u : (dp == 3u ? 7u : 0u));
      }
      if (same) {
        // omega' = 2^{-1/2} (-1)^alpha (1 + i^delta), delta odd; s' = t.
        if (!(delta & 1u)) e = 1u;
        a = 0u;
        dw = delta == 1u ? 1u : 7u;
      }
      // V_C on the lane's rows (hrow.hpp); gamma's changes are collected as
      // bit j of gam2 (+2) and fbits (-1) and applied after the loop.
      const HRowMasks K = h_row_masks32(Wl, Wh, V1l, V1h, qbl, qbh, qs, hq, use0, a);
      // When no term of the wave in the V_0 case has W != 0 (|v| close to n
      // leaves V_0 with at most one bit), the W terms of that case vanish for
      // every term (wave-uniform test).
      const bool w_empty = __ballot(use0 && (Wl | Wh) != 0u) == 0ull;
      uint32_t gam2 = 0u, fbits = 0u;
      auto row = [&](uint32_t j, auto general) {
        const uint64_t F = LF[j * 64u], G = LG[j * 64u], M = LM[j * 64u];
        uint32_t Fl = (uint32_t)F, Fh = (uint32_t)(F >> 32);
        uint32_t Gl = (uint32_t)G, Gh = (uint32_t)(G >> 32);
        uint32_t Ml = (uint32_t)M, Mh = (uint32_t)(M >> 32);
        uint32_t g2, f1;
        h_row<decltype(general)::value>(K, Fl, Fh, Gl, Gh, Ml, Mh, g2, f1);
        const uint32_t bj = 1u << j;
        gam2 = bop3<kAndOr>(g2, bj, gam2);
        fbits = bop3<kAndOr>(f1, bj, fbits);
        LF[j * 64u] = ((uint64_t)Fh << 32) | Fl;
        LG[j * 64u] = ((uint64_t)Gh << 32) | Gl;
        LM[j * 64u] = ((uint64_t)Mh << 32) | Ml;
      };
      // Rows j < n / LPT exist in every lane (no per-lane bound in the loop);
      // row n / LPT only in lanes li < n % LPT.
      if (__ballot(!same) == 0ull) {
        // t = u for every term of the wave: no row changes.
      } else if (w_empty) {
#pragma unroll 2
        for (uint32_t j = 0; j < nfull; ++j) row(j, std::false_type{});
        if (li < ntail) row(nfull, std::false_type{});
      } else {
#pragma unroll 2
        for (uint32_t j = 0; j < nfull; ++j) row(j, std::true_type{});
        if (li < ntail) row(nfull, std::true_type{});
      }
      gw = gam_apply(gw, gam2, fbits);
      // s' = y with bit q set to c, where y = t, or u + e_q when t_q = 1 (so
      // y agrees with t + t_q d off bit q); v' = v with bit q set to b.
      const uint32_t tqm = tq ? ~0u : 0u, ccm = cc ? ~0u : 0u, bm = b ? ~0u : 0u;
      sl = ((tl ^ (tqm & dl)) & ~qbl) | (ccm & qbl);
      sh = ((th ^ (tqm & dh)) & ~qbh) | (ccm & qbh);
      vl = (vl & ~qbl) | (bm & qbl);
      vh = (vh & ~qbh) | (bm & qbh);
      w = (w + 4u * alpha + dw) & 7u;
      continue;
    }
    const bool wq = on && li == lq;
    if (op == OP_CX || op == OP_CZ) {
      const uint32_t r = (w0 >> 16) & 0xffu;
      const uint32_t kr = r / LPT, lr = r % LPT;
      const bool wr = on && li == lr;
      if (op == OP_CX) {
        // gamma_q += gamma_r + 2 (M_q . F_r); G_r ^= G_q; F_q ^= F_r; M_q ^= M_r.
        const uint32_t gr = gam_get(grp32<T>(gw, lr, tw), kr);
        if (wq) {
          const uint64_t Fr = RF[r * T], Mr = RM[r * T];
          const uint64_t Fq = RF[q * T], Mq = RM[q * T];
          RF[q * T] = Fq ^ Fr;
          RM[q * T] = Mq ^ Mr;
          gw = gam_add(gw, kq, gr + 2u * par64(Mq & Fr));
        }
        if (wr) RG[r * T] ^= RG[q * T];
      } else {
        // M_q ^= G_r, M_r ^= G_q.
        if (wq) RM[q * T] ^= RG[r * T];
        if (wr) RM[r * T] ^= RG[q * T];
      }
    } else if (wq) {
      // S^pw on q: M_q ^= G_q pw times, gamma_q -= pw.
      uint32_t pw = 1u;
      if (op == OP_SLOT_SPOW) pw = ((w0 >> 16) >> (2u * cur_b)) & 3u;
      else if (op == OP_SPOW) pw = w0 >> 24;
      if (pw & 1u) RM[q * T] ^= RG[q * T];
      gw = gam_add(gw, kq, (4u - pw) & 3u);
    }
  }
  if (live) {
    const uint64_t drs = J.dst_rs, dis = J.dst_is;
    for (uint32_t j = 0; j < rpl; ++j) {
      const uint32_t p = li + j * LPT;
      if (p >= n) break;
      const uint64_t off = (uint64_t)p * drs + item * dis;
      J.dst.F[off] = LF[j * 64u];
      J.dst.G[off] = LG[j * 64u];
      J.dst.M[off] = LM[j * 64u];
      J.dst.gamma[off] = (uint8_t)gam_get(gw, j);
    }
    if (li == 0) {
      J.dst.v[item] = ((uint64_t)vh << 32) | vl;
      J.dst.s[item] = ((uint64_t)sh << 32) | sl;
      J.dst.omega[item] = (uint8_t)w;
      if (e) atomicOr(err, 1u);
    }
  }
}

template <int LPT>
hipError_t launch_lds_t(const EvolveJob& J, const DGate* gates, uint32_t n_gates, bool from_zero,
                        uint32_t* err, hipStream_t st) {
  constexpr uint32_t T = 64 / LPT;
  constexpr uint32_t kTermsPerBlock = kLdsWaves * T;
  const uint32_t blocks = (uint32_t)((J.count + kTermsPerBlock - 1) / kTermsPerBlock);
  if (blocks == 0) return hipSuccess;
  const size_t smem = (size_t)kLdsWaves * 3u * J.dst.n * T * sizeof(uint64_t);
  static bool attr_set[2] = {false, false};
  const void* fn = from_zero ? reinterpret_cast<const void*>(&k_evolve_lds<LPT, true>)
                             : reinterpret_cast<const void*>(&k_evolve_lds<LPT, false>);
  if (smem > 65536 && !attr_set[from_zero]) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set[from_zero] = true;
  }
  if (from_zero)
    hipLaunchKernelGGL((k_evolve_lds<LPT, true>), dim3(blocks), dim3(256), smem, st, J, gates, n_gates, err);
  else
    hipLaunchKernelGGL((k_evolve_lds<LPT, false>), dim3(blocks), dim3(256), smem, st, J, gates, n_gates, err);
  return hipGetLastError();
}

}  // namespace

uint64_t evolve_lds_capacity(int lanes, uint32_t n) {
  int dev = 0, cus = 0;
  hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  const uint64_t T = 64u / (uint32_t)lanes;
  const uint64_t wg_bytes = (uint64_t)kLdsWaves * 3u * n * T * sizeof(uint64_t);
  const uint64_t per_cu = wg_bytes ? (160u * 1024u) / wg_bytes : 0u;
  return per_cu * kLdsWaves * T * (uint64_t)cus;
}

hipError_t launch_evolve_lds(int lanes, const EvolveJob& J, const DGate* gates, uint32_t n_gates,
                             bool from_zero, uint32_t* err, hipStream_t st) {
  switch (lanes) {
    case 4: return launch_lds_t<4>(J, gates, n_gates, from_zero, err, st);
    case 8: return launch_lds_t<8>(J, gates, n_gates, from_zero, err, st);
    case 16: return launch_lds_t<16>(J, gates, n_gates, from_zero, err, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace chsim
