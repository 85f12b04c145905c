// CH-form evolution with one term per wave and one tableau row per lane
// (step (a) of the hot path; the same gates and rules as evolve_kernel.hpp).
//
// Lane p holds row p (F_p, G_p, M_p, gamma_p; zero for p >= n).  A left rule
// reads rows q and r with v_readlane into scalar registers and the lanes
// p = q, r update their own row; the Hadamard update (Eqs. (H1)-(H7),
// Prop. H) takes row q the same way, computes t, u, alpha, beta and the case
// of Prop. H on the scalar unit (v, s, omega live there), and every lane
// applies the batch of commuting right rules of V_C to its row.  With one
// term per wave every branch is uniform, so a gate costs only its own
// instructions: this mapping serves spans with few items, where the time is
// the latency of one wave's gate chain.
#include "device_common.hpp"
#include "internal.hpp"

namespace chsim {
namespace {

constexpr uint32_t kW64Chunk = 2048;  // gates staged in LDS at a time (16 KiB)

// All ones if bit b (< 32) of x is set, else zero.
__device__ __forceinline__ uint32_t bmask(uint32_t x, uint32_t b) {
  return (uint32_t)__builtin_amdgcn_sbfe((int)x, b, 1u);
}

// CH form of (-1)^alpha 2^{-1/2} U_C U_H (|t> + i^delta |u>) for t != u, one
// tableau row per lane (Prop. H and its proof): V_C's batches of right rules
// applied to the lane's row, then the single-qubit part W_C = V_C S_q^a,
// W_H = U_H H_q^{b xor v_q}, s' and omega'.  t, u, alpha, delta, v, s, w are
// wave-uniform.
__device__ __forceinline__ void superpose_w64(uint64_t& F, uint64_t& G, uint64_t& M, uint32_t& g, uint64_t& v,
                                              uint64_t& s, uint32_t& w, uint64_t t, uint64_t u, uint32_t alpha,
                                              uint32_t delta) {
  const uint64_t nv = ~v;
  const uint64_t d = t ^ u, V0 = d & nv, V1 = d & v;
  const bool use0 = V0 != 0ull;
  const uint32_t qh = (uint32_t)__builtin_ctzll(use0 ? V0 : V1);
  const uint64_t qb = 1ull << qh;
  const uint64_t W = (use0 ? V0 : V1) & ~qb;
  // The lane's row as 32-bit halves; qs, hq locate bit qh.
  const uint32_t qs = qh & 31u;
  const bool hq = qh >= 32u;
  const uint32_t qbl = (uint32_t)qb, qbh = (uint32_t)(qb >> 32);
  const uint32_t Wl = (uint32_t)W, Wh = (uint32_t)(W >> 32);
  uint32_t Fl = (uint32_t)F, Fh = (uint32_t)(F >> 32);
  uint32_t Gl = (uint32_t)G, Gh = (uint32_t)(G >> 32);
  uint32_t Ml = (uint32_t)M, Mh = (uint32_t)(M >> 32);
  if (use0 && W == 0ull) {
    // W empty (V_0 = {q}): only R[CZ_{q,i}], i in V_1.
    const uint32_t V1l = (uint32_t)V1, V1h = (uint32_t)(V1 >> 32);
    const uint32_t mf = bmask(hq ? Fh : Fl, qs);
    const uint32_t c = (uint32_t)__popc(Fl & V1l) + (uint32_t)__popc(Fh & V1h);
    const uint32_t mm = bmask(c, 0u);
    Ml ^= (qbl & mm) ^ (V1l & mf);
    Mh ^= (qbh & mm) ^ (V1h & mf);
    g = (g + 2u * (mf & c & 1u)) & 3u;
  } else if (use0) {
    // R[CX_{q,i}], i in W: G_{.,q} ^= G_{.,i}; F_{.,i} ^= F_{.,q}; M_{.,q} ^= M_{.,i}.
    // R[CZ_{q,i}], i in V_1: M_{.,q} ^= F_{.,i}; M_{.,i} ^= F_{.,q}; gamma += 2 F_{.,q} F_{.,i}.
    const uint32_t V1l = (uint32_t)V1, V1h = (uint32_t)(V1 >> 32);
    const uint32_t mf = bmask(hq ? Fh : Fl, qs);
    const uint32_t mg = bmask((uint32_t)__popc(Gl & Wl) + (uint32_t)__popc(Gh & Wh), 0u);
    Gl ^= qbl & mg;
    Gh ^= qbh & mg;
    Fl ^= Wl & mf;
    Fh ^= Wh & mf;
    const uint32_t c = (uint32_t)__popc(Fl & V1l) + (uint32_t)__popc(Fh & V1h);
    const uint32_t mm = bmask(c + (uint32_t)__popc(Ml & Wl) + (uint32_t)__popc(Mh & Wh), 0u);
    Ml ^= (qbl & mm) ^ (V1l & mf);
    Mh ^= (qbh & mm) ^ (V1h & mf);
    g = (g + 2u * (mf & c & 1u)) & 3u;
  } else {
    // R[CX_{i,q}], i in W: G_{.,i} ^= G_{.,q}; F_{.,q} ^= F_{.,i}; M_{.,i} ^= M_{.,q}.
    const uint32_t mg = bmask(hq ? Gh : Gl, qs), mm = bmask(hq ? Mh : Ml, qs);
    const uint32_t mf = bmask((uint32_t)__popc(Fl & Wl) + (uint32_t)__popc(Fh & Wh), 0u);
    Gl ^= Wl & mg;
    Gh ^= Wh & mg;
    Fl ^= qbl & mf;
    Fh ^= qbh & mf;
    Ml ^= Wl & mm;
    Mh ^= Wh & mm;
  }
  const uint32_t tq = (uint32_t)((t >> qh) & 1ull);
  const uint64_t y = tq ? (u ^ qb) : t;  // y and z differ only in bit qh; y_qh = t_qh
  const uint32_t vq = (uint32_t)((v >> qh) & 1ull);
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
  if (a) {
    // R[S_q]: M_{.,q} ^= F_{.,q}; gamma -= F_{.,q}.
    const uint32_t fb = ((hq ? Fh : Fl) >> qs) & 1u;
    const uint32_t mfb = 0u - fb;
    Ml ^= qbl & mfb;
    Mh ^= qbh & mfb;
    g = (g - fb) & 3u;
  }
  F = ((uint64_t)Fh << 32) | Fl;
  G = ((uint64_t)Gh << 32) | Gl;
  M = ((uint64_t)Mh << 32) | Ml;
  s = (y & ~qb) | ((uint64_t)cc << qh);
  v = (v & ~qb) | ((uint64_t)b << qh);
  w = (w + 4u * alpha + dw) & 7u;
}

template <bool kFromZero>
__global__ __launch_bounds__(256) void k_evolve_w64(EvolveJob J, const DGate* __restrict__ gates,
                                                    uint32_t n_gates, uint32_t* __restrict__ err) {
  const uint64_t count = J.count_dev ? (uint64_t)*J.count_dev : J.count;
  if ((uint64_t)blockIdx.x * 4u >= count) return;  // whole block: no barrier skipped
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = uniform32(threadIdx.x >> 6);
  const uint64_t item = (uint64_t)blockIdx.x * 4u + wave;
  const bool live = item < count;
  // A dead wave (ragged last block) evolves a copy of item 0 and stores nothing.
  const uint64_t it = live ? item : 0;
  const uint64_t sa = uniform64(J.src_idx ? (uint64_t)J.src_idx[it] : it);  // input state
  const uint64_t ba = uniform64(J.br_idx ? (uint64_t)J.br_idx[it] : it);    // branch choices
  const uint64_t chb = J.chi_br;
  const uint8_t* __restrict__ branch = J.branch;
  const uint32_t n = J.dst.n;
  const bool act = lane < n;
  uint64_t F, G, M;
  uint32_t g;
  uint64_t v, s;
  uint32_t w;
  if (kFromZero) {
    F = act ? (1ull << lane) : 0ull;
    G = F;
    M = 0ull;
    g = 0u;
    v = 0ull;
    s = 0ull;
    w = 0u;
  } else {
    const uint64_t off = (uint64_t)lane * J.src_rs + sa * J.src_is;
    F = act ? J.src.F[off] : 0ull;
    G = act ? J.src.G[off] : 0ull;
    M = act ? J.src.M[off] : 0ull;
    g = act ? (uint32_t)J.src.gamma[off] : 0u;
    v = uniform64(J.src.v[sa]);
    s = uniform64(J.src.s[sa]);
    w = uniform32(J.src.omega[sa]);
  }
  uint32_t e = 0u;
  const uint32_t* __restrict__ seq = J.slot_seq;
  const uint32_t n_occ = J.n_occ;
  uint32_t next_b = n_occ ? uniform32(branch[(uint64_t)seq[0] * chb + ba]) : 0u;
  uint32_t cur_b = 0u, occ = 1u;
  const uint2* __restrict__ g2 = reinterpret_cast<const uint2*>(gates);
  __shared__ uint2 sg[kW64Chunk + 1];  // one entry past the chunk, so the next gate is always read in bounds
  for (uint32_t c0 = 0; c0 < n_gates; c0 += kW64Chunk) {
    const uint32_t cn = min(kW64Chunk, n_gates - c0);
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < cn; t += 256u) sg[t] = g2[c0 + t];
    if (threadIdx.x == 0) sg[cn] = make_uint2(0u, 0u);
    __syncthreads();
    uint2 nxt = sg[0];
    for (uint32_t i = 0; i < cn; ++i) {
      const uint32_t w0 = uniform32(nxt.x), w1 = uniform32(nxt.y);
      nxt = sg[i + 1];
      const uint32_t op = w0 & 0xffu, q = (w0 >> 8) & 0xffu, r = (w0 >> 16) & 0xffu;
      const uint32_t cond = (w1 >> 16) & 0xffu;
      if (cond) {  // a slot's first gate, or a gate of some branches only (uniform here)
        if (cond & kSlotStart) {
          cur_b = next_b;
          if (occ < n_occ) next_b = uniform32(branch[(uint64_t)seq[occ] * chb + ba]);
          ++occ;
        }
        if ((cond & kCondApply) && !(((w1 >> 24) >> cur_b) & 1u)) continue;
      }
      switch (op) {
        case OP_CZ: {
          // M_q ^= G_r, M_r ^= G_q.
          const uint64_t Gq = rl64(G, q), Gr = rl64(G, r);
          if (lane == q) M ^= Gr;
          if (lane == r) M ^= Gq;
          break;
        }
        case OP_CX: {
          // gamma_q += gamma_r + 2 (M_q . F_r) (M_q before the update);
          // G_r ^= G_q; F_q ^= F_r; M_q ^= M_r.
          const uint64_t Fr = rl64(F, r), Mr = rl64(M, r), Gq = rl64(G, q), Mq = rl64(M, q);
          const uint32_t gr = rl32(g, r);
          if (lane == q) {
            g = (g + gr + 2u * par64(Mq & Fr)) & 3u;
            F ^= Fr;
            M ^= Mr;
          }
          if (lane == r) G ^= Gq;
          break;
        }
        case OP_H: {
          // Hadamard on qubit q: Eqs. (H2), (H4), the t = u case, Prop. H.
          const uint64_t Fp = rl64(F, q), Gp = rl64(G, q), Mp = rl64(M, q);
          const uint32_t gp = rl32(g, q);
          const uint64_t nv = ~v;
          const uint64_t t = s ^ (Gp & v);
          const uint64_t u = s ^ (Fp & nv) ^ (Mp & v);
          const uint32_t alpha = par64(Gp & nv & s);
          const uint32_t beta = par64(Mp & nv & s) ^ par64(Fp & v & (Mp ^ s));
          const uint32_t delta = (gp + 2u * (alpha + beta)) & 3u;
          if (t == u) {
            // omega' = 2^{-1/2} (-1)^alpha (1 + i^delta), delta odd.
            if (!(delta & 1u)) e = 1u;
            w = (w + 4u * alpha + (delta == 1u ? 1u : 7u)) & 7u;
            s = t;
            break;
          }
          superpose_w64(F, G, M, g, v, s, w, t, u, alpha, delta);
          break;
        }
        default: {
          // S^pw on q: M_q ^= G_q pw times, gamma_q -= pw.
          const uint32_t pw = op == OP_SLOT_SPOW ? ((w0 >> 16) >> (2u * cur_b)) & 3u : op == OP_SPOW ? (w0 >> 24) : 1u;
          if (lane == q) {
            if (pw & 1u) M ^= G;
            g = (g - pw) & 3u;
          }
          break;
        }
      }
    }
  }
  if (live) {
    if (act) {
      const uint64_t off = (uint64_t)lane * J.dst_rs + item * J.dst_is;
      J.dst.F[off] = F;
      J.dst.G[off] = G;
      J.dst.M[off] = M;
      J.dst.gamma[off] = (uint8_t)g;
    }
    if (lane == 0) {
      J.dst.v[item] = v;
      J.dst.s[item] = s;
      J.dst.omega[item] = (uint8_t)w;
      if (e) atomicOr(err, 1u);
    }
  }
}

// Projective gates prod_j (I + P_j) / 2 on every term of the store (end of Sec.
// "Phase-sensitive Clifford simulator"), P_j = i^a X(x) Z(z) Hermitian, one
// term per wave, lane p holding row p.  By Eq. (tableaux)
//   U_C^{-1} P U_C = i^a prod_{p in x} i^{gamma_p} X(F_p) Z(M_p) prod_{p in z} Z(G_p),
// accumulated on the scalar unit as i^c X(u) Z(w) over the set bits of x
// (rows by readlane; X(u) Z(w) X(f) Z(m) = (-1)^{w.f} X(u ^ f) Z(w ^ m)).
// Conjugation by U_H = H(v) swaps X and Z on the qubits in v (with a sign
// (-1)^{u_j w_j} each), so Q = U_H^{-1} U_C^{-1} P U_C U_H acts on |s> as
// (I + Q)|s> = |s> + i^delta |t>, t = s ^ u', u' = (u & ~v) | (w & v),
// delta = c + 2 par(u & w & v) + 2 par(w' & s), w' = (w & ~v) | (u & v).
// t = s: the term stays (delta = 0) or is projected to zero (delta = 2);
// otherwise Prop. H gives the CH form of 2^{-1/2} U_C U_H (|s> + i^delta |t>)
// and b is scaled by 2^{-1/2}.  A term with b = 0 is left as it is.  An odd
// delta with t = s (P not Hermitian) sets the error flag.
__global__ __launch_bounds__(256) void k_project_w64(TermsView T, ProjGates P, uint32_t* __restrict__ err) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t item = (uint64_t)blockIdx.x * 4u + uniform32(threadIdx.x >> 6);
  if (item >= T.chi) return;  // whole waves; the kernel has no barrier
  const uint32_t n = T.n;
  const bool act = lane < n;
  const uint64_t off = (uint64_t)lane * T.chi + item;
  uint64_t F = act ? T.F[off] : 0ull, G = act ? T.G[off] : 0ull, M = act ? T.M[off] : 0ull;
  uint32_t g = act ? (uint32_t)T.gamma[off] : 0u;
  uint64_t v = uniform64(T.v[item]), s = uniform64(T.s[item]);
  uint32_t w = uniform32(T.omega[item]);
  double2 b = T.b[item];
  bool zero = b.x == 0.0 && b.y == 0.0;
  bool changed = false;
  for (uint32_t j = 0; j < P.count && !zero; ++j) {
    uint32_t c = P.a[j];
    uint64_t xu = 0ull, zw = 0ull;
    for (uint64_t xm = P.x[j]; xm; xm &= xm - 1ull) {
      const uint32_t p = (uint32_t)__builtin_ctzll(xm);
      const uint64_t Fp = rl64(F, p);
      c += rl32(g, p) + 2u * par64(zw & Fp);
      xu ^= Fp;
      zw ^= rl64(M, p);
    }
    for (uint64_t zm = P.z[j]; zm; zm &= zm - 1ull) zw ^= rl64(G, (uint32_t)__builtin_ctzll(zm));
    const uint64_t up = (xu & ~v) | (zw & v), wp = (zw & ~v) | (xu & v);
    const uint32_t delta = (c + 2u * par64(xu & zw & v) + 2u * par64(wp & s)) & 3u;
    if (up == 0ull) {
      if (delta & 1u) {
        if (lane == 0) atomicOr(err, 1u);
        break;
      }
      zero = delta == 2u;
      continue;
    }
    superpose_w64(F, G, M, g, v, s, w, s, s ^ up, 0u, delta);
    b.x *= 0.70710678118654752440;
    b.y *= 0.70710678118654752440;
    changed = true;
  }
  if (changed) {
    if (act) {
      T.F[off] = F;
      T.G[off] = G;
      T.M[off] = M;
      T.gamma[off] = (uint8_t)g;
    }
    if (lane == 0) {
      T.v[item] = v;
      T.s[item] = s;
      T.omega[item] = (uint8_t)w;
    }
  }
  if (lane == 0) T.b[item] = zero ? make_double2(0.0, 0.0) : b;
}

}  // namespace

hipError_t launch_evolve_w64(const EvolveJob& J, const DGate* gates, uint32_t n_gates, bool from_zero,
                             uint32_t* err, hipStream_t st) {
  const uint32_t blocks = (uint32_t)((J.count + 3) / 4);
  if (blocks == 0) return hipSuccess;
  if (from_zero)
    hipLaunchKernelGGL(k_evolve_w64<true>, dim3(blocks), dim3(256), 0, st, J, gates, n_gates, err);
  else
    hipLaunchKernelGGL(k_evolve_w64<false>, dim3(blocks), dim3(256), 0, st, J, gates, n_gates, err);
  return hipGetLastError();
}

hipError_t launch_project(const TermsView& T, const ProjGates& P, uint32_t* err, hipStream_t st) {
  const uint64_t blocks = (T.chi + 3) / 4;
  if (blocks == 0 || P.count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_project_w64, dim3((uint32_t)blocks), dim3(256), 0, st, T, P, err);
  return hipGetLastError();
}

}  // namespace chsim
