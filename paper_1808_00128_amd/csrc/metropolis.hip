// Metropolis chain over n-bit outputs (Sec. "Heuristic Metropolis simulator").
//
// Each chain c keeps, per term alpha, the Pauli Q_x = i^mu Z(t) X(u) of its
// current string x, stored as the word u | mu << 62 (t is not needed for the
// amplitude, and the product with U_C^{-1} X_j U_C is taken on the right:
// the two factors commute, so Q_x P_j = P_j Q_x).  A step proposes y = x ^ e_j:
//   u' = u ^ F_j,  mu' = mu + gamma_j + 2 par(u' & M_j),
// and <y|phi_alpha> follows from (u', mu') as in Eq. (amplitude1), O(1) words
// per term and chain.
//
// Kernels per step: (1) k_propose_gather (single flips; the cache is brought
// up to date once per window of kMetroWin steps, in place) or k_propose (flip
// masks: the tile's rows staged in LDS; the cache is brought up to date with
// an accepted mask at the next step, in place): lanes over terms, reduce
// sum_alpha b_alpha <y|phi_alpha> over the 256-term tile in FP64; (2) one workgroup per chain: add the tiles' partials in a fixed
// order, r = |A(y)|^2 / |A(x)|^2 in FP64, accept iff U < r.
#include "device_common.hpp"
#include "internal.hpp"

namespace chsim {

namespace {

struct TermAmpConst {
  uint64_t v, s;
  uint32_t w;
  double w0r, w0i;  // b_alpha 2^{-|v|/2}
};

__device__ __forceinline__ TermAmpConst load_const(const TermsView& T, uint64_t a) {
  TermAmpConst c;
  c.v = T.v[a];
  c.s = T.s[a];
  c.w = T.omega[a];
  const double2 b = T.b[a];
  const int vc = __popcll(c.v);
  const double h = 0.70710678118654752440;
  const double mag = ldexp(1.0, -(vc >> 1)) * ((vc & 1) ? h : 1.0);
  c.w0r = b.x * mag;
  c.w0i = b.y * mag;
  return c;
}

// b <x|phi> from the cached (u, mu), without branches: the rotation by
// e^{i pi k / 4} (an odd k first multiplies by e^{i pi / 4}, then i^{k >> 1}
// swaps and negates), and zero when x is outside the term's support.
__device__ __forceinline__ double2 term_value(const TermAmpConst& c, uint64_t u, uint32_t mu) {
  // u and s have no bits at or above n, so outside supp(v) is ~v.
  const bool off = ((u ^ c.s) & ~c.v) != 0ull;
  const uint32_t k = (c.w + 2u * mu + 4u * __popcll(u & c.v & c.s)) & 7u;
  const double h = 0.70710678118654752440;
  const double a = (k & 1u) ? (c.w0r - c.w0i) * h : c.w0r;
  const double b = (k & 1u) ? (c.w0r + c.w0i) * h : c.w0i;
  const uint32_t m = k >> 1;
  double re = (m & 1u) ? b : a, im = (m & 1u) ? a : b;
  re = __longlong_as_double(__double_as_longlong(re) ^ ((long long)((m ^ (m >> 1)) & 1u) << 63));
  im = __longlong_as_double(__double_as_longlong(im) ^ ((long long)(m >> 1) << 63));
  return make_double2(off ? 0.0 : re, off ? 0.0 : im);
}

constexpr uint64_t kUMask = (1ull << 62) - 1ull;

// A double moved between lanes by DPP (two 32-bit moves on the VALU).
template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, kCtrl, 0xF, 0xF, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), kCtrl, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum of x over the wave's 64 lanes, valid in lane 0, in a fixed order:
// within quads (lane ^ 1, lane ^ 2) and rows of 16 (half-row and row
// mirrors) by DPP moves, across the two rows of each half by one swizzle,
// and the halves by a read of lane 32.
__device__ __forceinline__ double wave_sum0(double x) {
  x += dpp_f64<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x += dpp_f64<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  x += dpp_f64<0x141>(x);  // row_half_mirror
  x += dpp_f64<0x140>(x);  // row_mirror
  x += __shfl_xor(x, 16);
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 32);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 32);
  return x + __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum of a double2 over the 256-thread block (fixed order); result in thread 0.
__device__ __forceinline__ double2 block_sum(double2 v, double2* scratch) {
  for (int m = 32; m >= 1; m >>= 1) {
    v.x += __shfl_down(v.x, m);
    v.y += __shfl_down(v.y, m);
  }
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  double2 r = make_double2(0.0, 0.0);
  if (threadIdx.x == 0) {
    for (int w = 0; w < 4; ++w) {
      r.x += scratch[w].x;
      r.y += scratch[w].y;
    }
  }
  return r;
}

// Initial Q_x for every chain (the O(k n^2) start-up cost) and the tile sums of
// <x_c|psi>.
__global__ __launch_bounds__(256) void k_metro_init(TermsView T, MetroView Mv) {
  __shared__ double2 scratch[4];
  const uint64_t a = (uint64_t)blockIdx.x * kMetroTile + threadIdx.x;
  const bool live = a < T.chi;
  const uint64_t chi = T.chi;
  TermAmpConst c;
  if (live) c = load_const(T, a);
  for (uint32_t ch = 0; ch < Mv.n_chain; ++ch) {
    const uint32_t n = T.n;
    const uint64_t x = Mv.x[ch] & ((n == 64) ? ~0ull : ((1ull << n) - 1ull));
    double2 val = make_double2(0.0, 0.0);
    if (live) {
      uint64_t u = 0, xm = x;
      uint32_t mu = 0;
      while (xm) {
        const uint32_t p = (uint32_t)__builtin_ctzll(xm);
        xm &= xm - 1ull;
        u ^= T.F[(uint64_t)p * chi + a];
        mu += T.gamma[(uint64_t)p * chi + a] + 2u * par64(u & T.M[(uint64_t)p * chi + a]);
      }
      mu &= 3u;
      Mv.state[(uint64_t)ch * chi + a] = (u & kUMask) | ((uint64_t)mu << 62);
      val = term_value(c, u, mu);
    }
    const double2 tot = block_sum(val, scratch);
    if (threadIdx.x == 0) Mv.partial[(uint64_t)ch * Mv.n_tiles + blockIdx.x] = tot;
  }
}

__global__ __launch_bounds__(256) void k_chain_amp(MetroView Mv) {
  __shared__ double2 scratch[4];
  const uint32_t ch = blockIdx.x;
  double2 acc = make_double2(0.0, 0.0);
  for (uint32_t t = threadIdx.x; t < Mv.n_tiles; t += 256u) {
    const double2 v = Mv.partial[(uint64_t)ch * Mv.n_tiles + t];
    acc.x += v.x;
    acc.y += v.y;
  }
  const double2 tot = block_sum(acc, scratch);
  if (threadIdx.x == 0) Mv.amp[ch] = tot;
}


// Flip-mask proposal step y = x ^ m for every chain, per term: the chain's
// cache is first brought up to date with the mask it accepted at the
// previous step (pmask, when the mode says so; written back in place, so a
// cache word is written only after an accepted move), then Q_y = Q_x
// prod_{j in m} P_j (right products; the factors commute) and
// sum_a b_a <y|phi_a> per chain over the block's 256 terms.  The block walks
// its tile in sub-tiles of 64 terms: the rows F_p, M_p, gamma_p of the
// sub-tile are staged in LDS once ([p][term], so a wave reading row j for
// its 64 terms is conflict-free), and wave w of 8 takes the chains c = w,
// w + 8, ...; a chain's masks are wave-uniform, so the loops over their set
// bits do not diverge and each term's rows leave HBM once per step for all
// chains.
constexpr uint32_t kSub = 64;
constexpr int kCW = 8;           // chains per wave in one pass
constexpr uint32_t kPWaves = 8;  // waves per block: kPWaves * kCW = 64 chains per pass
constexpr uint32_t kPThreads = 64 * kPWaves;
constexpr int kStage = (int)((64 * kSub + kPThreads - 1) / kPThreads);  // staging loads per thread
static_assert(kStage % 2 == 0, "staged in two halves");

__global__ __launch_bounds__(kPThreads) void k_propose(TermsView T, MetroView Mv,
                                                       const uint64_t* __restrict__ mask,
                                                       uint32_t mode) {
  extern __shared__ __align__(16) uint8_t smem[];
  const uint32_t n = T.n;
  uint64_t* sF = reinterpret_cast<uint64_t*>(smem);  // [n][64]
  uint64_t* sM = sF + (size_t)n * kSub;               // [n][64]
  uint8_t* sG = reinterpret_cast<uint8_t*>(sM + (size_t)n * kSub);  // [n][64]
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = uniform32(tid >> 6);
  const uint64_t chi = T.chi;
  const bool pend = mode & kProposeApplyPending, prop = mode & kProposeMasks;
  // Right product by P_j for every set bit j of mm.
  auto apply = [&](uint64_t& u, uint32_t& mu, uint64_t mm) {
    while (mm) {
      const uint32_t j = (uint32_t)__builtin_ctzll(mm);
      mm &= mm - 1ull;
      u ^= sF[j * kSub + lane];
      mu += (uint32_t)sG[j * kSub + lane] + 2u * par64(u & sM[j * kSub + lane]);
    }
  };
  for (uint32_t cg = 0; cg < Mv.n_chain; cg += kPWaves * kCW) {
    // This wave's chains in the pass: cg + wave + kPWaves k, k < kCW (wave-uniform).
    uint64_t m[kCW], pm[kCW];
    double accr[kCW], acci[kCW];
#pragma unroll
    for (int k = 0; k < kCW; ++k) {
      const uint32_t ch = cg + wave + kPWaves * (uint32_t)k;
      const bool on = ch < Mv.n_chain;
      m[k] = on && prop ? uniform64(mask[ch]) : 0ull;
      pm[k] = on && pend ? uniform64(Mv.pmask[ch]) : 0ull;
      accr[k] = 0.0;
      acci[k] = 0.0;
    }
    for (uint32_t sub = 0; sub < kMetroTile / kSub; ++sub) {
      const uint64_t base = (uint64_t)blockIdx.x * kMetroTile + (uint64_t)sub * kSub;
      if (base >= chi) break;  // block-uniform
      __syncthreads();         // the previous sub-tile's readers are done
      // The thread's share of the sub-tile is staged in two halves; within a
      // half every load is issued before the first store to LDS.
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        uint64_t rf[kStage / 2], rm[kStage / 2];
        uint32_t rg[kStage / 2];
#pragma unroll
        for (int r = 0; r < kStage / 2; ++r) {
          const uint32_t i = tid + (uint32_t)(half * (kStage / 2) + r) * kPThreads;
          const uint32_t p = i / kSub, t = i % kSub;
          const uint64_t at = base + t;
          const bool in = i < n * kSub && at < chi;
          rf[r] = in ? T.F[(uint64_t)p * chi + at] : 0ull;
          rm[r] = in ? T.M[(uint64_t)p * chi + at] : 0ull;
          rg[r] = in ? T.gamma[(uint64_t)p * chi + at] : 0u;
        }
#pragma unroll
        for (int r = 0; r < kStage / 2; ++r) {
          const uint32_t i = tid + (uint32_t)(half * (kStage / 2) + r) * kPThreads;
          if (i < n * kSub) {
            sF[i] = rf[r];
            sM[i] = rm[r];
            sG[i] = (uint8_t)rg[r];
          }
        }
      }
      const uint64_t a = base + lane;
      const bool live = a < chi;
      // Every cache word of this wave's chains is requested before any is used.
      uint64_t st[kCW];
#pragma unroll
      for (int k = 0; k < kCW; ++k) {
        const uint32_t ch = cg + wave + kPWaves * (uint32_t)k;
        st[k] = (live && (m[k] | pm[k]) != 0ull) ? Mv.state[(uint64_t)ch * chi + a] : 0ull;
      }
      TermAmpConst c{};
      if (live && prop) c = load_const(T, a);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kCW; ++k) {
        if ((m[k] | pm[k]) == 0ull || !live) continue;  // nothing to do, no such chain, or past chi
        const uint32_t ch = cg + wave + kPWaves * (uint32_t)k;
        uint64_t u = st[k] & kUMask;
        uint32_t mu = (uint32_t)(st[k] >> 62);
        if (pm[k]) {
          apply(u, mu, pm[k]);
          mu &= 3u;
          Mv.state[(uint64_t)ch * chi + a] = u | ((uint64_t)mu << 62);
        }
        if (m[k] == 0ull) continue;  // y = x: no proposal
        apply(u, mu, m[k]);
        const double2 val = term_value(c, u, mu & 3u);
        accr[k] += val.x;
        acci[k] += val.y;
      }
    }
    // One reduction over the lanes (terms) per chain.
#pragma unroll
    for (int k = 0; k < kCW; ++k) {
      const uint32_t ch = cg + wave + kPWaves * (uint32_t)k;
      if (ch >= Mv.n_chain || !prop) continue;  // wave-uniform
      double re = accr[k], im = acci[k];
      re = wave_sum0(re);
      im = wave_sum0(im);
      if (lane == 0) Mv.partial[(uint64_t)ch * Mv.n_tiles + blockIdx.x] = make_double2(re, im);
    }
  }
}

// Single-flip proposal step with deferred cache updates.  Lanes over terms
// (each lane takes four terms of the 256-term tile), waves over chains.  A
// chain's cached (u, mu) is brought up to date only once per window of
// kMetroWin steps: step t of the window that starts at t0 reads the cache as
// of t0, applies the flips the chain accepted at steps t0 .. t-1 (right
// products by their P_j in step order: the same arithmetic as updating after
// every accepted step), then the proposal's P_j.  The first step of the next
// window (and a final pass without a proposal at the end of a call) writes
// the brought-up-to-date cache back in place.  The tile's rows of chain 0's
// flip bits at the pending steps are staged in LDS once and serve every
// chain whose bit at that step is the same (every chain, when the chains
// share the flip bit of a step); a chain with another bit reads its row from
// the term store.  So per chain and step only the 8-byte cache word of each
// term is read, and it is written once per window.
constexpr uint32_t kGWaves = 4;
constexpr uint32_t kGSub = kMetroTile / 64;  // terms per lane
constexpr uint32_t kModeWrite = 1u, kModePropose = 2u;

template <int CP>
__global__ __launch_bounds__(64 * kGWaves) void k_propose_gather(TermsView T, MetroView Mv,
                                                                 uint32_t step, uint32_t pbase,
                                                                 uint32_t npend, uint32_t mode) {
  // Slots 0 .. npend-1: rows of chain 0's bits at the pending steps; slot
  // kMetroWin: the row of chain 0's proposal bit.
  constexpr uint32_t kSlots = kMetroWin + 1;
  __shared__ uint64_t sF[kSlots][kMetroTile], sM[kSlots][kMetroTile];
  __shared__ uint8_t sG[kSlots][kMetroTile];
  const uint32_t lane = threadIdx.x & 63u, wave = uniform32(threadIdx.x >> 6);
  const uint32_t n = T.n, nc = Mv.n_chain;
  const uint64_t chi = T.chi;
  const uint64_t tile0 = (uint64_t)blockIdx.x * kMetroTile;
  const bool full = tile0 + kMetroTile <= chi;  // block-uniform
  const bool write = mode & kModeWrite, prop = mode & kModePropose;
  // Term offsets within the tile, clamped to the last term in a partial tile:
  // past chi a lane reads that term's words and contributes zero (its
  // weight is zero) and writes nothing.
  const uint32_t last = (uint32_t)(chi - 1ull - tile0);
  uint32_t ao[kGSub];
#pragma unroll
  for (uint32_t sb = 0; sb < kGSub; ++sb) ao[sb] = min(sb * 64u + lane, last);
  uint32_t Wj[kSlots];
#pragma unroll
  for (uint32_t s = 0; s < kSlots; ++s) {
    Wj[s] = ~0u;
    const bool use = s < kMetroWin ? s < npend : prop;
    if (use) {
      Wj[s] = uniform32(Mv.jstream[s < kMetroWin ? pbase + s : step]) % n;
      const uint64_t off = (uint64_t)Wj[s] * chi + tile0 + min(threadIdx.x, last);
      sF[s][threadIdx.x] = T.F[off];
      sM[s][threadIdx.x] = T.M[off];
      sG[s][threadIdx.x] = T.gamma[off];
    }
  }
  __syncthreads();
  TermAmpConst c[kGSub];
#pragma unroll
  for (uint32_t sb = 0; sb < kGSub; ++sb) {
    if (prop) c[sb] = load_const(T, tile0 + ao[sb]);
    if (sb * 64u + lane > last) c[sb].w0r = c[sb].w0i = 0.0;
  }
  const uint32_t pmask = (1u << npend) - 1u;  // npend <= kMetroWin < 32
  // Right product by P_j of step slot s for the lane's terms: the staged row
  // when the chain's bit j is chain 0's, else the term store's.
  auto flip = [&](uint64_t (&u)[kGSub], uint32_t (&mu)[kGSub], uint32_t s, uint32_t j) {
    if (j == Wj[s]) {  // wave-uniform
#pragma unroll
      for (uint32_t sb = 0; sb < kGSub; ++sb) {
        u[sb] ^= sF[s][sb * 64u + lane];
        mu[sb] += (uint32_t)sG[s][sb * 64u + lane] + 2u * __popcll(u[sb] & sM[s][sb * 64u + lane]);
      }
    } else {
      const uint64_t* F = T.F + ((uint64_t)j * chi + tile0);
      const uint64_t* M = T.M + ((uint64_t)j * chi + tile0);
      const uint8_t* g = T.gamma + ((uint64_t)j * chi + tile0);
#pragma unroll
      for (uint32_t sb = 0; sb < kGSub; ++sb) {
        u[sb] ^= F[ao[sb]];
        mu[sb] += (uint32_t)g[ao[sb]] + 2u * __popcll(u[sb] & M[ao[sb]]);
      }
    }
  };
  // The wave's chains are ch = wave + kGWaves i.  Their per-chain words (the
  // pending mask, the proposal bit and the pending steps' bits) are read for
  // 64 chains at once, chain i % 64 in lane i % 64, and taken from there by
  // lane reads, so that no wait for them also waits for the cache words in
  // flight.
  const uint32_t n_mine = nc > wave ? (nc - wave + kGWaves - 1u) / kGWaves : 0u;
  uint32_t m_pm = 0u, m_j = 0u, m_js[kMetroWin];
  for (uint32_t i0 = 0; i0 < n_mine; i0 += 64u) {
    {
      const uint32_t i = i0 + lane;
      const bool ok = i < n_mine;
      const uint32_t ch = ok ? wave + kGWaves * i : wave;
      const uint64_t jrow = (uint64_t)ch * Mv.n_steps;
      m_pm = npend ? Mv.pend[ch] & pmask : 0u;
      m_j = prop ? Mv.jstream[jrow + step] % n : 0u;
#pragma unroll
      for (uint32_t s = 0; s < kMetroWin; ++s) m_js[s] = s < npend ? Mv.jstream[jrow + pbase + s] % n : 0u;
    }
    const uint32_t i_end = min(n_mine - i0, 64u);
    // CP chains per pass: all their cache words are requested before any is
    // combined.
    for (uint32_t k0 = 0; k0 < i_end; k0 += (uint32_t)CP) {
      uint64_t st[CP][kGSub];
#pragma unroll
      for (int h = 0; h < CP; ++h) {
        const uint32_t k = k0 + (uint32_t)h < i_end ? k0 + (uint32_t)h : k0;
        const uint32_t ch = wave + kGWaves * (i0 + k);
        const uint64_t* sp = Mv.state + ((uint64_t)ch * chi + tile0);
#pragma unroll
        for (uint32_t sb = 0; sb < kGSub; ++sb) st[h][sb] = sp[ao[sb]];
      }
#pragma unroll
      for (int h = 0; h < CP; ++h) {
        const uint32_t k = k0 + (uint32_t)h;
        if (k >= i_end) break;  // wave-uniform
        const uint32_t ch = wave + kGWaves * (i0 + k);
        uint64_t u[kGSub];
        uint32_t mu[kGSub];
#pragma unroll
        for (uint32_t sb = 0; sb < kGSub; ++sb) {
          u[sb] = st[h][sb] & kUMask;
          mu[sb] = (uint32_t)(st[h][sb] >> 62);
        }
        const uint32_t pm = (uint32_t)__builtin_amdgcn_readlane((int)m_pm, (int)k);
#pragma unroll
        for (uint32_t s = 0; s < kMetroWin; ++s)
          if ((pm >> s) & 1u) flip(u, mu, s, (uint32_t)__builtin_amdgcn_readlane((int)m_js[s], (int)k));
        if (write) {
          uint64_t* sp = Mv.state + ((uint64_t)ch * chi + tile0);
          if (full) {
#pragma unroll
            for (uint32_t sb = 0; sb < kGSub; ++sb) sp[sb * 64u + lane] = u[sb] | ((uint64_t)(mu[sb] & 3u) << 62);
          } else {
#pragma unroll
            for (uint32_t sb = 0; sb < kGSub; ++sb)
              if (sb * 64u + lane <= last) sp[sb * 64u + lane] = u[sb] | ((uint64_t)(mu[sb] & 3u) << 62);
          }
        }
        if (!prop) continue;
        flip(u, mu, kMetroWin, (uint32_t)__builtin_amdgcn_readlane((int)m_j, (int)k));
        double2 t0 = term_value(c[0], u[0], mu[0] & 3u);
        double re = t0.x, im = t0.y;
#pragma unroll
        for (uint32_t sb = 1; sb < kGSub; ++sb) {
          const double2 val = term_value(c[sb], u[sb], mu[sb] & 3u);
          re += val.x;
          im += val.y;
        }
        re = wave_sum0(re);
        im = wave_sum0(im);
        if (lane == 0) Mv.partial[(uint64_t)ch * Mv.n_tiles + blockIdx.x] = make_double2(re, im);
      }
    }
  }
}

// Single flips gather rows per term (deferred cache updates); flip masks
// (several rows per chain) read the tile's rows once through LDS.
hipError_t launch_gather(const TermsView& T, MetroView& Mv, uint32_t step, uint32_t pbase,
                         uint32_t npend, uint32_t mode, hipStream_t st) {
  hipLaunchKernelGGL(k_propose_gather<2>, dim3(Mv.n_tiles), dim3(64 * kGWaves), 0, st, T, Mv, step,
                     pbase, npend, mode);
  return hipGetLastError();
}

hipError_t launch_masks(const TermsView& T, MetroView& Mv, const uint64_t* mask, uint32_t mode,
                        hipStream_t st) {
  const size_t sm = (size_t)T.n * kSub * 17;
  if (sm > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_propose,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_propose, dim3(Mv.n_tiles), dim3(kPThreads), sm, st, T, Mv, mask, mode);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_metro_accept(MetroView Mv, uint32_t step) {
  __shared__ double2 scratch[4];
  const uint32_t ch = blockIdx.x;
  double2 acc = make_double2(0.0, 0.0);
  for (uint32_t t = threadIdx.x; t < Mv.n_tiles; t += 256u) {
    const double2 v = Mv.partial[(uint64_t)ch * Mv.n_tiles + t];
    acc.x += v.x;
    acc.y += v.y;
  }
  const double2 ay = block_sum(acc, scratch);
  if (threadIdx.x == 0) {
    const uint64_t idx = (uint64_t)ch * Mv.n_steps + step;
    const double2 ax = Mv.amp[ch];
    const double px = ax.x * ax.x + ax.y * ax.y;
    const double py = ay.x * ay.x + ay.y * ay.y;
    const double r = py / px;
    const double U = Mv.ustream[idx];
    const uint32_t acc_ = (px > 0.0) && (r >= 1.0 || U < r);
    uint64_t x = Mv.x[ch];
    // The step's bit in the chain's window of deferred cache updates.
    const uint32_t w = step % kMetroWin;
    uint32_t pend = w ? Mv.pend[ch] : 0u;
    if (acc_) {
      x ^= 1ull << (Mv.jstream[idx] % Mv.n_qubits);
      Mv.x[ch] = x;
      Mv.amp[ch] = ay;
      pend |= 1u << w;
    }
    Mv.pend[ch] = pend;
    if (Mv.trace) Mv.trace[idx] = x;
    if (Mv.accepted) Mv.accepted[idx] = (uint8_t)acc_;
  }
}

}  // namespace

hipError_t launch_metro_init(const TermsView& T, MetroView& Mv, hipStream_t st) {
  const uint32_t tiles = Mv.n_tiles;
  hipLaunchKernelGGL(k_metro_init, dim3(tiles), dim3(kMetroTile), 0, st, T, Mv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chain_amp, dim3(Mv.n_chain), dim3(256), 0, st, Mv);
  return hipGetLastError();
}

hipError_t launch_metro_steps(const TermsView& T, MetroView& Mv, uint32_t n_steps, hipStream_t st) {
  if (n_steps == 0) return hipSuccess;
  for (uint32_t t = 0; t < n_steps; ++t) {
    // Step t applies the accepted flips of its window's earlier steps; the
    // first step of a window (t > 0) applies the whole previous window and
    // writes the caches back.
    const uint32_t w = t % kMetroWin;
    const bool close = w == 0 && t > 0;
    const uint32_t pbase = close ? t - kMetroWin : t - w, npend = close ? kMetroWin : w;
    hipError_t e = launch_gather(T, Mv, t, pbase, npend,
                                 kModePropose | (close ? kModeWrite : 0u), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_metro_accept, dim3(Mv.n_chain), dim3(256), 0, st, Mv, t);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // The last window's accepted flips, so that every chain's current cache is
  // up to date when the call returns.
  const uint32_t t0 = (n_steps - 1u) / kMetroWin * kMetroWin;
  return launch_gather(T, Mv, 0, t0, n_steps - t0, kModeWrite, st);
}

hipError_t launch_propose(const TermsView& T, MetroView& Mv, const uint64_t* mask, uint32_t mode,
                          hipStream_t st) {
  return launch_masks(T, Mv, mask, mode, st);
}

}  // namespace chsim
