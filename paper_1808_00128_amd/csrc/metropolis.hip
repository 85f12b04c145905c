// Metropolis chain over n-bit outputs (Sec. "Heuristic Metropolis simulator").
//
// Each chain c keeps, per term alpha, the Pauli Q_x = i^mu Z(t) X(u) of its
// current string x, stored as the word u | mu << 62 (t is not needed for the
// amplitude, and the product with U_C^{-1} X_j U_C is taken on the right:
// the two factors commute, so Q_x P_j = P_j Q_x).  A step proposes y = x ^ e_j:
//   u' = u ^ F_j,  mu' = mu + gamma_j + 2 par(u' & M_j),
// and <y|phi_alpha> follows from (u', mu') as in Eq. (amplitude1), O(1) words
// per term and chain.  The proposal words are written to the chain's second
// buffer; accepting the move flips which buffer is current, so no term data
// is rewritten at accept time.
//
// Kernels per step: (1) k_propose_gather (single flips: each chain gathers
// its one row) or k_propose (flip masks: the tile's rows staged in LDS):
// lanes over terms, waves over chains: propose, write the proposal word, and
// reduce sum_alpha b_alpha <y|phi_alpha> over the 256-term tile in FP64; (2) one
// workgroup per chain: add the tiles' partials in a fixed order,
// r = |A(y)|^2 / |A(x)|^2 in FP64, accept iff U < r.
#include "device_common.hpp"
#include "internal.hpp"

namespace chsim {

namespace {

struct TermAmpConst {
  uint64_t s, nv, vs;
  uint32_t w;
  double w0r, w0i, w1r, w1i;
};

__device__ __forceinline__ TermAmpConst load_const(const TermsView& T, uint64_t a) {
  TermAmpConst c;
  const uint64_t v = T.v[a], s = T.s[a];
  const uint32_t n = T.n;
  const uint64_t nmask = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
  c.s = s;
  c.nv = ~v & nmask;
  c.vs = v & s;
  c.w = T.omega[a];
  const double2 b = T.b[a];
  const int vc = __popcll(v);
  const double h = 0.70710678118654752440;
  const double mag = ldexp(1.0, -(vc >> 1)) * ((vc & 1) ? h : 1.0);
  c.w0r = b.x * mag;
  c.w0i = b.y * mag;
  c.w1r = (c.w0r - c.w0i) * h;
  c.w1i = (c.w0r + c.w0i) * h;
  return c;
}

// b <x|phi> from the cached (u, mu).
__device__ __forceinline__ double2 term_value(const TermAmpConst& c, uint64_t u, uint32_t mu) {
  if ((u ^ c.s) & c.nv) return make_double2(0.0, 0.0);
  const uint32_t k = (c.w + 2u * mu + 4u * par64(u & c.vs)) & 7u;
  double re = (k & 1u) ? c.w1r : c.w0r;
  double im = (k & 1u) ? c.w1i : c.w0i;
  const uint32_t m = k >> 1;
  if (m & 1u) {
    const double t = re;
    re = im;
    im = t;
  }
  if ((m ^ (m >> 1)) & 1u) re = -re;
  if (m & 2u) im = -im;
  return make_double2(re, im);
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
      Mv.state[0][(uint64_t)ch * chi + a] = (u & kUMask) | ((uint64_t)mu << 62);
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
  if (threadIdx.x == 0) {
    Mv.amp[ch] = tot;
    Mv.parity[ch] = 0u;
  }
}


// Proposal step y = x ^ m for every chain, per term: Q_y = Q_x prod_{j in m} P_j
// (right products), the new cached (u, mu) into the other state buffer, and
// sum_a b_a <y|phi_a> per chain over the block's 256 terms.  The block walks
// its tile in sub-tiles of 64 terms: the rows F_p, M_p, gamma_p of the
// sub-tile are staged in LDS once ([p][term], so a wave reading row j for its
// 64 terms is conflict-free), and wave w of 8 takes the chains c = w,
// w + 8, ...; a chain's mask is wave-uniform, so the loop over its set bits does not
// diverge and each term's rows leave HBM once per step for all chains.  The
// masks are an array (learned proposal) or the single flips e_{j % n} of the
// chains' j stream at `step` (the paper's chain).
constexpr uint32_t kSub = 64;
constexpr int kCW = 8;           // chains per wave in one pass
constexpr uint32_t kPWaves = 8;  // waves per block: kPWaves * kCW = 64 chains per pass
constexpr uint32_t kPThreads = 64 * kPWaves;
constexpr int kStage = (int)((64 * kSub + kPThreads - 1) / kPThreads);  // staging loads per thread
static_assert(kStage % 2 == 0, "staged in two halves");

template <bool kSingle>
__global__ __launch_bounds__(kPThreads) void k_propose(TermsView T, MetroView Mv,
                                                       const uint64_t* __restrict__ mask,
                                                       uint32_t step) {
  extern __shared__ __align__(16) uint8_t smem[];
  const uint32_t n = T.n;
  uint64_t* sF = reinterpret_cast<uint64_t*>(smem);  // [n][64]
  uint64_t* sM = sF + (size_t)n * kSub;               // [n][64]
  uint8_t* sG = reinterpret_cast<uint8_t*>(sM + (size_t)n * kSub);  // [n][64]
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = uniform32(tid >> 6);
  const uint64_t chi = T.chi;
  for (uint32_t cg = 0; cg < Mv.n_chain; cg += kPWaves * kCW) {
    // This wave's chains in the pass: cg + wave + kPWaves k, k < kCW (wave-uniform).
    uint64_t m[kCW];
    uint32_t cur[kCW];
    double accr[kCW], acci[kCW];
#pragma unroll
    for (int k = 0; k < kCW; ++k) {
      const uint32_t ch = cg + wave + kPWaves * (uint32_t)k;
      m[k] = 0ull;
      if (ch < Mv.n_chain) {
        if (kSingle) m[k] = 1ull << (uniform32(Mv.jstream[(uint64_t)ch * Mv.n_steps + step]) % n);
        else m[k] = uniform64(mask[ch]);
      }
      cur[k] = ch < Mv.n_chain ? uniform32(Mv.parity[ch]) : 0u;
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
      // Every state word of this wave's chains is requested before any is used.
      uint64_t st[kCW];
#pragma unroll
      for (int k = 0; k < kCW; ++k) {
        const uint32_t ch = cg + wave + kPWaves * (uint32_t)k;
        st[k] = (live && m[k] != 0ull) ? Mv.state[cur[k]][(uint64_t)ch * chi + a] : 0ull;
      }
      TermAmpConst c{};
      if (live) c = load_const(T, a);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kCW; ++k) {
        if (m[k] == 0ull || !live) continue;  // y = x, no such chain, or past chi
        const uint32_t ch = cg + wave + kPWaves * (uint32_t)k;
        uint64_t u = st[k] & kUMask;
        uint32_t mu = (uint32_t)(st[k] >> 62);
        uint64_t mm = m[k];
        while (mm) {
          const uint32_t j = (uint32_t)__builtin_ctzll(mm);
          mm &= mm - 1ull;
          u ^= sF[j * kSub + lane];
          mu += (uint32_t)sG[j * kSub + lane] + 2u * par64(u & sM[j * kSub + lane]);
        }
        mu &= 3u;
        Mv.state[cur[k] ^ 1u][(uint64_t)ch * chi + a] = u | ((uint64_t)mu << 62);
        const double2 val = term_value(c, u, mu);
        accr[k] += val.x;
        acci[k] += val.y;
      }
    }
    // One reduction over the lanes (terms) per chain.
#pragma unroll
    for (int k = 0; k < kCW; ++k) {
      const uint32_t ch = cg + wave + kPWaves * (uint32_t)k;
      if (ch >= Mv.n_chain) continue;  // wave-uniform
      double re = accr[k], im = acci[k];
      re = wave_sum0(re);
      im = wave_sum0(im);
      if (lane == 0) Mv.partial[(uint64_t)ch * Mv.n_tiles + blockIdx.x] = make_double2(re, im);
    }
  }
}

// Single-flip proposal step without LDS: lanes over terms, waves over
// chains; each chain gathers the words of its flipped row F_j, M_j, gamma_j
// straight from the term store (rows that several chains flip are served by
// L2), so no barrier separates loading from computing and only the touched
// rows are read.  Each lane adds its terms of the 256-term tile in the same
// order, and the lane sums are reduced with the same butterfly, as k_propose.
constexpr uint32_t kGWaves = 4;
constexpr uint32_t kGSub = kMetroTile / 64;  // 64-term sub-tiles per tile

template <int CP>
__global__ __launch_bounds__(64 * kGWaves) void k_propose_gather(TermsView T, MetroView Mv,
                                                                 uint32_t step) {
  const uint32_t lane = threadIdx.x & 63u, wave = uniform32(threadIdx.x >> 6);
  const uint32_t n = T.n;
  const uint64_t chi = T.chi;
  const uint64_t tile0 = (uint64_t)blockIdx.x * kMetroTile;
  TermAmpConst c[kGSub];
  bool live[kGSub];
#pragma unroll
  for (uint32_t sb = 0; sb < kGSub; ++sb) {
    const uint64_t a = tile0 + sb * 64u + lane;
    live[sb] = a < chi;
    c[sb] = TermAmpConst{};
    if (live[sb]) c[sb] = load_const(T, a);
  }
  // CP chains per pass: all their state words and rows are requested before
  // any is combined (more loads in flight when the grid is small).  A chain
  // whose flip bit equals the previous chain's (one bit per step shared by
  // the chains) reuses the rows already loaded.
  uint64_t Fr[CP][kGSub], Mr[CP][kGSub];
  uint32_t gr[CP][kGSub], jprev[CP];
#pragma unroll
  for (int h = 0; h < CP; ++h) jprev[h] = ~0u;
  for (uint32_t c0 = wave; c0 < Mv.n_chain; c0 += (uint32_t)CP * kGWaves) {
    uint64_t st[CP][kGSub];
    uint32_t cur[CP];
#pragma unroll
    for (int h = 0; h < CP; ++h) {
      const bool on = c0 + (uint32_t)h * kGWaves < Mv.n_chain;  // wave-uniform
      const uint32_t ch = on ? c0 + (uint32_t)h * kGWaves : c0;
      const uint32_t j = uniform32(Mv.jstream[(uint64_t)ch * Mv.n_steps + step]) % n;
      cur[h] = uniform32(Mv.parity[ch]);
      const bool rows = j != jprev[h];  // wave-uniform
      jprev[h] = j;
#pragma unroll
      for (uint32_t sb = 0; sb < kGSub; ++sb) {
        const uint64_t a = tile0 + sb * 64u + lane;
        const bool ld = on && live[sb];
        const uint64_t off = (uint64_t)j * chi + a;
        st[h][sb] = ld ? Mv.state[cur[h]][(uint64_t)ch * chi + a] : 0ull;
        if (rows) {
          Fr[h][sb] = live[sb] ? T.F[off] : 0ull;
          Mr[h][sb] = live[sb] ? T.M[off] : 0ull;
          gr[h][sb] = live[sb] ? (uint32_t)T.gamma[off] : 0u;
        }
      }
    }
#pragma unroll
    for (int h = 0; h < CP; ++h) {
      const uint32_t ch = c0 + (uint32_t)h * kGWaves;
      if (ch >= Mv.n_chain) break;
      double re = 0.0, im = 0.0;
#pragma unroll
      for (uint32_t sb = 0; sb < kGSub; ++sb) {
        if (!live[sb]) continue;
        const uint64_t a = tile0 + sb * 64u + lane;
        uint64_t u = st[h][sb] & kUMask;
        uint32_t mu = (uint32_t)(st[h][sb] >> 62);
        u ^= Fr[h][sb];
        mu += gr[h][sb] + 2u * par64(u & Mr[h][sb]);
        mu &= 3u;
        Mv.state[cur[h] ^ 1u][(uint64_t)ch * chi + a] = u | ((uint64_t)mu << 62);
        const double2 val = term_value(c[sb], u, mu);
        re += val.x;
        im += val.y;
      }
      re = wave_sum0(re);
      im = wave_sum0(im);
      if (lane == 0) Mv.partial[(uint64_t)ch * Mv.n_tiles + blockIdx.x] = make_double2(re, im);
    }
  }
}

// Single flips gather their one row per chain; flip masks (several rows per
// chain) read the tile's rows once through LDS.
template <bool kSingle>
hipError_t launch_propose_t(const TermsView& T, MetroView& Mv, const uint64_t* mask, uint32_t step,
                            hipStream_t st) {
  if (kSingle) {
    // Small grids (fewer than 2048 tiles) take two chains per pass per wave.
    if (Mv.n_tiles < 2048u)
      hipLaunchKernelGGL(k_propose_gather<2>, dim3(Mv.n_tiles), dim3(64 * kGWaves), 0, st, T, Mv, step);
    else
      hipLaunchKernelGGL(k_propose_gather<1>, dim3(Mv.n_tiles), dim3(64 * kGWaves), 0, st, T, Mv, step);
    return hipGetLastError();
  }
  const size_t sm = (size_t)T.n * kSub * 17;
  if (sm > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_propose<false>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_propose<false>, dim3(Mv.n_tiles), dim3(kPThreads), sm, st, T, Mv, mask, step);
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
    if (acc_) {
      x ^= 1ull << (Mv.jstream[idx] % Mv.n_qubits);
      Mv.x[ch] = x;
      Mv.amp[ch] = ay;
      Mv.parity[ch] ^= 1u;
    }
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
  for (uint32_t t = 0; t < n_steps; ++t) {
    hipError_t e = launch_propose_t<true>(T, Mv, nullptr, t, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_metro_accept, dim3(Mv.n_chain), dim3(256), 0, st, Mv, t);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_propose(const TermsView& T, MetroView& Mv, const uint64_t* mask, uint32_t step,
                          hipStream_t st) {
  return launch_propose_t<false>(T, Mv, mask, step, st);
}

}  // namespace chsim
