// Amplitudes <x|psi> = sum_alpha b_alpha <x|phi_alpha> (step (b) of the hot path).
//
// Per (term, x), Eqs. (amplitude), (amplitude1): Q = prod_{p: x_p = 1}
// U_C^{-1} X_p U_C = i^mu Z(t) X(u) is built by right multiplication,
//   u ^= F_p;  mu += gamma_p + 2 par(u & M_p)       (u already updated),
// and <x|phi> = 0 if (u ^ s) & ~v != 0, else e^{i pi k/4} 2^{-|v|/2} with
// k = omega + 2 mu + 4 par(u & v & s) (mod 8).
//
// Reformulation used here (exact, same k).  Only the parity of the M part of
// mu enters k (it is multiplied by 4 mod 8), and summing over the set bits
// q of x in order gives
//   sum_q par(u_{<=q} & M_q) = sum_{p <= q, both in x} par(F_p & M_q)
// = x^T B x (mod 2) with the upper-triangular GF(2) matrix
// B_pq = par(F_p & M_q), p <= q.  par(u & v & s) = sum_{p in x} par(F_p & v & s)
// and the gamma high bits are x-linear too, so both fold into the diagonal
// of B.  With the column words c_q = sum_p B_pq e_p, w = XOR_{q in x} c_q and
//   k = omega + 2 popc(x & gamma_lo) + 4 popc(x & w)   (mod 8),
//   <x|phi> != 0  iff  ((XOR_{p in x} F_p) ^ s) & ~v == 0.
// Both XOR sums are GF(2)-linear in x, so each is read from per-term tables
// of 4-bit chunks of x: table c, entry e = XOR of the rows 4c + b, b in e.
// A prologue kernel computes the c_q rows and per-term constants once per
// term set; the amplitude kernel builds the tables of 8 terms at a time in
// LDS and lanes run over bitstrings (2 per lane): 2 ceil(n/4) LDS lookups
// and 64-bit XORs per (term, x) instead of a loop over the set bits of x.
// The table for u has s folded into chunk 0 and is masked with ~v, so the
// zero test is u == 0; a wave skips the phase work of a term for which all
// its lanes' amplitudes vanish.  Only the n - |v| positions outside v matter
// in u; when n - |v| <= 64 - n the prologue gathers them, in increasing
// order, into bits n, n + 1, ... of the c_q rows (gathering is linear, so a
// table of the combined rows yields both sums at once) and such a packed
// term has one table: the zero test reads the bits above n, and x & w never
// sees them.  Deep circuits leave |v| close to n, so most terms are packed
// and take half the lookups.
//
// Work items (request, range of 8-term tiles, chunk of 512 bitstrings) are
// pulled from a queue by a persistent grid, so one launch serves any mix of
// instances.  Per tile, the terms' constants are staged in LDS beside the
// tables, with the eight values a term can take (omega folded in), so a
// lane's value is one more lookup.  Each lane sums its bitstrings' values
// over the item's terms (FP32: plain within a tile, the tile sums with a
// two-sum compensation term; or FP64), the item writes one partial per
// bitstring, and a second kernel adds the ranges in FP64 in a fixed order.
#include <algorithm>
#include <vector>

#include "device_common.hpp"
#include "internal.hpp"

namespace chsim {

namespace {

constexpr int kTT = 8;                    // terms per table tile
constexpr int kMaxCh = 16;                // 4-bit chunks of a 64-bit string
constexpr int kTabWords = kMaxCh * 16;    // one table (u or w) of one term, in 64-bit words
static_assert(kTT * 2 * kMaxCh == 256, "one builder thread per (term, table, chunk)");
// Bitstrings per lane XPL (1 or 2): a work item holds 256 XPL bitstrings.

// Bits of a at the set positions of m, packed in increasing order into the
// low popcount(m) bits.
__device__ __forceinline__ uint64_t gather_bits(uint64_t a, uint64_t m) {
  uint64_t r = 0;
  for (uint32_t k = 0; m != 0ull; ++k, m &= m - 1ull) r |= ((a >> __builtin_ctzll(m)) & 1ull) << k;
  return r;
}

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

template <typename T>
struct Acc;

// FP32: the terms of one 8-term tile are added plainly (term), and the tile
// sum joins a running sum with a compensation term per component (flush).
template <>
struct Acc<float> {
  float sr = 0.f, er = 0.f, si = 0.f, ei = 0.f;
  float br = 0.f, bi = 0.f;
  __device__ __forceinline__ void term(float r, float i) {
    br += r;
    bi += i;
  }
  __device__ __forceinline__ void flush() {
    float s, e;
    two_sum(sr, br, s, e);
    sr = s;
    er += e;
    two_sum(si, bi, s, e);
    si = s;
    ei += e;
    br = bi = 0.f;
  }
  __device__ __forceinline__ double2 value() const {
    return make_double2((double)sr + (double)er, (double)si + (double)ei);
  }
};

template <>
struct Acc<double> {
  double sr = 0.0, si = 0.0;
  __device__ __forceinline__ void term(double r, double i) {
    sr += r;
    si += i;
  }
  __device__ __forceinline__ void flush() {}
  __device__ __forceinline__ double2 value() const { return make_double2(sr, si); }
};

// Per-term constants of one tile, staged in LDS next to the tables: the gamma
// low-bit plane, whether the term is packed, and the nine values a term can
// add, ph[k] = b_alpha 2^{-|v|/2} e^{i pi (k + omega) / 4} for k = 0..7 and
// ph[8] = 0, so that a lane picks its value with one lookup.
template <typename T>
struct TileTerm {
  uint64_t glo;
  uint32_t packed, pad;
  T ph[9][2];
};

// Prologue: per term, the rows c_q of B (stored like F: c[q * chi + a]), for
// a packed term with F_q gathered from the ~v positions above bit n, and the
// constants.  kPrepSplit threads per term, thread (part, lane) of a 256-thread
// block taking rows q = part (mod kPrepSplit) of term kPrepTerms block + lane
// (short serial chains: a row costs q + 1 parities); F rows of the block's
// terms are parked in LDS, and the low bits of gamma are gathered by the same
// split and combined through LDS.
constexpr uint32_t kPrepTerms = 16;
constexpr uint32_t kPrepSplit = 256 / kPrepTerms;
__global__ __launch_bounds__(256) void k_amp_prep(TermsView T, uint64_t* __restrict__ crow,
                                                  AmpTerm* __restrict__ cst) {
  extern __shared__ __align__(16) uint8_t smem[];
  uint64_t* gpart = reinterpret_cast<uint64_t*>(smem);  // [kPrepSplit][kPrepTerms]
  uint64_t* Fs = gpart + kPrepSplit * kPrepTerms;       // [n][kPrepTerms]
  const uint32_t lane = threadIdx.x % kPrepTerms, part = threadIdx.x / kPrepTerms;
  const uint64_t chi = T.chi;
  const uint64_t a = (uint64_t)blockIdx.x * kPrepTerms + lane;
  const bool on = a < chi;
  const uint32_t n = T.n;
  uint64_t glo = 0;
  if (on)
    for (uint32_t p = part; p < n; p += kPrepSplit) {
      Fs[p * kPrepTerms + lane] = T.F[(uint64_t)p * chi + a];
      glo |= (uint64_t)(T.gamma[(uint64_t)p * chi + a] & 1u) << p;
    }
  gpart[part * kPrepTerms + lane] = glo;
  __syncthreads();
  if (!on) return;  // no barrier follows
  const uint64_t xm = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
  const uint64_t v = T.v[a], s = T.s[a];
  const uint64_t vs = v & s;
  const uint64_t nv = ~v & xm;
  const uint32_t nfree = (uint32_t)__popcll(nv);
  const bool packed = nfree <= 64u - n;  // n + nfree <= 64; nfree > 0 implies n < 64
  for (uint32_t q = part; q < n; q += kPrepSplit) {
    const uint64_t Mq = T.M[(uint64_t)q * chi + a];
    const uint32_t ghi_q = (T.gamma[(uint64_t)q * chi + a] >> 1) & 1u;
    uint64_t col = 0;
    for (uint32_t p = 0; p <= q; ++p) col |= (uint64_t)par64(Fs[p * kPrepTerms + lane] & Mq) << p;
    col ^= (uint64_t)(ghi_q ^ par64(Fs[q * kPrepTerms + lane] & vs)) << q;
    if (packed && nfree != 0u) col |= gather_bits(Fs[q * kPrepTerms + lane], nv) << n;
    crow[(uint64_t)q * chi + a] = col;
  }
  if (part != 0) return;
  glo = 0;
  for (uint32_t k = 0; k < kPrepSplit; ++k) glo |= gpart[k * kPrepTerms + lane];
  AmpTerm c;
  c.nv = nv;
  c.snv = !packed ? (s & nv) : (nfree != 0u ? gather_bits(s, nv) << n : 0ull);
  c.glo = glo;
  c.w = T.omega[a];
  c.packed = packed ? 1u : 0u;
  const double2 b = T.b[a];
  const int vc = __popcll(v);
  const double h = 0.70710678118654752440;
  const double mag = ldexp(1.0, -(vc >> 1)) * ((vc & 1) ? h : 1.0);
  c.w0r = b.x * mag;
  c.w0i = b.y * mag;
  c.w1r = (c.w0r - c.w0i) * h;
  c.w1i = (c.w0r + c.w0i) * h;
  cst[a] = c;
}

// Build the tables of terms base .. base + kTT - 1.  Thread (t, kind, c)
// builds chunk c of term t's table `kind` (0: u from F with s folded into
// chunk 0 and masked with ~v, not built for a packed term; 1: w from the c
// rows, for a packed term with the gathered s folded into chunk 0), 16 entries by the
// recurrence e[j] = e[j & (j - 1)] ^ row[ctz j].  Entry e of chunk c sits at
// word c * 16 + (e ^ c): the 16 lanes writing one entry index of 16 chunks,
// and the lanes reading 16 different entries of one chunk, hit distinct banks.
template <typename T>
__device__ __forceinline__ void build_tables(uint64_t* tab, TileTerm<T>* tt, const AmpInst& I,
                                             uint64_t base, uint32_t nch, uint32_t tid) {
  const uint32_t t = tid >> 5, kind = (tid >> 4) & 1u, c = tid & 15u;
  const uint64_t chi = I.T.chi;
  const uint64_t a = base + t;
  if (a >= chi) return;
  const AmpTerm& C = I.cst[a];
  if (kind == 1 && c < 9) {
    // Value k of the term: w0 (k even) or w1 (k odd) times i^(k >> 1), with
    // k counted from omega; exact in T (a rounding, then a swap and signs).
    T re = (T)0, im = (T)0;
    if (c < 8) {
      const uint32_t k = (c + C.w) & 7u;
      re = (k & 1u) ? (T)C.w1r : (T)C.w0r;
      im = (k & 1u) ? (T)C.w1i : (T)C.w0i;
      const uint32_t m = k >> 1;
      if (m & 1u) {
        const T tmp = re;
        re = im;
        im = tmp;
      }
      if ((m ^ (m >> 1)) & 1u) re = -re;
      if (m & 2u) im = -im;
    }
    tt[t].ph[c][0] = re;
    tt[t].ph[c][1] = im;
    if (c == 0) {
      tt[t].glo = C.glo;
      tt[t].packed = C.packed;
    }
  }
  if (c >= nch) return;
  const uint32_t n = I.T.n;
  const uint64_t* rows = kind ? I.crow : I.T.F;
  if (kind == 0 && C.packed) return;
  uint64_t r[4];
  uint64_t mask = ~0ull, e0 = 0;
  if (kind == 0) mask = C.nv;
  if (kind == 0 || C.packed) e0 = (c == 0) ? C.snv : 0ull;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const uint32_t p = 4u * c + (uint32_t)b;
    r[b] = (p < n) ? (rows[(uint64_t)p * chi + a] & mask) : 0ull;
  }
  uint64_t e[16];
  e[0] = e0;
#pragma unroll
  for (int j = 1; j < 16; ++j) e[j] = e[j & (j - 1)] ^ r[__builtin_ctz(j)];
  uint64_t* dst = tab + (t * 2u + kind) * kTabWords + c * 16u;
#pragma unroll
  for (int j = 0; j < 16; ++j) dst[(uint32_t)j ^ c] = e[j];
}

// Terms of one tile against the lane's XPL bitstrings.  off[j][c] is the
// swizzled word offset of chunk c's entry for bitstring j; hi masks the bits
// above n, where a packed term keeps its zero test.
template <typename T>
__device__ __forceinline__ void add_term(const TileTerm<T>& K, uint64_t glo, uint64_t x, uint64_t w,
                                         bool nz, Acc<T>& acc) {
  const uint32_t k = (2u * (uint32_t)__popcll(x & glo) + 4u * (uint32_t)__popcll(x & w)) & 7u;
  const uint32_t idx = nz ? k : 8u;
  acc.term(K.ph[idx][0], K.ph[idx][1]);
}

template <typename T, int NCH, int XPL>
__device__ __forceinline__ void run_tile(const uint64_t* tab, const TileTerm<T>* tt,
                                         uint32_t tcount, uint64_t hi,
                                         const uint32_t (&off)[XPL][kMaxCh],
                                         const uint64_t (&x)[XPL], const bool (&live)[XPL],
                                         Acc<T> (&acc)[XPL]) {
#pragma unroll
  for (int t = 0; t < kTT; ++t) {
    if ((uint32_t)t >= tcount) break;
    const uint64_t* tu = tab + (t * 2) * kTabWords;
    const uint64_t* tw = tu + kTabWords;
    const TileTerm<T>& K = tt[t];
    const uint64_t glo = uniform64(K.glo);
    if (uniform32(K.packed)) {
#pragma unroll
      for (int j = 0; j < XPL; ++j) {
        uint64_t w = 0;
#pragma unroll
        for (int c = 0; c < NCH; ++c) w ^= tw[off[j][c]];
        const bool nz = live[j] && (w & hi) == 0ull;
        if (__ballot(nz) == 0ull) continue;
        add_term<T>(K, glo, x[j], w, nz, acc[j]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < XPL; ++j) {
        uint64_t u = 0;
#pragma unroll
        for (int c = 0; c < NCH; ++c) u ^= tu[off[j][c]];
        const bool nz = live[j] && u == 0ull;
        if (__ballot(nz) == 0ull) continue;
        uint64_t w = 0;
#pragma unroll
        for (int c = 0; c < NCH; ++c) w ^= tw[off[j][c]];
        add_term<T>(K, glo, x[j], w, nz, acc[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < XPL; ++j) acc[j].flush();
}

template <typename T, int XPL>
__global__ __launch_bounds__(256) void k_amp(const AmpInst* __restrict__ insts,
                                             const AmpItem* __restrict__ items, uint32_t n_items,
                                             uint32_t* __restrict__ counter) {
  __shared__ __align__(16) uint64_t tab[kTT * 2 * kTabWords];  // 32 KiB
  __shared__ __align__(16) TileTerm<T> tt[kTT];
  __shared__ uint32_t s_item;
  const uint32_t tid = threadIdx.x;

  for (;;) {
    // Persistent workgroups pull (request, tile range, bitstring chunk) items.
    if (tid == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t it = uniform32(s_item);
    __syncthreads();
    if (it >= n_items) break;
    const AmpItem item = items[it];
    const AmpInst& I = insts[item.inst];
    const uint32_t n = I.T.n;
    const uint64_t chi = I.T.chi;
    const uint32_t nch = (n + 3u) / 4u;
    const uint64_t xmask = (n == 64) ? ~0ull : ((1ull << n) - 1ull);

    uint64_t x[XPL];
    bool live[XPL];
    uint32_t off[XPL][kMaxCh];
    Acc<T> acc[XPL];
#pragma unroll
    for (int j = 0; j < XPL; ++j) {
      const uint32_t xi = item.x0 + (uint32_t)j * 256u + tid;
      live[j] = xi < item.x1;
      x[j] = live[j] ? (I.x[xi] & xmask) : 0ull;  // bits >= n never index a row
#pragma unroll
      for (int c = 0; c < kMaxCh; ++c)
        off[j][c] = (uint32_t)c * 16u + (((uint32_t)(x[j] >> (4 * c)) & 15u) ^ (uint32_t)c);
    }

    const uint64_t tiles = (chi + kTT - 1) / kTT;
    const uint64_t t0 = (uint64_t)item.range * I.tiles_per_range;
    const uint64_t t1 = std::min<uint64_t>(tiles, t0 + I.tiles_per_range);
    for (uint64_t tile = t0; tile < t1; ++tile) {
      const uint64_t base = tile * kTT;
      const uint32_t tcount = (uint32_t)std::min<uint64_t>((uint64_t)kTT, chi - base);
      __syncthreads();  // the previous tile's readers are done
      build_tables<T>(tab, tt, I, base, nch, tid);
      __syncthreads();
      switch (nch) {
#define CHSIM_AMP_CASE(K)                                         \
  case K:                                                         \
    run_tile<T, K, XPL>(tab, tt, tcount, ~xmask, off, x, live, acc); \
    break;
        CHSIM_AMP_CASE(1) CHSIM_AMP_CASE(2) CHSIM_AMP_CASE(3) CHSIM_AMP_CASE(4)
        CHSIM_AMP_CASE(5) CHSIM_AMP_CASE(6) CHSIM_AMP_CASE(7) CHSIM_AMP_CASE(8)
        CHSIM_AMP_CASE(9) CHSIM_AMP_CASE(10) CHSIM_AMP_CASE(11) CHSIM_AMP_CASE(12)
        CHSIM_AMP_CASE(13) CHSIM_AMP_CASE(14) CHSIM_AMP_CASE(15) CHSIM_AMP_CASE(16)
#undef CHSIM_AMP_CASE
        default:
          break;
      }
    }
#pragma unroll
    for (int j = 0; j < XPL; ++j) {
      const uint32_t xi = item.x0 + (uint32_t)j * 256u + tid;
      if (live[j]) I.partial[(uint64_t)item.range * I.n_x + xi] = acc[j].value();
    }
  }
}

__global__ void k_reset_counter(uint32_t* counter) { *counter = 0u; }

// out[i] = sum over tile ranges of partial[range][i], FP64, in a fixed order:
// a 256-thread block takes 16 bitstrings (over all requests) and 16 slices of
// their ranges; a thread sums its slice in range order, and the slice sums
// are added in slice order.
constexpr uint32_t kRedX = 16, kRedSlices = 16;
__global__ __launch_bounds__(256) void k_reduce_ranges(const AmpInst* __restrict__ insts,
                                                       const uint64_t* __restrict__ prefix,
                                                       uint32_t n_inst) {
  __shared__ double2 part[kRedSlices][kRedX];
  const uint32_t xl = threadIdx.x % kRedX, sl = threadIdx.x / kRedX;
  const uint64_t g = (uint64_t)blockIdx.x * kRedX + xl;
  const bool on = g < prefix[n_inst];
  uint32_t lo = 0;
  uint64_t i = 0;
  double r = 0.0, im = 0.0;
  if (on) {
    uint32_t hi = n_inst;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (prefix[mid] <= g) lo = mid;
      else hi = mid;
    }
    const AmpInst& I = insts[lo];
    i = g - prefix[lo];
    const uint32_t r0 = (uint32_t)((uint64_t)I.n_ranges * sl / kRedSlices);
    const uint32_t r1 = (uint32_t)((uint64_t)I.n_ranges * (sl + 1) / kRedSlices);
    for (uint32_t t = r0; t < r1; ++t) {
      const double2 v = I.partial[(uint64_t)t * I.n_x + i];
      r += v.x;
      im += v.y;
    }
  }
  part[sl][xl] = make_double2(r, im);
  __syncthreads();
  if (sl != 0 || !on) return;
  double sr = 0.0, si = 0.0;
  for (uint32_t k = 0; k < kRedSlices; ++k) {
    sr += part[k][xl].x;
    si += part[k][xl].y;
  }
  insts[lo].out[i] = make_double2(sr, si);
}

}  // namespace

hipError_t launch_amp_prep(const TermsView& T, uint64_t* crow, AmpTerm* cst, hipStream_t st) {
  const uint32_t blocks = (uint32_t)((T.chi + kPrepTerms - 1) / kPrepTerms);
  const size_t sm = ((size_t)T.n + kPrepSplit) * kPrepTerms * sizeof(uint64_t);
  hipLaunchKernelGGL(k_amp_prep, dim3(blocks), dim3(256), sm, st, T, crow, cst);
  return hipGetLastError();
}

void amp_plan(const std::vector<AmpRequestPlan>& reqs, uint32_t target_items, uint32_t xpl,
              std::vector<AmpItem>& items, std::vector<uint32_t>& tiles_per_range,
              std::vector<uint32_t>& n_ranges) {
  const uint32_t kXChunk = 256u * xpl;  // bitstrings per work item
  uint64_t total_tiles = 0, chunks_total = 0;
  for (const auto& r : reqs) {
    total_tiles += (r.chi + kTT - 1) / kTT;
    chunks_total += (r.n_x + kXChunk - 1) / kXChunk;
  }
  items.clear();
  tiles_per_range.assign(reqs.size(), 1);
  n_ranges.assign(reqs.size(), 1);
  // One range length for all requests, so that the item count reaches the
  // target; between 1 and 512 tiles per range.
  uint64_t per = 1;
  if (total_tiles > 0 && chunks_total > 0) {
    const double avg_chunks = (double)chunks_total / (double)reqs.size();
    const double want_ranges = (double)target_items / avg_chunks;
    per = (uint64_t)((double)total_tiles / want_ranges);
    per = std::min<uint64_t>(std::max<uint64_t>(per, 1), 512);
  }
  for (uint32_t q = 0; q < reqs.size(); ++q) {
    const auto& r = reqs[q];
    const uint64_t tiles = (r.chi + kTT - 1) / kTT;
    tiles_per_range[q] = (uint32_t)per;
    n_ranges[q] = (uint32_t)((tiles + per - 1) / per);
    for (uint32_t rg = 0; rg < n_ranges[q]; ++rg)
      for (uint32_t x0 = 0; x0 < r.n_x; x0 += kXChunk)
        items.push_back(AmpItem{q, rg, x0, std::min<uint32_t>(r.n_x, x0 + kXChunk)});
  }
  // Longest first: cost ~ terms x bitstrings x (ceil(n / 4) lookups + constant).
  auto cost = [&](const AmpItem& it) {
    const auto& r = reqs[it.inst];
    const uint64_t tiles = (r.chi + kTT - 1) / kTT;
    const uint64_t t0 = (uint64_t)it.range * tiles_per_range[it.inst];
    const uint64_t nt = std::min<uint64_t>(tiles, t0 + tiles_per_range[it.inst]) - t0;
    return (double)nt * (double)(it.x1 - it.x0) * (double)((r.n + 3) / 4 + 4);
  };
  std::stable_sort(items.begin(), items.end(),
                   [&](const AmpItem& a, const AmpItem& b) { return cost(a) > cost(b); });
}

namespace {

// Plan of one request written on the device: the request record, the
// bitstring prefix [0, n_x], and item i = (range i / chunks, chunk i % chunks).
// Items are independent (each writes its own partials), so their order does
// not change the result.
__global__ __launch_bounds__(256) void k_fill_single_plan(AmpInst inst, AmpInst* insts_d, AmpItem* items_d,
                                                          uint64_t* prefix_d, uint32_t n_items,
                                                          uint32_t chunks, uint32_t x_chunk) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    insts_d[0] = inst;
    prefix_d[0] = 0ull;
    prefix_d[1] = inst.n_x;
  }
  if (i >= n_items) return;
  const uint32_t rg = i / chunks, c = i % chunks;
  const uint32_t x0 = c * x_chunk;
  const uint32_t x1 = x0 + x_chunk < inst.n_x ? x0 + x_chunk : inst.n_x;
  items_d[i] = AmpItem{0u, rg, x0, x1};
}

}  // namespace

void amp_plan_single(uint64_t chi, uint32_t n_x, uint32_t target_items, uint32_t xpl, uint32_t* tiles_per_range,
                     uint32_t* n_ranges, uint32_t* chunks) {
  // The range length amp_plan chooses for one request.
  const uint32_t x_chunk = 256u * xpl;
  const uint64_t tiles = (chi + kTT - 1) / kTT;
  const uint64_t ch = (n_x + x_chunk - 1) / x_chunk;
  uint64_t per = 1;
  if (tiles > 0 && ch > 0) {
    const double want_ranges = (double)target_items / (double)ch;
    per = (uint64_t)((double)tiles / want_ranges);
    per = std::min<uint64_t>(std::max<uint64_t>(per, 1), 512);
  }
  *tiles_per_range = (uint32_t)per;
  *n_ranges = (uint32_t)((tiles + per - 1) / per);
  *chunks = (uint32_t)ch;
}

hipError_t launch_amp_fill_single(const AmpInst& inst, AmpInst* insts_d, AmpItem* items_d, uint64_t* prefix_d,
                                  uint32_t n_items, uint32_t chunks, uint32_t xpl, hipStream_t st) {
  const uint32_t blocks = (n_items + 255u) / 256u;
  hipLaunchKernelGGL(k_fill_single_plan, dim3(blocks ? blocks : 1), dim3(256), 0, st, inst, insts_d, items_d,
                     prefix_d, n_items, chunks, 256u * xpl);
  return hipGetLastError();
}

hipError_t launch_amp_items(const AmpInst* insts_d, const AmpItem* items_d, uint32_t n_items,
                            uint32_t* counter, bool fp32c, uint32_t xpl, const uint64_t* prefix_d,
                            uint32_t n_inst, uint64_t total_x, hipStream_t st) {
  if (xpl != 1u && xpl != 2u) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Kernel variant (FP32C or FP64, 1 or 2 bitstrings per lane).
  const int var = (fp32c ? 2 : 0) + (int)(xpl - 1u);
  const void* fns[4] = {(const void*)k_amp<double, 1>, (const void*)k_amp<double, 2>,
                        (const void*)k_amp<float, 1>, (const void*)k_amp<float, 2>};
  // Compute units and resident workgroups per unit, queried once per device.
  constexpr int kMaxDev = 64;
  static int cached_cus[kMaxDev] = {}, cached_per_cu[kMaxDev][4] = {};
  int dev = 0;
  hipGetDevice(&dev);
  const int di = (dev >= 0 && dev < kMaxDev) ? dev : 0;
  int cus = cached_cus[di];
  if (cus <= 0) {
    cus = 256;
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    cached_cus[di] = cus;
  }
  int per_cu = cached_per_cu[di][var];
  if (per_cu <= 0) {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fns[var], 256, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    cached_per_cu[di][var] = per_cu;
  }
  uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)n_items, (uint64_t)cus * per_cu);
  if (grid == 0) grid = 1;
  switch (var) {
    case 0: hipLaunchKernelGGL((k_amp<double, 1>), dim3(grid), dim3(256), 0, st, insts_d, items_d, n_items, counter); break;
    case 1: hipLaunchKernelGGL((k_amp<double, 2>), dim3(grid), dim3(256), 0, st, insts_d, items_d, n_items, counter); break;
    case 2: hipLaunchKernelGGL((k_amp<float, 1>), dim3(grid), dim3(256), 0, st, insts_d, items_d, n_items, counter); break;
    default: hipLaunchKernelGGL((k_amp<float, 2>), dim3(grid), dim3(256), 0, st, insts_d, items_d, n_items, counter); break;
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint32_t blocks = (uint32_t)((total_x + kRedX - 1) / kRedX);
  hipLaunchKernelGGL(k_reduce_ranges, dim3(blocks), dim3(256), 0, st, insts_d, prefix_d, n_inst);
  return hipGetLastError();
}

}  // namespace chsim
