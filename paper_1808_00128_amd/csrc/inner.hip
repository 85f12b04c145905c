// Inner products <phi_A|phi_alpha> with equatorial states and the norm
// estimate (step (c) of the hot path).
//
// Lemma (Inner Product): with J = diag(gamma) + offdiag(M F^T mod 2) and
// K = G^T (A + J) G (off-diagonal mod 2, diagonal mod 4),
//   <phi|phi_A> = 2^{-(n+|v|)/2} i^{s K s^T} (-1)^{s.v} Z(B),
// B = K + 2 diag(s + sK) restricted to supp(v).  Lemma (Exponential Sum):
// Z(B) through the Z_2 form on |v| + 1 variables of Eq. (Q) and its real and
// imaginary parts, Eq. (real), each evaluated by eliminating pairs of
// variables with the identity sum_{x1,x2} (-1)^{x1 x2 + mu1 x1 + mu2 x2} =
// 2 (-1)^{mu1 mu2} (Eq. (eq5)).
//
// Mapping.  A per-term prologue (one wave per term, lane = row) stores the
// term's rows and columns of G and K_J = G^T J G with the vectors the pair
// step needs, restricted to supp(v) and compressed to |v| bits (only the
// variables in supp(v) enter B); K_J is shared by every equatorial state
// since K is linear in A + J.  The pair kernel gives each lane one
// equatorial state A (64 per wave) and walks the terms (pair_term below);
// with |v| < 32 every word of a term's Z_2 form fits 32 bits.
#include <algorithm>

#include "device_common.hpp"
#include "internal.hpp"

namespace chsim {

// All ones if bit b (< 32) of x is set, else zero.
__device__ __forceinline__ uint32_t bit_mask32(uint32_t x, uint32_t b) {
  return (uint32_t)__builtin_amdgcn_sbfe((int)x, b, 1u);
}

namespace {

constexpr int kWaves = 4;

// OR of x over the wave's lanes (a superset when some lanes are inactive:
// DPP and swizzles read their registers as they are).
__device__ __forceinline__ uint32_t wave_or32(uint32_t x) {
  x |= (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, true);
  x |= (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, true);
  x |= (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x141, 0xF, 0xF, true);
  x |= (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x140, 0xF, 0xF, true);
  x |= (uint32_t)__shfl_xor((int)x, 16);
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 0) | (uint32_t)__builtin_amdgcn_readlane((int)x, 32);
}

// K = G^T X G for X in M_n given by rows: lane c holds Xoff_c (bit d = X_cd,
// d != c) and Xdiag_c in Z_4.  G: lane c holds row G_c; Gt: lane a holds
// column a of G (bit c = G_ca).  Returns lane a's row of K (off-diagonal bits)
// and K_aa mod 4.
__device__ __forceinline__ void conj_gxg(uint64_t G, uint64_t Gt, uint64_t Xoff, uint32_t Xdiag,
                                         uint32_t lane, uint32_t n, uint64_t& Koff,
                                         uint32_t& Kdiag) {
  const uint64_t lb = 1ull << lane;
  const bool act = lane < n;
  const uint64_t Xrow = act ? ((Xoff & ~lb) | ((uint64_t)(Xdiag & 1u) << lane)) : 0ull;
  const uint64_t upper = (lane == 63u) ? 0ull : (~0ull << (lane + 1u));
  const uint64_t Urow = act ? (Xoff & upper) : 0ull;
  uint64_t Y = 0, YU = 0;
  for (uint32_t c = 0; c < n; ++c) {
    const uint64_t Xc = rl64(Xrow, c), Uc = rl64(Urow, c);
    const uint64_t m = bitmask64(Gt, c);
    Y ^= Xc & m;
    YU ^= Uc & m;
  }
  uint64_t K = 0;
  for (uint32_t d = 0; d < n; ++d) {
    const uint64_t Gd = rl64(G, d);
    K ^= Gd & bitmask64(Y, d);
  }
  const uint64_t xdlo = ballot64(act && (Xdiag & 1u)), xdhi = ballot64(act && (Xdiag & 2u));
  Kdiag = ((uint32_t)__popcll(Gt & xdlo) + 2u * (uint32_t)__popcll(Gt & xdhi) +
           2u * par64(YU & Gt)) & 3u;
  Koff = act ? (K & ~lb) : 0ull;
}

struct InnerRec {
  uint32_t nonzero, k8;
  int e2;
};

__device__ __forceinline__ double2 rec_value(const InnerRec& r, double2 b) {
  const double h = 0.70710678118654752440;
  const int e2 = r.e2;
  // 2^{e2/2}; for odd e2 it is 2^{(e2-1)/2} sqrt(2) ((e2 - 1) is even, so the division is exact).
  const double mag = (e2 & 1) ? ldexp(1.41421356237309504880, (e2 - 1) / 2) : ldexp(1.0, e2 / 2);
  double cr, ci;
  switch (r.k8) {
    case 0: cr = 1; ci = 0; break;
    case 1: cr = h; ci = h; break;
    case 2: cr = 0; ci = 1; break;
    case 3: cr = -h; ci = h; break;
    case 4: cr = -1; ci = 0; break;
    case 5: cr = -h; ci = -h; break;
    case 6: cr = 0; ci = -1; break;
    default: cr = h; ci = -h; break;
  }
  return make_double2(mag * (b.x * cr - b.y * ci), mag * (b.x * ci + b.y * cr));
}

// Per-term record (words), in the term's compressed variables: bit a' of a
// compressed word stands for the a'-th qubit of supp(v) (in increasing
// order), and the pair step's Z_2 form has one more variable, index |v|.
//   [0, n):      row c of G restricted to supp(v), compressed (lane c);
//   [n, 2n):     column a of G for the a'-th qubit a of supp(v), at a' (zero
//                past |v|);
//   [2n, 3n):    row a of K_J off its diagonal, restricted to supp(v) and
//                compressed, at a';
//   3n, 3n + 1:  diag(K_J) low and high bit planes, compressed;
//   3n + 2:      (s K_J) with the diagonal low bits, compressed;
//   3n + 3:      y = G s (over all rows);
//   3n + 4:      s K_J s^T mod 4;
//   3n + 5:      s, compressed.
__host__ __device__ constexpr uint32_t inner_rec_words(uint32_t n) { return 3u * n + 6u; }

// The bits of x at the set positions of m, packed from bit 0 up (m
// wave-uniform).
__device__ __forceinline__ uint64_t gather_bits(uint64_t x, uint64_t m) {
  uint64_t out = 0;
  for (uint32_t k = 0; m; m &= m - 1ull, ++k) out |= ((x >> __builtin_ctzll(m)) & 1ull) << k;
  return out;
}

__global__ __launch_bounds__(256) void k_inner_prep(TermsView Tv, uint64_t* __restrict__ rec) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t n = Tv.n;
  const bool act = lane < n;
  const uint64_t term = (uint64_t)blockIdx.x * kWaves + uniform32(tid >> 6);
  if (term >= Tv.chi) return;  // whole wave
  const uint64_t chi = Tv.chi;
  const uint64_t off = (uint64_t)lane * chi + term;
  const uint64_t F = act ? Tv.F[off] : 0ull;
  const uint64_t G = act ? Tv.G[off] : 0ull;
  const uint64_t M = act ? Tv.M[off] : 0ull;
  const uint32_t g = act ? Tv.gamma[off] : 0u;
  const uint64_t s = uniform64(Tv.s[term]);
  // Column `lane` of G.
  uint64_t Gt = 0;
  for (uint32_t a = 0; a < n; ++a) {
    const uint64_t col = ballot64(((G >> a) & 1ull) != 0ull);
    if (lane == a) Gt = col;
  }
  // J: diag gamma, J_ab = par(M_a & F_b) for a != b.
  uint64_t Joff = 0;
  for (uint32_t bb = 0; bb < n; ++bb) {
    const uint64_t Fb = rl64(F, bb);
    Joff |= (uint64_t)par64(M & Fb) << bb;
  }
  uint64_t KJoff;
  uint32_t KJdiag;
  conj_gxg(G, Gt, Joff, g, lane, n, KJoff, KJdiag);
  const uint64_t Krow = act ? (KJoff | ((uint64_t)(KJdiag & 1u) << lane)) : 0ull;
  const uint64_t kdlo = ballot64(act && (KJdiag & 1u)), kdhi = ballot64(act && (KJdiag & 2u));
  const uint64_t skj = ballot64(act && par64(s & Krow));
  const uint64_t upper = (lane == 63u) ? 0ull : (~0ull << (lane + 1u));
  const uint64_t pairs = ballot64(act && ((s >> lane) & 1ull) && par64(KJoff & s & upper));
  const uint32_t sks = ((uint32_t)__popcll(s & kdlo) + 2u * (uint32_t)__popcll(s & kdhi) +
                        2u * (uint32_t)__popcll(pairs)) & 3u;
  const uint64_t y = ballot64(act && par64(G & s));
  const uint64_t v = uniform64(Tv.v[term]);
  // Lane a' gathers column a and row a of K_J of the a'-th qubit a of supp(v).
  uint64_t colc = 0, kjc = 0;
  {
    uint32_t k = 0;
    for (uint64_t m = v; m; m &= m - 1ull, ++k) {
      const uint32_t a = (uint32_t)__builtin_ctzll(m);
      const uint64_t ca = rl64(Gt, a), ka = rl64(KJoff, a);
      if (lane == k) {
        colc = ca;
        kjc = ka;
      }
    }
  }
  uint64_t* r = rec + term * inner_rec_words(n);
  if (act) {
    r[lane] = gather_bits(G, v);
    r[n + lane] = colc;
    r[2u * n + lane] = gather_bits(kjc, v);  // K_J's diagonal is not in KJoff
  }
  if (lane == 0) {
    r[3u * n] = gather_bits(kdlo, v);
    r[3u * n + 1u] = gather_bits(kdhi, v);
    r[3u * n + 2u] = gather_bits(skj, v);
    r[3u * n + 3u] = y;
    r[3u * n + 4u] = sks;
    r[3u * n + 5u] = gather_bits(s, v);
  }
}

// A as 64-state columns: at[c][l] = row c of A_l with its diagonal low bit
// at c, and the diagonal bit planes of every state (zero past L).
__global__ __launch_bounds__(256) void k_inner_atrans(const uint64_t* __restrict__ Aoff,
                                                      const uint8_t* __restrict__ Adiag, uint32_t n,
                                                      uint32_t L, uint32_t Lp, uint64_t* __restrict__ at,
                                                      uint64_t* __restrict__ planes) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= Lp) return;
  uint64_t lo = 0, hi = 0;
  for (uint32_t c = 0; c < n; ++c) {
    uint64_t row = 0;
    if (l < L) {
      const uint32_t d = Adiag[(uint64_t)l * n + c];
      row = (Aoff[(uint64_t)l * n + c] & ~(1ull << c)) | ((uint64_t)(d & 1u) << c);
      lo |= (uint64_t)(d & 1u) << c;
      hi |= (uint64_t)((d >> 1) & 1u) << c;
    }
    at[(uint64_t)c * Lp + l] = row;
  }
  planes[l] = lo;
  planes[Lp + l] = hi;
}

template <typename Word>
__device__ __forceinline__ Word rlw(Word x, uint32_t src);
template <>
__device__ __forceinline__ uint32_t rlw<uint32_t>(uint32_t x, uint32_t src) {
  return rl32(x, src);
}
template <>
__device__ __forceinline__ uint64_t rlw<uint64_t>(uint64_t x, uint32_t src) {
  return rl64(x, src);
}
// All ones if bit 0 of b is set.
template <typename Word>
__device__ __forceinline__ Word wmask(uint64_t b) {
  return (Word)0 - (Word)(b & 1u);
}

// One term against the wave's 64 equatorial states (lane = state), in the
// term's compressed variables (bit a' = the a'-th qubit of supp(v)): Word is
// 32 bits when the Z_2 form's |v| + 1 variables fit, else 64.  Everything
// that depends only on the term is wave-uniform:
//   Z_c = A_c G and W_c = U_c G (U = strictly upper part of A) by lookup in
//   tables of XORs of G's rows, four rows per table (Four Russians);
//   K_A on supp(v): row a = XOR of Z_c over c with G_ca = 1;
//   diag(K_A) mod 4 = G-column popcounts against A's diagonal planes plus
//   2 (XOR_c G_c & W_c);  (s K_A) = XOR_c G_c [A_c . y] and
//   s K_A s^T = y^T A y mod 4 with y = G s.
// Each lane then eliminates its own Z_2 form (rows in LDS, pivots chosen per
// lane) and adds b_alpha <phi_A|phi_alpha> to its state's sum.
template <typename Word, int NS, int NMAX>
__device__ __forceinline__ void pair_term(const uint64_t* __restrict__ r, uint32_t n, uint32_t nv, uint32_t lane,
                                          uint32_t l, uint32_t L, const uint64_t* __restrict__ atl, uint32_t Lp,
                                          uint64_t adlo, uint64_t adhi, uint32_t omega, uint32_t sv, double2 bb,
                                          Word* __restrict__ gtab, void* __restrict__ srow, double& accr,
                                          double& acci) {
  constexpr uint32_t kChunks = (NMAX + 3) / 4;
  const Word Gl = lane < n ? (Word)r[lane] : (Word)0;
  const uint64_t Gtl = lane < nv ? r[n + lane] : 0ull;
  const Word KJl = lane < nv ? (Word)r[2u * n + lane] : (Word)0;
  const Word kjdlo = (Word)uniform64(r[3u * n]), kjdhi = (Word)uniform64(r[3u * n + 1u]);
  const Word skj = (Word)uniform64(r[3u * n + 2u]);
  const uint64_t y = uniform64(r[3u * n + 3u]);
  const uint32_t sksj = uniform32((uint32_t)r[3u * n + 4u]);
  const Word sc = (Word)uniform64(r[3u * n + 5u]);
  // Lookup tables: gtab[k][e] = XOR of G rows 4k + i over the bits i of e
  // (zero for chunks at or past n, so every chunk of NMAX can be looked up).
  for (uint32_t k = 0; k < kChunks; ++k) {
    Word t = 0;
    for (uint32_t i = 0; i < 4u; ++i) {
      const uint32_t row = 4u * k + i;
      if (row < n) t ^= rlw<Word>(Gl, row) & wmask<Word>(lane >> i);
    }
    if (lane < 16u) gtab[k * 16u + lane] = t;
  }
  __builtin_amdgcn_wave_barrier();
  // With 64-bit words the rows of only 32 lanes fit the LDS region at once:
  // the two halves of the wave take the term one after the other.
  constexpr bool kWide = sizeof(Word) == 8;
  const uint32_t stride = kWide ? 32u : 64u, slot = kWide ? (lane & 31u) : lane;
  Word* const S = reinterpret_cast<Word*>(srow);
  for (uint32_t h = 0; h < (kWide ? 2u : 1u); ++h) {
    if (kWide && (lane >> 5) != h) continue;
    // One pass over A's rows.
    Word Sacc[NS];
#pragma unroll
    for (int a = 0; a < NS; ++a) Sacc[a] = 0;
    Word D = 0, sKA = 0;
    uint64_t tU = 0;
    uint64_t Anext = atl[0];
    for (uint32_t c = 0; c < n; ++c) {
      const Word Gc = rlw<Word>(Gl, c);
      const uint64_t Ac = Anext;
      if (c + 1u < n) Anext = atl[(uint64_t)(c + 1u) * Lp];  // next row in flight
      const uint64_t upc = (c == 63u) ? 0ull : (~0ull << (c + 1u));
      const uint64_t Uc = Ac & upc;
      // Z_c = A_c G and W_c = U_c G from the tables: every chunk's lookup is
      // issued at once; above the chunk holding c the nibbles of A_c and U_c
      // agree, that chunk takes a lookup of its own, below it U_c is zero.
      const uint32_t kc = c >> 2;
      Word tz[kChunks];
#pragma unroll
      for (uint32_t k = 0; k < kChunks; ++k) tz[k] = gtab[k * 16u + (uint32_t)((Ac >> (4u * k)) & 15ull)];
      Word W = gtab[kc * 16u + (uint32_t)((Uc >> (4u * kc)) & 15ull)];
      Word Z = 0;
#pragma unroll
      for (uint32_t k = 0; k < kChunks; ++k) {
        Z ^= tz[k];
        W ^= tz[k] & wmask<Word>(k > kc);
      }
      D ^= Gc & W;
      sKA ^= Gc & wmask<Word>(par64(Ac & y));
      if ((y >> c) & 1ull) tU ^= Uc & y;
      // K_A rows on supp(v): S_a ^= Z_c for the a with G_ca = 1 (a uniform
      // test per row: only those rows do any vector work).
#pragma unroll
      for (int a = 0; a < NS; ++a)
        if ((Gc >> a) & 1u) Sacc[a] ^= Z;
    }
    // B on supp(v): Bd_a = K_aa + 2 (s_a + (sK)_a) with K = K_J + K_A.
    const Word skl = skj ^ sKA;
    Word kap = 0, lam = 0;
    for (uint32_t a = 0; a < nv; ++a) {
      const uint64_t ga = rl64(Gtl, a);
      const uint32_t kd = (uint32_t)((kjdlo >> a) & 1u) + 2u * (uint32_t)((kjdhi >> a) & 1u) +
                          (uint32_t)__popcll(ga & adlo) + 2u * (uint32_t)__popcll(ga & adhi) +
                          2u * (uint32_t)((D >> a) & 1u);
      const uint32_t bd = (kd + 2u * (uint32_t)(((sc ^ skl) >> a) & 1u)) & 3u;
      kap |= (Word)(bd & 1u) << a;
      lam |= (Word)(bd >> 1) << a;
    }
    const uint32_t sks = (sksj + (uint32_t)__popcll(y & adlo) + 2u * (uint32_t)__popcll(y & adhi) +
                          2u * par64(tU)) & 3u;
    // Z_2 form of Eq. (Q) on supp(v) and one extra variable e = |v|.
    const uint32_t e = nv;
    const Word eb = (Word)1 << e;
    const Word Rset = (Word)((eb << 1) - (Word)1);
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      if ((uint32_t)a < nv) {
        const Word odd = (kap >> a) & (Word)1;
        const Word row = (((rlw<Word>(KJl, (uint32_t)a) ^ Sacc[a]) ^ (kap & ((Word)0 - odd))) &
                          ~((Word)1 << a)) | (odd << e);
        S[(uint32_t)a * stride + slot] = row;
      }
    }
    S[e * stride + slot] = kap;
    Word lr = lam, li = lam | eb, rem = Rset, iso = 0;
    uint32_t sr = 0, si = 0, nel = 0;
    // Eliminate a pair (a, b) with S_ab = 1 at a time (Eq. (eq5)); pivots per
    // lane.  A variable whose row is zero has no neighbour and never gains
    // one (S stays symmetric and an update only joins neighbours of the
    // pair), and its linear coefficients no longer change: it is set aside.
    for (;;) {
      uint32_t a = 0;
      Word Sa = 0;
      while (rem != 0) {
        a = kWide ? (uint32_t)__builtin_ctzll((uint64_t)rem) : (uint32_t)__builtin_ctz((uint32_t)rem);
        Sa = S[a * stride + slot];
        if (Sa != 0) break;
        iso |= (Word)1 << a;
        rem &= ~((Word)1 << a);
      }
      if (!__builtin_amdgcn_ballot_w64(rem != 0)) break;
      // Rows that no lane still holds are zero in every lane: only the
      // union of the remaining variables needs the update.
      const uint32_t remUl = wave_or32((uint32_t)rem);
      const uint32_t remUh = kWide ? wave_or32((uint32_t)((uint64_t)rem >> 32)) : 0u;
      if (rem != 0) {
        const uint32_t b = kWide ? (uint32_t)__builtin_ctzll((uint64_t)Sa) : (uint32_t)__builtin_ctz((uint32_t)Sa);
        const Word Sb = S[b * stride + slot];
        const Word ab = ((Word)1 << a) | ((Word)1 << b);
        const Word m1 = Sa & ~ab, m2 = Sb & ~ab;
        // Row c ^= (S_ac ? row b : 0) ^ (S_bc ? row a : 0), outside a, b; on
        // 32-bit halves, the tests as sign-extending bit-field extracts (c is
        // wave-uniform, so rows c < 32 and c >= 32 take separate loops).
        const uint32_t m1l = (uint32_t)m1, m2l = (uint32_t)m2, nabl = ~(uint32_t)ab;
        if constexpr (kWide) {
          const uint32_t m1h = (uint32_t)((uint64_t)m1 >> 32), m2h = (uint32_t)((uint64_t)m2 >> 32);
          const uint32_t nabh = ~(uint32_t)((uint64_t)ab >> 32);
          auto upd = [&](uint32_t c, uint32_t k1, uint32_t k2) {
            const uint64_t Sc = S[c * stride + slot];
            const uint32_t Sl = ((uint32_t)Sc ^ (m2l & k1) ^ (m1l & k2)) & nabl;
            const uint32_t Sh = ((uint32_t)(Sc >> 32) ^ (m2h & k1) ^ (m1h & k2)) & nabh;
            S[c * stride + slot] = (Word)(((uint64_t)Sh << 32) | Sl);
          };
          for (uint32_t m = (uint32_t)Rset & remUl; m; m &= m - 1u) {
            const uint32_t c = (uint32_t)__builtin_ctz(m);
            upd(c, bit_mask32(m1l, c), bit_mask32(m2l, c));
          }
          for (uint32_t m = (uint32_t)((uint64_t)Rset >> 32) & remUh; m; m &= m - 1u) {
            const uint32_t c = (uint32_t)__builtin_ctz(m);
            upd(32u + c, bit_mask32(m1h, c), bit_mask32(m2h, c));
          }
        } else {
          for (uint32_t m = (uint32_t)Rset & remUl; m; m &= m - 1u) {
            const uint32_t c = (uint32_t)__builtin_ctz(m);
            const uint32_t Sc = (uint32_t)S[c * stride + slot];
            S[c * stride + slot] = (Word)((Sc ^ (m2l & bit_mask32(m1l, c)) ^ (m1l & bit_mask32(m2l, c))) & nabl);
          }
        }
        S[a * stride + slot] = 0;
        S[b * stride + slot] = 0;
        {
          const Word la = (lr >> a) & (Word)1, lbb = (lr >> b) & (Word)1;
          sr ^= (uint32_t)(la & lbb);
          lr ^= (m2 & ((Word)0 - la)) ^ (m1 & ((Word)0 - lbb)) ^ (m1 & m2);
          lr &= ~ab;
        }
        {
          const Word la = (li >> a) & (Word)1, lbb = (li >> b) & (Word)1;
          si ^= (uint32_t)(la & lbb);
          li ^= (m2 & ((Word)0 - la)) ^ (m1 & ((Word)0 - lbb)) ^ (m1 & m2);
          li &= ~ab;
        }
        rem &= ~ab;
        ++nel;
      }
    }
    __builtin_amdgcn_wave_barrier();
    const int rr = kWide ? __popcll((uint64_t)iso) : __popc((uint32_t)iso);
    const bool re_nz = (lr & iso) == 0, im_nz = (li & iso) == 0;
    // Re Z = (-1)^sr 2^{nel + r - 1}, Im Z likewise; both non-zero only with equal exponents.
    if (l < L && (re_nz || im_nz)) {
      const int ez0 = (int)nel + rr - 1;
      uint32_t kz;
      int ez;
      if (re_nz && im_nz) {
        kz = sr ? (si ? 5u : 3u) : (si ? 7u : 1u);
        ez = 2 * ez0 + 1;
      } else if (re_nz) {
        kz = sr ? 4u : 0u;
        ez = 2 * ez0;
      } else {
        kz = si ? 6u : 2u;
        ez = 2 * ez0;
      }
      const uint32_t kin = (2u * sks + 4u * sv + kz) & 7u;
      InnerRec rc;
      rc.nonzero = 1u;
      rc.k8 = (omega - kin) & 7u;  // <phi_A|omega phi> = omega conj(<phi|phi_A>)
      rc.e2 = ez - (int)(n + nv);
      const double2 val = rec_value(rc, bb);
      accr += val.x;
      acci += val.y;
    }
  }
}

// LDS of one pair wave: the lookup tables (NMAX <= 64: 16 chunks of 16
// 64-bit entries) and the elimination rows, 64 lanes x 32 variables of 32
// bits or 32 lanes x (n + 1) variables of 64 bits.
__host__ __device__ constexpr uint32_t inner_gtab_bytes() { return 16u * 16u * 8u; }
__host__ __device__ constexpr uint32_t inner_srow_bytes(uint32_t n) {
  return (n + 1u) * 32u * 8u > 32u * 64u * 4u ? (n + 1u) * 32u * 8u : 32u * 64u * 4u;
}

// One wave per (term group, batch of 64 states); lane = state.  The block
// index maps XCD-aware: workgroups are dealt to the 8 XCDs in turn, and the
// batches of one term group are consecutive on one XCD, so a term's record
// is read from HBM once per XCD-resident group rather than once per batch.
template <int NMAX>
__global__ __launch_bounds__(64, NMAX <= 40 ? 3 : 2) void k_inner_pairs(TermsView Tv, const uint64_t* __restrict__ rec,
                                                    const uint64_t* __restrict__ at,
                                                    const uint64_t* __restrict__ planes, uint32_t L,
                                                    uint32_t Lp, uint32_t n_groups, uint32_t n_batches,
                                                    double2* __restrict__ partial, uint32_t* __restrict__ err) {
  extern __shared__ __align__(16) uint64_t lds_w[];
  const uint32_t n = Tv.n;
  const uint32_t lane = threadIdx.x;
  uint32_t group, batch;
  if (n_groups % 8u == 0u) {
    const uint32_t xcd = blockIdx.x % 8u, k = blockIdx.x / 8u;
    group = (k / n_batches) * 8u + xcd;
    batch = k % n_batches;
  } else {
    group = blockIdx.x % n_groups;
    batch = blockIdx.x / n_groups;
  }
  const uint32_t l = batch * 64u + lane;
  const uint64_t adlo = planes[l], adhi = planes[Lp + l];
  const uint64_t* __restrict__ atl = at + l;
  const uint32_t R = inner_rec_words(n);
  void* const gtab = lds_w;
  void* const srow = reinterpret_cast<unsigned char*>(lds_w) + inner_gtab_bytes();
  double accr = 0.0, acci = 0.0;
  uint32_t bad = 0;
  for (uint64_t term = group; term < Tv.chi; term += n_groups) {
    const uint64_t* r = rec + term * R;
    const uint64_t v = uniform64(Tv.v[term]);
    const uint32_t omega = uniform32(Tv.omega[term]);
    const double2 bb = Tv.b[term];
    if (v == ~0ull) {
      bad = 1u;
      continue;
    }
    const uint32_t nv = (uint32_t)__popcll(v);
    const uint32_t sv = par64(Tv.s[term] & v);
    if (nv < 32u)
      pair_term<uint32_t, (NMAX < 32 ? NMAX : 32), NMAX>(r, n, nv, lane, l, L, atl, Lp, adlo, adhi, omega, sv, bb,
                                                         reinterpret_cast<uint32_t*>(gtab), srow, accr, acci);
    else
      pair_term<uint64_t, NMAX, NMAX>(r, n, nv, lane, l, L, atl, Lp, adlo, adhi, omega, sv, bb,
                                      reinterpret_cast<uint64_t*>(gtab), srow, accr, acci);
  }
  if (bad && lane == 0u) atomicOr(err, 1u);
  if (l < L) partial[(uint64_t)group * L + l] = make_double2(accr, acci);
}

__global__ __launch_bounds__(256) void k_inner_reduce(const double2* __restrict__ partial,
                                                      uint32_t n_blocks, uint32_t L, uint32_t n,
                                                      double2* __restrict__ overlap,
                                                      double* __restrict__ eta) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= L) return;
  double re = 0.0, im = 0.0;
  for (uint32_t b = 0; b < n_blocks; ++b) {
    const double2 v = partial[(uint64_t)b * L + l];
    re += v.x;
    im += v.y;
  }
  overlap[l] = make_double2(re, im);
  eta[l] = ldexp(re * re + im * im, (int)n);
}

// Mean of eta in FP64 with a fixed summation order.
__global__ __launch_bounds__(256) void k_eta_sum(const double* __restrict__ eta, uint32_t L,
                                                 double* __restrict__ out) {
  __shared__ double part[256];
  double acc = 0.0;
  for (uint32_t l = threadIdx.x; l < L; l += 256u) acc += eta[l];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (uint32_t w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0];
}

}  // namespace

constexpr uint32_t kTermGroups = 512;  // waves per batch of 64 states, each over chi / 512 terms

InnerPlan inner_plan(const TermsView& T, uint32_t L) {
  InnerPlan P;
  P.Lp = (L + 63u) / 64u * 64u;
  P.n_batches = P.Lp / 64u;
  P.n_groups = (uint32_t)std::min<uint64_t>(kTermGroups, T.chi);
  P.partial_elems = (size_t)P.n_groups * L;
  P.work_words = (size_t)T.chi * inner_rec_words(T.n) + (size_t)T.n * P.Lp + 2u * (size_t)P.Lp;
  return P;
}

hipError_t launch_inner(const TermsView& T, const uint64_t* Aoff, const uint8_t* Adiag, uint32_t L,
                        const InnerPlan& P, double2* partial, uint64_t* work, double2* overlap,
                        double* eta, double* eta_sum, uint32_t* err, hipStream_t st) {
  const uint32_t n = T.n;
  uint64_t* rec = work;
  uint64_t* at = rec + (size_t)T.chi * inner_rec_words(n);
  uint64_t* planes = at + (size_t)n * P.Lp;
  hipLaunchKernelGGL(k_inner_prep, dim3((uint32_t)((T.chi + kWaves - 1) / kWaves)), dim3(64 * kWaves), 0, st,
                     T, rec);
  hipLaunchKernelGGL(k_inner_atrans, dim3((P.Lp + 255u) / 256u), dim3(256), 0, st, Aoff, Adiag, n, L, P.Lp,
                     at, planes);
  const size_t sm = (size_t)inner_gtab_bytes() + inner_srow_bytes(n);
  const dim3 grid(P.n_groups * P.n_batches);
  switch ((n + 7u) / 8u) {
#define CHSIM_INNER_CASE(k)                                                                          \
  case k:                                                                                            \
    hipLaunchKernelGGL(k_inner_pairs<8 * k>, grid, dim3(64), sm, st, T, rec, at, planes, L, P.Lp,     \
                       P.n_groups, P.n_batches, partial, err);                                       \
    break;
    CHSIM_INNER_CASE(1)
    CHSIM_INNER_CASE(2)
    CHSIM_INNER_CASE(3)
    CHSIM_INNER_CASE(4)
    CHSIM_INNER_CASE(5)
    CHSIM_INNER_CASE(6)
    CHSIM_INNER_CASE(7)
    CHSIM_INNER_CASE(8)
#undef CHSIM_INNER_CASE
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_inner_reduce, dim3((L + 255) / 256), dim3(256), 0, st, partial, P.n_groups, L,
                     T.n, overlap, eta);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_eta_sum, dim3(1), dim3(256), 0, st, eta, L, eta_sum);
  return hipGetLastError();
}

}  // namespace chsim
