// Inner products of two CH forms (general stabilizer states):
//   overlap_l = <theta_l|psi> = sum_alpha b_alpha <theta_l|phi_alpha>,
// theta_l the CH form of term l of a second term set (the "bra" set).
//
// Method.  <theta|phi> = sum_x conj(<x|theta>) <x|phi> with the amplitudes of
// Eqs. (amplitude), (amplitude1).  In the quadratic-form view of those
// amplitudes (the same one the amplitude kernel uses), a CH form gives
//   <x|phi> = 2^{-|v|/2} e^{i pi k(x)/4},  k(x) = omega + 2 popc(x & glo) + 4 x^T B x
// on its support, with B_pq = par(F_p & M_q) for p < q and
// B_pp = par(F_p & M_p) + gamma_hi,p + par(F_p & v & s) (mod 2); the support is
// x = (s + y) G^T for y on v (F G^T = I makes u = x F = s + y).  The sum over
// the intersection of the two supports:
//   * the ket's support is x1 + span{column i of G : i in v} (x1 = s G^T);
//   * the bra's support is (x F_b)_j = s_b,j for j outside v_b, i.e.
//     equations sum_i y_i (G^T F_b)_ij = s_b,j + par(x1 & column j of F_b);
//   * GF(2) elimination gives x = x0 + sum_f z_f d_f over the free variables f;
//   * the phase k_ket - k_bra on it is e^{i pi K0/4} i^{E(z)} with E a Z_4
//     quadratic form of Lemma (Exponential Sum): diagonal
//     l_f + 2 (par(x0 & t_f) + q(d_f)), off-diagonal
//     par(d_f & d_g & (glo_ket ^ glo_bra)) + par(d_f & t_g), where t = Bs d
//     (Bs = B + B^T of both states, the bilinear form of x^T B x),
//     q(d) = d^T B d and l_f the signed count of d_f's bits in the glo planes
//     (signs flipped where x0 has a 1);
//   * Z(E) by the lift of Eq. (Q) and pair elimination (Eqs. (identity), (eq5)).
// The paper states the O(n^3) cost and defers this method to earlier work.
//
// Mapping.  A prologue writes a record per term (one wave per term, lane =
// row): the columns and rows of G, the columns of F, the rows of Bs and a few
// words.  The pair kernel runs one wave per (bra state, group of ket terms),
// lane i holding row or variable i, so every step is O(1) or O(n) wave-wide
// instructions with uniform control flow.
#include <algorithm>

#include "device_common.hpp"
#include "internal.hpp"

namespace chsim {

namespace {

constexpr int kCHWaves = 4;

__host__ __device__ constexpr uint32_t chrec_words(uint32_t n) { return 6u * n + 6u; }

// Record of one term: colG [0, n), rows of G [n, 2n), colF [2n, 3n), rows of
// Bs [3n, 4n), Bs colG_i [4n, 5n), Bu colG_i [5n, 6n) (Bu: the strictly
// upper part of Bs, row q below bit q), then diag(B), glo, x1 = s G^T, s, v,
// omega.
__global__ __launch_bounds__(64 * kCHWaves) void k_chrec(TermsView T, uint64_t* __restrict__ rec) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t term = (uint64_t)blockIdx.x * kCHWaves + uniform32(threadIdx.x >> 6);
  if (term >= T.chi) return;  // whole waves
  const uint32_t n = T.n;
  const bool act = lane < n;
  const uint64_t off = (uint64_t)lane * T.chi + term;
  const uint64_t F = act ? T.F[off] : 0ull, G = act ? T.G[off] : 0ull, M = act ? T.M[off] : 0ull;
  const uint32_t g = act ? (uint32_t)T.gamma[off] : 0u;
  const uint64_t v = uniform64(T.v[term]), s = uniform64(T.s[term]);
  uint64_t colG = 0, colF = 0, P = 0;
  for (uint32_t q = 0; q < n; ++q) {
    const uint64_t cg = ballot64(((G >> q) & 1ull) != 0ull);
    const uint64_t cf = ballot64(((F >> q) & 1ull) != 0ull);
    if (lane == q) {
      colG = cg;
      colF = cf;
    }
    P |= (uint64_t)par64(F & rl64(M, q)) << q;  // P_pq = par(F_p & M_q)
  }
  // Bs_pq = P_{min(p,q), max(p,q)} for p != q.
  uint64_t low = 0;
  for (uint32_t q = 0; q < n; ++q) low |= ((rl64(P, q) >> lane) & 1ull) << q;
  const uint64_t above = (lane >= 63u) ? 0ull : (~0ull << (lane + 1u));
  const uint64_t below = (1ull << lane) - 1ull;
  const uint64_t Bs = act ? ((P & above) | (low & below)) : 0ull;
  const uint64_t diag = ballot64(act && (((P >> lane) & 1ull) ^ (uint64_t)((g >> 1) & 1u) ^
                                         (uint64_t)par64(F & v & s)) != 0ull);
  const uint64_t glo = ballot64(act && (g & 1u));
  const uint64_t x1 = ballot64(act && par64(G & s));
  // The term's own part of t = Bs d and tu = Bu d for d = column i of G
  // (lane i); a pair's directions are sums of such columns.
  uint64_t W = 0, Wu = 0;
  for (uint32_t q = 0; q < n; ++q) {
    const uint64_t Bq = rl64(Bs, q) & bitmask64(colG, q);
    W ^= Bq;
    Wu ^= Bq & ((1ull << q) - 1ull);
  }
  uint64_t* r = rec + term * chrec_words(n);
  if (act) {
    r[lane] = colG;
    r[n + lane] = G;
    r[2u * n + lane] = colF;
    r[3u * n + lane] = Bs;
    r[4u * n + lane] = W;
    r[5u * n + lane] = Wu;
  }
  if (lane == 0) {
    r[6u * n] = diag;
    r[6u * n + 1u] = glo;
    r[6u * n + 2u] = x1;
    r[6u * n + 3u] = s;
    r[6u * n + 4u] = v;
    r[6u * n + 5u] = T.omega[term];
  }
}

__device__ __forceinline__ double2 scaled_root(uint32_t k8, int e2, double2 b) {
  const double h = 0.70710678118654752440;
  const double mag = (e2 & 1) ? ldexp(1.41421356237309504880, (e2 - 1) / 2) : ldexp(1.0, e2 / 2);
  double cr, ci;
  switch (k8 & 7u) {
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

// What the pair elimination of a lifted form leaves: eliminated pairs, the
// isolated variables, the two lifted sums' signs and which of them vanish.
struct LiftOut {
  uint32_t nel, sr, si;
  int niso;
  bool re_nz, im_nz;
};

template <typename Word>
__device__ __forceinline__ Word rl_word(Word x, uint32_t src) {
  if constexpr (sizeof(Word) == 4) return rl32(x, src);
  else return rl64(x, src);
}
template <typename Word>
__device__ __forceinline__ uint32_t ctz_word(Word x) {
  if constexpr (sizeof(Word) == 4) return (uint32_t)__builtin_ctz(x);
  else return (uint32_t)__builtin_ctzll(x);
}

// Z of the Z_2 form of Eq. (Q) that lifts a Z_4 form (kap: odd diagonal,
// lam: diagonal high bits, S: off-diagonal rows, lane v holding row v) onto
// the variables Rset, of which e is the extra one, by pair elimination
// (Eqs. (identity), (eq5)); Word holds a row (bit v = variable v, lane v < its
// width).
template <typename Word>
__device__ __forceinline__ LiftOut lift_eliminate(Word S, Word kap, Word lam, Word Rset, uint32_t e, uint32_t lane) {
  constexpr uint32_t kBits = sizeof(Word) * 8u;
  const bool inw = lane < kBits;
  const Word lbw = inw ? (Word)((Word)1 << (lane & (kBits - 1u))) : (Word)0;
  const Word eb = (Word)((Word)1 << e);
  const Word odd = inw ? (Word)((kap >> (lane & (kBits - 1u))) & (Word)1) : (Word)0;
  const bool var = (Rset & ~eb & lbw) != (Word)0;
  Word row = var ? (Word)(((S ^ (kap & (Word)((Word)0 - odd))) & ~lbw) | (Word)(odd << e)) : (Word)0;
  if (lane == e) row = kap;
  Word lr = lam, li = lam | eb, rem = Rset, iso = 0;
  LiftOut o{0u, 0u, 0u, 0, false, false};
  for (;;) {
    // First remaining variable with a non-zero row; variables with zero rows
    // are isolated for good.
    const Word nz = (Word)ballot64((rem & lbw) != (Word)0 && row != (Word)0);
    const Word zr = rem & ~nz;
    if (nz == (Word)0) {
      iso |= zr;
      break;
    }
    const uint32_t va = ctz_word(nz);
    const Word below = (Word)(((Word)1 << va) - (Word)1);
    iso |= zr & below;
    rem &= ~(zr & below);
    const Word Sa = rl_word(row, va);
    const uint32_t vb = ctz_word(Sa);
    const Word Sb = rl_word(row, vb);
    const Word ab = (Word)(((Word)1 << va) | ((Word)1 << vb));
    const Word m1 = Sa & ~ab, m2 = Sb & ~ab;
    const Word b1 = inw ? (Word)((Word)0 - ((m1 >> (lane & (kBits - 1u))) & (Word)1)) : (Word)0;
    const Word b2 = inw ? (Word)((Word)0 - ((m2 >> (lane & (kBits - 1u))) & (Word)1)) : (Word)0;
    row ^= (m2 & b1) ^ (m1 & b2);
    row &= ~ab;
    if (lane == va || lane == vb) row = 0;
    {
      const Word la = (lr >> va) & (Word)1, lbb = (lr >> vb) & (Word)1;
      o.sr ^= (uint32_t)(la & lbb);
      lr ^= (m2 & (Word)((Word)0 - la)) ^ (m1 & (Word)((Word)0 - lbb)) ^ (m1 & m2);
      lr &= ~ab;
    }
    {
      const Word la = (li >> va) & (Word)1, lbb = (li >> vb) & (Word)1;
      o.si ^= (uint32_t)(la & lbb);
      li ^= (m2 & (Word)((Word)0 - la)) ^ (m1 & (Word)((Word)0 - lbb)) ^ (m1 & m2);
      li &= ~ab;
    }
    rem &= ~ab;
    ++o.nel;
  }
  o.niso = __popcll((uint64_t)iso);
  o.re_nz = (lr & iso) == (Word)0;
  o.im_nz = (li & iso) == (Word)0;
  return o;
}

// One wave per (bra state l = bra block * kCHWaves + wave, ket group g):
// the ket terms g, g + groups, ...; lane i holds row/variable i
// (a pair's free variables are moved to lanes 0, 1, ... when at most 31 of
// them, so that the Z_4 form's rows and its elimination use 32-bit words).
// Eight waves per SIMD (the LDS of the tables and the scratch allows eight).
// The block index maps XCD-aware: workgroups are dealt to the 8 XCDs in turn,
// and the bra blocks of one ket group are consecutive on one XCD, so a ket
// record is read from HBM about once per XCD-resident group.
__global__ __launch_bounds__(64 * kCHWaves, 8) void k_inner_ch_pairs(
    const uint64_t* __restrict__ rec_k, const double2* __restrict__ b_k, uint64_t chi_k,
    const uint64_t* __restrict__ rec_b, uint32_t L, uint32_t n, uint32_t groups, uint32_t bra_blocks,
    double2* __restrict__ partial, uint32_t* __restrict__ err) {
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t group, bblock;
  if (groups % 8u == 0u) {
    const uint32_t xcd = blockIdx.x % 8u, k = blockIdx.x / 8u;
    group = (k / bra_blocks) * 8u + xcd;
    bblock = k % bra_blocks;
  } else {
    group = blockIdx.x % groups;
    bblock = blockIdx.x / groups;
  }
  const uint32_t l = bblock * kCHWaves + uniform32(threadIdx.x >> 6);
  if (l >= L) return;  // whole waves
  const uint32_t R = chrec_words(n);
  const bool act = lane < n;
  const uint64_t lb = 1ull << lane;
  // Bra record (held for the whole wave).
  const uint64_t* rb = rec_b + (uint64_t)l * R;
  const uint64_t colFb = act ? rb[2u * n + lane] : 0ull;
  const uint64_t Bsb = act ? rb[3u * n + lane] : 0ull;
  const uint64_t diag_b = uniform64(rb[6u * n]), glo_b = uniform64(rb[6u * n + 1u]);
  const uint64_t s_b = uniform64(rb[6u * n + 3u]), v_b = uniform64(rb[6u * n + 4u]);
  const uint32_t om_b = uniform32((uint32_t)rb[6u * n + 5u]);
  const uint64_t neq_mask = ~v_b & ((n == 64u) ? ~0ull : ((1ull << n) - 1ull));  // equations j outside v_b
  // The bra's part of t = Bs d and tu = Bu d by nibbles of d: tables of the
  // XOR of each subset of 4 consecutive rows of Bs_b (and of Bu_b), built once
  // for the wave's bra state and read with a lane's own index (t_d = XOR over
  // nibble groups g of tab[g][nibble g of d]); an entry holds the Bs and Bu
  // words side by side, so one 16-byte read serves both.
  __shared__ __align__(16) uint64_t tabs[kCHWaves][16][16][2];
  uint64_t(*const tab)[16][2] = tabs[uniform32(threadIdx.x >> 6)];
  // Scratch for moving a pair's free variables to lanes 0, 1, ...
  __shared__ uint64_t cds[kCHWaves][32], cws[kCHWaves][32];
  __shared__ uint32_t ces[kCHWaves][32];
  uint64_t* const cd = cds[uniform32(threadIdx.x >> 6)];
  uint64_t* const cw = cws[uniform32(threadIdx.x >> 6)];
  uint32_t* const ce = ces[uniform32(threadIdx.x >> 6)];
  const uint32_t ngrp = (n + 3u) / 4u;
  for (uint32_t g = 0; g < ngrp; ++g) {
    uint64_t acc = 0;
    for (uint32_t b = 0; b < 4u; ++b) {
      const uint32_t q = 4u * g + b;
      if (q >= n) break;
      const uint64_t R = rl64(Bsb, q);
      const uint64_t val = lane < 16u ? R : (R & ((1ull << q) - 1ull));
      if (((lane & 15u) >> b) & 1u) acc ^= val;
    }
    if (lane < 32u) tab[g][lane & 15u][lane >> 4] = acc;
  }
  // (Bs_b d, Bu_b d) for one d.
  auto lookup2 = [&](uint64_t x, uint64_t& rs, uint64_t& ru) {
    rs = 0;
    ru = 0;
    for (uint32_t g = 0; g < ngrp; ++g) {
      const ulonglong2 e = *reinterpret_cast<const ulonglong2*>(tab[g][(x >> (4u * g)) & 15u]);
      rs ^= e.x;
      ru ^= e.y;
    }
  };
  double accr = 0.0, acci = 0.0;
  uint32_t bad = 0;
  for (uint64_t a = group; a < chi_k; a += groups) {
    const uint64_t* rk = rec_k + a * R;
    const uint64_t colGk = act ? rk[lane] : 0ull;
    const uint64_t Growk = act ? rk[n + lane] : 0ull;
    const uint64_t Bsk = act ? rk[3u * n + lane] : 0ull;
    const uint64_t Wk = act ? rk[4u * n + lane] : 0ull, Wuk = act ? rk[5u * n + lane] : 0ull;
    const uint64_t diag_k = uniform64(rk[6u * n]), glo_k = uniform64(rk[6u * n + 1u]);
    const uint64_t x1 = uniform64(rk[6u * n + 2u]);
    const uint64_t v_k = uniform64(rk[6u * n + 4u]);
    const uint32_t om_k = uniform32((uint32_t)rk[6u * n + 5u]);
    // Equations: lane j (j outside v_b): E_j = XOR of G rows p with F_b[p][j] = 1,
    // restricted to the unknowns v_k; rhs_j = s_b,j + par(x1 & colF_b,j).
    // E_j restricted to v_k has bit i = par(column j of F_b & column i of G_k):
    // with few equations, one ballot per equation over the lanes i; else
    // lane j adds the G rows p its column selects.
    const bool eq = ((neq_mask >> lane) & 1ull) != 0ull;
    uint64_t E = 0;
    if (5u * (uint32_t)__popcll(neq_mask) < 4u * n) {
      const bool unk = ((v_k >> lane) & 1ull) != 0ull;
      for (uint64_t em = neq_mask; em; em &= em - 1ull) {
        const uint32_t j = (uint32_t)__builtin_ctzll(em);
        const uint64_t Ej = ballot64(unk && par64(rl64(colFb, j) & colGk));
        if (lane == j) E = Ej;
      }
    } else {
      for (uint32_t p = 0; p < n; ++p) E ^= rl64(Growk, p) & bitmask64(colFb, p);
      E &= v_k;
    }
    uint32_t rhs = (uint32_t)((s_b >> lane) & 1ull) ^ par64(x1 & colFb);
    if (!eq) {
      E = 0;
      rhs = 0;
    }
    // Reduced row echelon form: a pivot lane per step, eliminated from all others.
    uint64_t used = 0, pivmask = 0;
    uint32_t pivvar = 0;
    for (;;) {
      const uint64_t cand = ballot64(eq && !((used >> lane) & 1ull) && E != 0ull);
      if (cand == 0ull) break;
      const uint32_t j = (uint32_t)__builtin_ctzll(cand);
      const uint64_t Ej = rl64(E, j);
      const uint32_t rj = rl32(rhs, j);
      const uint32_t pv = (uint32_t)__builtin_ctzll(Ej);
      if (lane != j && ((E >> pv) & 1ull)) {
        E ^= Ej;
        rhs ^= rj;
      }
      if (lane == j) pivvar = pv;
      used |= 1ull << j;
      pivmask |= 1ull << pv;
    }
    if (ballot64(eq && E == 0ull && rhs != 0u)) continue;  // the supports do not meet
    // Free variables f (lanes) and their directions d_f in x-space; x0.
    // Directions d_f of the free variables f (column f of G plus the pivot
    // columns its equations bring in), with the ket's parts of Bs d_f and
    // Bu d_f from the same columns' record words.
    const uint64_t Fr = v_k & ~pivmask;
    const bool fr = ((Fr >> lane) & 1ull) != 0ull;
    uint64_t d = fr ? colGk : 0ull, tk = fr ? Wk : 0ull, tuk = fr ? Wuk : 0ull;
    uint64_t x0 = x1;
    for (uint64_t u = used; u; u &= u - 1ull) {
      const uint32_t j = (uint32_t)__builtin_ctzll(u);
      const uint64_t Ej = rl64(E, j);
      const uint32_t pv = rl32(pivvar, j);
      const uint64_t cg = rl64(colGk, pv), cw = rl64(Wk, pv), cwu = rl64(Wuk, pv);
      if (fr && ((Ej >> lane) & 1ull)) {
        d ^= cg;
        tk ^= cw;
        tuk ^= cwu;
      }
      if (rl32(rhs, j)) x0 ^= cg;
    }
    // t_f = Bs d_f with Bs = Bs_ket + Bs_bra (the bilinear form), and
    // tu_f = Bu d_f with Bu its strictly upper part (column q of Bu is row q of
    // Bs below bit q), so that d^T B d = par(d & diag) + par(d & Bu d).
    const uint64_t Bs = Bsk ^ Bsb;
    uint64_t tb, tub;
    lookup2(d, tb, tub);
    const uint64_t t = tk ^ tb, tu = tuk ^ tub;
    const uint64_t above = (lane >= 63u) ? 0ull : (~0ull << (lane + 1u));
    const uint64_t tu0 = ballot64(act && par64(Bs & above & x0));
    const uint64_t Bd = diag_k ^ diag_b, gd = glo_k ^ glo_b;
    const uint64_t pa = glo_k & ~glo_b, pb = glo_b & ~glo_k;
    const uint64_t Pp = (pa & ~x0) | (pb & x0), Pm = (pb & ~x0) | (pa & x0);
    // Constant phase K0 = k_ket(x0) - k_bra(x0) (units of pi/4).
    const uint32_t qx0 = par64(Bd & x0) ^ par64(x0 & tu0);
    const uint32_t K0 = (om_k + 8u - om_b + 2u * ((uint32_t)__popcll(x0 & pa) + 3u * (uint32_t)__popcll(x0 & pb)) +
                         4u * qx0) & 7u;
    // Z_4 form on the free variables: diagonal e (lane f), rows S.
    const bool fv = ((Fr >> lane) & 1ull) != 0ull;
    const uint32_t lf = ((uint32_t)__popcll(d & Pp) + 3u * (uint32_t)__popcll(d & Pm)) & 3u;
    const uint32_t qd = par64(Bd & d) ^ par64(d & tu);
    const uint32_t ef = (lf + 2u * (par64(x0 & t) ^ qd)) & 3u;
    if (Fr == ~0ull) {
      bad = 1u;
      continue;
    }
    // S_fg = par(d_f & w_g) with w_g = (d_g & gd) ^ t_g, formed by each lane
    // for its own variable.
    const uint64_t wv = (d & gd) ^ t;
    const uint32_t nf = (uint32_t)__popcll(Fr);
    LiftOut lo;
    if (nf < 32u) {
      // At most 31 free variables: move variable f to lane c = (its rank in
      // Fr), so that rows are 32-bit words over c and the extra variable is
      // c = nf.
      const uint32_t c = (uint32_t)__popcll(Fr & (lb - 1ull));
      if (fv) {
        cd[c] = d;
        cw[c] = wv;
        ce[c] = ef;
      }
      __builtin_amdgcn_wave_barrier();
      const bool fc = lane < nf;
      const uint64_t dc = fc ? cd[lane] : 0ull, wc = fc ? cw[lane] : 0ull;
      const uint32_t ec = fc ? ce[lane] : 0u;
      __builtin_amdgcn_wave_barrier();
      uint32_t S = 0;
      for (uint32_t c2 = 0; c2 < nf; ++c2) S |= par64(dc & rl64(wc, c2)) << c2;
      const uint32_t lb32 = lane < 32u ? (1u << lane) : 0u;
      S = fc ? (S & ~lb32) : 0u;
      lo = lift_eliminate<uint32_t>(S, (uint32_t)ballot64(fc && (ec & 1u)), (uint32_t)ballot64(fc && (ec & 2u)),
                                    (2u << nf) - 1u, nf, lane);
    } else {
      uint64_t S = 0;
      for (uint64_t u = Fr; u; u &= u - 1ull) {
        const uint32_t f2 = (uint32_t)__builtin_ctzll(u);
        S |= (uint64_t)par64(d & rl64(wv, f2)) << f2;
      }
      S = fv ? (S & ~lb) : 0ull;
      const uint32_t e = (uint32_t)__builtin_ctzll(~Fr);
      lo = lift_eliminate<uint64_t>(S, ballot64(fv && (ef & 1u)), ballot64(fv && (ef & 2u)), Fr | (1ull << e), e,
                                    lane);
    }
    const bool re_nz = lo.re_nz, im_nz = lo.im_nz;
    if (!(re_nz || im_nz)) continue;
    const int ez0 = (int)lo.nel + lo.niso - 1;
    uint32_t kz;
    int ez;
    if (re_nz && im_nz) {
      kz = lo.sr ? (lo.si ? 5u : 3u) : (lo.si ? 7u : 1u);
      ez = 2 * ez0 + 1;
    } else if (re_nz) {
      kz = lo.sr ? 4u : 0u;
      ez = 2 * ez0;
    } else {
      kz = lo.si ? 6u : 2u;
      ez = 2 * ez0;
    }
    const int e2 = ez - (int)((uint32_t)__popcll(v_k) + (uint32_t)__popcll(v_b));
    const double2 val = scaled_root(K0 + kz, e2, b_k[a]);
    accr += val.x;
    acci += val.y;
  }
  if (bad && lane == 0u) atomicOr(err, 1u);
  if (lane == 0u) partial[(uint64_t)group * L + l] = make_double2(accr, acci);
}

__global__ __launch_bounds__(256) void k_inner_ch_reduce(const double2* __restrict__ partial, uint32_t groups,
                                                         uint32_t L, double2* __restrict__ overlap) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= L) return;
  double re = 0.0, im = 0.0;
  for (uint32_t g = 0; g < groups; ++g) {
    const double2 v = partial[(uint64_t)g * L + l];
    re += v.x;
    im += v.y;
  }
  overlap[l] = make_double2(re, im);
}

// total = sum_l conj(b_l) overlap_l in FP64, fixed order (one block).
__global__ __launch_bounds__(256) void k_inner_ch_total(const double2* __restrict__ overlap,
                                                        const double2* __restrict__ b_bra, uint32_t L,
                                                        double2* __restrict__ total) {
  __shared__ double pr[256], pi[256];
  double re = 0.0, im = 0.0;
  for (uint32_t l = threadIdx.x; l < L; l += 256u) {
    const double2 o = overlap[l], c = b_bra[l];
    re += c.x * o.x + c.y * o.y;
    im += c.x * o.y - c.y * o.x;
  }
  pr[threadIdx.x] = re;
  pi[threadIdx.x] = im;
  __syncthreads();
  for (uint32_t w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      pr[threadIdx.x] += pr[threadIdx.x + w];
      pi[threadIdx.x] += pi[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = make_double2(pr[0], pi[0]);
}

}  // namespace

size_t inner_ch_record_words(uint32_t n, uint64_t chi) { return (size_t)chi * chrec_words(n); }

hipError_t launch_inner_ch_records(const TermsView& T, uint64_t* rec, hipStream_t st) {
  const uint64_t blocks = (T.chi + kCHWaves - 1) / kCHWaves;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chrec, dim3((uint32_t)blocks), dim3(64 * kCHWaves), 0, st, T, rec);
  return hipGetLastError();
}

uint32_t inner_ch_groups(uint64_t chi_k, uint32_t L) {
  // About 2^17 waves in all, at least one ket term per group, a multiple of
  // 8 groups when there are 8 or more (the XCD-aware block order).
  const uint64_t want = std::max<uint64_t>(1, (uint64_t)(1u << 17) / std::max<uint32_t>(L, 1u));
  const uint64_t g = std::min<uint64_t>(std::min<uint64_t>(want, 4096), chi_k);
  return (uint32_t)(g >= 8 ? g & ~7ull : g);
}

hipError_t launch_inner_ch(const uint64_t* rec_k, const double2* b_k, uint64_t chi_k, const uint64_t* rec_b,
                           const double2* b_bra, uint32_t L, uint32_t n, uint32_t groups, double2* partial,
                           double2* overlap, double2* total, uint32_t* err, hipStream_t st) {
  const uint32_t bra_blocks = (L + kCHWaves - 1) / kCHWaves;
  const uint64_t blocks = (uint64_t)bra_blocks * groups;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_inner_ch_pairs, dim3((uint32_t)blocks), dim3(64 * kCHWaves), 0, st, rec_k, b_k, chi_k, rec_b,
                     L, n, groups, bra_blocks, partial, err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_inner_ch_reduce, dim3((L + 255u) / 256u), dim3(256), 0, st, partial, groups, L, overlap);
  e = hipGetLastError();
  if (e != hipSuccess || !total) return e;
  hipLaunchKernelGGL(k_inner_ch_total, dim3(1), dim3(256), 0, st, overlap, b_bra, L, total);
  return hipGetLastError();
}

}  // namespace chsim
