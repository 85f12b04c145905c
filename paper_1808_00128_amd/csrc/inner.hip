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
// Mapping: one wave per term, lane a holds row a of every n x n bit matrix.
// K = G^T X G splits into Y = G^T X (row a = XOR of the rows X_c with c in
// column a of G) and K = Y G (row a = XOR of the rows G_d with d in row a of
// Y); the rows of the other operand come by readlane.  The diagonal mod 4
// uses popcounts of G's column against X's diagonal bit-planes and the parity
// of the strictly-upper part.  The elimination keeps the symmetric Z_2
// adjacency S in the lanes (lane c = row c); a pivot pair (a, b) is found by
// ballot + find-first-set, and the rank-2 update S_c ^= [c in m1] m2 ^
// [c in m2] m1 is one masked XOR per lane.  K_J is computed once per term and
// every equatorial state reuses it (K is linear in A + J).
#include "device_common.hpp"
#include "internal.hpp"

namespace chsim {

namespace {

constexpr int kWaves = 4;

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
  uint32_t bad;
};

// Evaluate one pair from the term's K (lane rows).  Wave-uniform result:
// <phi_A|phi> = 0 or e^{i pi k8/4} 2^{e2/2} (omega included).
__device__ __forceinline__ InnerRec pair_record(uint64_t Koff, uint32_t Kdiag, uint64_t v,
                                                uint64_t s, uint32_t omega, uint32_t lane,
                                                uint32_t n) {
  InnerRec rec{0u, 0u, 0, 0u};
  const bool act = lane < n;
  const uint64_t lb = 1ull << lane;
  const uint32_t sl = (uint32_t)((s >> lane) & 1ull);
  const uint64_t Krow = act ? (Koff | ((uint64_t)(Kdiag & 1u) << lane)) : 0ull;
  // (sK)_a = par(s & K_a) (K symmetric); s K s^T mod 4.
  const uint32_t skl = par64(s & Krow);
  const uint64_t upper = (lane == 63u) ? 0ull : (~0ull << (lane + 1u));
  const uint64_t kdlo = ballot64(act && (Kdiag & 1u)), kdhi = ballot64(act && (Kdiag & 2u));
  const uint64_t pairs = ballot64(act && sl && par64(Koff & s & upper));
  const uint32_t sks =
      ((uint32_t)__popcll(s & kdlo) + 2u * (uint32_t)__popcll(s & kdhi) + 2u * (uint32_t)__popcll(pairs)) & 3u;
  const uint32_t sv = par64(s & v);
  // B on supp(v): diagonal K_aa + 2 (s_a + (sK)_a), off-diagonal K_ab.
  const bool inv = act && ((v >> lane) & 1ull);
  const uint32_t Bd = (Kdiag + 2u * (sl ^ skl)) & 3u;
  // Z_2 lift (Eq. (Q)): kappa_a = B_aa & 1, lambda_a = B_aa >> 1; extra variable e.
  const uint64_t kap = ballot64(inv && (Bd & 1u));
  const uint64_t lam = ballot64(inv && (Bd & 2u));
  if (v == ~0ull) {
    rec.bad = 1u;
    return rec;
  }
  const uint32_t e = (uint32_t)__builtin_ctzll(~v);
  const uint64_t eb = 1ull << e;
  uint64_t S = 0;
  if (inv) S = (((Koff & v) ^ (((Bd & 1u) ? kap : 0ull))) & ~lb) | ((uint64_t)(Bd & 1u) << e);
  if (lane == e) S = kap;
  uint64_t lr = lam, li = lam | eb;  // linear parts for Re (x_e coefficient 0) and Im (1)
  uint64_t rem = v | eb;
  uint32_t sr = 0, si = 0, nel = 0;
  for (;;) {
    const uint64_t nz = ballot64(S != 0ull);
    if (!nz) break;
    const uint32_t a = (uint32_t)__builtin_ctzll(nz);
    const uint64_t Sa = rl64(S, a);
    const uint32_t b = (uint32_t)__builtin_ctzll(Sa);
    const uint64_t Sb = rl64(S, b);
    const uint64_t ab = (1ull << a) | (1ull << b);
    const uint64_t m1 = Sa & ~ab, m2 = Sb & ~ab;
    S ^= (m2 & bitmask64(m1, lane)) ^ (m1 & bitmask64(m2, lane));
    S &= ~ab;
    if (lane == a || lane == b) S = 0ull;
    {
      const uint64_t la = (lr >> a) & 1ull, lbb = (lr >> b) & 1ull;
      sr ^= (uint32_t)(la & lbb);
      lr ^= (m2 & (0ull - la)) ^ (m1 & (0ull - lbb)) ^ (m1 & m2);
      lr &= ~ab;
    }
    {
      const uint64_t la = (li >> a) & 1ull, lbb = (li >> b) & 1ull;
      si ^= (uint32_t)(la & lbb);
      li ^= (m2 & (0ull - la)) ^ (m1 & (0ull - lbb)) ^ (m1 & m2);
      li &= ~ab;
    }
    rem &= ~ab;
    ++nel;
  }
  const int r = __popcll(rem);
  const bool re_nz = (lr & rem) == 0ull, im_nz = (li & rem) == 0ull;
  // Re Z = (-1)^sr 2^{nel + r - 1}, Im Z likewise; both non-zero only with equal exponents.
  const int ez0 = (int)nel + r - 1;
  if (!re_nz && !im_nz) return rec;
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
  rec.nonzero = 1u;
  rec.k8 = (omega - kin) & 7u;  // <phi_A|omega phi> = omega conj(<phi|phi_A>)
  rec.e2 = ez - (int)(n + (uint32_t)__popcll(v));
  return rec;
}

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

__global__ __launch_bounds__(256) void k_inner(TermsView Tv, const uint64_t* __restrict__ Aoff,
                                               const uint8_t* __restrict__ Adiag, uint32_t L,
                                               double2* __restrict__ partial,
                                               uint32_t* __restrict__ err) {
  extern __shared__ __align__(16) double2 acc[];  // [kWaves][L]
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t wave = uniform32(tid >> 6);
  double2* my = acc + (size_t)wave * L;
  for (uint32_t l = lane; l < L; l += 64u) my[l] = make_double2(0.0, 0.0);
  const uint32_t n = Tv.n;
  const bool act = lane < n;
  const uint64_t chi = Tv.chi;
  uint32_t bad = 0;
  for (uint64_t term = (uint64_t)blockIdx.x * kWaves + wave; term < chi;
       term += (uint64_t)gridDim.x * kWaves) {
    const uint64_t off = (uint64_t)lane * chi + term;
    const uint64_t F = act ? Tv.F[off] : 0ull;
    const uint64_t G = act ? Tv.G[off] : 0ull;
    const uint64_t M = act ? Tv.M[off] : 0ull;
    const uint32_t g = act ? Tv.gamma[off] : 0u;
    const uint64_t v = uniform64(Tv.v[term]), s = uniform64(Tv.s[term]);
    const uint32_t omega = uniform32(Tv.omega[term]);
    const double2 b = Tv.b[term];
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
    for (uint32_t l = 0; l < L; ++l) {
      const uint64_t Ao = act ? Aoff[(uint64_t)l * n + lane] : 0ull;
      const uint32_t Ad = act ? Adiag[(uint64_t)l * n + lane] : 0u;
      uint64_t KAoff;
      uint32_t KAdiag;
      conj_gxg(G, Gt, Ao, Ad, lane, n, KAoff, KAdiag);
      const uint64_t Koff = KJoff ^ KAoff;
      const uint32_t Kdiag = (KJdiag + KAdiag) & 3u;
      const InnerRec rec = pair_record(Koff, Kdiag, v, s, omega, lane, n);
      bad |= rec.bad;
      if (rec.nonzero && lane == 0u) {
        const double2 val = rec_value(rec, b);
        double2 cur = my[l];
        cur.x += val.x;
        cur.y += val.y;
        my[l] = cur;
      }
    }
  }
  if (bad && lane == 0u) atomicOr(err, 1u);
  __syncthreads();
  for (uint32_t l = tid; l < L; l += 256u) {
    double re = 0.0, im = 0.0;
    for (int w = 0; w < kWaves; ++w) {
      re += acc[(size_t)w * L + l].x;
      im += acc[(size_t)w * L + l].y;
    }
    partial[(uint64_t)blockIdx.x * L + l] = make_double2(re, im);
  }
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

size_t inner_partial_elems(const TermsView& T, uint32_t L, uint32_t* n_blocks) {
  uint64_t waves = T.chi;
  uint64_t blocks = (waves + kWaves - 1) / kWaves;
  if (blocks > 2048) blocks = 2048;
  *n_blocks = (uint32_t)blocks;
  return (size_t)blocks * L;
}

hipError_t launch_inner(const TermsView& T, const uint64_t* Aoff, const uint8_t* Adiag, uint32_t L,
                        double2* partial, uint32_t n_blocks, double2* overlap, double* eta,
                        double* eta_sum, uint32_t* err, hipStream_t st) {
  const size_t sm = (size_t)kWaves * L * sizeof(double2);
  if (sm > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_inner, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_inner, dim3(n_blocks), dim3(256), sm, st, T, Aoff, Adiag, L, partial, err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_inner_reduce, dim3((L + 255) / 256), dim3(256), 0, st, partial, n_blocks, L,
                     T.n, overlap, eta);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_eta_sum, dim3(1), dim3(256), 0, st, eta, L, eta_sum);
  return hipGetLastError();
}

}  // namespace chsim
