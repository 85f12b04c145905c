// CH-form invariant check (debug call chsim_validate).
//
// A CH form |phi> = omega U_C U_H |s> stores the tableaux of U_C (Eq.
// (tableaux)): U_C^{-1} Z_p U_C = Z(G_p) and U_C^{-1} X_p U_C =
// i^{gamma_p} X(F_p) Z(M_p).  Conjugation keeps the Pauli commutation
// relations and Hermiticity, which gives three invariants of every term
// produced by unitary evolution:
//   (1) F G^T = I (X_p and Z_q anticommute iff p = q);
//   (2) M F^T is symmetric (X_p and X_q commute);
//   (3) gamma_p = F_p . M_p (mod 2) (the row i^gamma X(F) Z(M) is Hermitian).
// Stored words must also be in range: rows, v and s below bit n, gamma in
// Z_4, omega in Z_8.
//
// Mapping: one wave per term, lane p holds row p; the rows of other lanes
// arrive by readlane, so each test is O(n) per lane.
#include "device_common.hpp"
#include "internal.hpp"

namespace chsim {

namespace {

__global__ __launch_bounds__(256) void k_validate(TermsView T, uint64_t first, uint64_t count,
                                                  unsigned long long* out) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t item = (uint64_t)blockIdx.x * 4u + uniform32(threadIdx.x >> 6);
  if (item >= count) return;  // wave-uniform
  const uint64_t a = first + item;
  const uint32_t n = T.n;
  const uint64_t chi = T.chi;
  const uint64_t nmask = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
  const bool row = lane < n;
  const uint64_t off = (uint64_t)lane * chi + a;
  const uint64_t F = row ? T.F[off] : 0ull;
  const uint64_t G = row ? T.G[off] : 0ull;
  const uint64_t M = row ? T.M[off] : 0ull;
  const uint32_t g = row ? (uint32_t)T.gamma[off] : 0u;
  uint32_t what = 0;
  if (row && ((((F | G | M) & ~nmask) != 0ull) || g > 3u)) what |= CHSIM_BAD_RANGE;
  if (lane == 0 && ((((T.v[a] | T.s[a]) & ~nmask) != 0ull) || T.omega[a] > 7u)) what |= CHSIM_BAD_RANGE;
  // (1) and the rows of M F^T: bit q of R = par(M_p & F_q).
  uint64_t R = 0ull;
  bool fg = true;
  for (uint32_t q = 0; q < n; ++q) {
    const uint64_t Gq = rl64(G, q), Fq = rl64(F, q);
    if (par64(F & Gq) != (lane == q ? 1u : 0u)) fg = false;
    R |= (uint64_t)par64(M & Fq) << q;
  }
  if (row && !fg) what |= CHSIM_BAD_TABLEAU;
  // (2) bit q of R_p equals bit p of R_q.
  bool sym = true;
  for (uint32_t q = 0; q < n; ++q) {
    const uint64_t Rq = rl64(R, q);
    if (((R >> q) & 1ull) != ((Rq >> lane) & 1ull)) sym = false;
  }
  if (row && !sym) what |= CHSIM_BAD_SYMMETRY;
  // (3)
  if (row && par64(F & M) != (g & 1u)) what |= CHSIM_BAD_GAMMA;
  uint32_t all = 0;
  for (uint32_t b = 1; b <= CHSIM_BAD_GAMMA; b <<= 1)
    if (ballot64((what & b) != 0u)) all |= b;
  if (lane == 0 && all) {
    atomicAdd(&out[0], 1ull);
    atomicMin(&out[1], (unsigned long long)a);
    atomicOr(&out[2], (unsigned long long)all);
  }
}

__global__ void k_validate_clear(unsigned long long* out) {
  if (threadIdx.x == 0) {
    out[0] = 0ull;
    out[1] = ~0ull;
    out[2] = 0ull;
  }
}

}  // namespace

hipError_t launch_validate(const TermsView& T, uint64_t first, uint64_t count, unsigned long long* out,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_validate_clear, dim3(1), dim3(64), 0, st, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || count == 0) return e;
  const uint64_t blocks = (count + 3) / 4;
  for (uint64_t b0 = 0; b0 < blocks; b0 += (1u << 30)) {
    const uint64_t nb = blocks - b0 < (1u << 30) ? blocks - b0 : (1u << 30);
    const uint64_t f = first + b0 * 4u, c = count - b0 * 4u;
    hipLaunchKernelGGL(k_validate, dim3((uint32_t)nb), dim3(256), 0, st, T, f, c, out);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace chsim
