// CPU oracle for the sum-over-Cliffords hot path of Bravyi, Browne, Calpin,
// Campbell, Gosset, Howard, "Simulation of quantum circuits by low-rank
// stabilizer decompositions" (Quantum 3, 181 (2019); arXiv:1808.00128).
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  The product library
// never links, loads or calls it, and the two share no code, headers, tables
// or generators.
//
// Style: plain and slow on purpose.  Every binary matrix is one byte per
// entry, indexed the way the paper writes it (row p, column j), and every
// step follows the paper's definitions in the paper's order:
//   * CH-form data (F, G, M, gamma, v, s, omega) and its initialisation:
//     Sec. "Phase-sensitive Clifford simulator", Eqs. (phi), (tableaux), (Htype).
//   * Left/right multiplication rules L[S], L[CZ], L[CX], R[S], R[CZ], R[CX]:
//     the rule table at the end of that section.
//   * Hadamard update: Eqs. (H1)-(H7) and Proposition H with its proof.
//   * Amplitude <x|phi>: Eqs. (amplitude), (amplitude1).
//   * Sampling from one CH-form: the three-step sampler after Eq. (amplitude1).
//   * Sum-over-Cliffords expansion: Eqs. (Udecomp), (Vphi) and the per-gate
//     product formula; R(theta) decomposition: Eq. (Rtheta).
//   * Sparsification: Lemma (Sparsification) and its proof, Eq. (Omega).
//   * Inner product with an equatorial state: Lemma (Inner Product), Eq. (eqa1).
//   * Exponential sum: Lemma (Exponential Sum) and its proof, Eqs. (q), (Zreal),
//     (identity), (eq5), (Q), (real).
//   * Norm estimation: Lemma (Norm Estimation), Eq. (xi).
//   * Metropolis chain: Sec. "Heuristic Metropolis simulator", with the cached
//     Pauli Q_x updated by left multiplication as the paper describes.
//
// Readings where the paper is silent or ambiguous (each also listed in the
// design notes):
//   * qubit p <-> bit p of a uint64 bitstring; a row of a binary matrix is
//     exported as a uint64 with bit j = entry (p, j).
//   * inside a tableau row the X part stands left of the Z part.
//   * the global phase omega is kept as an integer k mod 8 (omega = e^{i pi k/4});
//     every factor the paper computes as a complex number is checked to be an
//     eighth root of unity before it is folded in.
//   * L[CX] uses the value of M_q before the update in (MF^T)_{q,r}.
//   * Prop. H: "first qubit" = lowest index; the single-qubit CH-form
//     omega S^a H^b |c> is found by search with a = 0 preferred.
//   * phase gate = diag(1, e^{i theta}); theta = theta' + k pi/2 with
//     theta' in [0, pi/2); S^k goes into both branches, and Eq. (Rtheta) for
//     theta' is multiplied by e^{i theta'/2}.
//   * Exponential sum outputs Re and Im as 0 or +-2^e (signs in {-1,0,1}).

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

typedef std::complex<double> cplx;
typedef long double ldbl;

static const double kPi = 3.14159265358979323846264338327950288;

// Branch coverage of the Hadamard update, for the exhaustive tests:
// [0] t == u; [1] V_0 non-empty; [2] V_0 empty; [3 + 8*y_q + 2*delta + v_q]
// the single-qubit case (y_q, delta, v_q).
#include <atomic>
static std::atomic<long> g_cover[3 + 16];

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator, written from its published definition
// (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC'11): 10 rounds; round multipliers 0xD2511F53 and 0xCD9E8D57; key bumped by
// the Weyl constants 0x9E3779B9 and 0xBB67AE85 before every round but the first.
// ---------------------------------------------------------------------------
static void philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

// Uniform double in [0,1) for (seed, index, sub, stream): counter
// (index_lo, index_hi, sub, stream), key (seed_lo, seed_hi); the first two
// output words give 53 bits: (w0 << 21) | (w1 >> 11), scaled by 2^-53.
static double uniform53(uint64_t seed, uint64_t index, uint32_t sub, uint32_t stream) {
  uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), sub, stream};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  philox(ctr, key, w);
  uint64_t bits = ((uint64_t)w[0] << 21) | (uint64_t)(w[1] >> 11);
  return (double)bits * (1.0 / 9007199254740992.0);
}

static const uint32_t kStreamSparsify = 0x53504152u;  // "SPAR"

// ---------------------------------------------------------------------------
// Eighth roots of unity.
// ---------------------------------------------------------------------------
static cplx root8(int k) {
  k = ((k % 8) + 8) % 8;
  return std::polar(1.0, kPi * k / 4.0);
}

// The paper computes several phase factors as complex numbers; under unitary
// evolution each one is an eighth root of unity.  Return k with z = e^{i pi k/4},
// or -1 if z is not one (the caller turns that into an error).
static int to_z8(cplx z) {
  for (int k = 0; k < 8; ++k)
    if (std::abs(z - root8(k)) < 1e-9) return k;
  return -1;
}

// ---------------------------------------------------------------------------
// CH-form, Sec. "Phase-sensitive Clifford simulator":
//   |phi> = omega U_C U_H |s>,  U_C^{-1} Z_p U_C = prod_j Z_j^{G_pj},
//   U_C^{-1} X_p U_C = i^{gamma_p} prod_j X_j^{F_pj} Z_j^{M_pj},  U_H = H(v).
// ---------------------------------------------------------------------------
struct CH {
  int n = 0;
  std::vector<uint8_t> F, G, M;  // n*n, entry (p, j) at [p*n + j]
  std::vector<int> gamma;        // Z_4
  std::vector<uint8_t> v, s;     // length n
  int omega = 0;                 // Z_8
  int error = 0;                 // set when a paper invariant is violated

  explicit CH(int n_) : n(n_) { reset(); }
  // Initial state |0^n>: G = F = I, M = 0, gamma = v = s = 0, omega = 1.
  void reset() {
    F.assign(n * n, 0); G.assign(n * n, 0); M.assign(n * n, 0);
    for (int p = 0; p < n; ++p) { F[p * n + p] = 1; G[p * n + p] = 1; }
    gamma.assign(n, 0); v.assign(n, 0); s.assign(n, 0);
    omega = 0; error = 0;
  }
  uint8_t& f(int p, int j) { return F[p * n + j]; }
  uint8_t& g(int p, int j) { return G[p * n + j]; }
  uint8_t& m(int p, int j) { return M[p * n + j]; }

  // ---- left multiplication U_C <- Gamma U_C (rule table) ----
  void L_S(int q) {
    for (int p = 0; p < n; ++p) m(q, p) ^= g(q, p);
    gamma[q] = (gamma[q] + 3) % 4;  // gamma_q - 1
  }
  void L_CZ(int q, int r) {
    for (int p = 0; p < n; ++p) {
      m(q, p) ^= g(r, p);
      m(r, p) ^= g(q, p);
    }
  }
  void L_CX(int q, int r) {
    // (M F^T)_{q,r} with M taken before the update of row q.
    int mf = 0;
    for (int j = 0; j < n; ++j) mf += m(q, j) * f(r, j);
    gamma[q] = (gamma[q] + gamma[r] + 2 * (mf % 2)) % 4;
    for (int p = 0; p < n; ++p) {
      g(r, p) ^= g(q, p);
      f(q, p) ^= f(r, p);
      m(q, p) ^= m(r, p);
    }
  }
  // ---- right multiplication U_C <- U_C Gamma (rule table) ----
  void R_S(int q) {
    for (int p = 0; p < n; ++p) {
      m(p, q) ^= f(p, q);
      gamma[p] = (gamma[p] - f(p, q) + 4) % 4;
    }
  }
  void R_CZ(int q, int r) {
    for (int p = 0; p < n; ++p) {
      m(p, q) ^= f(p, r);
      m(p, r) ^= f(p, q);
      gamma[p] = (gamma[p] + 2 * f(p, q) * f(p, r)) % 4;
    }
  }
  void R_CX(int q, int r) {
    for (int p = 0; p < n; ++p) {
      g(p, q) ^= g(p, r);
      f(p, r) ^= f(p, q);
      m(p, q) ^= m(p, r);
    }
  }

  // ---- Hadamard on qubit p: Eqs. (H1)-(H7), Proposition H ----
  void H(int p) {
    std::vector<uint8_t> t(n), u(n);
    int alpha = 0, beta = 0;
    for (int j = 0; j < n; ++j) {
      int vb = 1 - v[j];
      t[j] = s[j] ^ (g(p, j) & v[j]);                        // Eq. (H2)
      u[j] = s[j] ^ (f(p, j) & vb) ^ (m(p, j) & v[j]);       // Eq. (H2)
      alpha += g(p, j) * vb * s[j];                          // Eq. (H4)
      beta += m(p, j) * vb * s[j] + f(p, j) * v[j] * (m(p, j) + s[j]);
    }
    alpha %= 2;
    beta %= 2;
    const cplx I(0.0, 1.0);
    cplx ig = std::pow(I, gamma[p]);
    if (t == u) {
      // omega' = 2^{-1/2} [(-1)^alpha + i^{gamma_p} (-1)^beta], s' = t.
      cplx w = (1.0 / std::sqrt(2.0)) * ((alpha ? -1.0 : 1.0) + ig * (beta ? -1.0 : 1.0));
      int k = to_z8(w);
      if (k < 0) { error = 1; return; }
      omega = (omega + k) % 8;
      s = t;
      g_cover[0]++;
      return;
    }
    int delta = (gamma[p] + 2 * (alpha + beta)) % 4;
    superpose(t, u, alpha, delta);
  }

  // CH form of (-1)^alpha 2^{-1/2} U_C U_H (|t> + i^delta |u>) for t != u, by
  // Proposition H and its proof (the second half of the Hadamard update).
  void superpose(const std::vector<uint8_t>& t, const std::vector<uint8_t>& u, int alpha, int delta) {
    const cplx I(0.0, 1.0);
    // Proof of Prop. H: subsets V_0, V_1 and the C-type circuit V_C.
    std::vector<int> V0, V1;
    for (int i = 0; i < n; ++i)
      if (t[i] != u[i]) (v[i] ? V1 : V0).push_back(i);
    int q;
    g_cover[V0.empty() ? 2 : 1]++;
    if (!V0.empty()) {
      q = V0[0];
      // V_C = prod_{i in V0 \ q} CX_{q,i} * prod_{i in V1} CZ_{q,i}; U_C <- U_C V_C.
      for (size_t a = 1; a < V0.size(); ++a) R_CX(q, V0[a]);
      for (size_t a = 0; a < V1.size(); ++a) R_CZ(q, V1[a]);
    } else {
      q = V1[0];
      // V_C = prod_{i in V1 \ q} CX_{i,q}.
      for (size_t a = 1; a < V1.size(); ++a) R_CX(V1[a], q);
    }
    std::vector<uint8_t> y(n), z(n);
    if (t[q] == 1) { y = u; y[q] ^= 1; z = u; }
    else { y = t; z = t; z[q] ^= 1; }
    // Single-qubit state H^{v_q}(|y_q> + i^delta |z_q>) = w S^a H^b |c>: find
    // (a, b, c, w) by trying every candidate, a = 0 first.
    const double h = 1.0 / std::sqrt(2.0);
    cplx tv[2] = {0.0, 0.0};
    tv[y[q]] += 1.0;
    tv[z[q]] += std::pow(I, delta);
    if (v[q]) {
      cplx a0 = h * (tv[0] + tv[1]), a1 = h * (tv[0] - tv[1]);
      tv[0] = a0; tv[1] = a1;
    }
    int fa = -1, fb = -1, fc = -1;
    cplx fw = 0.0;
    for (int a = 0; a < 2 && fa < 0; ++a)
      for (int b = 0; b < 2 && fa < 0; ++b)
        for (int c = 0; c < 2 && fa < 0; ++c) {
          cplx cv[2] = {0.0, 0.0};
          if (b) { cv[0] = h; cv[1] = c ? -h : h; } else { cv[c] = 1.0; }
          if (a) cv[1] *= I;
          cplx w = std::conj(cv[0]) * tv[0] + std::conj(cv[1]) * tv[1];  // <cand|target>
          if (std::abs(tv[0] - w * cv[0]) < 1e-9 && std::abs(tv[1] - w * cv[1]) < 1e-9) {
            fa = a; fb = b; fc = c; fw = w;
          }
        }
    if (fa < 0) { error = 2; return; }
    g_cover[3 + 8 * y[q] + 2 * delta + v[q]]++;
    if (fa) R_S(q);  // W_C = V_C S_q^a
    // Eq. (H7): omega' = 2^{-1/2} (-1)^alpha w.
    int k = to_z8(h * (alpha ? -1.0 : 1.0) * fw);
    if (k < 0) { error = 3; return; }
    omega = (omega + k) % 8;
    s = y;
    s[q] = (uint8_t)fc;
    v[q] = (uint8_t)fb;  // W_H = U_H H_q^{b xor v_q}
  }

  // ---- projective gate (I + (-1)^bit Z_q) / 2, end of Sec. "Phase-sensitive
  // Clifford simulator" ----
  // Gamma U_C U_H |s> = (1/2) U_C U_H (I + Q) |s> with Q = U_H^-1 U_C^-1 P U_C U_H.
  // U_C^-1 Z_q U_C = Z(G_q) (Eq. (tableaux)); conjugating by U_H = H(v) turns the
  // Z on qubits with v_j = 1 into X: Q = (-1)^bit X(G_q & v) Z(G_q & ~v), so
  // (I + Q)|s> = |s> + i^delta |t>, t = s + (G_q & v), i^delta = (-1)^{bit + (G_q & ~v).s}.
  // Returns 1: state unchanged (t = s, i^delta = 1); 0: the projection is zero
  // (t = s, i^delta = -1); 2: the state becomes 2^{-1/2} times the CH form of
  // 2^{-1/2} U_C U_H (|s> + i^delta |t>) (Prop. H, as for the Hadamard).
  int project_z(int q, int bit) {
    std::vector<uint8_t> t(n);
    int sign = bit;
    bool same = true;
    for (int j = 0; j < n; ++j) {
      int gq = g(q, j);
      t[j] = s[j] ^ (gq & v[j]);
      if (t[j] != s[j]) same = false;
      sign += gq * (1 - v[j]) * s[j];
    }
    sign %= 2;
    if (same) return sign ? 0 : 1;
    std::vector<uint8_t> s0 = s;
    superpose(s0, t, 0, 2 * sign);
    return 2;
  }

  // ---- projective gate (I + P) / 2 for any Hermitian Pauli P = i^a X(x) Z(z)
  // (a = x.z mod 2; X part left of the Z part), end of Sec. "Phase-sensitive
  // Clifford simulator" ----
  // Gamma U_C U_H |s> = (1/2) U_C U_H (I + Q) |s>, Q = U_H^-1 U_C^-1 P U_C U_H.
  // By Eq. (tableaux), U_C^-1 P U_C = i^a prod_{p in x} i^{gamma_p} X(F_p) Z(M_p)
  // prod_{p in z} Z(G_p); the product is kept as i^c X(u) Z(w), using
  // X(u) Z(w) X(f) Z(m) = (-1)^{w.f} X(u + f) Z(w + m).  U_H = H(v) swaps X and
  // Z on the qubits with v_j = 1 (H X^u Z^w H = (-1)^{u w} X^w Z^u), so
  // Q = i^c (-1)^{sum_{j: v_j = 1} u_j w_j} X(u') Z(w') and
  // (I + Q)|s> = |s> + i^delta |t>, t = s + u', i^delta = i^c (-1)^{... + w'.s}.
  // Returns 1 (state unchanged), 0 (projected to zero) or 2 (the state becomes
  // 2^{-1/2} times the CH form of 2^{-1/2} U_C U_H (|s> + i^delta |t>), Prop. H).
  int project_pauli(int a, const std::vector<uint8_t>& px, const std::vector<uint8_t>& pz) {
    std::vector<uint8_t> u(n, 0), w(n, 0);
    int c = ((a % 4) + 4) % 4;
    for (int p = 0; p < n; ++p) {
      if (!px[p]) continue;
      int dot = 0;
      for (int j = 0; j < n; ++j) dot += w[j] * f(p, j);
      c = (c + gamma[p] + 2 * (dot % 2)) % 4;
      for (int j = 0; j < n; ++j) {
        u[j] ^= f(p, j);
        w[j] ^= m(p, j);
      }
    }
    for (int p = 0; p < n; ++p)
      if (pz[p])
        for (int j = 0; j < n; ++j) w[j] ^= g(p, j);
    std::vector<uint8_t> u2(n), w2(n), t(n);
    int sw = 0, ws = 0;
    bool same = true;
    for (int j = 0; j < n; ++j) {
      if (v[j]) { u2[j] = w[j]; w2[j] = u[j]; sw += u[j] * w[j]; }
      else { u2[j] = u[j]; w2[j] = w[j]; }
      t[j] = s[j] ^ u2[j];
      if (u2[j]) same = false;
      ws += w2[j] * s[j];
    }
    int delta = (c + 2 * (sw % 2) + 2 * (ws % 2)) % 4;
    if (same) {
      // Q|s> = i^delta |s>: a Hermitian Q has eigenvalue +1 or -1.
      if (delta % 2) { error = 4; return -1; }
      return delta == 0 ? 1 : 0;
    }
    std::vector<uint8_t> s0 = s;
    superpose(s0, t, 0, delta);
    return 2;
  }

  // ---- amplitude <x|phi>, Eqs. (amplitude), (amplitude1) ----
  // Returns 1 if nonzero; then <x|phi> = e^{i pi k8/4} 2^{-vcount/2}.
  int amplitude(uint64_t x, int* k8, int* vcount) const {
    std::vector<uint8_t> t(n, 0), u(n, 0);
    int mu = 0;
    for (int p = 0; p < n; ++p) {
      if (!((x >> p) & 1)) continue;
      // Q <- Q * i^{gamma_p} X(F_p) Z(M_p), with Q = i^mu Z(t) X(u):
      // Z(t) X(u) X(f) Z(m) = (-1)^{(u+f).m} Z(t+m) X(u+f).
      int dot = 0;
      for (int j = 0; j < n; ++j) {
        u[j] ^= F[p * n + j];
        dot += u[j] * M[p * n + j];
        t[j] ^= M[p * n + j];
      }
      mu = (mu + gamma[p] + 2 * (dot % 2)) % 4;
    }
    int sign = 0, vc = 0;
    for (int j = 0; j < n; ++j) {
      if (v[j]) { sign += u[j] * s[j]; ++vc; }
      else if (u[j] != s[j]) return 0;
    }
    *k8 = (omega + 2 * mu + 4 * (sign % 2)) % 8;
    *vcount = vc;
    return 1;
  }

  // ---- sampling from |<x|phi>|^2 (three-step sampler) ----
  // flips: bit j flips w_j where v_j = 1 (the random coin tosses).
  uint64_t sample(uint64_t flips) const {
    std::vector<uint8_t> w(s);
    for (int j = 0; j < n; ++j)
      if (v[j] && ((flips >> j) & 1)) w[j] ^= 1;
    uint64_t x = 0;
    for (int i = 0; i < n; ++i) {  // x = w G^T (mod 2)
      int acc = 0;
      for (int j = 0; j < n; ++j) acc += w[j] * G[i * n + j];
      if (acc % 2) x |= (uint64_t)1 << i;
    }
    return x;
  }

  // Invariants: F G^T = I (mod 2); M F^T symmetric (mod 2); gamma_p = F_p.M_p (mod 2).
  int check() const {
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        int fg = 0, mf = 0, mf2 = 0;
        for (int j = 0; j < n; ++j) {
          fg += F[a * n + j] * G[b * n + j];
          mf += M[a * n + j] * F[b * n + j];
          mf2 += M[b * n + j] * F[a * n + j];
        }
        if (fg % 2 != (a == b ? 1 : 0)) return 1;
        if (mf % 2 != mf2 % 2) return 2;
      }
    for (int p = 0; p < n; ++p) {
      int fm = 0;
      for (int j = 0; j < n; ++j) fm += F[p * n + j] * M[p * n + j];
      if ((gamma[p] - fm) % 2 != 0) return 3;
    }
    return error ? 10 + error : 0;
  }

  void export_packed(uint64_t* Fo, uint64_t* Go, uint64_t* Mo, uint8_t* go, uint64_t* vo,
                     uint64_t* so, int* wo) const {
    for (int p = 0; p < n; ++p) {
      uint64_t fr = 0, gr = 0, mr = 0;
      for (int j = 0; j < n; ++j) {
        fr |= (uint64_t)F[p * n + j] << j;
        gr |= (uint64_t)G[p * n + j] << j;
        mr |= (uint64_t)M[p * n + j] << j;
      }
      if (Fo) Fo[p] = fr;
      if (Go) Go[p] = gr;
      if (Mo) Mo[p] = mr;
      if (go) go[p] = (uint8_t)gamma[p];
    }
    uint64_t vv = 0, ss = 0;
    for (int j = 0; j < n; ++j) {
      vv |= (uint64_t)v[j] << j;
      ss |= (uint64_t)s[j] << j;
    }
    if (vo) *vo = vv;
    if (so) *so = ss;
    if (wo) *wo = omega;
  }
};

// Gate codes of the circuit interface.
enum { OP_H = 0, OP_S = 1, OP_CX = 2, OP_CZ = 3, OP_SLOT = 4, OP_CCZ = 5 };

static int ch_apply(CH& c, int op, int q, int r) {
  if (q < 0 || q >= c.n) return 1;
  switch (op) {
    case OP_H: c.H(q); return c.error ? 2 : 0;
    case OP_S: c.L_S(q); return 0;
    case OP_CX: if (r < 0 || r >= c.n || r == q) return 1; c.L_CX(q, r); return 0;
    case OP_CZ: if (r < 0 || r >= c.n || r == q) return 1; c.L_CZ(q, r); return 0;
    default: return 1;
  }
}

// ---------------------------------------------------------------------------
// Decomposition of the phase gate diag(1, e^{i theta}), Eq. (Rtheta).
// theta = theta' + k pi/2, theta' in [0, pi/2): diag(1,e^{i theta}) = S^k diag(1, e^{i theta'})
// and diag(1,e^{i theta'}) = e^{i theta'/2} R(theta') = c0 I + c1 S with
//   c0 = e^{i theta'/2} (cos(theta'/2) - sin(theta'/2)),
//   c1 = e^{i theta'/2} sqrt(2) e^{-i pi/4} sin(theta'/2).
// Branch 0 is S^k with weight c0, branch 1 is S^{k+1} with weight c1.
// ---------------------------------------------------------------------------
static void phase_decomp(double theta, cplx* c0, cplx* c1, int* k) {
  double quarter = kPi / 2.0;
  double kf = std::floor(theta / quarter);
  double tp = theta - kf * quarter;
  if (tp < 0.0) { tp += quarter; kf -= 1.0; }
  if (tp >= quarter) { tp -= quarter; kf += 1.0; }
  long long kk = (long long)kf;
  *k = (int)(((kk % 4) + 4) % 4);
  cplx ph = std::polar(1.0, tp / 2.0);
  *c0 = ph * (std::cos(tp / 2.0) - std::sin(tp / 2.0));
  *c1 = ph * std::sqrt(2.0) * std::polar(1.0, -kPi / 4.0) * std::sin(tp / 2.0);
}

// ---------------------------------------------------------------------------
// Sum-over-Cliffords terms: U = sum_j c_j K_j built from per-slot decompositions
// (Eqs. (Udecomp), (Vphi)); exact enumeration or the Sparsification Lemma's
// random Omega = (||c||_1 / k) sum_alpha omega_alpha (Eq. (Omega)).
// ---------------------------------------------------------------------------
struct Slot {
  int nb = 0;                                // number of branches j
  cplx c[8];                                 // coefficient c_j
  std::vector<std::array<int, 3>> k[8];      // Clifford K_j as (op, q, r), applied in order
};

// Slot for diag(1, e^{i theta}) on qubit q: branch 0 = S^k, branch 1 = S^{k+1}.
static void phase_slot(double theta, int q, Slot* sl) {
  int k;
  phase_decomp(theta, &sl->c[0], &sl->c[1], &k);
  sl->nb = 2;
  for (int j = 0; j < 2; ++j) {
    sl->k[j].clear();
    for (int a = 0; a < (k + j) % 4; ++a) sl->k[j].push_back({OP_S, q, 0});
  }
}

// CCZ on qubits (a, b, c) by the lifting lemma, Eq. (CCZ decomposition):
// CCZ = (1/6) [ I + CZ_ab + CZ_ac + CZ_bc + CZ_ab CZ_ac Z_a + CZ_ab CZ_bc Z_b
//               + CZ_ac CZ_bc Z_c - CZ_ab CZ_ac CZ_bc Z_a Z_b Z_c ],
// branches in that order, Z = S S.  The paper prints the prefactor 2/9; with
// 2/9 the sum is 4/3 on |000>, while 1/6 gives CCZ exactly and
// ||c||_1^2 = (8/6)^2 = 16/9, the paper's value of xi(CCZ), and matches its
// state decomposition |CCZ> = (1/6) sum_Q Q |+++>.
static void ccz_slot(int a, int b, int c, Slot* sl) {
  sl->nb = 8;
  const int pair[3][2] = {{a, b}, {a, c}, {b, c}};
  // cz[j]: which of the pairs (ab, ac, bc) branch j applies; zq[j]: qubits with Z.
  const int cz[8] = {0, 1, 2, 4, 1 | 2, 1 | 4, 2 | 4, 1 | 2 | 4};
  const int zq[8][3] = {{-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1},
                        {a, -1, -1},  {b, -1, -1},  {c, -1, -1},  {a, b, c}};
  for (int j = 0; j < 8; ++j) {
    sl->c[j] = cplx(j == 7 ? -1.0 / 6.0 : 1.0 / 6.0, 0.0);
    sl->k[j].clear();
    for (int e = 0; e < 3; ++e)
      if (cz[j] >> e & 1) sl->k[j].push_back({OP_CZ, pair[e][0], pair[e][1]});
    for (int e = 0; e < 3; ++e)
      if (zq[j][e] >= 0) {
        sl->k[j].push_back({OP_S, zq[j][e], 0});
        sl->k[j].push_back({OP_S, zq[j][e], 0});
      }
  }
}

struct Terms {
  int n = 0;
  std::vector<int> op, q, r;  // circuit (SLOT entries refer to slots in order)
  std::vector<Slot> slots;
  uint64_t chi = 0;
  int mode = 0;  // 0 exact, 1 sparsify
  uint64_t seed = 0;
  double l1 = 0.0;                   // ||c||_1 of the full product decomposition
  std::vector<uint64_t> index;       // term indices alpha that were built
  std::vector<CH> ch;                // their CH-forms
  std::vector<cplx> b;               // their coefficients b_alpha
  std::vector<std::vector<uint8_t>> branch;  // branch choice per slot
  int error = 0;
};

static void choose_branches(const Terms& T, uint64_t alpha, std::vector<uint8_t>& br, cplx& b) {
  size_t m = T.slots.size();
  br.assign(m, 0);
  if (T.mode == 0) {
    // Exact expansion: alpha's digits in the mixed radix (nb_0, nb_1, ...),
    // slot 0 least significant, pick the branch of each slot; b = prod_p c_j.
    b = 1.0;
    uint64_t rem = alpha;
    for (size_t p = 0; p < m; ++p) {
      br[p] = (uint8_t)(rem % (uint64_t)T.slots[p].nb);
      rem /= (uint64_t)T.slots[p].nb;
      b *= T.slots[p].c[br[p]];
    }
  } else {
    // Sparsification: j ~ |c_j| / ||c||_1 independently per slot (product form of
    // p_j), b = (||c||_1 / k) prod_p c_j / |c_j|.  Branch rule: the smallest j with
    // u * W < sum_{i<=j} w_i, where w_i = |c_i| and W = sum_i w_i.
    cplx ph = 1.0;
    for (size_t p = 0; p < m; ++p) {
      const Slot& sl = T.slots[p];
      double w[8], W = 0.0;
      for (int j = 0; j < sl.nb; ++j) {
        w[j] = std::sqrt(sl.c[j].real() * sl.c[j].real() + sl.c[j].imag() * sl.c[j].imag());
        W += w[j];
      }
      double u = uniform53(T.seed, alpha, (uint32_t)p, kStreamSparsify);
      int j = sl.nb - 1;
      double cum = 0.0;
      for (int i = 0; i + 1 < sl.nb; ++i) {
        cum += w[i];
        if (u * W < cum) { j = i; break; }
      }
      br[p] = (uint8_t)j;
      ph *= sl.c[j] / w[j];
    }
    b = (T.l1 / (double)T.chi) * ph;
  }
}

static void evolve_term(const Terms& T, const std::vector<uint8_t>& br, CH& c, int* err) {
  c.reset();
  size_t slot = 0;
  for (size_t g = 0; g < T.op.size(); ++g) {
    if (T.op[g] == OP_SLOT || T.op[g] == OP_CCZ) {
      for (const auto& k : T.slots[slot].k[br[slot]])
        if (ch_apply(c, k[0], k[1], k[2])) {
          *err = 1;
          return;
        }
      ++slot;
    } else if (ch_apply(c, T.op[g], T.q[g], T.r[g])) {
      *err = 1;
      return;
    }
  }
}

template <class Fn>
static void parallel_for(size_t count, int threads, Fn fn) {
  if (threads <= 1 || count < 2) {
    for (size_t i = 0; i < count; ++i) fn(i, 0);
    return;
  }
  std::vector<std::thread> pool;
  size_t chunk = (count + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    size_t lo = t * chunk, hi = std::min(count, lo + chunk);
    if (lo >= hi) break;
    pool.emplace_back([=, &fn]() {
      for (size_t i = lo; i < hi; ++i) fn(i, t);
    });
  }
  for (auto& th : pool) th.join();
}

// Compensated (Neumaier) accumulation in long double.
struct CSum {
  ldbl s = 0, c = 0;
  void add(ldbl x) {
    ldbl t = s + x;
    if (std::fabs((double)s) >= std::fabs((double)x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
  }
  ldbl value() const { return s + c; }
};

// Value of a term record e^{i pi k/4} 2^{-vc/2} times b, in long double.
static void record_value(cplx b, int k, int vc, ldbl* re, ldbl* im) {
  const ldbl h = 0.707106781186547524400844362104849039L;
  ldbl mag = std::ldexp((ldbl)1.0, -(vc / 2));
  if (vc % 2) mag *= h;
  ldbl cr, ci;
  switch (((k % 8) + 8) % 8) {
    case 0: cr = 1; ci = 0; break;
    case 1: cr = h; ci = h; break;
    case 2: cr = 0; ci = 1; break;
    case 3: cr = -h; ci = h; break;
    case 4: cr = -1; ci = 0; break;
    case 5: cr = -h; ci = -h; break;
    case 6: cr = 0; ci = -1; break;
    default: cr = h; ci = -h; break;
  }
  ldbl br = b.real(), bi = b.imag();
  *re = mag * (br * cr - bi * ci);
  *im = mag * (br * ci + bi * cr);
}

// ---------------------------------------------------------------------------
// Exponential sum Z(B) = sum_x i^{x B x^T}, Lemma (Exponential Sum).
// ---------------------------------------------------------------------------
// Z_2 sum of (-1)^{Q(x)}, Q(x) = x M x^T + L x^T (mod 2), M a general binary
// matrix (non-symmetric, non-zero diagonal allowed).  Result 0 or sign*2^exp.
static void z2_sum(int n, std::vector<uint8_t> M, std::vector<uint8_t> L, int* zero, int* sign,
                   int* expo) {
  int sg = 0, ex = 0;
  for (;;) {
    // Find a pair a != b with M_ab != M_ba ("otherwise permute the variables").
    int pa = -1, pb = -1;
    for (int a = 0; a < n && pa < 0; ++a)
      for (int b = a + 1; b < n; ++b)
        if (M[a * n + b] != M[b * n + a]) { pa = a; pb = b; break; }
    if (pa < 0) {
      // M symmetric: Q(x) = sum_a (M_aa + L_a) x_a is linear.
      for (int a = 0; a < n; ++a)
        if ((M[a * n + a] ^ L[a]) & 1) { *zero = 1; *sign = 0; *expo = 0; return; }
      *zero = 0; *sign = sg ? -1 : 1; *expo = ex + n;
      return;
    }
    // x = (x_a, x_b, y).  mu_1(y) = L_a + M_aa + m1.y, mu_2(y) = L_b + M_bb + m2.y,
    // identity (identity): sum over x_a, x_b = 2 (-1)^{mu_1 mu_2}; Eq. (eq5) for Q'(y).
    std::vector<int> rest;
    for (int a = 0; a < n; ++a)
      if (a != pa && a != pb) rest.push_back(a);
    int n2 = n - 2;
    int c1 = (L[pa] + M[pa * n + pa]) & 1;
    int c2 = (L[pb] + M[pb * n + pb]) & 1;
    std::vector<uint8_t> m1(n2), m2(n2);
    for (int i = 0; i < n2; ++i) {
      int y = rest[i];
      m1[i] = (M[pa * n + y] + M[y * n + pa]) & 1;
      m2[i] = (M[pb * n + y] + M[y * n + pb]) & 1;
    }
    std::vector<uint8_t> M2(n2 * n2), L2(n2);
    for (int i = 0; i < n2; ++i) {
      for (int j = 0; j < n2; ++j)
        M2[i * n2 + j] = (M[rest[i] * n + rest[j]] + m1[i] * m2[j]) & 1;
      L2[i] = (L[rest[i]] + c1 * m2[i] + c2 * m1[i]) & 1;
    }
    sg ^= (c1 * c2) & 1;
    ex += 1;
    M.swap(M2);
    L.swap(L2);
    n = n2;
  }
}

// B: N x N, symmetric, off-diagonal entries in {0,1}, diagonal in Z_4 (byte matrix).
// Re Z = re_sign 2^re_exp (0 if re_sign == 0), likewise Im.
static void expsum(int N, const uint8_t* B, int* re_sign, int* re_exp, int* im_sign, int* im_exp) {
  // Eq. (q): M upper triangular from B; B_aa = 2 L_a + K_a.  Eq. (Q): Z_2 form on
  // N + 1 variables with quadratic part M_ab + K_a K_b (a < b) and K_a x_a x_{N+1}.
  int n1 = N + 1;
  std::vector<uint8_t> Mq(n1 * n1, 0), Lq(n1, 0);
  std::vector<int> Kv(N), Lv(N);
  for (int a = 0; a < N; ++a) {
    int d = B[a * N + a] % 4;
    Lv[a] = d / 2;
    Kv[a] = d % 2;
  }
  for (int a = 0; a < N; ++a) {
    for (int b = a + 1; b < N; ++b) Mq[a * n1 + b] = (uint8_t)((B[a * N + b] + Kv[a] * Kv[b]) & 1);
    Mq[a * n1 + N] = (uint8_t)Kv[a];
    Lq[a] = (uint8_t)Lv[a];
  }
  // Eq. (real): Re Z = 1/2 sum (-1)^Q, Im Z = 1/2 sum (-1)^{Q + x_{N+1}}.
  for (int part = 0; part < 2; ++part) {
    Lq[N] = (uint8_t)part;
    int zero, sign, ex;
    z2_sum(n1, Mq, Lq, &zero, &sign, &ex);
    int* so = part ? im_sign : re_sign;
    int* eo = part ? im_exp : re_exp;
    if (zero) { *so = 0; *eo = 0; }
    else { *so = sign; *eo = ex - 1; }
  }
}

// ---------------------------------------------------------------------------
// Inner product <phi_A | phi> with an equatorial state, Lemma (Inner Product).
// A: off-diagonal rows as uint64 (bit b of row a = A_ab) and diagonal in Z_4.
// Result record: 0, or e^{i pi k/4} 2^{e2/2}, for <phi_A | phi> including omega.
// ---------------------------------------------------------------------------
static int inner_record(const CH& c, const uint64_t* Aoff, const uint8_t* Adiag, int* k8, int* e2) {
  int n = c.n;
  // J in M_n: diag(J) = gamma, J_ab = (M F^T)_ab mod 2 for a != b.
  std::vector<int> AJ(n * n);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      int jab;
      if (a == b) jab = c.gamma[a];
      else {
        int acc = 0;
        for (int k = 0; k < n; ++k) acc += c.M[a * n + k] * c.F[b * n + k];
        jab = acc % 2;
      }
      int aab = (a == b) ? (Adiag[a] % 4) : (int)((Aoff[a] >> b) & 1);
      AJ[a * n + b] = aab + jab;
    }
  // K = G^T (A + J) G over the integers; off-diagonal mod 2, diagonal mod 4.
  std::vector<long long> T1(n * n, 0), K(n * n, 0);
  for (int c1 = 0; c1 < n; ++c1)
    for (int b = 0; b < n; ++b) {
      long long acc = 0;
      for (int d = 0; d < n; ++d) acc += (long long)AJ[c1 * n + d] * c.G[d * n + b];
      T1[c1 * n + b] = acc;
    }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      long long acc = 0;
      for (int c1 = 0; c1 < n; ++c1) acc += (long long)c.G[c1 * n + a] * T1[c1 * n + b];
      K[a * n + b] = (a == b) ? (acc % 4) : (acc % 2);
    }
  // s K s^T (mod 4) and s + sK (mod 2).
  long long sks = 0;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) sks += (long long)c.s[a] * K[a * n + b] * c.s[b];
  std::vector<int> ssk(n);
  for (int b = 0; b < n; ++b) {
    long long acc = c.s[b];
    for (int a = 0; a < n; ++a) acc += (long long)c.s[a] * K[a * n + b];
    ssk[b] = (int)(acc % 2);
  }
  int sv = 0;
  for (int j = 0; j < n; ++j) sv += c.s[j] * c.v[j];
  // B = restriction of K + 2 diag(s + sK) to the support of v.
  std::vector<int> sup;
  for (int j = 0; j < n; ++j)
    if (c.v[j]) sup.push_back(j);
  int N = (int)sup.size();
  std::vector<uint8_t> B(N * N);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      int a = sup[i], b = sup[j];
      if (i == j) B[i * N + j] = (uint8_t)((K[a * n + a] + 2 * ssk[a]) % 4);
      else B[i * N + j] = (uint8_t)(K[a * n + b] % 2);
    }
  int rs, re, is, ie;
  expsum(N, B.data(), &rs, &re, &is, &ie);
  // Z = rs 2^re + i is 2^ie as e^{i pi kz/4} 2^{ez/2}.
  int kz, ez;
  if (rs == 0 && is == 0) return 0;
  if (is == 0) { kz = rs > 0 ? 0 : 4; ez = 2 * re; }
  else if (rs == 0) { kz = is > 0 ? 2 : 6; ez = 2 * ie; }
  else {
    if (re != ie) return -1;  // cannot happen for a Gauss sum; flagged as an error
    if (rs > 0 && is > 0) kz = 1;
    else if (rs < 0 && is > 0) kz = 3;
    else if (rs < 0 && is < 0) kz = 5;
    else kz = 7;
    ez = 2 * re + 1;
  }
  // <phi|phi_A> = 2^{-(n+|v|)/2} i^{sKs^T} (-1)^{s.v} Z(B) for omega = 1;
  // <phi_A | omega phi> = omega conj(<phi|phi_A>).
  int kin = (int)((2 * (sks % 4) + 4 * (sv % 2) + kz) % 8);
  *k8 = ((c.omega - kin) % 8 + 8) % 8;
  *e2 = ez - (n + N);
  return 1;
}

// ---------------------------------------------------------------------------
// Inner product <a|b> of two CH forms (general stabilizer states).  The paper
// states the O(n^3) cost and defers the method to earlier work (Sec. "Fast
// norm estimation" and the introduction); the definition is the sum
// <a|b> = sum_x conj(<x|a>) <x|b> with each amplitude from Eqs. (amplitude),
// (amplitude1).  Two routes:
//   ch_inner_brute: that sum over all 2^n strings (small n; the definition).
//   ch_inner: the same sum restricted to where both amplitudes are non-zero.
// <x|a> != 0 iff x = (s_a + y) G_a^T with y supported on v_a (the three-step
// sampler's parametrization; u = x F_a = s_a + y since F_a G_a^T = I), and
// <x|b> != 0 iff (x F_b)_j = (s_b)_j for every j outside v_b.  Their
// intersection is x(z) = x_0 + sum_k z_k d_k (Gaussian elimination over GF(2)
// in y), an affine space of dimension N.  On it the phase
// conj(<x|a>) <x|b> / |.| = e^{i pi h(x)/4} has h(x(z)) - h(x_0) even, and
// q(z) = (h(x(z)) - h(x_0)) / 2 (mod 4) is a quadratic form of the kind of
// Lemma (Exponential Sum) (each amplitude's exponent is, and composing with an
// affine map keeps that form), so
//   <a|b> = e^{i pi h(x_0)/4} 2^{-(|v_a| + |v_b|)/2} Z(B_q),
// with B_q read off q at z = 0, e_k and e_k + e_l, and Z by the exponential
// sum of Lemma (Exponential Sum).  q is checked against B_q on further points.
// ---------------------------------------------------------------------------
static cplx ch_inner_brute(const CH& a, const CH& b) {
  const int n = a.n;
  CSum sr, si;
  for (uint64_t x = 0; x < ((uint64_t)1 << n); ++x) {
    int ka, va, kb, vb;
    if (!a.amplitude(x, &ka, &va) || !b.amplitude(x, &kb, &vb)) continue;
    ldbl re, im;
    record_value(cplx(1.0, 0.0), kb - ka, va + vb, &re, &im);
    sr.add(re);
    si.add(im);
  }
  return cplx((double)sr.value(), (double)si.value());
}

// Returns 1 with <a|b> = e^{i pi k8/4} 2^{e2/2}, 0 if <a|b> = 0, < 0 on an
// internal inconsistency.
static int ch_inner(const CH& a, const CH& b, int* k8, int* e2) {
  const int n = a.n;
  if (b.n != n) return -1;
  // Columns of G_a: x(y) = sum_j (s_a + y)_j colG_j.
  auto colG = [&](int j) {
    std::vector<uint8_t> c(n);
    for (int i = 0; i < n; ++i) c[i] = a.G[i * n + j];
    return c;
  };
  std::vector<uint8_t> x1(n, 0);
  for (int j = 0; j < n; ++j)
    if (a.s[j]) {
      std::vector<uint8_t> c = colG(j);
      for (int i = 0; i < n; ++i) x1[i] ^= c[i];
    }
  // Unknowns y_i, i in v_a; equations (x(y) F_b)_j = s_b[j] for j outside v_b.
  std::vector<int> var;
  for (int i = 0; i < n; ++i)
    if (a.v[i]) var.push_back(i);
  const int nv = (int)var.size();
  std::vector<std::vector<uint8_t>> eq;  // nv coefficients + rhs
  for (int j = 0; j < n; ++j) {
    if (b.v[j]) continue;
    std::vector<uint8_t> row(nv + 1, 0);
    for (int k = 0; k < nv; ++k) {
      std::vector<uint8_t> c = colG(var[k]);
      int acc = 0;
      for (int p = 0; p < n; ++p) acc += c[p] * b.F[p * n + j];
      row[k] = (uint8_t)(acc & 1);
    }
    int acc = 0;
    for (int p = 0; p < n; ++p) acc += x1[p] * b.F[p * n + j];
    row[nv] = (uint8_t)((b.s[j] + acc) & 1);
    eq.push_back(row);
  }
  // Reduced row echelon form.
  std::vector<int> pivcol;
  int r = 0;
  for (int k = 0; k < nv && r < (int)eq.size(); ++k) {
    int piv = -1;
    for (int i = r; i < (int)eq.size(); ++i)
      if (eq[i][k]) { piv = i; break; }
    if (piv < 0) continue;
    std::swap(eq[r], eq[piv]);
    for (int i = 0; i < (int)eq.size(); ++i)
      if (i != r && eq[i][k])
        for (int c = 0; c <= nv; ++c) eq[i][c] ^= eq[r][c];
    pivcol.push_back(k);
    ++r;
  }
  for (int i = r; i < (int)eq.size(); ++i)
    if (eq[i][nv]) return 0;  // the supports do not meet
  std::vector<uint8_t> is_piv(nv, 0);
  for (int k : pivcol) is_piv[k] = 1;
  // y_0: pivots from the right-hand side, free variables 0.  Null vector of
  // free variable f: e_f plus the pivots whose row has f.
  std::vector<uint8_t> y0(nv, 0);
  for (int i = 0; i < r; ++i) y0[pivcol[i]] = eq[i][nv];
  std::vector<std::vector<uint8_t>> dirs;  // in x-space
  auto x_of_y = [&](const std::vector<uint8_t>& y, bool affine) {
    std::vector<uint8_t> x = affine ? x1 : std::vector<uint8_t>(n, 0);
    for (int k = 0; k < nv; ++k)
      if (y[k]) {
        std::vector<uint8_t> c = colG(var[k]);
        for (int i = 0; i < n; ++i) x[i] ^= c[i];
      }
    return x;
  };
  for (int f = 0; f < nv; ++f) {
    if (is_piv[f]) continue;
    std::vector<uint8_t> y(nv, 0);
    y[f] = 1;
    for (int i = 0; i < r; ++i)
      if (eq[i][f]) y[pivcol[i]] = 1;
    dirs.push_back(x_of_y(y, false));
  }
  const std::vector<uint8_t> x0 = x_of_y(y0, true);
  const int N = (int)dirs.size();
  auto pack = [&](const std::vector<uint8_t>& x) {
    uint64_t w = 0;
    for (int i = 0; i < n; ++i) w |= (uint64_t)x[i] << i;
    return w;
  };
  // h(x) = phase of conj(<x|a>) <x|b> in units of pi/4.
  int va = 0, vb = 0;
  auto h = [&](const std::vector<uint8_t>& x, int* out) {
    int ka, kb;
    if (!a.amplitude(pack(x), &ka, &va) || !b.amplitude(pack(x), &kb, &vb)) return false;
    *out = ((kb - ka) % 8 + 8) % 8;
    return true;
  };
  auto point = [&](const std::vector<int>& on) {
    std::vector<uint8_t> x = x0;
    for (int k : on)
      for (int i = 0; i < n; ++i) x[i] ^= dirs[k][i];
    return x;
  };
  int h0;
  if (!h(x0, &h0)) return -2;
  auto qval = [&](const std::vector<int>& on, int* out) {
    int hz;
    if (!h(point(on), &hz)) return false;
    int d = ((hz - h0) % 8 + 8) % 8;
    if (d % 2) return false;
    *out = d / 2;
    return true;
  };
  std::vector<uint8_t> Bq(N * N, 0);
  std::vector<int> qk(N);
  for (int k = 0; k < N; ++k) {
    if (!qval({k}, &qk[k])) return -3;
    Bq[k * N + k] = (uint8_t)qk[k];
  }
  for (int k = 0; k < N; ++k)
    for (int l = k + 1; l < N; ++l) {
      int q2;
      if (!qval({k, l}, &q2)) return -3;
      int c = ((q2 - qk[k] - qk[l]) % 4 + 4) % 4;
      if (c % 2) return -4;
      Bq[k * N + l] = Bq[l * N + k] = (uint8_t)(c / 2);
    }
  // Check q(z) = z^T B_q z (mod 4) on every z (N <= 10) or on 64 pseudo-random z.
  const int checks = N <= 10 ? (1 << N) : 64;
  uint64_t st = 0x9E3779B97F4A7C15ull ^ (uint64_t)N;
  for (int c = 0; c < checks; ++c) {
    std::vector<int> on;
    if (N <= 10) {
      for (int k = 0; k < N; ++k)
        if ((c >> k) & 1) on.push_back(k);
    } else {
      st ^= st << 13; st ^= st >> 7; st ^= st << 17;
      for (int k = 0; k < N; ++k)
        if ((st >> (k % 64)) & 1) on.push_back(k);
    }
    int qz;
    if (!qval(on, &qz)) return -3;
    int form = 0;
    for (size_t i = 0; i < on.size(); ++i) {
      form += Bq[on[i] * N + on[i]];
      for (size_t j = i + 1; j < on.size(); ++j) form += 2 * Bq[on[i] * N + on[j]];
    }
    if ((form - qz) % 4 != 0) return -5;
  }
  int rs, re, is, ie;
  expsum(N, Bq.data(), &rs, &re, &is, &ie);
  int kz, ez;
  if (rs == 0 && is == 0) return 0;
  if (is == 0) { kz = rs > 0 ? 0 : 4; ez = 2 * re; }
  else if (rs == 0) { kz = is > 0 ? 2 : 6; ez = 2 * ie; }
  else {
    if (re != ie) return -6;
    if (rs > 0 && is > 0) kz = 1;
    else if (rs < 0 && is > 0) kz = 3;
    else if (rs < 0 && is < 0) kz = 5;
    else kz = 7;
    ez = 2 * re + 1;
  }
  *k8 = (h0 + kz) % 8;
  *e2 = ez - (va + vb);
  return 1;
}

// ---------------------------------------------------------------------------
// C interface (ctypes).
// ---------------------------------------------------------------------------
extern "C" {

void orc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { philox(ctr, key, out); }

double orc_uniform(uint64_t seed, uint64_t index, uint32_t sub, uint32_t stream) {
  return uniform53(seed, index, sub, stream);
}

uint32_t orc_stream_sparsify(void) { return kStreamSparsify; }

void orc_coverage(long* out, int reset) {
  for (int i = 0; i < 19; ++i) {
    out[i] = g_cover[i].load();
    if (reset) g_cover[i] = 0;
  }
}

// ---- single CH-form ----
void* orc_ch_new(int n) {
  if (n < 1 || n > 64) return nullptr;
  return new CH(n);
}
void orc_ch_free(void* h) { delete (CH*)h; }
int orc_ch_apply(void* h, int op, int q, int r) { return ch_apply(*(CH*)h, op, q, r); }
int orc_ch_apply_right(void* h, int op, int q, int r) {
  CH& c = *(CH*)h;
  if (op == OP_S) c.R_S(q);
  else if (op == OP_CZ) c.R_CZ(q, r);
  else if (op == OP_CX) c.R_CX(q, r);
  else return 1;
  return 0;
}
void orc_ch_export(void* h, uint64_t* F, uint64_t* G, uint64_t* M, uint8_t* gamma, uint64_t* v,
                   uint64_t* s, int* omega) {
  ((CH*)h)->export_packed(F, G, M, gamma, v, s, omega);
}
int orc_ch_amplitude(void* h, uint64_t x, int* k8, int* vcount) {
  return ((CH*)h)->amplitude(x, k8, vcount);
}
uint64_t orc_ch_sample(void* h, uint64_t flips) { return ((CH*)h)->sample(flips); }
int orc_ch_check(void* h) { return ((CH*)h)->check(); }
int orc_ch_inner(void* h, const uint64_t* Aoff, const uint8_t* Adiag, int* k8, int* e2) {
  return inner_record(*(CH*)h, Aoff, Adiag, k8, e2);
}

// <a|b> of two CH forms: rc 1 with e^{i pi k8/4} 2^{e2/2}, 0 for zero, < 0 on error.
int orc_ch_inner_ch(void* ha, void* hb, int* k8, int* e2) {
  return ch_inner(*(CH*)ha, *(CH*)hb, k8, e2);
}
// The same by the definition, summing over all 2^n strings.
void orc_ch_inner_brute(void* ha, void* hb, double* out) {
  cplx z = ch_inner_brute(*(CH*)ha, *(CH*)hb);
  out[0] = z.real();
  out[1] = z.imag();
}

// ---- decomposition and exponential sum ----
void orc_phase_decomp(double theta, double* c, int* k) {
  cplx c0, c1;
  phase_decomp(theta, &c0, &c1, k);
  c[0] = c0.real(); c[1] = c0.imag(); c[2] = c1.real(); c[3] = c1.imag();
}
void orc_expsum(int N, const uint8_t* B, int* out4) {
  expsum(N, B, &out4[0], &out4[1], &out4[2], &out4[3]);
}

// ---- sum-over-Cliffords terms ----
// Circuit: n_gates entries (op, q, r, t).  Slots are the SLOT entries (phase
// gate on q, consuming theta[] in order) and the CCZ entries (qubits q, r, t),
// numbered together in circuit order; a CCZ slot's theta entry is unused.
// alphas: the term indices to build (NULL = all chi terms).
void* orc_terms_build(int n, int n_gates, const uint8_t* op, const uint8_t* q, const uint8_t* r,
                      const uint8_t* t, int n_slot, const double* theta, uint64_t chi, int mode,
                      uint64_t seed, const uint64_t* alphas, uint64_t n_alpha, int threads) {
  Terms* T = new Terms();
  T->n = n;
  T->chi = chi;
  T->mode = mode;
  T->seed = seed;
  int slot_seen = 0;
  for (int g = 0; g < n_gates; ++g) {
    T->op.push_back(op[g]);
    T->q.push_back(q[g]);
    T->r.push_back(r[g]);
    if (op[g] == OP_SLOT || op[g] == OP_CCZ) {
      if (slot_seen >= n_slot) { T->error = 1; return T; }
      Slot sl;
      if (op[g] == OP_SLOT) {
        phase_slot(theta[slot_seen], q[g], &sl);
      } else {
        int a = q[g], b = r[g], c = t ? t[g] : 0;
        if (a >= n || b >= n || c >= n || a == b || a == c || b == c) { T->error = 1; return T; }
        ccz_slot(a, b, c, &sl);
      }
      T->slots.push_back(sl);
      ++slot_seen;
    }
  }
  if (slot_seen != n_slot) { T->error = 1; return T; }
  double l1 = 1.0;
  long double prod = 1.0L;
  for (const Slot& sl : T->slots) {
    double W = 0.0;
    for (int j = 0; j < sl.nb; ++j) W += std::abs(sl.c[j]);
    l1 *= W;
    prod *= (long double)sl.nb;
  }
  T->l1 = l1;
  if (mode == 0 && prod != (long double)chi) { T->error = 2; return T; }
  uint64_t cnt = alphas ? n_alpha : chi;
  T->index.resize(cnt);
  for (uint64_t i = 0; i < cnt; ++i) T->index[i] = alphas ? alphas[i] : i;
  T->ch.assign(cnt, CH(n));
  T->b.assign(cnt, 0.0);
  T->branch.assign(cnt, {});
  std::vector<int> errs(cnt, 0);
  parallel_for(cnt, threads, [&](size_t i, int) {
    choose_branches(*T, T->index[i], T->branch[i], T->b[i]);
    evolve_term(*T, T->branch[i], T->ch[i], &errs[i]);
    if (T->ch[i].error) errs[i] = 2;
  });
  for (uint64_t i = 0; i < cnt; ++i)
    if (errs[i]) T->error = 3;
  return T;
}
// The CCZ decomposition table: coeff[2j], coeff[2j+1] = (re, im) of c_j; branch j
// is gates[off[j] .. off[j+1]) with gate i = (op, q, r) in gates[3i .. 3i+2].
// Returns the total gate count (gates must hold 3 * 32 ints).
int orc_ccz_decomp(int a, int b, int c, double* coeff, uint32_t* off, int32_t* gates) {
  Slot sl;
  ccz_slot(a, b, c, &sl);
  int cnt = 0;
  off[0] = 0;
  for (int j = 0; j < sl.nb; ++j) {
    coeff[2 * j] = sl.c[j].real();
    coeff[2 * j + 1] = sl.c[j].imag();
    for (const auto& k : sl.k[j]) {
      gates[3 * cnt] = k[0];
      gates[3 * cnt + 1] = k[1];
      gates[3 * cnt + 2] = k[2];
      ++cnt;
    }
    off[j + 1] = (uint32_t)cnt;
  }
  return cnt;
}
// Apply prod_j (I + (-1)^{bits[j]} Z_{qubits[j]}) / 2 to every built term in order:
// each CH form is updated and b_alpha scaled by 2^{-1/2} per code-2 step or set
// to zero.  Returns the number of terms whose CH form went invalid (0 expected).
int orc_terms_project(void* h, int w, const int32_t* qubits, const uint8_t* bits, int threads) {
  Terms* T = (Terms*)h;
  std::vector<int> bad(T->ch.size(), 0);
  parallel_for(T->ch.size(), threads, [&](size_t a, int) {
    for (int j = 0; j < w; ++j) {
      if (T->b[a] == cplx(0.0, 0.0)) break;  // already projected away
      int code = T->ch[a].project_z(qubits[j], bits[j]);
      if (T->ch[a].error) { bad[a] = 1; return; }
      if (code == 0) T->b[a] = 0.0;
      else if (code == 2) T->b[a] *= 1.0 / std::sqrt(2.0);
    }
  });
  int nb = 0;
  for (int x : bad) nb += x;
  return nb;
}
// Apply prod_j (I + P_j) / 2, P_j = i^{a[j]} X(x[j]) Z(z[j]) (Hermitian), to every
// built term in order, as orc_terms_project does for Z-type projectors.
int orc_terms_project_pauli(void* h, int w, const uint8_t* a, const uint64_t* x, const uint64_t* z,
                            int threads) {
  Terms* T = (Terms*)h;
  const int n = T->n;
  std::vector<int> bad(T->ch.size(), 0);
  parallel_for(T->ch.size(), threads, [&](size_t t, int) {
    for (int j = 0; j < w; ++j) {
      if (T->b[t] == cplx(0.0, 0.0)) break;  // already projected away
      std::vector<uint8_t> px(n), pz(n);
      for (int q = 0; q < n; ++q) {
        px[q] = (uint8_t)((x[j] >> q) & 1);
        pz[q] = (uint8_t)((z[j] >> q) & 1);
      }
      int code = T->ch[t].project_pauli(a[j], px, pz);
      if (T->ch[t].error || code < 0) { bad[t] = 1; return; }
      if (code == 0) T->b[t] = 0.0;
      else if (code == 2) T->b[t] *= 1.0 / std::sqrt(2.0);
    }
  });
  int nb = 0;
  for (int e : bad) nb += e;
  return nb;
}
// One CH form: code of project_pauli (-1 on an invalid state or a non-Hermitian P).
int orc_ch_project_pauli(void* h, int a, uint64_t x, uint64_t z) {
  CH* c = (CH*)h;
  std::vector<uint8_t> px(c->n), pz(c->n);
  for (int q = 0; q < c->n; ++q) {
    px[q] = (uint8_t)((x >> q) & 1);
    pz[q] = (uint8_t)((z >> q) & 1);
  }
  int code = c->project_pauli(a, px, pz);
  return c->error ? -1 : code;
}
// One CH form: returns the code of project_z (and -1 on an invalid state).
int orc_ch_project(void* h, int q, int bit) {
  CH* c = (CH*)h;
  int code = c->project_z(q, bit);
  return c->error ? -1 : code;
}
// Copy of a term set (same circuit, same built terms).
void* orc_terms_clone(void* h) { return new Terms(*(Terms*)h); }
void orc_terms_free(void* h) { delete (Terms*)h; }
int orc_terms_error(void* h) { return ((Terms*)h)->error; }
double orc_terms_l1(void* h) { return ((Terms*)h)->l1; }
uint64_t orc_terms_count(void* h) { return ((Terms*)h)->ch.size(); }
void* orc_terms_ch(void* h, uint64_t i) { return &((Terms*)h)->ch[i]; }
void orc_terms_b(void* h, uint64_t i, double* b) {
  b[0] = ((Terms*)h)->b[i].real();
  b[1] = ((Terms*)h)->b[i].imag();
}
void orc_terms_branch(void* h, uint64_t i, uint8_t* out) {
  const auto& br = ((Terms*)h)->branch[i];
  for (size_t p = 0; p < br.size(); ++p) out[p] = br[p];
}

// <x|psi> = sum_alpha b_alpha <x|phi_alpha> over the built terms.
void orc_terms_amplitudes(void* h, const uint64_t* x, uint64_t n_x, double* out, int threads) {
  Terms* T = (Terms*)h;
  parallel_for(n_x, threads, [&](size_t i, int) {
    CSum sr, si;
    for (size_t a = 0; a < T->ch.size(); ++a) {
      int k, vc;
      if (!T->ch[a].amplitude(x[i], &k, &vc)) continue;
      ldbl re, im;
      record_value(T->b[a], k, vc, &re, &im);
      sr.add(re);
      si.add(im);
    }
    out[2 * i] = (double)sr.value();
    out[2 * i + 1] = (double)si.value();
  });
}

// Norm estimation: overlap_l = <phi_{A_l}|psi> = sum_alpha b_alpha <phi_{A_l}|phi_alpha>,
// eta_l = 2^n |overlap_l|^2 (Lemma (Norm Estimation)).  Returns the number of
// failed records (0 expected).
int orc_terms_inner(void* h, const uint64_t* Aoff, const uint8_t* Adiag, uint64_t L,
                    double* overlap, double* eta, int threads) {
  Terms* T = (Terms*)h;
  int n = T->n;
  std::vector<int> bad(L, 0);
  parallel_for(L, threads, [&](size_t l, int) {
    CSum sr, si;
    for (size_t a = 0; a < T->ch.size(); ++a) {
      int k, e2;
      int rc = inner_record(T->ch[a], Aoff + l * n, Adiag + l * n, &k, &e2);
      if (rc < 0) { bad[l] = 1; continue; }
      if (rc == 0) continue;
      // value = b e^{i pi k/4} 2^{e2/2}; reuse record_value with vc = -e2.
      ldbl re, im;
      record_value(T->b[a], k, -e2, &re, &im);
      sr.add(re);
      si.add(im);
    }
    double o_re = (double)sr.value(), o_im = (double)si.value();
    overlap[2 * l] = o_re;
    overlap[2 * l + 1] = o_im;
    eta[l] = (double)(std::ldexp((ldbl)1.0, n) * ((ldbl)o_re * o_re + (ldbl)o_im * o_im));
  });
  int nb = 0;
  for (uint64_t l = 0; l < L; ++l) nb += bad[l];
  return nb;
}

// overlap_l = <theta_l|psi> = sum_alpha b_alpha <theta_l|phi_alpha>, theta_l the
// CH form of term l of hb (its b not included), psi the terms of ha; and
// *total = sum_l conj(b^hb_l) overlap_l = <psi_hb|psi_ha>.  Returns the number
// of failed pair records (0 expected).
int orc_terms_inner_ch(void* ha, void* hb, double* overlap, double* total, int threads) {
  Terms* A = (Terms*)ha;
  Terms* Bt = (Terms*)hb;
  const size_t L = Bt->ch.size();
  std::vector<int> bad(L, 0);
  parallel_for(L, threads, [&](size_t l, int) {
    CSum sr, si;
    for (size_t a = 0; a < A->ch.size(); ++a) {
      int k, e2;
      int rc = ch_inner(Bt->ch[l], A->ch[a], &k, &e2);
      if (rc < 0) { bad[l] = 1; continue; }
      if (rc == 0) continue;
      ldbl re, im;
      record_value(A->b[a], k, -e2, &re, &im);
      sr.add(re);
      si.add(im);
    }
    overlap[2 * l] = (double)sr.value();
    overlap[2 * l + 1] = (double)si.value();
  });
  CSum tr, ti;
  for (size_t l = 0; l < L; ++l) {
    const cplx c = std::conj(Bt->b[l]);
    const ldbl orr = overlap[2 * l], oi = overlap[2 * l + 1];
    tr.add((ldbl)c.real() * orr - (ldbl)c.imag() * oi);
    ti.add((ldbl)c.real() * oi + (ldbl)c.imag() * orr);
  }
  total[0] = (double)tr.value();
  total[1] = (double)ti.value();
  int nb = 0;
  for (int e : bad) nb += e;
  return nb;
}

// ---- Metropolis chain, Sec. "Heuristic Metropolis simulator" ----
// One chain per x_init entry.  Per step s: proposal bit j = jstream[c*steps + s],
// y = x xor e_j; accept iff U < P(y)/P(x) with U = ustream[c*steps + s]
// (r >= 1 always accepts).  Q_x per term is cached as (mu, t, u) and updated by
// Q_y = (U_C^{-1} X_j U_C) Q_x.  Outputs the chain state after every step,
// accept flags, and the final amplitude <x|psi>.
int orc_metropolis(void* h, uint32_t n_chain, uint32_t steps, const uint64_t* x_init,
                   const uint32_t* jstream, const double* ustream, uint64_t* x_trace,
                   uint8_t* accepted, double* amp_final, int threads) {
  Terms* T = (Terms*)h;
  int n = T->n;
  std::vector<int> bad(n_chain, 0);
  parallel_for(n_chain, threads, [&](size_t c, int) {
    size_t k = T->ch.size();
    std::vector<std::vector<uint8_t>> tt(k, std::vector<uint8_t>(n, 0)), uu(k, std::vector<uint8_t>(n, 0));
    std::vector<int> mu(k, 0);
    uint64_t x = x_init[c];
    // Initial Q_x for every term (the O(k n^2) part).
    for (size_t a = 0; a < k; ++a) {
      const CH& ch = T->ch[a];
      for (int p = 0; p < n; ++p) {
        if (!((x >> p) & 1)) continue;
        // Q <- Q * P_p (right multiplication while building the product in order).
        int dot = 0;
        for (int j = 0; j < n; ++j) {
          uu[a][j] ^= ch.F[p * n + j];
          dot += uu[a][j] * ch.M[p * n + j];
          tt[a][j] ^= ch.M[p * n + j];
        }
        mu[a] = (mu[a] + ch.gamma[p] + 2 * (dot % 2)) % 4;
      }
    }
    auto amp_of = [&](size_t a, const std::vector<uint8_t>& u, int m, ldbl* re, ldbl* im) -> int {
      const CH& ch = T->ch[a];
      int sign = 0, vc = 0;
      for (int j = 0; j < n; ++j) {
        if (ch.v[j]) { sign += u[j] * ch.s[j]; ++vc; }
        else if (u[j] != ch.s[j]) return 0;
      }
      int kk = (ch.omega + 2 * m + 4 * (sign % 2)) % 8;
      record_value(T->b[a], kk, vc, re, im);
      return 1;
    };
    CSum ax_r, ax_i;
    for (size_t a = 0; a < k; ++a) {
      ldbl re, im;
      if (amp_of(a, uu[a], mu[a], &re, &im)) { ax_r.add(re); ax_i.add(im); }
    }
    ldbl axr = ax_r.value(), axi = ax_i.value();
    ldbl px = axr * axr + axi * axi;
    if (px == 0) bad[c] = 1;
    std::vector<uint8_t> nt(n), nu(n);
    std::vector<std::vector<uint8_t>> pt(k), pu(k);
    std::vector<int> pm(k);
    for (uint32_t st = 0; st < steps; ++st) {
      uint32_t j = jstream[(size_t)c * steps + st];
      double U = ustream[(size_t)c * steps + st];
      CSum ay_r, ay_i;
      for (size_t a = 0; a < k; ++a) {
        const CH& ch = T->ch[a];
        // P_j Q_x = i^{gamma_j} X(F_j) Z(M_j) i^mu Z(t) X(u)
        //         = i^{gamma_j + mu} (-1)^{(M_j + t).F_j} Z(M_j + t) X(F_j + u).
        int dot = 0;
        for (int q = 0; q < n; ++q) {
          nt[q] = ch.M[j * n + q] ^ tt[a][q];
          nu[q] = ch.F[j * n + q] ^ uu[a][q];
          dot += nt[q] * ch.F[j * n + q];
        }
        int m2 = (mu[a] + ch.gamma[j] + 2 * (dot % 2)) % 4;
        pt[a] = nt;
        pu[a] = nu;
        pm[a] = m2;
        ldbl re, im;
        if (amp_of(a, nu, m2, &re, &im)) { ay_r.add(re); ay_i.add(im); }
      }
      ldbl ayr = ay_r.value(), ayi = ay_i.value();
      ldbl py = ayr * ayr + ayi * ayi;
      double ratio = (double)(py / px);
      int acc = (px > 0) && (ratio >= 1.0 || U < ratio);
      if (acc) {
        x ^= (uint64_t)1 << j;
        for (size_t a = 0; a < k; ++a) { tt[a] = pt[a]; uu[a] = pu[a]; mu[a] = pm[a]; }
        axr = ayr; axi = ayi; px = py;
      }
      x_trace[(size_t)c * steps + st] = x;
      accepted[(size_t)c * steps + st] = (uint8_t)acc;
    }
    amp_final[2 * c] = (double)axr;
    amp_final[2 * c + 1] = (double)axi;
  });
  int nb = 0;
  for (uint32_t c = 0; c < n_chain; ++c) nb += bad[c];
  return nb;
}

}  // extern "C"
