/* chsim.h — C ABI of the MI355X (gfx950) sum-over-Cliffords hot path.
 *
 * Implements the data-parallel core of Bravyi, Browne, Calpin, Campbell,
 * Gosset, Howard, "Simulation of quantum circuits by low-rank stabilizer
 * decompositions" (Quantum 3, 181 (2019), arXiv:1808.00128):
 *   (a) evolve chi CH-form stabilizer terms through their sampled Clifford
 *       circuits (Sec. "Phase-sensitive Clifford simulator");
 *   (b) amplitudes <x|psi> = sum_j b_j <x|phi_j> (Eqs. (amplitude), (amplitude1));
 *   (c) inner products <phi_A|psi> with equatorial states and the norm
 *       estimate (Lemmas (Inner Product), (Exponential Sum), (Norm Estimation));
 *   and the Metropolis chain over n-bit outputs (Sec. "Heuristic Metropolis
 *   simulator").
 *
 * Conventions (shared by every call):
 *   - qubit p is bit p of a uint64 bitstring; 1 <= n <= 64.
 *   - a binary matrix row is a uint64 with bit j = entry (p, j).
 *   - complex numbers are two doubles (re, im).
 *   - every call returns a chsim_status; on failure nothing is written to
 *     caller outputs that the status does not describe, and
 *     chsim_last_error() returns a message (thread-local).
 *   - the caller owns every pointer it passes; the library reads or writes
 *     them only during the call.  The library owns all device memory behind
 *     a chsim_ctx.
 *   - `stream` is a hipStream_t or NULL (the default stream).  Without
 *     CHSIM_DEVICE_PTRS, pointer arguments are host pointers and the call
 *     returns after the results are in host memory.  With CHSIM_DEVICE_PTRS
 *     they are device pointers on the context's device, and the call only
 *     enqueues work on `stream`.
 */
#ifndef CHSIM_H_INCLUDED
#define CHSIM_H_INCLUDED

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t chsim_status;
#define CHSIM_OK 0
#define CHSIM_EINVAL 1       /* an argument is out of range or inconsistent */
#define CHSIM_ENOMEM 2       /* device or host allocation failed */
#define CHSIM_EDEVICE 3      /* a HIP runtime call failed */
#define CHSIM_EUNSUPPORTED 4 /* valid request outside what this build supports */
#define CHSIM_ESTATE 5       /* a term violated a CH-form invariant */

/* Gate codes.  CX: q = control, r = target.  SLOT: a non-Clifford gate whose
 * Clifford decomposition is the instance's slot_decomp[slot]. */
enum { CHSIM_H = 0, CHSIM_S = 1, CHSIM_CX = 2, CHSIM_CZ = 3, CHSIM_SLOT = 4 };

typedef struct chsim_gate {
  uint8_t op, q, r, pad;
  uint32_t slot;
} chsim_gate;

#define CHSIM_MAX_BRANCH 8

/* Clifford decomposition of one non-Clifford gate, V = sum_j coeff_j K_j
 * (Eq. (Udecomp) per gate; the lifting lemma gives such decompositions for
 * diagonal gates).  K_j is the gate sequence gates[off[j] .. off[j+1]),
 * applied in order (ops in {H, S, CX, CZ}).  1 <= n_branch <= CHSIM_MAX_BRANCH. */
typedef struct chsim_decomp {
  uint32_t n_branch;
  const double* coeff;     /* 2 * n_branch: (re, im) of c_j */
  const uint32_t* off;     /* n_branch + 1 offsets into gates, off[0] = 0 */
  const chsim_gate* gates; /* off[n_branch] gates */
} chsim_decomp;

#define CHSIM_EXACT 0    /* all prod_p n_branch(p) products, b = prod c (Eq. (Vphi)) */
#define CHSIM_SPARSIFY 1 /* chi i.i.d. draws, Lemma (Sparsification), Eq. (Omega) */

/* One circuit instance: its qubit count, slot decompositions and term set.
 * EXACT requires chi == prod_p n_branch(p); term alpha takes for slot p the
 * branch given by digit p of alpha in the mixed radix (n_branch(0),
 * n_branch(1), ...), slot 0 least significant.  SPARSIFY draws, per term alpha and
 * slot p, a uniform u from Philox4x32-10 with counter (alpha_lo, alpha_hi, p,
 * 0x53504152) and key (seed_lo, seed_hi) (53 bits: (w0 << 21) | (w1 >> 11));
 * branch = smallest j with u * W_p < sum_{i<=j} |c_i|, W_p = sum_i |c_i|, and
 * b_alpha = (prod_p W_p / chi) prod_p c_j / |c_j|. */
typedef struct chsim_instance {
  uint32_t n;
  uint32_t n_slot;
  const chsim_decomp* slot_decomp; /* n_slot entries (may be NULL if n_slot == 0) */
  uint64_t chi;
  uint32_t mode;
  uint64_t seed;
} chsim_instance;

typedef struct chsim_ctx chsim_ctx;

/* Flags. */
#define CHSIM_FP64 0u          /* amplitudes summed in FP64 */
#define CHSIM_FP32C 1u         /* FP32 with per-block two-sum, FP64 across blocks */
#define CHSIM_DEVICE_PTRS 0x100u
/* chsim_metropolis_step: record the n_steps steps' kernel launches once in a
 * HIP graph and replay it while the call's sizes and buffers stay the same
 * (one graph launch per call instead of two kernel launches per step). */
#define CHSIM_GRAPH 0x200u

/* Create a context on HIP device `device` holding n_inst instances; for each,
 * choose every term's branches and coefficient b_alpha (exact enumeration or
 * sparsification, see chsim_instance) and set every term to |0^n> (F = G = I,
 * M = 0, gamma = v = s = 0, omega = 1; CH-form initialisation of the
 * Clifford-simulator section).  EINVAL: n outside [1, 64], chi = 0, bad
 * decomposition, EXACT with chi != prod n_branch.  ENOMEM: term store does not
 * fit.  On failure *ctx is NULL. */
chsim_status chsim_terms_init(chsim_ctx** ctx, int device, uint32_t n_inst,
                              const chsim_instance* inst);

/* Re-draw instance `inst`'s terms in place with a new seed (SPARSIFY; EXACT
 * re-enumerates) and return every term to |0^n>, without reallocating: the
 * term-generation step of chsim_terms_init on existing storage.  Enqueued on
 * `stream`. */
chsim_status chsim_terms_reset(chsim_ctx* ctx, uint32_t inst, uint64_t seed, void* stream);

/* Left-multiply every term of instance `inst` by the gate sequence (Clifford
 * gates by the rules L[S], L[CZ], L[CX]; H by Eqs. (H1)-(H7) and Prop. H; a
 * SLOT applies the term's chosen branch K_j of that slot's decomposition).
 * May be called repeatedly on consecutive circuit segments.  EINVAL: qubit
 * >= n, q == r on a 2-qubit gate, slot >= n_slot.  ESTATE: a term hit a case
 * that unitary evolution cannot produce (reported after the call). */
chsim_status chsim_apply_clifford(chsim_ctx* ctx, uint32_t inst, const chsim_gate* gates,
                                  size_t n_gates, void* stream);

/* out[2i], out[2i+1] = <x_i|psi>, psi = sum_alpha b_alpha |phi_alpha> (not
 * normalised), per Eqs. (amplitude), (amplitude1).  flags: CHSIM_FP64 or
 * CHSIM_FP32C, optionally | CHSIM_DEVICE_PTRS.  EINVAL: a bitstring has a bit
 * >= n set (checked for host pointers only), n_x == 0. */
chsim_status chsim_amplitudes(chsim_ctx* ctx, uint32_t inst, const uint64_t* x, size_t n_x,
                              double* out, uint32_t flags, void* stream);

/* One request of a batched amplitude call: out[2i], out[2i+1] = <x_i|psi_inst>
 * for i < n_x.  x and out are host or device pointers as the call's flags say;
 * requests may name the same instance; output arrays must not overlap. */
typedef struct chsim_amp_request {
  uint32_t inst;
  uint32_t reserved;
  const uint64_t* x;
  size_t n_x;
  double* out;
} chsim_amp_request;

/* chsim_amplitudes for several requests in one launch (instances of
 * different n, chi and bitstring counts share one persistent grid that pulls
 * (request, term range, bitstring chunk) work items), same formula, flags and
 * results as one call per request.  Host bitstring arrays are checked as in
 * chsim_amplitudes.  EINVAL: n_req == 0, a request with a bad instance, a null
 * array or n_x == 0.  The plan is cached in the context: a context must not be
 * used from two streams at once. */
chsim_status chsim_amplitudes_batch(chsim_ctx* ctx, const chsim_amp_request* reqs, size_t n_req,
                                    uint32_t flags, void* stream);

/* chsim_amplitudes for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same formula, kernels and results as chsim_amplitudes with the same
 * flags, but every intermediate (the prologue rows and term constants, the
 * per-range partial sums, the work items and the queue counter) lives in a
 * fixed device array of 64 MiB that the library's code object holds on each
 * GPU until the process ends; no hipMalloc, hipFree or other allocating call
 * is made.  Requires CHSIM_DEVICE_PTRS (x and out are device pointers) and
 * enqueues only.  Uses the context's current bitstrings-per-item value and
 * never runs the autotuner.  The array is shared by every call on one GPU and
 * keeps the last call's contents: two calls that overlap in time on the same
 * GPU (different streams, threads or contexts) race and give wrong results.
 * EINVAL: host pointers, n_x == 0, null arrays, or a request whose
 * intermediates exceed the array (about 8 n chi + 64 chi + 16 n_x ranges
 * bytes; n = 50, chi = 2^16, 4096 strings needs 47 MB). */
chsim_status chsim_amplitudes_noalloc(chsim_ctx* ctx, uint32_t inst, const uint64_t* x, size_t n_x,
                                      double* out, uint32_t flags, void* stream);

/* Norm estimation with equatorial states phi_A, A in M_n (Eq. (eqa1)):
 * A_off[l*n + a] = row a of the off-diagonal part of A_l (bit b = A_ab; bit a
 * ignored), A_diag[l*n + a] = A_aa in {0..3}.  overlap[2l..2l+1] = <phi_{A_l}|psi>
 * (Lemma (Inner Product) with the exponential sum of Lemma (Exponential Sum));
 * eta[l] = 2^n |overlap_l|^2; *eta_mean = mean_l eta[l] (FP64), the estimator of
 * ||psi||^2 of Lemma (Norm Estimation).  eta and eta_mean may be NULL.
 * EINVAL: L == 0, asymmetric A (host pointers only).  EUNSUPPORTED: n == 64
 * with a term whose |v| == 64. */
chsim_status chsim_inner_products(chsim_ctx* ctx, uint32_t inst, const uint64_t* A_off,
                                  const uint8_t* A_diag, size_t L, double* overlap, double* eta,
                                  double* eta_mean, uint32_t flags, void* stream);

/* Inner products with general stabilizer states given as CH forms: for every
 * term l of instance bra_inst (its CH form theta_l; its coefficient b_l not
 * included), overlap[2l], overlap[2l+1] = <theta_l|psi> = sum_alpha b_alpha
 * <theta_l|phi_alpha> over the terms of instance inst, and, if total is not
 * NULL, total[0..1] = sum_l conj(b_l) <theta_l|psi> = <psi_bra|psi> (with
 * bra_inst == inst: <psi|psi> exactly, chi^2 pairs).  Each pair is the sum of
 * conj(<x|theta>) <x|phi> (Eqs. (amplitude), (amplitude1)) over the
 * intersection of the two supports, an exponential sum of Lemma (Exponential
 * Sum); the paper gives its O(n^3) cost (Sec. "Fast norm estimation") and
 * defers the method to earlier work.  overlap has 2 chi_bra doubles; with
 * CHSIM_DEVICE_PTRS overlap and total are device pointers and the call only
 * enqueues, else it returns after copying.  EINVAL: instances of different n,
 * null overlap.  EUNSUPPORTED: n = 64 with a ket term whose |v| = 64. */
chsim_status chsim_inner_products_ch(chsim_ctx* ctx, uint32_t inst, uint32_t bra_inst, double* overlap,
                                     double* total, uint32_t flags, void* stream);

/* Projective gates (I + (-1)^{bits[j]} Z_{qubits[j]}) / 2, j < w, applied in order
 * to every term of the instance in place (end of Sec. "Phase-sensitive Clifford
 * simulator": Gamma|phi> = (1/2) U_C U_H (I + Q)|s>, with Q from the tableau
 * row G_q and the CH form of the result by Prop. H).  A term is kept, scaled by
 * 2^{-1/2} (b_alpha and its CH form updated), or projected to zero (b_alpha = 0),
 * so the instance then holds Pi psi.  qubits, bits: host arrays of w entries.
 * The same as chsim_project_pauli with a = 2 bits[j], x = 0, z = e_{qubits[j]}.
 * EINVAL: w > 64, a qubit >= n, a bit > 1, null arrays with w > 0. */
chsim_status chsim_project_z(chsim_ctx* ctx, uint32_t inst, const uint32_t* qubits, const uint8_t* bits,
                             uint32_t w, void* stream);

/* Projective gates (I + P_j) / 2 for Hermitian Paulis P_j = i^{a[j]} X(x[j]) Z(z[j])
 * (X part left of the Z part; bit q of x[j], z[j] = qubit q), j < w, applied in
 * order to every term of the instance in place (end of Sec. "Phase-sensitive
 * Clifford simulator": Gamma|phi> = (1/2) U_C U_H (I + Q)|s> with
 * Q = U_H^{-1} U_C^{-1} P U_C U_H, U_C^{-1} P U_C read off the tableaux of Eq.
 * (tableaux) in O(n^2), and the CH form of the result by Prop. H).  A term is
 * kept, scaled by 2^{-1/2} (b_alpha and its CH form updated), or projected to
 * zero (b_alpha = 0), so the instance then holds prod_j (I + P_j)/2 psi.
 * a, x, z: host arrays of w entries.  EINVAL: w > 64, a[j] > 3, a bit >= n in
 * x[j] or z[j], a[j] != popcount(x[j] & z[j]) mod 2 (P_j not Hermitian), null
 * arrays with w > 0.  Chains started on the instance are dropped. */
chsim_status chsim_project_pauli(chsim_ctx* ctx, uint32_t inst, const uint8_t* a, const uint64_t* x,
                                 const uint64_t* z, uint32_t w, void* stream);

/* Copy the term store (CH forms, b_alpha, and the branch choices when both
 * have the same slot count) of src_inst into dst_inst, device to device.
 * EINVAL: the instances differ in n or chi. */
chsim_status chsim_terms_copy(chsim_ctx* ctx, uint32_t src_inst, uint32_t dst_inst, void* stream);

/* Chain-rule sampling of w output bits by norm estimation (Sec. "Fast norm
 * estimation", sampling paragraph: P_w(x) = ||Pi psi||^2 / ||psi||^2,
 * Pi = prod_j (I + (-1)^{x_j} Z_j) / 2, bits drawn one by one).  For bit j the
 * terms are copied into scratch_inst (same n and chi), projected onto
 * (x_0..x_{j-1}, b) for b = 0 and 1, and their norms estimated over the L
 * equatorial states (layout of chsim_inner_products, host arrays); the
 * conditional probability of 0 is e_0 / (e_0 + e_1) (1/2 if both are zero),
 * and x_j = 0 iff u[j] < it.  Writes bits_out[w], prob_out[w] (probability of
 * each chosen bit given the previous ones) and, if est_out is not NULL,
 * est_out[2j + b] = e_b.  Host arrays; synchronous; scratch_inst's terms are
 * overwritten.  EINVAL: w not in 1..64, a qubit >= n, u[j] not in [0, 1),
 * scratch_inst == inst or of another shape, null arrays, L == 0. */
chsim_status chsim_sample_marginal(chsim_ctx* ctx, uint32_t inst, uint32_t scratch_inst, const uint32_t* qubits,
                                   uint32_t w, const uint64_t* A_off, const uint8_t* A_diag, size_t L,
                                   const double* u, uint8_t* bits_out, double* prob_out, double* est_out,
                                   void* stream);

/* Sparsification tail bound (Lemma (Sparsification tail bound), Eq. (event)):
 * for a normalised psi and chi >= ||c||_1^2 / delta^2 sparsified terms,
 * ||psi - Omega||^2 <= <Omega|Omega> - 1 + delta^2 with probability at least
 * 1 - 2 exp(-delta^2 / (8 F(psi))).  <Omega|Omega> is estimated by norm
 * estimation over the L equatorial states given (same layout and checks as
 * chsim_inner_products, host arrays only) and delta^2 = ||c||_1^2 / chi.
 * Writes out[0] = the estimate of <Omega|Omega> (mean of eta_l),
 * out[1] = its standard error over the L states, out[2] = delta^2,
 * out[3] = out[0] - 1 + out[2], the bound on ||psi - Omega||^2.  Synchronous.
 * EINVAL: an EXACT instance (Omega = psi), L < 2, a null output, or the
 * errors of chsim_inner_products. */
chsim_status chsim_sparsification_bound(chsim_ctx* ctx, uint32_t inst, const uint64_t* A_off,
                                        const uint8_t* A_diag, size_t L, double out[4], void* stream);

/* Start n_chain Metropolis chains at x0[c] (Sec. "Heuristic Metropolis
 * simulator"): caches, per chain and term, the Pauli Q_x as (u, mu) and
 * writes amp[2c..2c+1] = <x0_c|psi>.  Requires n <= 62.  EINVAL: some
 * <x0_c|psi> == 0 (P(x0) must be > 0).  The cache describes the terms as
 * they are now: every call that changes them (chsim_apply_clifford,
 * chsim_set_terms, chsim_project_z, chsim_terms_copy into the instance,
 * chsim_terms_reset) drops the chains, and a later step returns EINVAL until
 * chsim_metropolis_init runs again. */
chsim_status chsim_metropolis_init(chsim_ctx* ctx, uint32_t inst, uint32_t n_chain,
                                   const uint64_t* x0, double* amp, uint32_t flags, void* stream);

/* Advance every chain n_steps single-bit-flip steps.  Step t of chain c flips
 * bit j = j_stream[c*n_steps + t] (< n; checked for host pointers, reduced mod n
 * on the device for device pointers) and accepts iff
 * u_stream[c*n_steps + t] < |<y|psi>|^2 / |<x|psi>|^2 (FP64 sums, FP64
 * ratio).  x_trace[c*n_steps + t] receives the state after step t, accepted[...]
 * 1/0 (both may be NULL); amp (may be NULL) receives the final <x_c|psi>.
 * flags: CHSIM_DEVICE_PTRS, CHSIM_GRAPH (same results, launched from a cached
 * graph of the n_steps steps; the graph is kept per instance until the
 * buffers, n_steps or the chains change, or the context is destroyed). */
chsim_status chsim_metropolis_step(chsim_ctx* ctx, uint32_t inst, uint32_t n_steps,
                                   const uint32_t* j_stream, const double* u_stream,
                                   uint64_t* x_trace, uint8_t* accepted, double* amp,
                                   uint32_t flags, void* stream);

/* ---- Learned proposal -------------------------------------------------
 * A flip-mask proposal from a small network f: {0,1}^n -> R^n (n -> H -> H
 * -> n, ReLU) on BF16 matrix cores with FP32 accumulation.  Features
 * s_j = 1 - 2 x_j.  pi_j(x) = clip(sigmoid(f(x)_j), pi_min, pi_max).  The
 * chain proposes y = x ^ m from the mixture
 *   q(y|x) = eps [|m| = 1] / n + (1 - eps) prod_j pi_j^{m_j} (1 - pi_j)^{1 - m_j}
 * and accepts iff U < P(y) q(x|y) / (P(x) q(y|x)) (Metropolis-Hastings with the
 * exact amplitude ratio of Sec. "Heuristic Metropolis simulator"), so the
 * stationary law is the paper's P(x).  Parameters are packed in FP32 as
 * W1 [H][n], b1 [H], W2 [H][H], b2 [H], W3 [n][H], b3 [n]. */
typedef struct chsim_mlp chsim_mlp;

/* Create a network on the context's device for batches up to max_batch,
 * initialised from params (packed, see above).  EINVAL: n outside [1, 64],
 * hidden not a positive multiple of 16 or above 1024, max_batch == 0. */
chsim_status chsim_mlp_create(chsim_ctx* ctx, uint32_t n, uint32_t hidden, uint32_t max_batch,
                              const float* params, chsim_mlp** out);
chsim_status chsim_mlp_destroy(chsim_mlp* mlp);
/* Copy the FP32 parameters out / in (setting resets the optimiser state). */
chsim_status chsim_mlp_get_params(chsim_mlp* mlp, float* params);
chsim_status chsim_mlp_set_params(chsim_mlp* mlp, const float* params);
/* logits[b*n + j] = f(x_b)_j for batch <= max_batch strings. */
chsim_status chsim_mlp_forward(chsim_mlp* mlp, const uint64_t* x, uint32_t batch, float* logits,
                               uint32_t flags, void* stream);
/* Binary cross-entropy with logits against target flip bits t_b,
 * L = mean_{b,j} softplus(l_bj) - t_bj l_bj, and its gradient with respect to
 * every parameter (packed like the parameters; FP32).  Either output may be
 * NULL. */
chsim_status chsim_mlp_loss_grad(chsim_mlp* mlp, const uint64_t* x, const uint64_t* target,
                                 uint32_t batch, double* loss, float* grads, uint32_t flags,
                                 void* stream);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8) over `epochs` passes of
 * consecutive minibatches of (x, target) pairs; epoch_loss[e] (may be NULL)
 * receives the mean loss of epoch e. */
chsim_status chsim_mlp_train(chsim_mlp* mlp, const uint64_t* x, const uint64_t* target,
                             uint64_t count, uint32_t batch, uint32_t epochs, float lr,
                             double* epoch_loss, uint32_t flags, void* stream);

/* Random inputs of the learned chain, [chains][steps] (u_bits [chains][steps][n]):
 * u_mix < eps selects the single flip of bit j; otherwise bit k flips iff
 * u_bits < pi_k(x); u is the accept uniform. */
typedef struct chsim_learned_args {
  float eps, pi_min, pi_max;
  const double* u_mix;
  const uint32_t* j;
  const double* u_bits;
  const double* u;
} chsim_learned_args;

/* Advance the chains started by chsim_metropolis_init with the learned
 * proposal (requires n <= 62 and the network's n equal to the instance's).
 * Outputs as chsim_metropolis_step, plus n_flips[c*n_steps + t] = |m| (may be
 * NULL; a step with |m| = 0 leaves the chain in place and counts as
 * accepted). */
chsim_status chsim_metropolis_step_learned(chsim_ctx* ctx, uint32_t inst, chsim_mlp* mlp,
                                           uint32_t n_steps, const chsim_learned_args* args,
                                           uint64_t* x_trace, uint8_t* accepted,
                                           uint32_t* n_flips, double* amp, uint32_t flags,
                                           void* stream);

/* Sample one bitstring per request from a single term's |<x|phi_alpha>|^2 (the
 * three-step sampler of the Clifford-simulator section: w = s, flip w_j where
 * v_j = 1 and bit j of flips[i] is set, x = w G^T).  Host pointers. */
chsim_status chsim_sample_terms(chsim_ctx* ctx, uint32_t inst, size_t count,
                                const uint64_t* alpha, const uint64_t* flips, uint64_t* x_out);

/* Download terms [first, first + count) to host arrays laid out per term:
 * F, G, M: count*n rows; gamma: count*n; v, s: count; omega: count (Z_8,
 * omega = e^{i pi k/4}); b: 2*count; branch: count*n_slot.  NULL skips a field. */
chsim_status chsim_get_terms(chsim_ctx* ctx, uint32_t inst, uint64_t first, uint64_t count,
                             uint64_t* F, uint64_t* G, uint64_t* M, uint8_t* gamma, uint64_t* v,
                             uint64_t* s, uint8_t* omega, double* b, uint8_t* branch);

/* Upload terms (same layout as chsim_get_terms; every field required except
 * branch).  Lets the query kernels run on CH-forms built elsewhere.  EINVAL:
 * a row, v or s with a bit >= n, gamma > 3 or omega > 7 (nothing is written
 * then).  The invariants of Eq. (tableaux) are not checked here (see
 * chsim_validate).  Chains started on the instance are dropped. */
chsim_status chsim_set_terms(chsim_ctx* ctx, uint32_t inst, uint64_t first, uint64_t count,
                             const uint64_t* F, const uint64_t* G, const uint64_t* M,
                             const uint8_t* gamma, const uint64_t* v, const uint64_t* s,
                             const uint8_t* omega, const double* b);

/* Debug check of the CH-form invariants of terms [first, first + count) of
 * instance `inst` (Sec. "Phase-sensitive Clifford simulator", Eq. (tableaux):
 * U_C^{-1} Z_p U_C = Z(G_p), U_C^{-1} X_p U_C = i^{gamma_p} X(F_p) Z(M_p)).
 * Conjugation by U_C preserves the Pauli commutation relations and
 * Hermiticity, so every term reachable by unitary evolution satisfies
 *   CHSIM_BAD_TABLEAU:  F G^T = I over GF(2);
 *   CHSIM_BAD_SYMMETRY: M F^T symmetric over GF(2);
 *   CHSIM_BAD_GAMMA:    gamma_p = F_p . M_p (mod 2) for every row p;
 *   CHSIM_BAD_RANGE:    rows, v and s have no bit >= n, gamma_p < 4, omega < 8.
 * Writes *n_bad = number of terms violating at least one, *first_bad = the
 * smallest such index (UINT64_MAX if none) and *what = OR of the flags seen;
 * each output may be NULL.  Synchronous.  Returns CHSIM_ESTATE if some term
 * is bad (outputs still written), EINVAL for a range beyond chi. */
#define CHSIM_BAD_TABLEAU 1u
#define CHSIM_BAD_SYMMETRY 2u
#define CHSIM_BAD_GAMMA 4u
#define CHSIM_BAD_RANGE 8u
chsim_status chsim_validate(chsim_ctx* ctx, uint32_t inst, uint64_t first, uint64_t count,
                            uint64_t* n_bad, uint64_t* first_bad, uint32_t* what);

/* Decomposition of the phase gate diag(1, e^{i theta}) on `qubit`, Eq. (Rtheta)
 * after writing theta = theta' + k pi/2 with theta' in [0, pi/2):
 * diag(1, e^{i theta}) = c0 S^k + c1 S^{k+1}, c0 = e^{i theta'/2}(cos - sin)(theta'/2),
 * c1 = e^{i theta'/2} sqrt(2) e^{-i pi/4} sin(theta'/2).  Writes coeff[4],
 * off[3] and up to 7 gates into gates[8]; fills *out to point at them. */
chsim_status chsim_decompose_phase(double theta, uint32_t qubit, double coeff[4], uint32_t off[3],
                                   chsim_gate gates[8], chsim_decomp* out);

/* Decomposition of CCZ on qubits (a, b, c) into eight diagonal Clifford
 * branches by the lifting lemma, Eq. (CCZ decomposition), in the order of the
 * paper's sum: I, CZ_ab, CZ_ac, CZ_bc, CZ_ab CZ_ac Z_a, CZ_ab CZ_bc Z_b,
 * CZ_ac CZ_bc Z_c (c_j = 1/6 each) and CZ_ab CZ_ac CZ_bc Z_a Z_b Z_c
 * (c_7 = -1/6), with Z written as S S.  The paper prints the prefactor 2/9;
 * only 1/6 makes the sum equal CCZ, and it gives ||c||_1^2 = 16/9 = xi(CCZ)
 * as the paper states.  Writes coeff[16], off[9] and 24 gates into gates[24]
 * (caller-owned); fills *out to point at them.  EINVAL: a null output, a
 * qubit >= 64 or two equal qubits.  Host only; no device work. */
chsim_status chsim_decompose_ccz(uint32_t a, uint32_t b, uint32_t c, double coeff[16], uint32_t off[9],
                                 chsim_gate gates[24], chsim_decomp* out);

/* Tuning knobs of one instance; value 0 restores the library default.
 * EVOLVE_LANES: lanes per term in the evolution kernel (4, 8, 16, 32 or 64;
 * a wave holds 64 / lanes terms, and each lane holds ceil(n / lanes) tableau
 * rows in registers; lanes * ceil(n / lanes) must not exceed 64), or
 * lanes | CHSIM_EVOLVE_LDS with lanes 4, 8 or 16 (lanes * 16 >= n): the rows
 * of every term stay in LDS and the lanes of a term share them.  -1 =
 * autotune: the next chsim_apply_clifford that starts from |0^n> times every
 * shape on the real gate list (hipEvents), keeps the fastest, and leaves the
 * same terms any shape would.  Results never depend on the knob.
 * EUNSUPPORTED: no compiled kernel for that value and n. */
#define CHSIM_TUNE_EVOLVE_LANES 1u
#define CHSIM_EVOLVE_LDS 0x100
/* PREFIX_SHARE: an evolution from |0^n> runs the gates before a checkpoint
 * slot once per distinct choice of branches up to that slot (terms that
 * agree on those choices have identical CH forms there) and continues every
 * term from its prefix's state; results are bit-identical to evolving each
 * term alone.  0 = off, 1 = auto (default: checkpoint slots chosen from the
 * slots' branch weights, chi and the gate mix to minimise estimated work;
 * none when it would not pay), 2 = checkpoint wherever it removes any work
 * (for testing).  EINVAL: value outside 0..2. */
#define CHSIM_TUNE_PREFIX_SHARE 2u
/* AMP_STRINGS: bitstrings per work item of the amplitude kernel, 256 or 512
 * (1 or 2 per lane of a 256-lane workgroup; default 512), for every
 * amplitude launch of the context (inst only selects a valid instance).  -1 =
 * autotune: the next chsim_amplitudes or chsim_amplitudes_batch call runs
 * twice per value (the second run timed with hipEvents) and keeps the
 * faster; every run leaves correct outputs.  Results agree to rounding across values (the
 * terms are cut into ranges that may differ).  EUNSUPPORTED: another value. */
#define CHSIM_TUNE_AMP_STRINGS 3u
chsim_status chsim_set_tuning(chsim_ctx* ctx, uint32_t inst, uint32_t knob, int32_t value);

/* Current value of a knob.  For EVOLVE_LANES, timings_ms[8] receives the
 * autotuner's timings in ms for lanes 4, 8, 16, 32, 64 with rows in
 * registers and lanes 4, 8, 16 with rows in LDS (0 where not timed); for
 * AMP_STRINGS, timings_ms[0..1] = the autotuner's timings for 256 and 512;
 * for PREFIX_SHARE, timings_ms[0] = checkpoint levels of the last planned
 * evolution and timings_ms[1] = its estimated cost relative to evolving
 * every term alone.  timings_ms may be NULL. */
chsim_status chsim_get_tuning(chsim_ctx* ctx, uint32_t inst, uint32_t knob, int32_t* value,
                              float* timings_ms);

/* Work of the last chsim_apply_clifford on instance inst, in gate
 * applications (one gate on one term or on one shared prefix state):
 * apps[0] H, apps[1] CX, apps[2] CZ, apps[3] S, runs of S and slot powers of
 * S, apps[4] gates of general slot branches (each counted on every item,
 * applied or not).  *levels (may be NULL) = checkpoint levels used, and
 * distinct[k] (may be NULL; k < max_levels) = distinct branch prefixes at
 * level k.  Waits for the device.  EINVAL: apps NULL. */
chsim_status chsim_evolution_stats(chsim_ctx* ctx, uint32_t inst, uint64_t apps[5], uint32_t* levels,
                                   uint64_t* distinct, uint32_t max_levels);

/* Instance metadata: n, chi and ||c||_1 = prod_p W_p. */
chsim_status chsim_instance_info(chsim_ctx* ctx, uint32_t inst, uint32_t* n, uint64_t* chi,
                                 double* l1);

/* Roofline peaks of HIP device `device`, measured by microbenchmarks (they
 * measure the machine, not the method): out[0] = int32 VALU operations per
 * second (independent v_xor_b32 / v_add_u32 chains in every lane of a full
 * grid, one operation per lane per instruction), out[1] = HBM bytes per
 * second of a device-to-device copy of 1 GiB (bytes read plus bytes written;
 * the faster of a streaming copy kernel and the runtime's copy),
 * out[2] = LDS bytes per second of conflict-free 8-byte reads.  Each is the
 * best of three timed runs after a warm-up run.  Allocates and frees about
 * 2 GiB of device memory; synchronous; changes the current device.  EINVAL:
 * no such device or a null out; ENOMEM, EDEVICE on runtime failures. */
chsim_status chsim_measure_peaks(int device, double out[3]);

/* Release the context and its device memory.  NULL is accepted. */
chsim_status chsim_destroy(chsim_ctx* ctx);

/* Message of the last failing call on this thread ("" if none). */
const char* chsim_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CHSIM_H_INCLUDED */
