// Internal types shared by the HIP kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "chsim.h"

namespace chsim {

// Device gate codes: the public codes plus SPOW (S applied `arg` times on q),
// which the host uses for runs of S gates, and SLOT_SPOW (a slot whose
// branches are all powers of S on qubit q: the power is spow[branch] of the
// slot's table, per term).
enum : uint8_t { OP_H = 0, OP_S = 1, OP_CX = 2, OP_CZ = 3, OP_SLOT = 4, OP_SPOW = 5,
                 OP_SLOT_SPOW = 6 };

// A gate of the flat device list (8 bytes, read by the kernels as two
// 32-bit words on the scalar unit).  `slot` is the slot index of a slot
// gate.  SLOT_SPOW: the slot's branches are powers of S on qubit q; branch j
// applies S^{(r | arg << 8) >> 2j & 3}.  A gate of a general slot branch has
// kCondApply in cond and applies only to terms whose choice j for the slot
// has bit j set in arg2 (a branch mask: one bit for a gate of one branch's
// list, several for a net gate shared by diagonal branches).  kSlotStart in cond marks the first gate of a slot occurrence, where
// the term's branch choice for that slot is needed.
struct DGate {
  uint8_t op, q, r, arg;
  uint16_t slot;
  uint8_t cond, arg2;
};
static_assert(sizeof(DGate) == 8, "DGate is 8 bytes");
constexpr uint8_t kCondApply = 1, kSlotStart = 2;

// One slot's decomposition as the kernels read it.
struct SlotTable {
  uint32_t n_branch;
  uint32_t goff[CHSIM_MAX_BRANCH + 1];  // branch j = bgates[goff[j] .. goff[j+1])
  double cum[CHSIM_MAX_BRANCH];         // sum_{i<=j} |c_i|
  double total;                         // W = sum_i |c_i|
  double unit_re[CHSIM_MAX_BRANCH];     // c_j / |c_j| (0 if c_j == 0)
  double unit_im[CHSIM_MAX_BRANCH];
  double coef_re[CHSIM_MAX_BRANCH];     // c_j
  double coef_im[CHSIM_MAX_BRANCH];
  int32_t spow_q;                       // >= 0: every branch is S^{spow[j]} on this qubit
  uint8_t spow[CHSIM_MAX_BRANCH];
};

// Structure-of-arrays term store of one instance.  Row p of term a of F is
// F[p * chi + a] (rows outer, terms inner: consecutive terms are consecutive
// words), and likewise G, M and gamma; per-term words v, s, omega, b.
struct TermsView {
  uint32_t n;
  uint32_t n_slot;
  uint64_t chi;
  uint64_t* F;
  uint64_t* G;
  uint64_t* M;
  uint8_t* gamma;   // Z_4
  uint64_t* v;
  uint64_t* s;
  uint8_t* omega;   // Z_8
  double2* b;
  uint8_t* branch;  // branch[p * chi + a]
};

// Metropolis chain state (one instance).
struct MetroView {
  uint32_t n_chain;
  uint32_t n_tiles;       // term tiles of kMetroTile terms
  uint64_t* state;        // [n_chain][chi]: u | mu << 62, brought up to date lazily
  uint32_t* pend;         // per chain: accepted steps of the open window (bit w: step t0 + w)
  uint64_t* pmask;        // per chain: flip mask accepted at the previous flip-mask step, or 0
  uint64_t* x;            // per chain
  double2* amp;           // per chain: <x|psi>
  double2* partial;       // [n_chain][n_tiles]
  const uint32_t* jstream;
  const double* ustream;
  uint64_t* trace;        // may be null
  uint8_t* accepted;      // may be null
  uint32_t n_steps;
  uint32_t n_qubits;
};

constexpr int kMetroTile = 256;
// Steps per window of deferred chain-cache updates (single-flip chains).
constexpr uint32_t kMetroWin = 4;
constexpr int kAmpTile = 64;

// ---- launchers (each returns the first HIP error) ----
hipError_t launch_choose(const TermsView& T, const SlotTable* slots, uint32_t mode, uint64_t seed,
                         double scale, hipStream_t st);
// Evolution mapping: `lanes` lanes per term (4, 8, 16, 32 or 64; 64 / lanes
// terms per wave) and `rows` = ceil(n / lanes) tableau rows per lane.  0 = choose.
// lds: rows resident in LDS (evolve_lds.hip) instead of registers.
struct EvolveShape {
  int lanes = 0, rows = 0;
  bool lds = false;
};
EvolveShape evolve_shape_for(uint32_t n, int lanes);
EvolveShape evolve_default_shape(uint32_t n);
// Items a mapping holds on the chip at once (0: not bounded by LDS).
uint64_t evolve_capacity(EvolveShape s, uint32_t n);
bool evolve_shape_supported(EvolveShape s, uint32_t n);
// One evolution launch: count work items (or *count_dev of them, count being
// the grid's bound); item i starts from |0^n> (from_zero) or from state
// src_idx[i] (i if null) of src, takes its branch choices from column
// br_idx[i] (i if null) of branch [slot][chi_br], and writes state i of dst.
// src may equal dst when src_idx is null (in-place update).
// slot_seq[k] is the slot of the k-th slot occurrence of the launch's gates
// (n_occ of them): the kernel prefetches each term's choice one occurrence
// ahead.
// Row p of state k of src sits at p * src_rs + k * src_is (term store:
// rs = chi, is = 1; checkpoint stores: rs = 1, is = n, a state's rows
// contiguous so that a gathered state is read in whole cache lines), and
// likewise for dst.
struct EvolveJob {
  TermsView src, dst;
  uint64_t src_rs, src_is, dst_rs, dst_is;
  const uint32_t* src_idx;
  const uint32_t* br_idx;
  const uint8_t* branch;
  uint64_t chi_br;
  const uint32_t* count_dev;
  uint64_t count;
  const uint32_t* slot_seq;
  uint32_t n_occ;
};
hipError_t launch_evolve_job(const EvolveJob& J, const DGate* gates, uint32_t n_gates, bool from_zero,
                             uint32_t* err, EvolveShape shape, hipStream_t st);
hipError_t launch_evolve_l4(int rows, const EvolveJob& J, const DGate* gates, uint32_t n_gates,
                            bool from_zero, uint32_t* err, hipStream_t st);
hipError_t launch_evolve_l8(int rows, const EvolveJob& J, const DGate* gates, uint32_t n_gates,
                            bool from_zero, uint32_t* err, hipStream_t st);
hipError_t launch_evolve_wide(int lanes, int rows, const EvolveJob& J, const DGate* gates,
                              uint32_t n_gates, bool from_zero, uint32_t* err, hipStream_t st);
hipError_t launch_evolve_lds(int lanes, const EvolveJob& J, const DGate* gates, uint32_t n_gates,
                             bool from_zero, uint32_t* err, hipStream_t st);
// Projective gates (I + P_j) / 2, j < count, applied in order to every term of
// T in place (CH forms and b), with the Hermitian Pauli
// P_j = i^{a[j]} X(x[j]) Z(z[j]) (a[j] = popcount(x[j] & z[j]) mod 2).
struct ProjGates {
  uint32_t count;
  uint8_t a[64];
  uint64_t x[64];
  uint64_t z[64];
};
hipError_t launch_project(const TermsView& T, const ProjGates& P, uint32_t* err, hipStream_t st);
hipError_t launch_evolve_w64(const EvolveJob& J, const DGate* gates, uint32_t n_gates, bool from_zero,
                             uint32_t* err, hipStream_t st);
uint64_t evolve_lds_capacity(int lanes, uint32_t n);
hipError_t launch_evolve(const TermsView& T, const DGate* gates, uint32_t n_gates,
                         const uint32_t* slot_seq, uint32_t n_occ, bool from_zero, uint32_t* err,
                         EvolveShape shape, hipStream_t st);
hipError_t launch_set_zero(const TermsView& T, hipStream_t st);

// One checkpoint level of shared-prefix evolution.  For every term a < chi:
// key = (prev_id[a] (0 if null) << 32) | the branch choices of the n_span
// slots slot[i] packed at width[i] bits each (at most 32 bits in all);
// id_out[a] = rank of the key among the distinct keys (ids 0 .. *counter - 1,
// arbitrary order), rep[id] = some term with that key, parent[id] = its
// prev_id.  table has table_mask + 1 >= 2 chi entries; ids and slot_of are
// scratch of table and chi entries.
struct PrefixLevelArgs {
  const uint8_t* branch;  // [slot][chi]
  uint64_t chi;
  const uint16_t* slot;
  const uint8_t* width;
  uint32_t n_span;
  const uint32_t* prev_id;
  uint64_t* table;
  uint64_t table_mask;
  uint32_t* ids;
  uint32_t* slot_of;
  uint32_t* counter;
  uint32_t* id_out;
  uint32_t* rep;
  uint32_t* parent;
  uint32_t first_counters;  // > 0 at the first level: clear the table and this many counters
};
hipError_t launch_prefix_level(const PrefixLevelArgs& A, hipStream_t st);
hipError_t launch_sample(const TermsView& T, const uint64_t* alpha, const uint64_t* flips,
                         uint64_t* x_out, uint32_t count, hipStream_t st);
// CH-form invariants of terms [first, first + count): out[0] = terms that
// violate one, out[1] = the smallest such index (~0 if none), out[2] = OR of
// the CHSIM_BAD_* flags seen.
hipError_t launch_validate(const TermsView& T, uint64_t first, uint64_t count, unsigned long long* out,
                           hipStream_t st);

// Amplitudes.  Per-term values the amplitude kernel reads, computed by a
// prologue kernel from the term store: ~v masked to n bits, the value folded
// into entry 0 of the first chunk table of the zero test (s & ~v, or, for a
// packed term, s gathered from the ~v positions and shifted above bit n), the
// gamma low-bit plane, omega, whether the term is packed (its zero test rides
// in the high bits of the quadratic-form rows) and b_alpha 2^{-|v|/2} (w0)
// and w0 e^{i pi/4} (w1).
struct AmpTerm {
  uint64_t nv, snv, glo;
  uint32_t w, packed;
  double w0r, w0i, w1r, w1i;
};
static_assert(sizeof(AmpTerm) == 64, "AmpTerm is 64 bytes");

// One request = one instance's terms and its bitstrings; the request's terms
// are cut into ranges of `tiles_per_range` 8-term tiles and its bitstrings
// into chunks, and each (range, chunk) is one work item that a persistent
// workgroup pulls from a queue.  partial[range * n_x + i] holds the range's
// sum; a second kernel adds the ranges in a fixed order into out.
struct AmpInst {
  TermsView T;
  const uint64_t* crow;  // [n][chi] rows of the quadratic form (prologue output)
  const AmpTerm* cst;    // [chi]
  const uint64_t* x;
  double2* partial;  // [n_ranges][n_x]
  double2* out;      // [n_x]
  uint32_t n_x;
  uint32_t tiles_per_range;
  uint32_t n_ranges;
  uint32_t pad;
};
struct AmpItem {
  uint32_t inst, range, x0, x1;
};
struct AmpRequestPlan {
  uint32_t n;
  uint32_t n_x;
  uint64_t chi;
};
hipError_t launch_amp_prep(const TermsView& T, uint64_t* crow, AmpTerm* cst, hipStream_t st);
// Cut the requests into work items of 256 xpl bitstrings (xpl = 1 or 2, the
// bitstrings per lane of the kernel) sorted by estimated cost, largest first.
void amp_plan(const std::vector<AmpRequestPlan>& reqs, uint32_t target_items, uint32_t xpl,
              std::vector<AmpItem>& items, std::vector<uint32_t>& tiles_per_range,
              std::vector<uint32_t>& n_ranges);
// The plan amp_plan makes for a single request (tiles per range, ranges,
// bitstring chunks of 256 xpl), computed without containers.
void amp_plan_single(uint64_t chi, uint32_t n_x, uint32_t target_items, uint32_t xpl, uint32_t* tiles_per_range,
                     uint32_t* n_ranges, uint32_t* chunks);
// Write that plan's request record, prefix and n_items = ranges x chunks
// work items into device memory with a kernel (no host copy).
hipError_t launch_amp_fill_single(const AmpInst& inst, AmpInst* insts_d, AmpItem* items_d, uint64_t* prefix_d,
                                  uint32_t n_items, uint32_t chunks, uint32_t xpl, hipStream_t st);
// Reset the queue counter, run the persistent kernel, reduce.  prefix_d[q] =
// bitstrings of requests before q (n_inst + 1 entries).
hipError_t launch_amp_items(const AmpInst* insts_d, const AmpItem* items_d, uint32_t n_items,
                            uint32_t* counter, bool fp32c, uint32_t xpl, const uint64_t* prefix_d,
                            uint32_t n_inst, uint64_t total_x, hipStream_t st);

// Inner products with equatorial states: L states in batches of 64 (Lp =
// L rounded up), partial sums per term group, and a device workspace of
// work_words 8-byte words (per-term records and A rearranged by state).
struct InnerPlan {
  uint32_t Lp, n_batches, n_groups;
  size_t partial_elems, work_words;
};
InnerPlan inner_plan(const TermsView& T, uint32_t L);
hipError_t launch_inner(const TermsView& T, const uint64_t* Aoff, const uint8_t* Adiag, uint32_t L,
                        const InnerPlan& P, double2* partial, uint64_t* work, double2* overlap,
                        double* eta, double* eta_sum, uint32_t* err, hipStream_t st);

// Inner products of two CH forms: per-term records (inner_ch_record_words
// words for chi terms), then overlap_l = sum_a b_k[a] <theta_l|phi_a> over
// `groups` ket-term groups (partial: groups x L), and optionally
// total = sum_l conj(b_bra[l]) overlap_l.  err: a ket term with |v| = n = 64
// and no free index for the Z_2 lift.
size_t inner_ch_record_words(uint32_t n, uint64_t chi);
hipError_t launch_inner_ch_records(const TermsView& T, uint64_t* rec, hipStream_t st);
uint32_t inner_ch_groups(uint64_t chi_k, uint32_t L);
hipError_t launch_inner_ch(const uint64_t* rec_k, const double2* b_k, uint64_t chi_k, const uint64_t* rec_b,
                           const double2* b_bra, uint32_t L, uint32_t n, uint32_t groups, double2* partial,
                           double2* overlap, double2* total, uint32_t* err, hipStream_t st);

// Metropolis.
hipError_t launch_metro_init(const TermsView& T, MetroView& Mv, hipStream_t st);
hipError_t launch_metro_steps(const TermsView& T, MetroView& Mv, uint32_t n_steps, hipStream_t st);
// One proposal step for every chain with flip masks mask[c] (0: no move).
// Flip-mask proposals (mask per chain; mode: kProposeApplyPending applies
// each chain's pmask first and writes its cache back, kProposeMasks proposes
// the masks).
constexpr uint32_t kProposeApplyPending = 1u, kProposeMasks = 2u;
hipError_t launch_propose(const TermsView& T, MetroView& Mv, const uint64_t* mask, uint32_t mode,
                          hipStream_t st);

}  // namespace chsim
