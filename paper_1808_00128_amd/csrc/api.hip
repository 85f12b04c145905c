// C ABI of libchsim (declared in include/chsim.h): argument checks, device
// memory of the term store, host-side decomposition tables, and the calls
// that launch the kernels.  Every step of the hot path runs in the HIP kernels;
// this file only validates, allocates, copies and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <vector>

#include "chsim.h"
#include "internal.hpp"
#include "mlp.hpp"

using namespace chsim;

namespace {

thread_local std::string g_err;

// Device scratch of chsim_amplitudes_noalloc: one array per GPU, part of the
// code object (no allocation call), shared by every call on that GPU.
constexpr size_t kNoAllocScratch = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];
// Its device address on each GPU, taken once with that GPU current.  In host
// code `scratch` names a host-side stand-in, never the device memory.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

chsim_status fail(chsim_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(CHSIM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t count) {
    if (count <= n) return hipSuccess;
    if (p) hipFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) n = count;
    return e;
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    n = 0;
  }
};

// Evolution shapes the autotuner times, in the order of the reported
// timings: lanes per term (| CHSIM_EVOLVE_LDS for rows in LDS).
constexpr int kTuneShapes = 8;
constexpr int kTuneLanes[kTuneShapes] = {4, 8, 16, 32, 64, 4 | CHSIM_EVOLVE_LDS, 8 | CHSIM_EVOLVE_LDS,
                                         16 | CHSIM_EVOLVE_LDS};

// EvolveShape of a tuning value (lanes, with CHSIM_EVOLVE_LDS for LDS rows).
EvolveShape shape_of_value(uint32_t n, int value) {
  EvolveShape s = evolve_shape_for(n, value & ~CHSIM_EVOLVE_LDS);
  s.lds = (value & CHSIM_EVOLVE_LDS) != 0;
  return s;
}

int value_of_shape(EvolveShape s) { return s.lanes | (s.lds ? CHSIM_EVOLVE_LDS : 0); }

struct Instance {
  uint32_t n = 0, n_slot = 0, mode = 0;
  uint64_t chi = 0, seed = 0;
  double l1 = 1.0;
  bool at_zero = true;  // every term is |0^n> and the store holds nothing yet
  bool amp_ready = false;  // the amplitude prologue output matches the terms
  EvolveShape shape;    // evolution mapping (0 = default for n)
  bool autotune = false;  // time every shape at the next from-|0^n> evolution
  float tuned_ms[kTuneShapes] = {};     // per tuned shape, kTuneLanes order (0 = not timed)
  std::vector<SlotTable> slots_h;
  // Per slot: when every branch is diagonal (powers of S and CZ), the union of
  // the branches' net gates, each with the mask of branches that apply it
  // (empty otherwise).
  std::vector<std::vector<DGate>> diag_h;
  std::vector<DGate> bgates_h;
  DevBuf<uint64_t> F, G, M, v, s;
  DevBuf<uint8_t> gamma, omega, branch;
  DevBuf<double2> b;
  DevBuf<SlotTable> slots;
  // amplitude prologue output
  DevBuf<uint64_t> acrow;
  DevBuf<AmpTerm> acst;
  // shared-prefix evolution: knob, cached plan of the last gate list
  int prefix_mode = 1;  // 0 off, 1 auto, 2 always when it saves any work
  bool plan_valid = false;
  uint64_t plan_key = 0;
  std::vector<uint32_t> plan_cut;       // gate position after each checkpoint level
  std::vector<int> plan_lanes;          // mapping of each checkpoint span (0: the instance's)
  std::vector<uint32_t> plan_span_off;  // level k's slots: [span_off[k], span_off[k+1])
  std::vector<uint16_t> plan_slot_h;
  std::vector<uint8_t> plan_width_h;
  double plan_frac = 1.0;               // estimated work relative to per-term evolution
  DevBuf<uint16_t> plan_slot;
  DevBuf<uint8_t> plan_width;
  DevBuf<uint32_t> plan_count;  // distinct prefixes per level of the last run
  // gate applications of the last evolution: per span, gate counts by kind
  // and the item count (fixed, or plan_count[level] when level >= 0)
  struct SpanStat {
    int level;
    uint64_t items;
    uint64_t kinds[5];
  };
  std::vector<SpanStat> last_spans;
  // Metropolis steps recorded as a graph, and what they were recorded with.
  // metro_done is recorded after every launch of the graph, so the graph is
  // destroyed only once its last launch has finished.
  hipGraphExec_t metro_exec = nullptr;
  hipEvent_t metro_done = nullptr;
  MetroView metro_key{};
  TermsView metro_tkey{};
  uint32_t metro_steps = 0;
  // metropolis
  uint32_t n_chain = 0;
  DevBuf<uint64_t> mstate0, mpmask, mx, mtrace;
  DevBuf<uint32_t> mpend, mj;
  DevBuf<double2> mamp, mpartial;
  DevBuf<double> mu;
  DevBuf<uint8_t> macc;
  // learned chain
  DevBuf<uint64_t> ly, lmask;
  DevBuf<float> logit_x, logit_y;
  DevBuf<double> lumix, lubits;
  DevBuf<uint32_t> lj, lflips;

  TermsView view() {
    TermsView t;
    t.n = n;
    t.n_slot = n_slot;
    t.chi = chi;
    t.F = F.p;
    t.G = G.p;
    t.M = M.p;
    t.gamma = gamma.p;
    t.v = v.p;
    t.s = s.p;
    t.omega = omega.p;
    t.b = b.p;
    t.branch = branch.p;
    return t;
  }
  void drop_graph() {
    if (metro_exec) {
      if (metro_done) hipEventSynchronize(metro_done);
      hipGraphExecDestroy(metro_exec);
    }
    metro_exec = nullptr;
  }
  // The chain cache (Q_x per chain and term, the chain amplitudes and the
  // recorded steps) describes the terms at chsim_metropolis_init; every call
  // that changes the terms drops it.
  void drop_chains() {
    n_chain = 0;
    drop_graph();
  }
  void release() {
    drop_graph();
    if (metro_done) hipEventDestroy(metro_done);
    metro_done = nullptr;
    F.release(); G.release(); M.release(); v.release(); s.release();
    gamma.release(); omega.release(); branch.release(); b.release();
    slots.release();
    acrow.release(); acst.release();
    plan_slot.release(); plan_width.release(); plan_count.release();
    mstate0.release(); mpmask.release(); mx.release(); mtrace.release();
    mpend.release(); mj.release(); mamp.release(); mpartial.release(); mu.release(); macc.release();
    ly.release(); lmask.release(); logit_x.release(); logit_y.release(); lumix.release();
    lubits.release(); lj.release(); lflips.release();
  }
};

}  // namespace

struct chsim_ctx {
  int device = 0;
  std::vector<Instance> inst;
  DevBuf<DGate> gates;
  DevBuf<uint32_t> err;
  DevBuf<uint64_t> xbuf;
  DevBuf<double2> partial, out;
  DevBuf<uint64_t> aoff, inner_work;
  DevBuf<uint8_t> adiag;
  DevBuf<double> eta;
  DevBuf<double> eta_sum;
  DevBuf<unsigned long long> vcheck;  // chsim_validate: bad count, first bad index, flags
  DevBuf<uint64_t> chrec_k, chrec_b;   // CH x CH inner products: per-term records
  DevBuf<double2> chtotal;
  // Amplitude work queue: device copies of the last plan, and its host key.
  DevBuf<AmpInst> amp_insts;
  DevBuf<AmpItem> amp_items;
  DevBuf<uint64_t> amp_prefix;
  DevBuf<uint32_t> amp_counter;
  std::vector<AmpInst> amp_key;
  uint32_t amp_n_items = 0;
  hipStream_t cap_stream = nullptr;  // stream the Metropolis graphs are recorded on
  // The last gate list as given (instance, raw gates) and as converted; a call
  // with the same list reuses the conversion and the device copy.
  uint32_t dg_inst = UINT32_MAX;
  std::vector<chsim_gate> dg_in;
  std::vector<DGate> dg;
  uint64_t dg_hash = 0;
  // Amplitude plan of the last request shapes (n, n_x, chi per request) and
  // bitstrings per lane it was cut for.
  std::vector<uint64_t> amp_shape_key;
  uint32_t amp_plan_xpl = 0, amp_key_xpl = 0;
  std::vector<AmpItem> amp_items_h;
  std::vector<uint32_t> amp_tpr, amp_nr;
  // Bitstrings per lane of the amplitude kernel (work items of 256 xpl
  // bitstrings); amp_tune: time both on the next call and keep the faster.
  uint32_t amp_xpl = 2;
  bool amp_tune = false;
  float amp_tune_ms[2] = {0.f, 0.f};
  // Slot occurrences of the last gate list: first gate index and slot.
  std::vector<uint32_t> occ_start;
  std::vector<uint32_t> slotseq_h;
  DevBuf<uint32_t> slotseq;
  // Shared-prefix evolution scratch (sized for the largest instance).
  DevBuf<uint64_t> pf_table;
  DevBuf<uint32_t> pf_ids, pf_slotof, pf_id[2], pf_rep, pf_parent;
  DevBuf<uint64_t> ck_F[2], ck_G[2], ck_M[2], ck_v[2], ck_s[2];
  DevBuf<uint8_t> ck_gamma[2], ck_omega[2];
};

namespace {

chsim_status check_ctx(chsim_ctx* ctx, uint32_t inst) {
  if (!ctx) return fail(CHSIM_EINVAL, "null context");
  if (inst >= ctx->inst.size()) return fail(CHSIM_EINVAL, "instance %u out of range", inst);
  return CHSIM_OK;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

bool valid_clifford(const chsim_gate& g, uint32_t n) {
  if (g.q >= n) return false;
  if (g.op == CHSIM_CX || g.op == CHSIM_CZ) return g.r < n && g.r != g.q;
  return g.op == CHSIM_H || g.op == CHSIM_S;
}

// Append a gate, folding runs of S on one qubit into one SPOW; gates before
// index `first` (an earlier branch) are never merged into.
void push_gate(std::vector<DGate>& out, const chsim_gate& g, size_t first = 0) {
  if (g.op == CHSIM_S) {
    if (out.size() > first && out.back().op == OP_SPOW && out.back().q == g.q && out.back().cond == 0) {
      out.back().arg = (uint8_t)((out.back().arg + 1) & 3);
      return;
    }
    out.push_back(DGate{OP_SPOW, g.q, 0, 1, 0, 0, 0});
    return;
  }
  out.push_back(DGate{g.op, g.q, g.r, 0, 0, 0, 0});
}

// Branches made only of S powers and CZ gates act on a CH form through L[S]
// (M_q ^= G_q, gamma_q -= 1) and L[CZ] (M_q ^= G_r, M_r ^= G_q), which commute
// and leave F, G, v, s and omega alone, so a branch is fixed by its net S
// power per qubit (mod 4) and its CZ parity per pair.  Each distinct net gate
// becomes one conditional gate whose mask holds the branches that apply it.
void merge_diagonal_branches(const Instance& I, const SlotTable& st, std::vector<DGate>& out) {
  std::map<std::pair<uint32_t, uint32_t>, uint8_t> mask;  // (q, r) -> branches; r = 64 + power for S^power
  for (uint32_t j = 0; j < st.n_branch; ++j) {
    std::map<uint32_t, uint32_t> pw;
    std::map<std::pair<uint32_t, uint32_t>, uint32_t> cz;
    for (uint32_t k = st.goff[j]; k < st.goff[j + 1]; ++k) {
      const DGate& g = I.bgates_h[k];
      if (g.op == OP_SPOW) pw[g.q] += g.arg;
      else if (g.op == OP_CZ) cz[{std::min(g.q, g.r), std::max(g.q, g.r)}] ^= 1u;
      else return;  // not diagonal: keep the per-branch gate lists
    }
    for (const auto& e : cz)
      if (e.second) mask[e.first] |= (uint8_t)(1u << j);
    for (const auto& e : pw)
      if (e.second & 3u) mask[{e.first, 64u + (e.second & 3u)}] |= (uint8_t)(1u << j);
  }
  for (const auto& e : mask) {
    const uint32_t q = e.first.first, r = e.first.second;
    if (r >= 64) out.push_back(DGate{OP_SPOW, (uint8_t)q, 0, (uint8_t)(r - 64), 0, kCondApply, e.second});
    else out.push_back(DGate{OP_CZ, (uint8_t)q, (uint8_t)r, 0, 0, kCondApply, e.second});
  }
}

chsim_status build_slots(Instance& I, const chsim_instance& in) {
  I.slots_h.clear();
  I.bgates_h.clear();
  I.diag_h.clear();
  double l1 = 1.0;
  for (uint32_t p = 0; p < in.n_slot; ++p) {
    const chsim_decomp& d = in.slot_decomp[p];
    if (d.n_branch < 1 || d.n_branch > CHSIM_MAX_BRANCH || !d.coeff || !d.off || (!d.gates && d.off[d.n_branch]))
      return fail(CHSIM_EINVAL, "slot %u: bad decomposition", p);
    if (d.off[0] != 0) return fail(CHSIM_EINVAL, "slot %u: off[0] must be 0", p);
    SlotTable st;
    std::memset(&st, 0, sizeof st);
    st.n_branch = d.n_branch;
    double cum = 0.0;
    for (uint32_t j = 0; j < d.n_branch; ++j) {
      if (d.off[j + 1] < d.off[j]) return fail(CHSIM_EINVAL, "slot %u: offsets decrease", p);
      st.goff[j] = (uint32_t)I.bgates_h.size();
      for (uint32_t k = d.off[j]; k < d.off[j + 1]; ++k) {
        const chsim_gate& g = d.gates[k];
        if (!valid_clifford(g, in.n)) return fail(CHSIM_EINVAL, "slot %u branch %u: bad gate %u", p, j, k);
        push_gate(I.bgates_h, g, st.goff[j]);
      }
      const double re = d.coeff[2 * j], im = d.coeff[2 * j + 1];
      const double w = std::sqrt(re * re + im * im);
      cum += w;
      st.cum[j] = cum;
      st.coef_re[j] = re;
      st.coef_im[j] = im;
      st.unit_re[j] = w > 0.0 ? re / w : 0.0;
      st.unit_im[j] = w > 0.0 ? im / w : 0.0;
    }
    st.goff[d.n_branch] = (uint32_t)I.bgates_h.size();
    // A family of S powers on one qubit (e.g. the phase-gate decomposition)
    // is applied as a per-term power, so terms never diverge on it.
    st.spow_q = -1;
    {
      int q = -1;
      bool fam = true;
      for (uint32_t j = 0; j < d.n_branch && fam; ++j) {
        const uint32_t len = st.goff[j + 1] - st.goff[j];
        if (len == 0) { st.spow[j] = 0; continue; }
        const DGate& g0 = I.bgates_h[st.goff[j]];
        if (len != 1 || g0.op != OP_SPOW || (q >= 0 && q != g0.q)) { fam = false; break; }
        q = g0.q;
        st.spow[j] = g0.arg;
      }
      if (fam && q >= 0) st.spow_q = q;
    }
    st.total = cum;
    if (!(cum > 0.0) || !std::isfinite(cum)) return fail(CHSIM_EINVAL, "slot %u: zero or non-finite weights", p);
    I.diag_h.emplace_back();
    if (st.spow_q < 0) merge_diagonal_branches(I, st, I.diag_h.back());
    l1 *= cum;
    I.slots_h.push_back(st);
  }
  I.l1 = l1;
  return CHSIM_OK;
}

// Upload a host or device input array into a device buffer; returns the device pointer.
template <typename T>
chsim_status stage_in(DevBuf<T>& buf, const T* src, size_t count, bool device_ptrs, hipStream_t st,
                      const T** out) {
  if (device_ptrs) {
    *out = src;
    return CHSIM_OK;
  }
  HIP_TRY(buf.ensure(count));
  HIP_TRY(hipMemcpyAsync(buf.p, src, count * sizeof(T), hipMemcpyHostToDevice, st));
  *out = buf.p;
  return CHSIM_OK;
}

chsim_status ensure_materialised(Instance& I, hipStream_t st) {
  if (!I.at_zero) return CHSIM_OK;
  HIP_TRY(launch_set_zero(I.view(), st));
  I.at_zero = false;
  I.amp_ready = false;
  return CHSIM_OK;
}

// Device address of `scratch` on the current device `device` (taken once).
chsim_status scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(CHSIM_EUNSUPPORTED, "device %d beyond %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(CHSIM_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return CHSIM_OK;
}

chsim_status check_err_flag(chsim_ctx* ctx, hipStream_t st, const char* what) {
  uint32_t flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, ctx->err.p, sizeof flag, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (flag) return fail(CHSIM_ESTATE, "%s: a term violated a CH-form invariant", what);
  return CHSIM_OK;
}

}  // namespace

extern "C" {

const char* chsim_last_error(void) { return g_err.c_str(); }

chsim_status chsim_terms_init(chsim_ctx** out, int device, uint32_t n_inst,
                              const chsim_instance* inst) {
  g_err.clear();
  if (!out) return fail(CHSIM_EINVAL, "null output pointer");
  *out = nullptr;
  if (n_inst == 0 || !inst) return fail(CHSIM_EINVAL, "no instances");
  // Validate everything before touching a device.
  for (uint32_t i = 0; i < n_inst; ++i) {
    const chsim_instance& in = inst[i];
    if (in.n < 1 || in.n > 64) return fail(CHSIM_EINVAL, "instance %u: n = %u outside [1, 64]", i, in.n);
    if (in.chi == 0) return fail(CHSIM_EINVAL, "instance %u: chi = 0", i);
    if (in.n_slot && !in.slot_decomp) return fail(CHSIM_EINVAL, "instance %u: missing decompositions", i);
    if (in.mode != CHSIM_EXACT && in.mode != CHSIM_SPARSIFY) return fail(CHSIM_EINVAL, "instance %u: bad mode", i);
    if (in.n_slot > 65535) return fail(CHSIM_EUNSUPPORTED, "instance %u: more than 65535 slots", i);
    if (in.mode == CHSIM_EXACT) {
      long double prod = 1.0L;
      for (uint32_t p = 0; p < in.n_slot; ++p) prod *= in.slot_decomp[p].n_branch;
      if (prod != (long double)in.chi) return fail(CHSIM_EINVAL, "instance %u: EXACT needs chi = prod n_branch", i);
    }
  }
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(CHSIM_EINVAL, "device %d not present", device);
  HIP_TRY(hipSetDevice(device));
  {
    void* sp = nullptr;
    chsim_status sst = scratch_address(device, &sp);
    if (sst) return sst;
  }
  chsim_ctx* ctx = new chsim_ctx();
  ctx->device = device;
  ctx->inst.resize(n_inst);
  auto cleanup = [&](chsim_status st) {
    chsim_destroy(ctx);
    return st;
  };
  if (ctx->err.ensure(1) != hipSuccess) return cleanup(fail(CHSIM_ENOMEM, "error flag allocation"));
  for (uint32_t i = 0; i < n_inst; ++i) {
    const chsim_instance& in = inst[i];
    Instance& I = ctx->inst[i];
    I.n = in.n;
    I.n_slot = in.n_slot;
    I.chi = in.chi;
    I.mode = in.mode;
    I.seed = in.seed;
    chsim_status st = build_slots(I, in);
    if (st != CHSIM_OK) return cleanup(st);
    const size_t rows = (size_t)in.n * in.chi;
    bool ok = I.F.ensure(rows) == hipSuccess && I.G.ensure(rows) == hipSuccess &&
              I.M.ensure(rows) == hipSuccess && I.gamma.ensure(rows) == hipSuccess &&
              I.v.ensure(in.chi) == hipSuccess && I.s.ensure(in.chi) == hipSuccess &&
              I.omega.ensure(in.chi) == hipSuccess && I.b.ensure(in.chi) == hipSuccess &&
              I.branch.ensure((size_t)std::max<uint32_t>(in.n_slot, 1) * in.chi) == hipSuccess &&
              I.slots.ensure(std::max<size_t>(I.slots_h.size(), 1)) == hipSuccess;
    if (!ok) return cleanup(fail(CHSIM_ENOMEM, "instance %u: term store (%zu rows) does not fit", i, rows));
    if (!I.slots_h.empty() &&
        hipMemcpy(I.slots.p, I.slots_h.data(), I.slots_h.size() * sizeof(SlotTable), hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(CHSIM_EDEVICE, "slot table upload"));
    const double scale = I.l1 / (double)I.chi;
    if (launch_choose(I.view(), I.slots.p, I.mode, I.seed, scale, nullptr) != hipSuccess)
      return cleanup(fail(CHSIM_EDEVICE, "branch choice kernel"));
    I.at_zero = true;
  }
  if (hipDeviceSynchronize() != hipSuccess) return cleanup(fail(CHSIM_EDEVICE, "init synchronize"));
  *out = ctx;
  return CHSIM_OK;
}

chsim_status chsim_terms_reset(chsim_ctx* ctx, uint32_t inst, uint64_t seed, void* stream) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  Instance& I = ctx->inst[inst];
  HIP_TRY(hipSetDevice(ctx->device));
  I.seed = seed;
  const double scale = I.l1 / (double)I.chi;
  HIP_TRY(launch_choose(I.view(), I.slots.p, I.mode, I.seed, scale, as_stream(stream)));
  I.at_zero = true;
  I.amp_ready = false;
  I.drop_chains();
  return CHSIM_OK;
}

namespace {

// ---- shared-prefix evolution: plan ----------------------------------------
// Evolution-kernel cost per gate, measured on MI355X at n = 50: the latency
// of one gate for a lone wave, and the time per gate for 65536 items at full
// occupancy, in microseconds, by kind (H, CX, CZ, S-type).
struct GateCost {
  double lat[4], thr[4];
};
constexpr GateCost kCostReg8 = {{0.87, 0.76, 0.67, 0.46}, {4.23, 2.52, 2.21, 1.57}};
constexpr GateCost kCostReg16 = {{0.70, 0.55, 0.50, 0.40}, {4.10, 2.70, 2.40, 1.80}};
constexpr GateCost kCostWave = {{0.47, 0.28, 0.28, 0.29}, {11.9, 5.04, 4.18, 4.32}};
constexpr GateCost kCostLds4 = {{2.32, 0.39, 0.30, 0.30}, {5.19, 0.80, 0.62, 0.63}};
constexpr GateCost kCostLds8 = {{1.48, 0.39, 0.30, 0.30}, {4.67, 0.95, 0.77, 0.78}};
constexpr GateCost kCostLds16 = {{1.05, 0.39, 0.30, 0.29}, {5.80, 1.43, 1.21, 1.26}};
constexpr double kLevelCostUs = 45.0;  // prefix-id kernels and a launch per level

// Cost table of the mapping a span would run with (the whole-wave mapping
// for lanes = 64, the register tables otherwise).
const GateCost& cost_of(EvolveShape s) {
  if (s.lds) return s.lanes == 4 ? kCostLds4 : s.lanes == 8 ? kCostLds8 : kCostLds16;
  if (s.lanes == 64 || s.lanes == 32) return kCostWave;
  return s.lanes >= 16 ? kCostReg16 : kCostReg8;
}

int gate_kind(const DGate& g) {
  return g.op == OP_H ? 0 : g.op == OP_CX ? 1 : g.op == OP_CZ ? 2 : 3;
}

// Estimated time of `items` work items through gates with `cnt[kind]` gates
// of each kind; the row count scales the per-item throughput term.  A
// mapping that holds at most `cap` items on the chip at once runs whole
// rounds of cap items at full throughput and a last partial round, which is
// charged like a launch of that many items alone (latency-bound when small).
double span_us(const GateCost& c, const double cnt[4], double items, double row_scale, double cap) {
  double full = 0.0, rest = items;
  if (cap > 0 && items > cap) {
    full = std::floor(items / cap) * cap;
    rest = items - full;
  }
  double t = 0.0;
  for (int k = 0; k < 4; ++k) {
    const double per = c.thr[k] * row_scale / 65536.0;
    t += cnt[k] * (full * per + (rest > 0 ? std::max(c.lat[k], rest * per) : 0.0));
  }
  return t;
}

uint32_t branch_bits(uint32_t nb) {
  uint32_t b = 0;
  while ((1u << b) < nb) ++b;
  return b;
}

// Expected number of distinct branch prefixes after each slot occurrence
// among chi terms.  EXACT enumerates every combination; SPARSIFY draws each
// slot's branch j with probability |c_j| / W independently, so
// E[#distinct] = sum over prefixes of 1 - (1 - P)^chi: prefixes of
// probability >= eps are kept explicitly, lighter ones are counted as chi P
// (each sample in them ends up distinct), and once the explicit list grows
// large every later level is taken as saturated.
std::vector<double> estimate_distinct(const Instance& I, const std::vector<uint16_t>& occ) {
  const double chi = (double)I.chi;
  std::vector<double> D(occ.size() + 1, chi);
  D[0] = 1.0;
  if (I.mode == CHSIM_EXACT) {
    double prod = 1.0;
    for (size_t j = 0; j < occ.size(); ++j) {
      prod *= (double)I.slots_h[occ[j]].n_branch;
      D[j + 1] = std::min(chi, prod);
    }
    return D;
  }
  const double eps = 4.0 / chi;
  const size_t kMaxList = (size_t)1 << 18;
  std::vector<double> P{1.0}, next;
  double pruned = 0.0;
  for (size_t j = 0; j < occ.size(); ++j) {
    const SlotTable& st = I.slots_h[occ[j]];
    next.clear();
    double prev_cum = 0.0;
    for (uint32_t b = 0; b < st.n_branch; ++b) {
      const double pb = (st.cum[b] - prev_cum) / st.total;
      prev_cum = st.cum[b];
      if (!(pb > 0.0)) continue;
      for (double x : P) {
        const double y = x * pb;
        if (y >= eps) next.push_back(y);
        else pruned += y;
      }
    }
    P.swap(next);
    double d = chi * pruned;
    for (double x : P) d += -std::expm1(chi * std::log1p(-std::min(x, 1.0 - 1e-16)));
    D[j + 1] = std::min(chi, d);
    if (P.size() > kMaxList) break;  // later levels stay at chi
  }
  return D;
}

// Choose checkpoint levels (slot occurrences) and the mapping of each span
// to minimise the estimated time: a span from level i to level j runs the
// gates between them on the (estimated) distinct prefixes at j, bounded
// below by the latency of the gates for a lone wave; every level adds a
// fixed cost; the last span runs chi terms.  Mode 2 drops the fixed cost and
// takes any plan that saves work, so that small tests exercise the path.
void plan_prefix(Instance& I, const std::vector<DGate>& dg, EvolveShape shape) {
  I.plan_cut.clear();
  I.plan_lanes.clear();
  I.plan_span_off.assign(1, 0);
  I.plan_slot_h.clear();
  I.plan_width_h.clear();
  I.plan_frac = 1.0;
  // Slot occurrences: a SLOT_SPOW gate, or a run of conditional gates of one slot.
  std::vector<uint16_t> occ;
  std::vector<uint32_t> end;
  for (size_t i = 0; i < dg.size(); ++i) {
    const DGate& g = dg[i];
    if (g.cond & kSlotStart) {
      occ.push_back(g.slot);
      end.push_back((uint32_t)(i + 1));
    } else if ((g.cond & kCondApply) && !end.empty() && end.back() == i) {
      end.back() = (uint32_t)(i + 1);
    }
  }
  const size_t m = occ.size();
  if (m == 0 || I.prefix_mode == 0) return;
  // Cumulative gate counts by kind at each level boundary.
  std::vector<std::array<double, 4>> C(m + 1), Cw(dg.size() + 1);
  Cw[0] = {0, 0, 0, 0};
  for (size_t i = 0; i < dg.size(); ++i) {
    Cw[i + 1] = Cw[i];
    Cw[i + 1][gate_kind(dg[i])] += 1.0;
  }
  C[0] = Cw[0];
  for (size_t j = 0; j < m; ++j) C[j + 1] = Cw[end[j]];
  const std::array<double, 4> Ct = Cw[dg.size()];
  const double chi = (double)I.chi;
  const double rows = (double)I.n / 50.0;  // the table was measured at n = 50
  const double cap = (double)evolve_capacity(shape, I.n);
  const std::vector<double> D = estimate_distinct(I, occ);
  const bool force = I.prefix_mode == 2;
  auto seg = [&](size_t i, size_t j, double items, int* lanes) {
    double cnt[4];
    for (int k = 0; k < 4; ++k) cnt[k] = (j <= m ? C[j][k] : Ct[k]) - C[i][k];
    const double tp = span_us(cost_of(shape), cnt, items, rows, cap);
    const double tw = span_us(kCostWave, cnt, items, rows, 0.0);
    if (lanes) *lanes = tw < tp ? 64 : 0;
    return std::min(tp, tw);
  };
  auto work = [&](size_t i, size_t j, double items) {  // weighted gate applications
    double w = 0;
    for (int k = 0; k < 4; ++k) w += ((j <= m ? C[j][k] : Ct[k]) - C[i][k]) * (k == 0 ? 8.0 : 1.0);
    return w * items;
  };
  std::vector<uint32_t> bits(m + 1, 0);
  for (size_t j = 0; j < m; ++j) bits[j + 1] = bits[j] + branch_bits(I.slots_h[occ[j]].n_branch);
  const double inf = 1e300;
  std::vector<double> best(m + 1, inf);
  std::vector<int> from(m + 1, -1);
  best[0] = 0.0;
  for (size_t j = 1; j <= m; ++j)
    for (size_t i = 0; i < j; ++i) {
      if (best[i] >= inf || bits[j] - bits[i] > 32) continue;
      const double c = best[i] + (force ? work(i, j, D[j]) : seg(i, j, D[j], nullptr) + kLevelCostUs);
      if (c < best[j]) {
        best[j] = c;
        from[j] = (int)i;
      }
    }
  const double plain = force ? work(0, m + 1, chi) : seg(0, m + 1, chi, nullptr);
  size_t last = 0;
  double total = plain;
  for (size_t i = 1; i <= m; ++i) {
    if (best[i] >= inf) continue;
    const double c = best[i] + (force ? work(i, m + 1, chi) : seg(i, m + 1, chi, nullptr));
    if (c < total) {
      total = c;
      last = i;
    }
  }
  if (last == 0) return;
  std::vector<size_t> levels;
  for (size_t j = last; j != 0; j = (size_t)from[j]) levels.push_back(j);
  std::reverse(levels.begin(), levels.end());
  size_t prev = 0;
  for (size_t j : levels) {
    for (size_t t = prev; t < j; ++t) {
      I.plan_slot_h.push_back(occ[t]);
      I.plan_width_h.push_back((uint8_t)branch_bits(I.slots_h[occ[t]].n_branch));
    }
    I.plan_span_off.push_back((uint32_t)I.plan_slot_h.size());
    I.plan_cut.push_back(end[j - 1]);
    int lanes = 0;
    seg(prev, j, D[j], &lanes);
    I.plan_lanes.push_back(lanes);
    prev = j;
  }
  I.plan_frac = plain > 0 ? total / plain : 1.0;
}

// 64-bit words of the gate list (8 bytes per gate) mixed one at a time.
uint64_t dg_hash(const std::vector<DGate>& dg) {
  uint64_t h = 1469598103934665603ull;
  for (const DGate& g : dg) {
    uint64_t w;
    std::memcpy(&w, &g, sizeof w);
    h = (h ^ w) * 0x9E3779B97F4A7C15ull;
    h ^= h >> 29;
  }
  return h;
}

uint64_t gates_key(const Instance& I, uint64_t gate_hash) {
  uint64_t h = gate_hash;
  auto mix = [&](uint64_t w) {
    h = (h ^ w) * 0x9E3779B97F4A7C15ull;
    h ^= h >> 29;
  };
  mix(I.chi);
  mix((uint64_t)I.mode);
  mix((uint64_t)I.prefix_mode);
  return h;
}

// ---- shared-prefix evolution: run ------------------------------------------
TermsView ckpt_view(chsim_ctx* ctx, const Instance& I, int k) {
  TermsView t;
  std::memset(&t, 0, sizeof t);
  t.n = I.n;
  t.n_slot = I.n_slot;
  t.chi = I.chi;
  t.F = ctx->ck_F[k].p;
  t.G = ctx->ck_G[k].p;
  t.M = ctx->ck_M[k].p;
  t.gamma = ctx->ck_gamma[k].p;
  t.v = ctx->ck_v[k].p;
  t.s = ctx->ck_s[k].p;
  t.omega = ctx->ck_omega[k].p;
  return t;
}

// Evolve every term of I through the device gate list (ctx->gates, dg on the
// host), from |0^n> or from the stored terms.
Instance::SpanStat span_stat(const std::vector<DGate>& dg, uint32_t g0, uint32_t g1, int level,
                             uint64_t items) {
  Instance::SpanStat st;
  st.level = level;
  st.items = items;
  for (auto& k : st.kinds) k = 0;
  for (uint32_t i = g0; i < g1; ++i) {
    const DGate& g = dg[i];
    const int kind = (g.cond & kCondApply) ? 4 : g.op == OP_H ? 0 : g.op == OP_CX ? 1 : g.op == OP_CZ ? 2 : 3;
    ++st.kinds[kind];
  }
  return st;
}

chsim_status evolve_all(chsim_ctx* ctx, Instance& I, const std::vector<DGate>& dg, EvolveShape shape,
                        bool from_zero, hipStream_t s) {
  if (shape.lanes == 0) shape = evolve_default_shape(I.n);
  const uint32_t ng = (uint32_t)dg.size();
  const uint32_t n_occ_all = (uint32_t)ctx->occ_start.size();
  // Slot occurrences whose first gate lies in [g0, g1).
  auto occ_range = [&](uint32_t g0, uint32_t g1, uint32_t* first) {
    const auto b = std::lower_bound(ctx->occ_start.begin(), ctx->occ_start.end(), g0);
    const auto e = std::lower_bound(ctx->occ_start.begin(), ctx->occ_start.end(), g1);
    *first = (uint32_t)(b - ctx->occ_start.begin());
    return (uint32_t)(e - b);
  };
  I.last_spans.clear();
  if (!from_zero || I.prefix_mode == 0) {
    I.last_spans.push_back(span_stat(dg, 0, ng, -1, I.chi));
    HIP_TRY(launch_evolve(I.view(), ctx->gates.p, ng, ctx->slotseq.p, n_occ_all, from_zero, ctx->err.p,
                          shape, s));
    return CHSIM_OK;
  }
  const uint64_t key = gates_key(I, ctx->dg_hash) ^ ((uint64_t)(shape.lanes | (shape.lds ? 0x100 : 0)) << 48);
  if (!I.plan_valid || I.plan_key != key) {
    plan_prefix(I, dg, shape);
    I.plan_key = key;
    I.plan_valid = true;
    if (!I.plan_cut.empty()) {
      HIP_TRY(I.plan_slot.ensure(I.plan_slot_h.size()));
      HIP_TRY(I.plan_width.ensure(I.plan_width_h.size()));
      HIP_TRY(hipMemcpy(I.plan_slot.p, I.plan_slot_h.data(), I.plan_slot_h.size() * sizeof(uint16_t),
                        hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(I.plan_width.p, I.plan_width_h.data(), I.plan_width_h.size(), hipMemcpyHostToDevice));
    }
  }
  const size_t K = I.plan_cut.size();
  if (K == 0) {
    I.last_spans.push_back(span_stat(dg, 0, ng, -1, I.chi));
    HIP_TRY(launch_evolve(I.view(), ctx->gates.p, ng, ctx->slotseq.p, n_occ_all, true, ctx->err.p, shape, s));
    return CHSIM_OK;
  }
  const uint64_t chi = I.chi, n = I.n;
  uint64_t ts = 1;
  while (ts < 2 * chi) ts <<= 1;
  HIP_TRY(ctx->pf_table.ensure(ts));
  HIP_TRY(ctx->pf_ids.ensure(ts));
  HIP_TRY(ctx->pf_slotof.ensure(chi));
  HIP_TRY(ctx->pf_rep.ensure(chi));
  HIP_TRY(ctx->pf_parent.ensure(chi));
  HIP_TRY(I.plan_count.ensure(K));
  for (int k = 0; k < 2; ++k) {
    HIP_TRY(ctx->pf_id[k].ensure(chi));
    HIP_TRY(ctx->ck_F[k].ensure(n * chi));
    HIP_TRY(ctx->ck_G[k].ensure(n * chi));
    HIP_TRY(ctx->ck_M[k].ensure(n * chi));
    HIP_TRY(ctx->ck_gamma[k].ensure(n * chi));
    HIP_TRY(ctx->ck_v[k].ensure(chi));
    HIP_TRY(ctx->ck_s[k].ensure(chi));
    HIP_TRY(ctx->ck_omega[k].ensure(chi));
  }
  const uint32_t* prev_id = nullptr;
  uint32_t g0 = 0;
  for (size_t k = 0; k < K; ++k) {
    PrefixLevelArgs A;
    A.branch = I.branch.p;
    A.chi = chi;
    A.slot = I.plan_slot.p + I.plan_span_off[k];
    A.width = I.plan_width.p + I.plan_span_off[k];
    A.n_span = I.plan_span_off[k + 1] - I.plan_span_off[k];
    A.prev_id = prev_id;
    A.table = ctx->pf_table.p;
    A.table_mask = ts - 1;
    A.ids = ctx->pf_ids.p;
    A.slot_of = ctx->pf_slotof.p;
    A.counter = I.plan_count.p + k;
    A.id_out = ctx->pf_id[k % 2].p;
    A.rep = ctx->pf_rep.p;
    A.parent = ctx->pf_parent.p;
    A.first_counters = k == 0 ? (uint32_t)K : 0u;
    HIP_TRY(launch_prefix_level(A, s));
    EvolveJob J;
    J.src = ckpt_view(ctx, I, (int)((k + 1) % 2));
    J.dst = ckpt_view(ctx, I, (int)(k % 2));
    J.src_rs = J.dst_rs = 1;  // checkpoint states: rows of a state contiguous
    J.src_is = J.dst_is = n;
    J.src_idx = ctx->pf_parent.p;
    J.br_idx = ctx->pf_rep.p;
    J.branch = I.branch.p;
    J.chi_br = chi;
    J.count_dev = I.plan_count.p + k;
    J.count = chi;
    const uint32_t g1 = I.plan_cut[k];
    uint32_t o0 = 0;
    J.n_occ = occ_range(g0, g1, &o0);
    J.slot_seq = ctx->slotseq.p + o0;
    I.last_spans.push_back(span_stat(dg, g0, g1, (int)k, 0));
    const EvolveShape span_shape = I.plan_lanes[k] ? evolve_shape_for(I.n, I.plan_lanes[k]) : shape;
    HIP_TRY(launch_evolve_job(J, ctx->gates.p + g0, g1 - g0, k == 0, ctx->err.p, span_shape, s));
    prev_id = ctx->pf_id[k % 2].p;
    g0 = g1;
  }
  EvolveJob J;
  J.src = ckpt_view(ctx, I, (int)((K - 1) % 2));
  J.dst = I.view();
  J.src_rs = 1;
  J.src_is = n;
  J.dst_rs = chi;
  J.dst_is = 1;
  J.src_idx = prev_id;
  J.br_idx = nullptr;
  J.branch = I.branch.p;
  J.chi_br = chi;
  J.count_dev = nullptr;
  J.count = chi;
  uint32_t o0 = 0;
  J.n_occ = occ_range(g0, ng, &o0);
  J.slot_seq = ctx->slotseq.p + o0;
  I.last_spans.push_back(span_stat(dg, g0, ng, -1, chi));
  HIP_TRY(launch_evolve_job(J, ctx->gates.p + g0, ng - g0, false, ctx->err.p, shape, s));
  return CHSIM_OK;
}

}  // namespace

chsim_status chsim_apply_clifford(chsim_ctx* ctx, uint32_t inst, const chsim_gate* gates,
                                  size_t n_gates, void* stream) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  if (n_gates == 0) return CHSIM_OK;
  if (!gates) return fail(CHSIM_EINVAL, "null gate list");
  Instance& I = ctx->inst[inst];
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  // The same list as the last call (same instance): its conversion and its
  // device copy are still current.
  const bool same = ctx->dg_inst == inst && ctx->dg_in.size() == n_gates &&
                    std::memcmp(ctx->dg_in.data(), gates, n_gates * sizeof(chsim_gate)) == 0;
  std::vector<DGate>& dg = ctx->dg;
  if (!same) {
    ctx->dg_inst = UINT32_MAX;  // invalid until the new list is converted and uploaded
    dg.clear();
    dg.reserve(n_gates);
    for (size_t i = 0; i < n_gates; ++i) {
      const chsim_gate& g = gates[i];
      if (g.op == CHSIM_SLOT) {
        if (g.slot >= I.n_slot) return fail(CHSIM_EINVAL, "gate %zu: slot %u >= n_slot %u", i, g.slot, I.n_slot);
        const SlotTable& tb = I.slots_h[g.slot];
        if (tb.spow_q >= 0) {
          uint32_t packed = 0;  // branch j -> S^{spow[j]}, two bits each
          for (uint32_t j = 0; j < tb.n_branch; ++j) packed |= (uint32_t)(tb.spow[j] & 3u) << (2 * j);
          dg.push_back(DGate{OP_SLOT_SPOW, (uint8_t)tb.spow_q, (uint8_t)(packed & 0xffu), (uint8_t)(packed >> 8),
                             (uint16_t)g.slot, kSlotStart, 0});
        } else if (!I.diag_h[g.slot].empty()) {
          // Diagonal branches: one conditional gate per distinct net gate.
          bool first = true;
          for (DGate bg : I.diag_h[g.slot]) {
            bg.slot = (uint16_t)g.slot;
            bg.cond = (uint8_t)(kCondApply | (first ? kSlotStart : 0));
            dg.push_back(bg);
            first = false;
          }
        } else {
          // A general branch list becomes conditional gates: each term applies
          // only the gates of its own branch.
          bool first = true;
          for (uint32_t j = 0; j < tb.n_branch; ++j)
            for (uint32_t k = tb.goff[j]; k < tb.goff[j + 1]; ++k) {
              DGate bg = I.bgates_h[k];
              bg.slot = (uint16_t)g.slot;
              bg.cond = (uint8_t)(kCondApply | (first ? kSlotStart : 0));
              bg.arg2 = (uint8_t)(1u << j);
              dg.push_back(bg);
              first = false;
            }
        }
      } else {
        if (!valid_clifford(g, I.n))
          return fail(CHSIM_EINVAL, "gate %zu: (%u, %u, %u) invalid for n = %u", i, g.op, g.q, g.r, I.n);
        push_gate(dg, g);
      }
    }
    // One padding entry past the last gate: the LDS kernel reads the gate
    // after the current one without a bound check.
    static const DGate kPadGate = {OP_S, 0, 0, 0, 0, 0, 0};
    HIP_TRY(ctx->gates.ensure(dg.size() + 1));
    HIP_TRY(hipMemcpyAsync(ctx->gates.p, dg.data(), dg.size() * sizeof(DGate), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ctx->gates.p + dg.size(), &kPadGate, sizeof(DGate), hipMemcpyHostToDevice, s));
    ctx->occ_start.clear();
    ctx->slotseq_h.clear();
    for (size_t i = 0; i < dg.size(); ++i)
      if (dg[i].cond & kSlotStart) {
        ctx->occ_start.push_back((uint32_t)i);
        ctx->slotseq_h.push_back(dg[i].slot);
      }
    HIP_TRY(ctx->slotseq.ensure(ctx->slotseq_h.size()));
    if (!ctx->slotseq_h.empty())
      HIP_TRY(hipMemcpyAsync(ctx->slotseq.p, ctx->slotseq_h.data(), ctx->slotseq_h.size() * sizeof(uint32_t),
                             hipMemcpyHostToDevice, s));
    ctx->dg_hash = dg_hash(dg);
    ctx->dg_in.assign(gates, gates + n_gates);
    ctx->dg_inst = inst;
  }
  I.drop_chains();
  HIP_TRY(hipMemsetAsync(ctx->err.p, 0, sizeof(uint32_t), s));
  if (I.autotune && I.at_zero) {
    // Every shape computes the same terms from |0^n>, so timing all of them in
    // turn leaves the store correct; keep the fastest.
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = 0.f;
    EvolveShape best_shape;
    for (int ci = 0; ci < kTuneShapes; ++ci) {
      const EvolveShape sh = shape_of_value(I.n, kTuneLanes[ci]);
      I.tuned_ms[ci] = 0.f;
      if (!evolve_shape_supported(sh, I.n)) continue;
      HIP_TRY(hipEventRecord(e0, s));
      st = evolve_all(ctx, I, dg, sh, true, s);
      if (st) return st;
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      I.tuned_ms[ci] = ms;
      if (best_shape.lanes == 0 || ms < best) {
        best = ms;
        best_shape = sh;
      }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    I.shape = best_shape;
    I.autotune = false;
    // Leave the store as the chosen shape computes it.
    st = evolve_all(ctx, I, dg, I.shape, true, s);
    if (st) return st;
  } else {
    st = evolve_all(ctx, I, dg, I.shape, I.at_zero, s);
    if (st) return st;
  }
  I.at_zero = false;
  I.amp_ready = false;
  return check_err_flag(ctx, s, "apply_clifford");
}

namespace {

constexpr uint32_t kAmpTargetItems = 2048;  // work items per launch to aim for

struct AmpReq {
  uint32_t inst;
  const uint64_t* x;  // device
  uint32_t n_x;
  double2* out;       // device
};

// Run the amplitude prologue of an instance if its terms changed since.
chsim_status ensure_amp_prep(Instance& I, hipStream_t s) {
  if (I.amp_ready) return CHSIM_OK;
  HIP_TRY(I.acrow.ensure((size_t)I.n * I.chi));
  HIP_TRY(I.acst.ensure(I.chi));
  HIP_TRY(launch_amp_prep(I.view(), I.acrow.p, I.acst.p, s));
  I.amp_ready = true;
  return CHSIM_OK;
}

// Plan, upload the plan if it differs from the last one, and launch.
chsim_status run_amplitudes_xpl(chsim_ctx* ctx, const std::vector<AmpReq>& reqs, bool fp32c, uint32_t xpl,
                                hipStream_t s) {
  for (const auto& r : reqs) {
    chsim_status st = ensure_amp_prep(ctx->inst[r.inst], s);
    if (st) return st;
  }
  std::vector<AmpRequestPlan> plan;
  uint64_t total_x = 0;
  for (const auto& r : reqs) {
    const Instance& I = ctx->inst[r.inst];
    plan.push_back(AmpRequestPlan{I.n, r.n_x, I.chi});
    total_x += r.n_x;
  }
  // The plan depends on the requests' shapes only; reuse the last one.
  std::vector<uint64_t> shape_key;
  shape_key.reserve(3 * plan.size());
  for (const auto& p : plan) {
    shape_key.push_back(p.n);
    shape_key.push_back(p.n_x);
    shape_key.push_back(p.chi);
  }
  if (shape_key != ctx->amp_shape_key || xpl != ctx->amp_plan_xpl) {
    amp_plan(plan, kAmpTargetItems, xpl, ctx->amp_items_h, ctx->amp_tpr, ctx->amp_nr);
    ctx->amp_shape_key = shape_key;
    ctx->amp_plan_xpl = xpl;
  }
  const std::vector<AmpItem>& items = ctx->amp_items_h;
  const std::vector<uint32_t>& tpr = ctx->amp_tpr;
  const std::vector<uint32_t>& nr = ctx->amp_nr;
  size_t part = 0;
  for (size_t q = 0; q < reqs.size(); ++q) part += (size_t)nr[q] * reqs[q].n_x;
  HIP_TRY(ctx->partial.ensure(part));
  std::vector<AmpInst> insts(reqs.size());
  std::vector<uint64_t> prefix(reqs.size() + 1, 0);
  size_t off = 0;
  for (size_t q = 0; q < reqs.size(); ++q) {
    AmpInst a;
    std::memset(&a, 0, sizeof a);
    Instance& I = ctx->inst[reqs[q].inst];
    a.T = I.view();
    a.crow = I.acrow.p;
    a.cst = I.acst.p;
    a.x = reqs[q].x;
    a.partial = ctx->partial.p + off;
    a.out = reqs[q].out;
    a.n_x = reqs[q].n_x;
    a.tiles_per_range = tpr[q];
    a.n_ranges = nr[q];
    insts[q] = a;
    off += (size_t)nr[q] * reqs[q].n_x;
    prefix[q + 1] = prefix[q] + reqs[q].n_x;
  }
  const bool same = insts.size() == ctx->amp_key.size() && ctx->amp_key_xpl == xpl &&
                    std::memcmp(insts.data(), ctx->amp_key.data(), insts.size() * sizeof(AmpInst)) == 0;
  if (!same) {
    HIP_TRY(ctx->amp_insts.ensure(insts.size()));
    HIP_TRY(ctx->amp_items.ensure(items.size()));
    HIP_TRY(ctx->amp_prefix.ensure(prefix.size()));
    HIP_TRY(ctx->amp_counter.ensure(1));
    HIP_TRY(hipMemcpyAsync(ctx->amp_insts.p, insts.data(), insts.size() * sizeof(AmpInst),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ctx->amp_items.p, items.data(), items.size() * sizeof(AmpItem),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ctx->amp_prefix.p, prefix.data(), prefix.size() * sizeof(uint64_t),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // the host vectors die with this call
    ctx->amp_key = insts;
    ctx->amp_key_xpl = xpl;
    ctx->amp_n_items = (uint32_t)items.size();
  }
  HIP_TRY(launch_amp_items(ctx->amp_insts.p, ctx->amp_items.p, ctx->amp_n_items, ctx->amp_counter.p,
                           fp32c, xpl, ctx->amp_prefix.p, (uint32_t)reqs.size(), total_x, s));
  return CHSIM_OK;
}

// With the autotuner armed, run the call twice per bitstrings-per-lane value
// (the first run plans and uploads the work items; every run leaves correct
// outputs), time the second with hipEvents, keep the faster.
chsim_status run_amplitudes(chsim_ctx* ctx, const std::vector<AmpReq>& reqs, bool fp32c, hipStream_t s) {
  if (!ctx->amp_tune) return run_amplitudes_xpl(ctx, reqs, fp32c, ctx->amp_xpl, s);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  uint32_t best = 2;
  for (uint32_t xpl = 1; xpl <= 2; ++xpl) {
    chsim_status st = run_amplitudes_xpl(ctx, reqs, fp32c, xpl, s);
    if (!st) {
      HIP_TRY(hipEventRecord(e0, s));
      st = run_amplitudes_xpl(ctx, reqs, fp32c, xpl, s);
    }
    if (st) {
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      return st;
    }
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    ctx->amp_tune_ms[xpl - 1] = ms;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  best = ctx->amp_tune_ms[0] < ctx->amp_tune_ms[1] ? 1u : 2u;
  ctx->amp_xpl = best;
  ctx->amp_tune = false;
  return CHSIM_OK;
}

chsim_status check_bits(const Instance& I, const uint64_t* x, size_t n_x, size_t req) {
  if (I.n >= 64) return CHSIM_OK;
  const uint64_t bad = ~((1ull << I.n) - 1ull);
  for (size_t i = 0; i < n_x; ++i)
    if (x[i] & bad) return fail(CHSIM_EINVAL, "request %zu: bitstring %zu has bits >= n = %u", req, i, I.n);
  return CHSIM_OK;
}

}  // namespace

chsim_status chsim_amplitudes(chsim_ctx* ctx, uint32_t inst, const uint64_t* x, size_t n_x,
                              double* out, uint32_t flags, void* stream) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  if (n_x == 0 || !x || !out) return fail(CHSIM_EINVAL, "empty or null bitstring/output arrays");
  if (n_x > 0xFFFFFFFFull) return fail(CHSIM_EINVAL, "too many bitstrings");
  Instance& I = ctx->inst[inst];
  const bool dev = flags & CHSIM_DEVICE_PTRS;
  if (!dev && (st = check_bits(I, x, n_x, 0))) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  st = ensure_materialised(I, s);
  if (st) return st;
  const uint64_t* xd;
  st = stage_in(ctx->xbuf, x, n_x, dev, s, &xd);
  if (st) return st;
  double2* outd;
  if (dev) outd = reinterpret_cast<double2*>(out);
  else {
    HIP_TRY(ctx->out.ensure(n_x));
    outd = ctx->out.p;
  }
  st = run_amplitudes(ctx, {AmpReq{inst, xd, (uint32_t)n_x, outd}}, (flags & CHSIM_FP32C) != 0, s);
  if (st) return st;
  if (!dev) {
    HIP_TRY(hipMemcpyAsync(out, outd, n_x * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return CHSIM_OK;
}

chsim_status chsim_amplitudes_batch(chsim_ctx* ctx, const chsim_amp_request* reqs, size_t n_req,
                                    uint32_t flags, void* stream) {
  g_err.clear();
  if (!ctx) return fail(CHSIM_EINVAL, "null context");
  if (n_req == 0 || !reqs) return fail(CHSIM_EINVAL, "empty or null request array");
  if (n_req > 0xFFFFFFFFull) return fail(CHSIM_EINVAL, "too many requests");
  const bool dev = flags & CHSIM_DEVICE_PTRS;
  size_t total = 0;
  for (size_t q = 0; q < n_req; ++q) {
    const chsim_amp_request& r = reqs[q];
    if (r.inst >= ctx->inst.size()) return fail(CHSIM_EINVAL, "request %zu: instance %u out of range", q, r.inst);
    if (r.n_x == 0 || !r.x || !r.out) return fail(CHSIM_EINVAL, "request %zu: empty or null arrays", q);
    if (r.n_x > 0xFFFFFFFFull) return fail(CHSIM_EINVAL, "request %zu: too many bitstrings", q);
    if (!dev) {
      chsim_status st = check_bits(ctx->inst[r.inst], r.x, r.n_x, q);
      if (st) return st;
    }
    total += r.n_x;
  }
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  for (size_t q = 0; q < n_req; ++q) {
    chsim_status st = ensure_materialised(ctx->inst[reqs[q].inst], s);
    if (st) return st;
  }
  std::vector<AmpReq> rq(n_req);
  if (dev) {
    for (size_t q = 0; q < n_req; ++q)
      rq[q] = AmpReq{reqs[q].inst, reqs[q].x, (uint32_t)reqs[q].n_x, reinterpret_cast<double2*>(reqs[q].out)};
  } else {
    HIP_TRY(ctx->xbuf.ensure(total));
    HIP_TRY(ctx->out.ensure(total));
    size_t off = 0;
    for (size_t q = 0; q < n_req; ++q) {
      HIP_TRY(hipMemcpyAsync(ctx->xbuf.p + off, reqs[q].x, reqs[q].n_x * sizeof(uint64_t),
                             hipMemcpyHostToDevice, s));
      rq[q] = AmpReq{reqs[q].inst, ctx->xbuf.p + off, (uint32_t)reqs[q].n_x, ctx->out.p + off};
      off += reqs[q].n_x;
    }
  }
  chsim_status st = run_amplitudes(ctx, rq, (flags & CHSIM_FP32C) != 0, s);
  if (st) return st;
  if (!dev) {
    for (size_t q = 0; q < n_req; ++q)
      HIP_TRY(hipMemcpyAsync(reqs[q].out, rq[q].out, reqs[q].n_x * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return CHSIM_OK;
}

chsim_status chsim_amplitudes_noalloc(chsim_ctx* ctx, uint32_t inst, const uint64_t* x, size_t n_x,
                                      double* out, uint32_t flags, void* stream) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  if (!(flags & CHSIM_DEVICE_PTRS)) return fail(CHSIM_EINVAL, "chsim_amplitudes_noalloc takes device pointers only");
  if (n_x == 0 || !x || !out) return fail(CHSIM_EINVAL, "empty or null bitstring/output arrays");
  if (n_x > 0xFFFFFFFFull) return fail(CHSIM_EINVAL, "too many bitstrings");
  Instance& I = ctx->inst[inst];
  // Scratch layout: prologue rows [n][chi], term constants [chi], partial
  // sums [ranges][n_x], the request record, the work items, the bitstring
  // prefix and the queue counter, each 256-byte aligned.
  const uint32_t xpl = ctx->amp_xpl;
  uint32_t tpr = 0, n_ranges = 0, chunks = 0;
  amp_plan_single(I.chi, (uint32_t)n_x, kAmpTargetItems, xpl, &tpr, &n_ranges, &chunks);
  const uint64_t n_items = (uint64_t)n_ranges * chunks;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t o_crow = 0;
  const size_t o_cst = o_crow + up((size_t)I.n * I.chi * sizeof(uint64_t));
  const size_t o_part = o_cst + up((size_t)I.chi * sizeof(AmpTerm));
  const size_t o_inst = o_part + up((size_t)n_ranges * n_x * sizeof(double2));
  const size_t o_items = o_inst + up(sizeof(AmpInst));
  const size_t o_prefix = o_items + up((size_t)n_items * sizeof(AmpItem));
  const size_t o_counter = o_prefix + up(2 * sizeof(uint64_t));
  const size_t need = o_counter + up(sizeof(uint32_t));
  if (n_items > 0xFFFFFFFFull || need > kNoAllocScratch)
    return fail(CHSIM_EINVAL, "request needs %zu bytes of scratch (n = %u, chi = %llu, %zu strings); the limit is %zu",
                need, I.n, (unsigned long long)I.chi, n_x, kNoAllocScratch);
  HIP_TRY(hipSetDevice(ctx->device));
  void* base = nullptr;
  if ((st = scratch_address(ctx->device, &base))) return st;
  unsigned char* sp = static_cast<unsigned char*>(base);
  hipStream_t s = as_stream(stream);
  st = ensure_materialised(I, s);
  if (st) return st;
  uint64_t* crow = reinterpret_cast<uint64_t*>(sp + o_crow);
  AmpTerm* cst = reinterpret_cast<AmpTerm*>(sp + o_cst);
  HIP_TRY(launch_amp_prep(I.view(), crow, cst, s));
  AmpInst a;
  std::memset(&a, 0, sizeof a);
  a.T = I.view();
  a.crow = crow;
  a.cst = cst;
  a.x = x;
  a.partial = reinterpret_cast<double2*>(sp + o_part);
  a.out = reinterpret_cast<double2*>(out);
  a.n_x = (uint32_t)n_x;
  a.tiles_per_range = tpr;
  a.n_ranges = n_ranges;
  AmpInst* insts_d = reinterpret_cast<AmpInst*>(sp + o_inst);
  AmpItem* items_d = reinterpret_cast<AmpItem*>(sp + o_items);
  uint64_t* prefix_d = reinterpret_cast<uint64_t*>(sp + o_prefix);
  uint32_t* counter_d = reinterpret_cast<uint32_t*>(sp + o_counter);
  HIP_TRY(launch_amp_fill_single(a, insts_d, items_d, prefix_d, (uint32_t)n_items, chunks, xpl, s));
  HIP_TRY(launch_amp_items(insts_d, items_d, (uint32_t)n_items, counter_d, (flags & CHSIM_FP32C) != 0, xpl,
                           prefix_d, 1u, n_x, s));
  return CHSIM_OK;
}

chsim_status chsim_inner_products(chsim_ctx* ctx, uint32_t inst, const uint64_t* A_off,
                                  const uint8_t* A_diag, size_t L, double* overlap, double* eta,
                                  double* eta_mean, uint32_t flags, void* stream) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  if (L == 0 || !A_off || !A_diag || !overlap) return fail(CHSIM_EINVAL, "empty or null inputs");
  Instance& I = ctx->inst[inst];
  const bool dev = flags & CHSIM_DEVICE_PTRS;
  const uint32_t n = I.n;
  if (!dev) {
    const uint64_t nm = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    for (size_t l = 0; l < L; ++l)
      for (uint32_t a = 0; a < n; ++a) {
        const uint64_t row = A_off[l * n + a] & ~(1ull << a);
        if (row & ~nm) return fail(CHSIM_EINVAL, "A_%zu row %u has bits >= n", l, a);
        if (A_diag[l * n + a] > 3) return fail(CHSIM_EINVAL, "A_%zu diagonal entry %u not in Z_4", l, a);
        for (uint32_t b = a + 1; b < n; ++b)
          if (((row >> b) & 1ull) != ((A_off[l * n + b] >> a) & 1ull))
            return fail(CHSIM_EINVAL, "A_%zu is not symmetric at (%u, %u)", l, a, b);
      }
  }
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  st = ensure_materialised(I, s);
  if (st) return st;
  HIP_TRY(hipMemsetAsync(ctx->err.p, 0, sizeof(uint32_t), s));
  HIP_TRY(ctx->eta_sum.ensure(1));
  double total = 0.0;
  // Chunks of equatorial states bound the LDS accumulator of the kernel.
  const size_t kChunk = 2048;
  std::vector<double> eta_host;
  for (size_t l0 = 0; l0 < L; l0 += kChunk) {
    const uint32_t Lc = (uint32_t)std::min(kChunk, L - l0);
    const uint64_t* ao;
    const uint8_t* ad;
    if (dev) {
      ao = A_off + l0 * n;
      ad = A_diag + l0 * n;
    } else {
      HIP_TRY(ctx->aoff.ensure((size_t)Lc * n));
      HIP_TRY(ctx->adiag.ensure((size_t)Lc * n));
      HIP_TRY(hipMemcpyAsync(ctx->aoff.p, A_off + l0 * n, (size_t)Lc * n * 8, hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(ctx->adiag.p, A_diag + l0 * n, (size_t)Lc * n, hipMemcpyHostToDevice, s));
      ao = ctx->aoff.p;
      ad = ctx->adiag.p;
    }
    const InnerPlan ip = inner_plan(I.view(), Lc);
    HIP_TRY(ctx->partial.ensure(ip.partial_elems));
    HIP_TRY(ctx->inner_work.ensure(ip.work_words));
    double2* ovd;
    double* etad;
    if (dev) {
      ovd = reinterpret_cast<double2*>(overlap) + l0;
      if (eta) etad = eta + l0;
      else {
        HIP_TRY(ctx->eta.ensure(Lc));
        etad = ctx->eta.p;
      }
    } else {
      HIP_TRY(ctx->out.ensure(Lc));
      HIP_TRY(ctx->eta.ensure(Lc));
      ovd = ctx->out.p;
      etad = ctx->eta.p;
    }
    HIP_TRY(launch_inner(I.view(), ao, ad, Lc, ip, ctx->partial.p, ctx->inner_work.p, ovd, etad, ctx->eta_sum.p,
                         ctx->err.p, s));
    double part = 0.0;
    HIP_TRY(hipMemcpyAsync(&part, ctx->eta_sum.p, sizeof(double), hipMemcpyDeviceToHost, s));
    if (!dev) {
      HIP_TRY(hipMemcpyAsync(overlap + 2 * l0, ovd, (size_t)Lc * sizeof(double2), hipMemcpyDeviceToHost, s));
      if (eta) HIP_TRY(hipMemcpyAsync(eta + l0, etad, (size_t)Lc * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    total += part;
  }
  if (eta_mean) *eta_mean = total / (double)L;
  uint32_t flag = 0;
  HIP_TRY(hipMemcpy(&flag, ctx->err.p, sizeof flag, hipMemcpyDeviceToHost));
  if (flag) return fail(CHSIM_EUNSUPPORTED, "a term has |v| = 64 (no free index for the Z_2 lift)");
  return CHSIM_OK;
}

chsim_status chsim_inner_products_ch(chsim_ctx* ctx, uint32_t inst, uint32_t bra_inst, double* overlap,
                                     double* total, uint32_t flags, void* stream) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  st = check_ctx(ctx, bra_inst);
  if (st) return st;
  if (!overlap) return fail(CHSIM_EINVAL, "null overlap array");
  Instance& K = ctx->inst[inst];
  Instance& Bt = ctx->inst[bra_inst];
  if (K.n != Bt.n) return fail(CHSIM_EINVAL, "instances differ in n (%u, %u)", K.n, Bt.n);
  if (Bt.chi > 0x7FFFFFF0ull) return fail(CHSIM_EUNSUPPORTED, "bra instance has more than 2^31 terms");
  const bool dev = flags & CHSIM_DEVICE_PTRS;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  if ((st = ensure_materialised(K, s))) return st;
  if ((st = ensure_materialised(Bt, s))) return st;
  const uint32_t n = K.n, L = (uint32_t)Bt.chi;
  HIP_TRY(ctx->chrec_k.ensure(inner_ch_record_words(n, K.chi)));
  HIP_TRY(launch_inner_ch_records(K.view(), ctx->chrec_k.p, s));
  const uint64_t* rec_b = ctx->chrec_k.p;
  if (bra_inst != inst) {
    HIP_TRY(ctx->chrec_b.ensure(inner_ch_record_words(n, Bt.chi)));
    HIP_TRY(launch_inner_ch_records(Bt.view(), ctx->chrec_b.p, s));
    rec_b = ctx->chrec_b.p;
  }
  const uint32_t groups = inner_ch_groups(K.chi, L);
  HIP_TRY(ctx->partial.ensure((size_t)groups * L));
  double2* ovd;
  if (dev) ovd = reinterpret_cast<double2*>(overlap);
  else {
    HIP_TRY(ctx->out.ensure(L));
    ovd = ctx->out.p;
  }
  double2* totd = nullptr;
  if (total) {
    if (dev) totd = reinterpret_cast<double2*>(total);
    else {
      HIP_TRY(ctx->chtotal.ensure(1));
      totd = ctx->chtotal.p;
    }
  }
  HIP_TRY(hipMemsetAsync(ctx->err.p, 0, sizeof(uint32_t), s));
  HIP_TRY(launch_inner_ch(ctx->chrec_k.p, K.b.p, K.chi, rec_b, Bt.b.p, L, n, groups, ctx->partial.p, ovd, totd,
                          ctx->err.p, s));
  if (!dev) {
    HIP_TRY(hipMemcpyAsync(overlap, ovd, (size_t)L * sizeof(double2), hipMemcpyDeviceToHost, s));
    if (total) HIP_TRY(hipMemcpyAsync(total, totd, sizeof(double2), hipMemcpyDeviceToHost, s));
  }
  uint32_t flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, ctx->err.p, sizeof flag, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (flag) return fail(CHSIM_EUNSUPPORTED, "a ket term has |v| = 64 (no free index for the Z_2 lift)");
  return CHSIM_OK;
}

static MetroView metro_view(Instance& I) {
  MetroView m;
  m.n_chain = I.n_chain;
  m.n_tiles = (uint32_t)((I.chi + kMetroTile - 1) / kMetroTile);
  m.state = I.mstate0.p;
  m.pend = I.mpend.p;
  m.pmask = I.mpmask.p;
  m.x = I.mx.p;
  m.amp = I.mamp.p;
  m.partial = I.mpartial.p;
  m.jstream = I.mj.p;
  m.ustream = I.mu.p;
  m.trace = nullptr;
  m.accepted = nullptr;
  m.n_steps = 0;
  m.n_qubits = I.n;
  return m;
}

chsim_status chsim_metropolis_init(chsim_ctx* ctx, uint32_t inst, uint32_t n_chain,
                                   const uint64_t* x0, double* amp, uint32_t flags, void* stream) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  Instance& I = ctx->inst[inst];
  if (n_chain == 0 || !x0) return fail(CHSIM_EINVAL, "no chains");
  if (I.n > 62) return fail(CHSIM_EUNSUPPORTED, "Metropolis state packs u and mu into 64 bits: needs n <= 62");
  const bool dev = flags & CHSIM_DEVICE_PTRS;
  if (!dev && I.n < 64) {
    const uint64_t bad = ~((1ull << I.n) - 1ull);
    for (uint32_t c = 0; c < n_chain; ++c)
      if (x0[c] & bad) return fail(CHSIM_EINVAL, "x0[%u] has bits >= n", c);
  }
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  st = ensure_materialised(I, s);
  if (st) return st;
  I.n_chain = n_chain;
  const size_t cells = (size_t)n_chain * I.chi;
  const uint32_t tiles = (uint32_t)((I.chi + kMetroTile - 1) / kMetroTile);
  if (I.mstate0.ensure(cells) != hipSuccess)
    return fail(CHSIM_ENOMEM, "chain state (%zu words) does not fit", cells);
  HIP_TRY(I.mpend.ensure(n_chain));
  HIP_TRY(I.mpmask.ensure(n_chain));
  HIP_TRY(hipMemsetAsync(I.mpend.p, 0, n_chain * sizeof(uint32_t), s));
  HIP_TRY(hipMemsetAsync(I.mpmask.p, 0, n_chain * sizeof(uint64_t), s));
  HIP_TRY(I.mx.ensure(n_chain));
  HIP_TRY(I.mamp.ensure(n_chain));
  HIP_TRY(I.mpartial.ensure((size_t)n_chain * tiles));
  HIP_TRY(hipMemcpyAsync(I.mx.p, x0, n_chain * 8, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  MetroView mv = metro_view(I);
  HIP_TRY(launch_metro_init(I.view(), mv, s));
  std::vector<double2> a(n_chain);
  HIP_TRY(hipMemcpyAsync(a.data(), I.mamp.p, n_chain * sizeof(double2), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (uint32_t c = 0; c < n_chain; ++c)
    if (a[c].x == 0.0 && a[c].y == 0.0) {
      I.n_chain = 0;
      return fail(CHSIM_EINVAL, "chain %u starts at a string with <x|psi> = 0", c);
    }
  if (amp) {
    if (dev) HIP_TRY(hipMemcpyAsync(amp, I.mamp.p, n_chain * sizeof(double2), hipMemcpyDeviceToDevice, s));
    else std::memcpy(amp, a.data(), n_chain * sizeof(double2));
  }
  return CHSIM_OK;
}

chsim_status chsim_metropolis_step(chsim_ctx* ctx, uint32_t inst, uint32_t n_steps,
                                   const uint32_t* j_stream, const double* u_stream,
                                   uint64_t* x_trace, uint8_t* accepted, double* amp,
                                   uint32_t flags, void* stream) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  Instance& I = ctx->inst[inst];
  if (I.n_chain == 0) return fail(CHSIM_EINVAL, "chains not initialised");
  if (n_steps == 0) return CHSIM_OK;
  if (!j_stream || !u_stream) return fail(CHSIM_EINVAL, "null random streams");
  const bool dev = flags & CHSIM_DEVICE_PTRS;
  const size_t cnt = (size_t)I.n_chain * n_steps;
  if (!dev)
    for (size_t i = 0; i < cnt; ++i)
      if (j_stream[i] >= I.n) return fail(CHSIM_EINVAL, "j_stream[%zu] = %u >= n", i, j_stream[i]);
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  MetroView mv = metro_view(I);
  mv.n_steps = n_steps;
  const uint32_t* jd;
  const double* ud;
  st = stage_in(I.mj, j_stream, cnt, dev, s, &jd);
  if (st) return st;
  st = stage_in(I.mu, u_stream, cnt, dev, s, &ud);
  if (st) return st;
  mv.jstream = jd;
  mv.ustream = ud;
  if (x_trace) {
    if (dev) mv.trace = x_trace;
    else {
      HIP_TRY(I.mtrace.ensure(cnt));
      mv.trace = I.mtrace.p;
    }
  }
  if (accepted) {
    if (dev) mv.accepted = accepted;
    else {
      HIP_TRY(I.macc.ensure(cnt));
      mv.accepted = I.macc.p;
    }
  }
  if (flags & CHSIM_GRAPH) {
    const TermsView tv = I.view();
    const bool same = I.metro_exec && I.metro_steps == n_steps &&
                      std::memcmp(&I.metro_key, &mv, sizeof mv) == 0 &&
                      std::memcmp(&I.metro_tkey, &tv, sizeof tv) == 0;
    if (!same) {
      I.drop_graph();
      if (!ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
      const hipError_t le = launch_metro_steps(tv, mv, n_steps, ctx->cap_stream);
      const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &g);
      HIP_TRY(le);
      HIP_TRY(ce);
      const hipError_t ie = hipGraphInstantiate(&I.metro_exec, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      HIP_TRY(ie);
      I.metro_key = mv;
      I.metro_tkey = tv;
      I.metro_steps = n_steps;
    }
    HIP_TRY(hipGraphLaunch(I.metro_exec, s));
    if (!I.metro_done) HIP_TRY(hipEventCreateWithFlags(&I.metro_done, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(I.metro_done, s));
  } else {
    HIP_TRY(launch_metro_steps(I.view(), mv, n_steps, s));
  }
  if (!dev) {
    if (x_trace) HIP_TRY(hipMemcpyAsync(x_trace, mv.trace, cnt * 8, hipMemcpyDeviceToHost, s));
    if (accepted) HIP_TRY(hipMemcpyAsync(accepted, mv.accepted, cnt, hipMemcpyDeviceToHost, s));
    if (amp) HIP_TRY(hipMemcpyAsync(amp, I.mamp.p, I.n_chain * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  } else if (amp) {
    HIP_TRY(hipMemcpyAsync(amp, I.mamp.p, I.n_chain * sizeof(double2), hipMemcpyDeviceToDevice, s));
  }
  return CHSIM_OK;
}

chsim_status chsim_sample_terms(chsim_ctx* ctx, uint32_t inst, size_t count, const uint64_t* alpha,
                                const uint64_t* flips, uint64_t* x_out) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  if (count == 0) return CHSIM_OK;
  if (!alpha || !flips || !x_out) return fail(CHSIM_EINVAL, "null arrays");
  Instance& I = ctx->inst[inst];
  for (size_t i = 0; i < count; ++i)
    if (alpha[i] >= I.chi) return fail(CHSIM_EINVAL, "term index %zu out of range", i);
  HIP_TRY(hipSetDevice(ctx->device));
  st = ensure_materialised(I, nullptr);
  if (st) return st;
  DevBuf<uint64_t> buf;
  HIP_TRY(buf.ensure(3 * count));
  HIP_TRY(hipMemcpy(buf.p, alpha, count * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(buf.p + count, flips, count * 8, hipMemcpyHostToDevice));
  hipError_t e = launch_sample(I.view(), buf.p, buf.p + count, buf.p + 2 * count, (uint32_t)count, nullptr);
  if (e == hipSuccess) e = hipMemcpy(x_out, buf.p + 2 * count, count * 8, hipMemcpyDeviceToHost);
  buf.release();
  if (e != hipSuccess) return fail(CHSIM_EDEVICE, "sample: %s", hipGetErrorString(e));
  return CHSIM_OK;
}

chsim_status chsim_get_terms(chsim_ctx* ctx, uint32_t inst, uint64_t first, uint64_t count,
                             uint64_t* F, uint64_t* G, uint64_t* M, uint8_t* gamma, uint64_t* v,
                             uint64_t* s, uint8_t* omega, double* b, uint8_t* branch) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  Instance& I = ctx->inst[inst];
  if (first > I.chi || count > I.chi - first) return fail(CHSIM_EINVAL, "term range out of bounds");
  if (count == 0) return CHSIM_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  st = ensure_materialised(I, nullptr);
  if (st) return st;
  HIP_TRY(hipDeviceSynchronize());
  const uint32_t n = I.n;
  // Rows are strided by chi on the device: copy each row's slice, then transpose.
  auto rows = [&](uint64_t* dst, const uint64_t* src) -> chsim_status {
    if (!dst) return CHSIM_OK;
    std::vector<uint64_t> tmp((size_t)n * count);
    HIP_TRY(hipMemcpy2D(tmp.data(), count * 8, src + first, I.chi * 8, count * 8, n, hipMemcpyDeviceToHost));
    for (uint32_t p = 0; p < n; ++p)
      for (uint64_t a = 0; a < count; ++a) dst[a * n + p] = tmp[(size_t)p * count + a];
    return CHSIM_OK;
  };
  if ((st = rows(F, I.F.p))) return st;
  if ((st = rows(G, I.G.p))) return st;
  if ((st = rows(M, I.M.p))) return st;
  if (gamma) {
    std::vector<uint8_t> tmp((size_t)n * count);
    HIP_TRY(hipMemcpy2D(tmp.data(), count, I.gamma.p + first, I.chi, count, n, hipMemcpyDeviceToHost));
    for (uint32_t p = 0; p < n; ++p)
      for (uint64_t a = 0; a < count; ++a) gamma[a * n + p] = tmp[(size_t)p * count + a];
  }
  if (v) HIP_TRY(hipMemcpy(v, I.v.p + first, count * 8, hipMemcpyDeviceToHost));
  if (s) HIP_TRY(hipMemcpy(s, I.s.p + first, count * 8, hipMemcpyDeviceToHost));
  if (omega) HIP_TRY(hipMemcpy(omega, I.omega.p + first, count, hipMemcpyDeviceToHost));
  if (b) HIP_TRY(hipMemcpy(b, I.b.p + first, count * 16, hipMemcpyDeviceToHost));
  if (branch && I.n_slot) {
    std::vector<uint8_t> tmp((size_t)I.n_slot * count);
    HIP_TRY(hipMemcpy2D(tmp.data(), count, I.branch.p + first, I.chi, count, I.n_slot, hipMemcpyDeviceToHost));
    for (uint32_t p = 0; p < I.n_slot; ++p)
      for (uint64_t a = 0; a < count; ++a) branch[a * I.n_slot + p] = tmp[(size_t)p * count + a];
  }
  return CHSIM_OK;
}

chsim_status chsim_set_terms(chsim_ctx* ctx, uint32_t inst, uint64_t first, uint64_t count,
                             const uint64_t* F, const uint64_t* G, const uint64_t* M,
                             const uint8_t* gamma, const uint64_t* v, const uint64_t* s,
                             const uint8_t* omega, const double* b) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  Instance& I = ctx->inst[inst];
  if (first > I.chi || count > I.chi - first) return fail(CHSIM_EINVAL, "term range out of bounds");
  if (!F || !G || !M || !gamma || !v || !s || !omega || !b) return fail(CHSIM_EINVAL, "null field");
  if (count == 0) return CHSIM_OK;
  const uint32_t n = I.n;
  {
    // Words the kernels index by (ctz of v-derived masks, row selections)
    // must stay below bit n; gamma is in Z_4 and omega in Z_8.
    const uint64_t hi = (n == 64) ? 0ull : ~((1ull << n) - 1ull);
    for (uint64_t a = 0; a < count; ++a) {
      if ((v[a] | s[a]) & hi) return fail(CHSIM_EINVAL, "term %llu: v or s has a bit >= n", (unsigned long long)a);
      if (omega[a] > 7) return fail(CHSIM_EINVAL, "term %llu: omega %u not in Z_8", (unsigned long long)a, omega[a]);
      for (uint32_t p = 0; p < n; ++p) {
        const size_t i = (size_t)a * n + p;
        if ((F[i] | G[i] | M[i]) & hi)
          return fail(CHSIM_EINVAL, "term %llu row %u has a bit >= n", (unsigned long long)a, p);
        if (gamma[i] > 3) return fail(CHSIM_EINVAL, "term %llu: gamma_%u not in Z_4", (unsigned long long)a, p);
      }
    }
  }
  HIP_TRY(hipSetDevice(ctx->device));
  st = ensure_materialised(I, nullptr);
  if (st) return st;
  I.drop_chains();
  HIP_TRY(hipDeviceSynchronize());
  auto rows = [&](uint64_t* dst, const uint64_t* src) -> chsim_status {
    std::vector<uint64_t> tmp((size_t)n * count);
    for (uint32_t p = 0; p < n; ++p)
      for (uint64_t a = 0; a < count; ++a) tmp[(size_t)p * count + a] = src[a * n + p];
    HIP_TRY(hipMemcpy2D(dst + first, I.chi * 8, tmp.data(), count * 8, count * 8, n, hipMemcpyHostToDevice));
    return CHSIM_OK;
  };
  if ((st = rows(I.F.p, F))) return st;
  if ((st = rows(I.G.p, G))) return st;
  if ((st = rows(I.M.p, M))) return st;
  {
    std::vector<uint8_t> tmp((size_t)n * count);
    for (uint32_t p = 0; p < n; ++p)
      for (uint64_t a = 0; a < count; ++a) tmp[(size_t)p * count + a] = gamma[a * n + p];
    HIP_TRY(hipMemcpy2D(I.gamma.p + first, I.chi, tmp.data(), count, count, n, hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMemcpy(I.v.p + first, v, count * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(I.s.p + first, s, count * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(I.omega.p + first, omega, count, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(I.b.p + first, b, count * 16, hipMemcpyHostToDevice));
  I.amp_ready = false;
  return CHSIM_OK;
}

chsim_status chsim_validate(chsim_ctx* ctx, uint32_t inst, uint64_t first, uint64_t count,
                            uint64_t* n_bad, uint64_t* first_bad, uint32_t* what) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  Instance& I = ctx->inst[inst];
  if (first > I.chi || count > I.chi - first) return fail(CHSIM_EINVAL, "term range out of bounds");
  HIP_TRY(hipSetDevice(ctx->device));
  st = ensure_materialised(I, nullptr);
  if (st) return st;
  HIP_TRY(ctx->vcheck.ensure(3));
  HIP_TRY(launch_validate(I.view(), first, count, ctx->vcheck.p, nullptr));
  unsigned long long h[3] = {0ull, ~0ull, 0ull};
  HIP_TRY(hipMemcpy(h, ctx->vcheck.p, sizeof h, hipMemcpyDeviceToHost));
  if (n_bad) *n_bad = h[0];
  if (first_bad) *first_bad = h[1];
  if (what) *what = (uint32_t)h[2];
  if (h[0]) return fail(CHSIM_ESTATE, "%llu of %llu terms violate a CH-form invariant (first %llu, flags %llu)",
                        h[0], (unsigned long long)count, h[1], h[2]);
  return CHSIM_OK;
}

chsim_status chsim_decompose_phase(double theta, uint32_t qubit, double coeff[4], uint32_t off[3],
                                   chsim_gate gates[8], chsim_decomp* out) {
  g_err.clear();
  if (!coeff || !off || !gates || !out) return fail(CHSIM_EINVAL, "null output");
  if (!std::isfinite(theta)) return fail(CHSIM_EINVAL, "theta not finite");
  if (qubit >= 64) return fail(CHSIM_EINVAL, "qubit >= 64");
  const double pi = 3.14159265358979323846264338327950288;
  const double quarter = pi / 2.0;
  double kf = std::floor(theta / quarter);
  double tp = theta - kf * quarter;
  if (tp < 0.0) {
    tp += quarter;
    kf -= 1.0;
  }
  if (tp >= quarter) {
    tp -= quarter;
    kf += 1.0;
  }
  const int k = (int)(((long long)kf % 4 + 4) % 4);
  const double half = tp / 2.0;
  const double cs = std::cos(half), sn = std::sin(half);
  // e^{i theta'/2}
  const double er = std::cos(half), ei = std::sin(half);
  // c0 = e^{i theta'/2} (cos - sin)
  coeff[0] = er * (cs - sn);
  coeff[1] = ei * (cs - sn);
  // c1 = e^{i theta'/2} sqrt(2) e^{-i pi/4} sin = e^{i theta'/2} (1 - i) sin
  const double ar = sn, ai = -sn;
  coeff[2] = er * ar - ei * ai;
  coeff[3] = er * ai + ei * ar;
  uint32_t g = 0;
  off[0] = 0;
  for (int i = 0; i < k; ++i) gates[g++] = chsim_gate{CHSIM_S, (uint8_t)qubit, 0, 0, 0};
  off[1] = g;
  for (int i = 0; i < ((k + 1) & 3); ++i) gates[g++] = chsim_gate{CHSIM_S, (uint8_t)qubit, 0, 0, 0};
  off[2] = g;
  out->n_branch = 2;
  out->coeff = coeff;
  out->off = off;
  out->gates = gates;
  return CHSIM_OK;
}

chsim_status chsim_decompose_ccz(uint32_t a, uint32_t b, uint32_t c, double coeff[16], uint32_t off[9],
                                 chsim_gate gates[24], chsim_decomp* out) {
  g_err.clear();
  if (!coeff || !off || !gates || !out) return fail(CHSIM_EINVAL, "null output");
  if (a >= 64 || b >= 64 || c >= 64) return fail(CHSIM_EINVAL, "qubit >= 64");
  if (a == b || a == c || b == c) return fail(CHSIM_EINVAL, "CCZ qubits must be distinct");
  // The group of CCZ X_j CCZ^dag has generators X_c CZ_ab, X_b CZ_ac, X_a CZ_bc.
  // Branch j keeps a subset of them (the X parts act trivially on |+++>):
  // CZ on the pair of every kept generator, Z (= S S) on every qubit that two
  // kept pairs share, and a minus sign when all three are kept.  Subsets in the
  // order of the paper's sum: {}, {ab}, {ac}, {bc}, {ab,ac}, {ab,bc}, {ac,bc}, all.
  const uint32_t pq[3][2] = {{a, b}, {a, c}, {b, c}};
  static const uint8_t kKeep[8] = {0, 1, 2, 4, 3, 5, 6, 7};
  uint32_t g = 0;
  off[0] = 0;
  for (int j = 0; j < 8; ++j) {
    const uint8_t keep = kKeep[j];
    for (int e = 0; e < 3; ++e)
      if (keep >> e & 1) gates[g++] = chsim_gate{CHSIM_CZ, (uint8_t)pq[e][0], (uint8_t)pq[e][1], 0, 0};
    const uint32_t qs[3] = {a, b, c};
    for (uint32_t x : qs) {
      int uses = 0;
      for (int e = 0; e < 3; ++e) uses += (keep >> e & 1) && (pq[e][0] == x || pq[e][1] == x);
      if (uses >= 2) {
        gates[g++] = chsim_gate{CHSIM_S, (uint8_t)x, 0, 0, 0};
        gates[g++] = chsim_gate{CHSIM_S, (uint8_t)x, 0, 0, 0};
      }
    }
    off[j + 1] = g;
    coeff[2 * j] = keep == 7 ? -1.0 / 6.0 : 1.0 / 6.0;
    coeff[2 * j + 1] = 0.0;
  }
  out->n_branch = 8;
  out->coeff = coeff;
  out->off = off;
  out->gates = gates;
  return CHSIM_OK;
}

chsim_status chsim_set_tuning(chsim_ctx* ctx, uint32_t inst, uint32_t knob, int32_t value) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  Instance& I = ctx->inst[inst];
  switch (knob) {
    case CHSIM_TUNE_EVOLVE_LANES: {
      I.autotune = false;
      if (value == 0) {
        I.shape = EvolveShape();
        return CHSIM_OK;
      }
      if (value == -1) {
        I.autotune = true;
        return CHSIM_OK;
      }
      const EvolveShape s = shape_of_value(I.n, value);
      if (value < 0 || !evolve_shape_supported(s, I.n))
        return fail(CHSIM_EUNSUPPORTED, "no evolution kernel for lanes value %d and n = %u", value, I.n);
      I.shape = s;
      return CHSIM_OK;
    }
    case CHSIM_TUNE_PREFIX_SHARE: {
      if (value < 0 || value > 2) return fail(CHSIM_EINVAL, "prefix-share mode %d not in 0..2", value);
      I.prefix_mode = value;
      I.plan_valid = false;
      return CHSIM_OK;
    }
    case CHSIM_TUNE_AMP_STRINGS: {
      if (value == -1) {
        ctx->amp_tune = true;
        return CHSIM_OK;
      }
      if (value != 0 && value != 256 && value != 512)
        return fail(CHSIM_EUNSUPPORTED, "no amplitude kernel for %d bitstrings per work item", value);
      ctx->amp_tune = false;
      ctx->amp_xpl = value == 256 ? 1u : 2u;
      return CHSIM_OK;
    }
    default:
      return fail(CHSIM_EINVAL, "unknown tuning knob %u", knob);
  }
}

chsim_status chsim_get_tuning(chsim_ctx* ctx, uint32_t inst, uint32_t knob, int32_t* value,
                              float* timings_ms) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  Instance& I = ctx->inst[inst];
  if (knob == CHSIM_TUNE_PREFIX_SHARE) {
    if (value) *value = I.prefix_mode;
    if (timings_ms) {
      timings_ms[0] = I.plan_valid ? (float)I.plan_cut.size() : 0.f;
      timings_ms[1] = I.plan_valid ? (float)I.plan_frac : 1.f;
    }
    return CHSIM_OK;
  }
  if (knob == CHSIM_TUNE_AMP_STRINGS) {
    if (value) *value = (int32_t)(256u * ctx->amp_xpl);
    if (timings_ms) {
      timings_ms[0] = ctx->amp_tune_ms[0];
      timings_ms[1] = ctx->amp_tune_ms[1];
    }
    return CHSIM_OK;
  }
  if (knob != CHSIM_TUNE_EVOLVE_LANES) return fail(CHSIM_EINVAL, "unknown tuning knob %u", knob);
  EvolveShape sh = I.shape.lanes ? I.shape : evolve_default_shape(I.n);
  if (value) *value = value_of_shape(sh);
  if (timings_ms)
    for (int i = 0; i < kTuneShapes; ++i) timings_ms[i] = I.tuned_ms[i];
  return CHSIM_OK;
}

chsim_status chsim_evolution_stats(chsim_ctx* ctx, uint32_t inst, uint64_t apps[5], uint32_t* levels,
                                   uint64_t* distinct, uint32_t max_levels) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  if (!apps) return fail(CHSIM_EINVAL, "null output");
  Instance& I = ctx->inst[inst];
  uint32_t K = 0;
  for (const auto& sp : I.last_spans) K = std::max<uint32_t>(K, (uint32_t)(sp.level + 1));
  std::vector<uint32_t> counts(K, 0);
  if (K) {
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(counts.data(), I.plan_count.p, K * sizeof(uint32_t), hipMemcpyDeviceToHost));
  }
  for (int k = 0; k < 5; ++k) apps[k] = 0;
  for (const auto& sp : I.last_spans) {
    const uint64_t items = sp.level >= 0 ? counts[sp.level] : sp.items;
    for (int k = 0; k < 5; ++k) apps[k] += items * sp.kinds[k];
  }
  if (levels) *levels = K;
  if (distinct)
    for (uint32_t k = 0; k < std::min(K, max_levels); ++k) distinct[k] = counts[k];
  return CHSIM_OK;
}

chsim_status chsim_sparsification_bound(chsim_ctx* ctx, uint32_t inst, const uint64_t* A_off,
                                        const uint8_t* A_diag, size_t L, double out[4], void* stream) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  if (!out) return fail(CHSIM_EINVAL, "null output");
  const Instance& I = ctx->inst[inst];
  if (I.mode != CHSIM_SPARSIFY) return fail(CHSIM_EINVAL, "the bound is for a sparsified instance");
  if (L < 2) return fail(CHSIM_EINVAL, "need at least two equatorial states");
  std::vector<double> ov(2 * L), eta(L);
  double mean = 0.0;
  st = chsim_inner_products(ctx, inst, A_off, A_diag, L, ov.data(), eta.data(), &mean, 0u, stream);
  if (st) return st;
  // Standard error of the mean of the L estimates eta_l (two-pass variance).
  double ss = 0.0;
  for (size_t l = 0; l < L; ++l) ss += (eta[l] - mean) * (eta[l] - mean);
  const double delta2 = I.l1 * I.l1 / (double)I.chi;  // chi = ||c||_1^2 / delta^2
  out[0] = mean;
  out[1] = std::sqrt(ss / (double)(L - 1) / (double)L);
  out[2] = delta2;
  out[3] = mean - 1.0 + delta2;
  return CHSIM_OK;
}

namespace {

chsim_status run_projection(chsim_ctx* ctx, uint32_t inst, const ProjGates& P, void* stream) {
  Instance& I = ctx->inst[inst];
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  chsim_status st = ensure_materialised(I, s);
  if (st) return st;
  I.drop_chains();
  HIP_TRY(hipMemsetAsync(ctx->err.p, 0, sizeof(uint32_t), s));
  HIP_TRY(launch_project(I.view(), P, ctx->err.p, s));
  I.amp_ready = false;
  return check_err_flag(ctx, s, "projection");
}

}  // namespace

chsim_status chsim_project_pauli(chsim_ctx* ctx, uint32_t inst, const uint8_t* a, const uint64_t* x,
                                 const uint64_t* z, uint32_t w, void* stream) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  if (w == 0) return CHSIM_OK;
  if (!a || !x || !z) return fail(CHSIM_EINVAL, "null input");
  if (w > 64) return fail(CHSIM_EINVAL, "at most 64 projectors per call");
  const Instance& I = ctx->inst[inst];
  const uint64_t hi = (I.n == 64) ? 0ull : ~((1ull << I.n) - 1ull);
  ProjGates P;
  std::memset(&P, 0, sizeof P);
  P.count = w;
  for (uint32_t j = 0; j < w; ++j) {
    if ((x[j] | z[j]) & hi) return fail(CHSIM_EINVAL, "projector %u: X or Z part has a qubit >= n %u", j, I.n);
    if (a[j] > 3) return fail(CHSIM_EINVAL, "projector %u: phase exponent %u not in Z_4", j, a[j]);
    if ((a[j] & 1u) != ((uint32_t)__builtin_popcountll(x[j] & z[j]) & 1u))
      return fail(CHSIM_EINVAL, "projector %u: i^a X(x) Z(z) is not Hermitian (a != x.z mod 2)", j);
    P.a[j] = a[j];
    P.x[j] = x[j];
    P.z[j] = z[j];
  }
  return run_projection(ctx, inst, P, stream);
}

chsim_status chsim_project_z(chsim_ctx* ctx, uint32_t inst, const uint32_t* qubits, const uint8_t* bits,
                             uint32_t w, void* stream) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  if (w == 0) return CHSIM_OK;
  if (!qubits || !bits) return fail(CHSIM_EINVAL, "null input");
  const Instance& I = ctx->inst[inst];
  if (w > 64) return fail(CHSIM_EINVAL, "at most 64 projectors per call");
  // (I + (-1)^b Z_q) / 2 is the Pauli projector with a = 2 b, x = 0, z = e_q.
  ProjGates P;
  std::memset(&P, 0, sizeof P);
  P.count = w;
  for (uint32_t j = 0; j < w; ++j) {
    if (qubits[j] >= I.n) return fail(CHSIM_EINVAL, "projector %u: qubit %u >= n %u", j, qubits[j], I.n);
    if (bits[j] > 1) return fail(CHSIM_EINVAL, "projector %u: bit must be 0 or 1", j);
    P.a[j] = (uint8_t)(2u * bits[j]);
    P.x[j] = 0ull;
    P.z[j] = 1ull << qubits[j];
  }
  return run_projection(ctx, inst, P, stream);
}

chsim_status chsim_terms_copy(chsim_ctx* ctx, uint32_t src_inst, uint32_t dst_inst, void* stream) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, src_inst);
  if (st) return st;
  st = check_ctx(ctx, dst_inst);
  if (st) return st;
  if (src_inst == dst_inst) return CHSIM_OK;
  Instance& A = ctx->inst[src_inst];
  Instance& D = ctx->inst[dst_inst];
  if (A.n != D.n || A.chi != D.chi) return fail(CHSIM_EINVAL, "instances differ in n or chi");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  st = ensure_materialised(A, s);
  if (st) return st;
  D.drop_chains();
  const TermsView a = A.view(), d = D.view();
  const size_t rows = (size_t)A.n * A.chi;
  HIP_TRY(hipMemcpyAsync(d.F, a.F, rows * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(d.G, a.G, rows * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(d.M, a.M, rows * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(d.gamma, a.gamma, rows, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(d.v, a.v, A.chi * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(d.s, a.s, A.chi * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(d.omega, a.omega, A.chi, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(d.b, a.b, A.chi * sizeof(double2), hipMemcpyDeviceToDevice, s));
  if (A.n_slot == D.n_slot && A.n_slot)
    HIP_TRY(hipMemcpyAsync(d.branch, a.branch, (size_t)A.n_slot * A.chi, hipMemcpyDeviceToDevice, s));
  D.at_zero = false;
  D.amp_ready = false;
  return CHSIM_OK;
}

chsim_status chsim_sample_marginal(chsim_ctx* ctx, uint32_t inst, uint32_t scratch_inst, const uint32_t* qubits,
                                   uint32_t w, const uint64_t* A_off, const uint8_t* A_diag, size_t L,
                                   const double* u, uint8_t* bits_out, double* prob_out, double* est_out,
                                   void* stream) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  st = check_ctx(ctx, scratch_inst);
  if (st) return st;
  if (scratch_inst == inst) return fail(CHSIM_EINVAL, "the scratch instance must differ from the sampled one");
  if (w == 0 || w > 64) return fail(CHSIM_EINVAL, "w must be in 1..64");
  if (!qubits || !u || !bits_out || !prob_out || !A_off || !A_diag || L == 0) return fail(CHSIM_EINVAL, "null input");
  const Instance& I = ctx->inst[inst];
  const Instance& S = ctx->inst[scratch_inst];
  if (I.n != S.n || I.chi != S.chi) return fail(CHSIM_EINVAL, "scratch instance differs in n or chi");
  for (uint32_t j = 0; j < w; ++j) {
    if (qubits[j] >= I.n) return fail(CHSIM_EINVAL, "qubit %u >= n", qubits[j]);
    if (!(u[j] >= 0.0 && u[j] < 1.0)) return fail(CHSIM_EINVAL, "uniform %u not in [0, 1)", j);
  }
  std::vector<double> ov(2 * L);
  uint8_t bits[64];
  for (uint32_t j = 0; j < w; ++j) {
    // P(x_j = b | x_0..x_{j-1}) from the norm estimates of the terms projected
    // onto (x_0..x_{j-1}, b), b = 0, 1.
    double e[2];
    for (uint8_t b = 0; b < 2; ++b) {
      bits[j] = b;
      st = chsim_terms_copy(ctx, inst, scratch_inst, stream);
      if (st) return st;
      st = chsim_project_z(ctx, scratch_inst, qubits, bits, j + 1, stream);
      if (st) return st;
      st = chsim_inner_products(ctx, scratch_inst, A_off, A_diag, L, ov.data(), nullptr, &e[b], 0u, stream);
      if (st) return st;
    }
    const double tot = e[0] + e[1];
    const double p0 = tot > 0.0 ? e[0] / tot : 0.5;
    bits[j] = u[j] < p0 ? 0 : 1;
    bits_out[j] = bits[j];
    prob_out[j] = bits[j] ? 1.0 - p0 : p0;
    if (est_out) {
      est_out[2 * j] = e[0];
      est_out[2 * j + 1] = e[1];
    }
  }
  return CHSIM_OK;
}

chsim_status chsim_instance_info(chsim_ctx* ctx, uint32_t inst, uint32_t* n, uint64_t* chi, double* l1) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  const Instance& I = ctx->inst[inst];
  if (n) *n = I.n;
  if (chi) *chi = I.chi;
  if (l1) *l1 = I.l1;
  return CHSIM_OK;
}

chsim_status chsim_destroy(chsim_ctx* ctx) {
  if (!ctx) return CHSIM_OK;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  for (auto& I : ctx->inst) I.release();
  if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
  ctx->cap_stream = nullptr;
  ctx->gates.release();
  ctx->err.release();
  ctx->xbuf.release();
  ctx->partial.release();
  ctx->amp_insts.release();
  ctx->amp_items.release();
  ctx->amp_prefix.release();
  ctx->amp_counter.release();
  ctx->slotseq.release();
  ctx->pf_table.release();
  ctx->pf_ids.release();
  ctx->pf_slotof.release();
  ctx->pf_rep.release();
  ctx->pf_parent.release();
  for (int k = 0; k < 2; ++k) {
    ctx->pf_id[k].release();
    ctx->ck_F[k].release();
    ctx->ck_G[k].release();
    ctx->ck_M[k].release();
    ctx->ck_v[k].release();
    ctx->ck_s[k].release();
    ctx->ck_gamma[k].release();
    ctx->ck_omega[k].release();
  }
  ctx->out.release();
  ctx->aoff.release();
  ctx->inner_work.release();
  ctx->adiag.release();
  ctx->eta.release();
  ctx->eta_sum.release();
  ctx->vcheck.release();
  ctx->chrec_k.release();
  ctx->chrec_b.release();
  ctx->chtotal.release();
  delete ctx;
  return CHSIM_OK;
}


}  // extern "C"

struct chsim_mlp {
  chsim_ctx* ctx = nullptr;
  MLPDev d;
  DevBuf<double> loss;
  DevBuf<uint64_t> xin, tin;
  std::vector<void*> owned;
  ~chsim_mlp() {
    for (void* q : owned)
      if (q) hipFree(q);
    loss.release();
    xin.release();
    tin.release();
  }
};

namespace {

template <typename T>
hipError_t mlp_alloc(chsim_mlp* m, T** p, size_t count) {
  hipError_t e = hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
  if (e == hipSuccess) m->owned.push_back((void*)*p);
  return e;
}

}  // namespace

extern "C" {

chsim_status chsim_mlp_create(chsim_ctx* ctx, uint32_t n, uint32_t hidden, uint32_t max_batch,
                              const float* params, chsim_mlp** out) {
  g_err.clear();
  if (!out) return fail(CHSIM_EINVAL, "null output");
  *out = nullptr;
  if (!ctx) return fail(CHSIM_EINVAL, "null context");
  if (n < 1 || n > 64) return fail(CHSIM_EINVAL, "n = %u outside [1, 64]", n);
  if (hidden == 0 || hidden % 16 || hidden > 1024) return fail(CHSIM_EINVAL, "hidden = %u", hidden);
  if (max_batch == 0) return fail(CHSIM_EINVAL, "max_batch = 0");
  if (!params) return fail(CHSIM_EINVAL, "null parameters");
  HIP_TRY(hipSetDevice(ctx->device));
  chsim_mlp* m = new chsim_mlp();
  m->ctx = ctx;
  MLPDev& d = m->d;
  d.L.n = n;
  d.L.H = hidden;
  d.cap = max_batch;
  const uint64_t cnt = d.L.count();
  const size_t B = max_batch, H = hidden;
  d.part_cap = (uint64_t)1 << 19;
  bool ok = mlp_alloc(m, &d.part, d.part_cap) == hipSuccess && mlp_alloc(m, &d.p, cnt) == hipSuccess && mlp_alloc(m, &d.grad, cnt) == hipSuccess &&
            mlp_alloc(m, &d.adam_m, cnt) == hipSuccess && mlp_alloc(m, &d.adam_v, cnt) == hipSuccess &&
            mlp_alloc(m, &d.wb, d.L.wb_count()) == hipSuccess &&
            mlp_alloc(m, &d.a0, B * n) == hipSuccess && mlp_alloc(m, &d.a1, B * H) == hipSuccess &&
            mlp_alloc(m, &d.a2, B * H) == hipSuccess && mlp_alloc(m, &d.z1, B * H) == hipSuccess &&
            mlp_alloc(m, &d.z2, B * H) == hipSuccess && mlp_alloc(m, &d.logits, B * n) == hipSuccess &&
            mlp_alloc(m, &d.gf, B * n) == hipSuccess && mlp_alloc(m, &d.dz1, B * H) == hipSuccess &&
            mlp_alloc(m, &d.dz2, B * H) == hipSuccess && mlp_alloc(m, &d.gb, B * n) == hipSuccess &&
            mlp_alloc(m, &d.gz1, B * H) == hipSuccess && mlp_alloc(m, &d.gz2, B * H) == hipSuccess &&
            m->loss.ensure(1) == hipSuccess;
  if (!ok) {
    delete m;
    return fail(CHSIM_ENOMEM, "network buffers do not fit");
  }
  *out = m;
  chsim_status st = chsim_mlp_set_params(m, params);
  if (st != CHSIM_OK) {
    delete m;
    *out = nullptr;
  }
  return st;
}

chsim_status chsim_mlp_destroy(chsim_mlp* mlp) {
  if (!mlp) return CHSIM_OK;
  hipSetDevice(mlp->ctx->device);
  hipDeviceSynchronize();
  delete mlp;
  return CHSIM_OK;
}

chsim_status chsim_mlp_get_params(chsim_mlp* mlp, float* params) {
  g_err.clear();
  if (!mlp || !params) return fail(CHSIM_EINVAL, "null argument");
  HIP_TRY(hipSetDevice(mlp->ctx->device));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(params, mlp->d.p, mlp->d.L.count() * sizeof(float), hipMemcpyDeviceToHost));
  return CHSIM_OK;
}

chsim_status chsim_mlp_set_params(chsim_mlp* mlp, const float* params) {
  g_err.clear();
  if (!mlp || !params) return fail(CHSIM_EINVAL, "null argument");
  MLPDev& d = mlp->d;
  HIP_TRY(hipSetDevice(mlp->ctx->device));
  const size_t bytes = d.L.count() * sizeof(float);
  HIP_TRY(hipMemcpy(d.p, params, bytes, hipMemcpyHostToDevice));
  std::vector<float> zero(d.L.count(), 0.f);
  HIP_TRY(hipMemcpy(d.adam_m, zero.data(), bytes, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d.adam_v, zero.data(), bytes, hipMemcpyHostToDevice));
  d.step = 0;
  HIP_TRY(mlp_refresh(d, nullptr));
  HIP_TRY(hipDeviceSynchronize());
  return CHSIM_OK;
}

chsim_status chsim_mlp_forward(chsim_mlp* mlp, const uint64_t* x, uint32_t batch, float* logits,
                               uint32_t flags, void* stream) {
  g_err.clear();
  if (!mlp || !x || !logits) return fail(CHSIM_EINVAL, "null argument");
  MLPDev& d = mlp->d;
  if (batch == 0 || batch > d.cap) return fail(CHSIM_EINVAL, "batch %u outside [1, %u]", batch, d.cap);
  const bool dev = flags & CHSIM_DEVICE_PTRS;
  HIP_TRY(hipSetDevice(mlp->ctx->device));
  hipStream_t s = as_stream(stream);
  const uint64_t* xd;
  chsim_status st = stage_in(mlp->xin, x, batch, dev, s, &xd);
  if (st) return st;
  float* out = dev ? logits : d.logits;
  HIP_TRY(mlp_forward(d, xd, batch, out, s));
  if (!dev) {
    HIP_TRY(hipMemcpyAsync(logits, out, (size_t)batch * d.L.n * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return CHSIM_OK;
}

chsim_status chsim_mlp_loss_grad(chsim_mlp* mlp, const uint64_t* x, const uint64_t* target,
                                 uint32_t batch, double* loss, float* grads, uint32_t flags,
                                 void* stream) {
  g_err.clear();
  if (!mlp || !x || !target) return fail(CHSIM_EINVAL, "null argument");
  MLPDev& d = mlp->d;
  if (batch == 0 || batch > d.cap) return fail(CHSIM_EINVAL, "batch %u outside [1, %u]", batch, d.cap);
  if (flags & CHSIM_DEVICE_PTRS) return fail(CHSIM_EUNSUPPORTED, "host pointers only");
  HIP_TRY(hipSetDevice(mlp->ctx->device));
  hipStream_t s = as_stream(stream);
  const uint64_t *xd, *td;
  chsim_status st = stage_in(mlp->xin, x, batch, false, s, &xd);
  if (st) return st;
  st = stage_in(mlp->tin, target, batch, false, s, &td);
  if (st) return st;
  double zero = 0.0;
  HIP_TRY(hipMemcpyAsync(mlp->loss.p, &zero, sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(mlp_loss_grad(d, xd, td, batch, mlp->loss.p, s));
  double lsum = 0.0;
  HIP_TRY(hipMemcpyAsync(&lsum, mlp->loss.p, sizeof(double), hipMemcpyDeviceToHost, s));
  if (grads) HIP_TRY(hipMemcpyAsync(grads, d.grad, d.L.count() * sizeof(float), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (loss) *loss = lsum / ((double)batch * d.L.n);
  return CHSIM_OK;
}

chsim_status chsim_mlp_train(chsim_mlp* mlp, const uint64_t* x, const uint64_t* target,
                             uint64_t count, uint32_t batch, uint32_t epochs, float lr,
                             double* epoch_loss, uint32_t flags, void* stream) {
  g_err.clear();
  if (!mlp || !x || !target) return fail(CHSIM_EINVAL, "null argument");
  MLPDev& d = mlp->d;
  if (count == 0 || batch == 0 || batch > d.cap) return fail(CHSIM_EINVAL, "bad count or batch");
  const bool dev = flags & CHSIM_DEVICE_PTRS;
  HIP_TRY(hipSetDevice(mlp->ctx->device));
  hipStream_t s = as_stream(stream);
  const uint64_t *xd, *td;
  chsim_status st = stage_in(mlp->xin, x, count, dev, s, &xd);
  if (st) return st;
  st = stage_in(mlp->tin, target, count, dev, s, &td);
  if (st) return st;
  for (uint32_t e = 0; e < epochs; ++e) {
    double zero = 0.0;
    HIP_TRY(hipMemcpyAsync(mlp->loss.p, &zero, sizeof(double), hipMemcpyHostToDevice, s));
    for (uint64_t b0 = 0; b0 < count; b0 += batch) {
      const uint32_t B = (uint32_t)std::min<uint64_t>(batch, count - b0);
      HIP_TRY(mlp_loss_grad(d, xd + b0, td + b0, B, mlp->loss.p, s));
      HIP_TRY(mlp_adam(d, lr, s));
    }
    if (epoch_loss) {
      double lsum = 0.0;
      HIP_TRY(hipMemcpyAsync(&lsum, mlp->loss.p, sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      epoch_loss[e] = lsum / ((double)count * d.L.n);
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  return CHSIM_OK;
}

chsim_status chsim_metropolis_step_learned(chsim_ctx* ctx, uint32_t inst, chsim_mlp* mlp,
                                           uint32_t n_steps, const chsim_learned_args* args,
                                           uint64_t* x_trace, uint8_t* accepted,
                                           uint32_t* n_flips, double* amp, uint32_t flags,
                                           void* stream) {
  g_err.clear();
  chsim_status st = check_ctx(ctx, inst);
  if (st) return st;
  Instance& I = ctx->inst[inst];
  if (!mlp || !args) return fail(CHSIM_EINVAL, "null network or arguments");
  if (mlp->ctx != ctx) return fail(CHSIM_EINVAL, "network belongs to another context");
  if (I.n_chain == 0) return fail(CHSIM_EINVAL, "chains not initialised");
  if (mlp->d.L.n != I.n) return fail(CHSIM_EINVAL, "network n = %u, instance n = %u", mlp->d.L.n, I.n);
  if (I.n_chain > mlp->d.cap) return fail(CHSIM_EINVAL, "network batch %u < %u chains", mlp->d.cap, I.n_chain);
  if (!(args->eps >= 0.f && args->eps <= 1.f) || !(args->pi_min > 0.f) || !(args->pi_max < 1.f) ||
      !(args->pi_min <= args->pi_max))
    return fail(CHSIM_EINVAL, "eps must be in [0, 1] and 0 < pi_min <= pi_max < 1");
  if (!args->u_mix || !args->j || !args->u_bits || !args->u) return fail(CHSIM_EINVAL, "null random inputs");
  if (n_steps == 0) return CHSIM_OK;
  const bool dev = flags & CHSIM_DEVICE_PTRS;
  const size_t C = I.n_chain, cnt = C * n_steps;
  if (!dev)
    for (size_t i = 0; i < cnt; ++i)
      if (args->j[i] >= I.n) return fail(CHSIM_EINVAL, "j[%zu] >= n", i);
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  MetroView mv = metro_view(I);
  mv.n_steps = n_steps;
  LearnedView lv;
  lv.n = I.n;
  lv.n_chain = I.n_chain;
  lv.n_steps = n_steps;
  lv.eps = args->eps;
  lv.pi_min = args->pi_min;
  lv.pi_max = args->pi_max;
  const double *umd, *ubd, *ud;
  const uint32_t* jd;
  if ((st = stage_in(I.lumix, args->u_mix, cnt, dev, s, &umd))) return st;
  if ((st = stage_in(I.lj, args->j, cnt, dev, s, &jd))) return st;
  if ((st = stage_in(I.lubits, args->u_bits, cnt * I.n, dev, s, &ubd))) return st;
  if ((st = stage_in(I.mu, args->u, cnt, dev, s, &ud))) return st;
  lv.u_mix = umd;
  lv.j = jd;
  lv.u_bits = ubd;
  lv.u = ud;
  HIP_TRY(I.ly.ensure(C));
  HIP_TRY(I.lmask.ensure(C));
  HIP_TRY(I.logit_x.ensure(C * I.n));
  HIP_TRY(I.logit_y.ensure(C * I.n));
  lv.x = I.mx.p;
  lv.y = I.ly.p;
  lv.mask = I.lmask.p;
  lv.logit_x = I.logit_x.p;
  lv.logit_y = I.logit_y.p;
  lv.n_flips = nullptr;
  if (x_trace) {
    if (dev) mv.trace = x_trace;
    else {
      HIP_TRY(I.mtrace.ensure(cnt));
      mv.trace = I.mtrace.p;
    }
  }
  if (accepted) {
    if (dev) mv.accepted = accepted;
    else {
      HIP_TRY(I.macc.ensure(cnt));
      mv.accepted = I.macc.p;
    }
  }
  if (n_flips) {
    if (dev) lv.n_flips = n_flips;
    else {
      HIP_TRY(I.lflips.ensure(cnt));
      lv.n_flips = I.lflips.p;
    }
  }
  // The network's output at the current states.
  HIP_TRY(mlp_forward(mlp->d, I.mx.p, I.n_chain, I.logit_x.p, s));
  HIP_TRY(launch_learned_steps(I.view(), mv, lv, mlp->d, n_steps, s));
  if (!dev) {
    if (x_trace) HIP_TRY(hipMemcpyAsync(x_trace, mv.trace, cnt * 8, hipMemcpyDeviceToHost, s));
    if (accepted) HIP_TRY(hipMemcpyAsync(accepted, mv.accepted, cnt, hipMemcpyDeviceToHost, s));
    if (n_flips) HIP_TRY(hipMemcpyAsync(n_flips, lv.n_flips, cnt * 4, hipMemcpyDeviceToHost, s));
    if (amp) HIP_TRY(hipMemcpyAsync(amp, I.mamp.p, C * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  } else if (amp) {
    HIP_TRY(hipMemcpyAsync(amp, I.mamp.p, C * sizeof(double2), hipMemcpyDeviceToDevice, s));
  }
  return CHSIM_OK;
}

}  // extern "C"

