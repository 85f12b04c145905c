// Shared-prefix evolution support: distinct branch prefixes at checkpoint
// levels.
//
// Every term is the same Clifford circuit with the slots' branch choices
// substituted (Sec. "Sum-over-Cliffords", Sparsification Lemma: i.i.d.
// choices per slot), so two terms that agree on the choices of the first j
// slots have bit-identical CH forms after the gates before slot j + 1: the
// update rules are deterministic functions of the state and the gate.  The
// evolution therefore runs once per distinct prefix up to a checkpoint
// level, and each term continues from its prefix's state.
//
// Level k's prefix id of term a is the rank of the pair (level k-1 id,
// branch bits of the slots between the two levels) among the distinct pairs:
// an open-addressing hash table of 64-bit keys assigns ids (in an arbitrary
// order; ids only address checkpoint states).
#include "device_common.hpp"
#include "internal.hpp"

namespace chsim {

namespace {

constexpr uint64_t kEmpty = ~0ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  // splitmix64 finaliser
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Before the first level: an empty table and zero id counters for every
// level (later levels find the table emptied by the previous level's
// k_prefix_assign).
__global__ __launch_bounds__(256) void k_prefix_clear(PrefixLevelArgs A) {
  const uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h <= A.table_mask) A.table[h] = kEmpty;
  if (h < A.first_counters) A.counter[h] = 0u;
}

__global__ __launch_bounds__(256) void k_prefix_insert(PrefixLevelArgs A) {
  const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = a < A.chi;
  const uint32_t lane = threadIdx.x & 63u;
  // The span's slots and widths, 64 at a time, one per lane, taken by lane
  // reads (a wait for them would also wait for the branch bytes in flight);
  // the branch bytes themselves eight slots at a time.
  uint32_t bits = 0, sh = 0;
  for (uint32_t c0 = 0; c0 < A.n_span; c0 += 64u) {
    const uint32_t cn = min(A.n_span - c0, 64u);
    const uint32_t my_slot = lane < cn ? (uint32_t)A.slot[c0 + lane] : 0u;
    const uint32_t my_w = lane < cn ? (uint32_t)A.width[c0 + lane] : 0u;
    for (uint32_t k0 = 0; k0 < cn; k0 += 8u) {
      uint32_t bv[8], wv[8];
#pragma unroll
      for (uint32_t k = 0; k < 8u; ++k) {
        const uint32_t i = k0 + k < cn ? k0 + k : cn - 1u;
        const uint32_t sl = (uint32_t)__builtin_amdgcn_readlane((int)my_slot, (int)i);
        wv[k] = k0 + k < cn ? (uint32_t)__builtin_amdgcn_readlane((int)my_w, (int)i) : 0u;
        // A one-branch slot (width 0) carries no choice.
        bv[k] = (live && wv[k] != 0u) ? (uint32_t)A.branch[(uint64_t)sl * A.chi + a] : 0u;
      }
#pragma unroll
      for (uint32_t k = 0; k < 8u; ++k) {
        bits |= bv[k] << sh;
        sh += wv[k];
      }
    }
  }
  if (!live) return;
  const uint64_t prev = A.prev_id ? (uint64_t)A.prev_id[a] : 0ull;
  const uint64_t key = (prev << 32) | bits;  // prev < 2^32 - 1, so key != kEmpty
  uint64_t h = mix64(key) & A.table_mask;
  // The table has at least twice as many entries as keys: a free or
  // matching entry is always reached within table_mask + 1 probes.
  for (uint64_t probe = 0; probe <= A.table_mask; ++probe) {
    // Many terms share a key: look before the atomic.
    const uint64_t seen = __atomic_load_n(&A.table[h], __ATOMIC_RELAXED);
    if (seen == key) break;
    if (seen == kEmpty) {
      const uint64_t old = atomicCAS((unsigned long long*)&A.table[h], (unsigned long long)kEmpty,
                                     (unsigned long long)key);
      if (old == kEmpty || old == key) break;
    }
    h = (h + 1) & A.table_mask;
  }
  A.slot_of[a] = (uint32_t)h;
}

// One atomic per workgroup: the occupied entries of a workgroup take
// consecutive ids, in wave order and lane order within a wave.  Each entry
// is emptied once read, which leaves the table clear for the next level.
constexpr uint32_t kAssignThreads = 1024;

__global__ __launch_bounds__(kAssignThreads) void k_prefix_assign(PrefixLevelArgs A) {
  __shared__ uint32_t wave_cnt[kAssignThreads / 64];
  __shared__ uint32_t block_base;
  const uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool occ = h <= A.table_mask && A.table[h] != kEmpty;
  if (occ) A.table[h] = kEmpty;
  const uint64_t m = ballot64(occ);
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  if (lane == 0) wave_cnt[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (uint32_t k = 0; k < kAssignThreads / 64; ++k) {
      const uint32_t c = wave_cnt[k];
      wave_cnt[k] = run;
      run += c;
    }
    block_base = run ? atomicAdd(A.counter, run) : 0u;
  }
  __syncthreads();
  if (occ) A.ids[h] = block_base + wave_cnt[wave] + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

// Term a's id, the representative term of each id (any term with that
// prefix: they all carry the same choices on the slots seen so far) and the
// id's parent at the previous level.
__global__ __launch_bounds__(256) void k_prefix_map(PrefixLevelArgs A) {
  const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= A.chi) return;
  const uint32_t id = A.ids[A.slot_of[a]];
  A.id_out[a] = id;
  A.rep[id] = (uint32_t)a;
  A.parent[id] = A.prev_id ? A.prev_id[a] : 0u;
}

}  // namespace

hipError_t launch_prefix_level(const PrefixLevelArgs& A, hipStream_t st) {
  const uint64_t ts = A.table_mask + 1ull;
  const uint32_t tb = (uint32_t)((ts + 255) / 256), cb = (uint32_t)((A.chi + 255) / 256);
  if (A.first_counters)
    hipLaunchKernelGGL(k_prefix_clear, dim3(tb), dim3(256), 0, st, A);
  hipLaunchKernelGGL(k_prefix_insert, dim3(cb), dim3(256), 0, st, A);
  hipLaunchKernelGGL(k_prefix_assign, dim3((uint32_t)((ts + kAssignThreads - 1) / kAssignThreads)),
                     dim3(kAssignThreads), 0, st, A);
  hipLaunchKernelGGL(k_prefix_map, dim3(cb), dim3(256), 0, st, A);
  return hipGetLastError();
}

}  // namespace chsim
