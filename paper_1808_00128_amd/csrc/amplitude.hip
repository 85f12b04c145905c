// Amplitudes <x|psi> = sum_alpha b_alpha <x|phi_alpha> (step (b) of the hot path).
//
// Per (term, x), Eqs. (amplitude), (amplitude1): Q = prod_{p: x_p = 1}
// U_C^{-1} X_p U_C = i^mu Z(t) X(u) is built by right multiplication,
//   u ^= F_p;  mu += gamma_p + 2 par(u & M_p)       (u already updated),
// and <x|phi> = 0 if (u ^ s) & ~v != 0, else e^{i pi k/4} 2^{-|v|/2} with
// k = omega + 2 mu + 4 par(u & v & s) (mod 8).  The gamma part of mu only needs
// sum_{p in x} gamma_p = popc(x & Glo) + 2 popc(x & Ghi) (gamma bit-planes), so
// the per-bit loop is XOR, AND, POPCOUNT on 64-bit words.
//
// Mapping: work items (request, range of 64-term tiles, chunk of bitstrings)
// are pulled from a queue by a persistent grid, so one launch serves any mix
// of instances (qubit counts, term counts, bitstring counts).  For each tile
// of its range a workgroup stages {F_p, M_p} pairs [p][lane] in LDS; lanes
// run over terms and the bitstring is uniform across the wave, so the loop
// over the set bits of x runs on the scalar unit and every lane reads its own
// term's row p from LDS.  Each wave takes a batch of XB bitstrings, parks the
// per-lane values in a padded LDS buffer and sums them transposed (lane =
// bitstring, sequential over terms) with per-lane two-sum compensation in
// FP32 (or plain FP64); the tile sums are added into an FP64 accumulator per
// bitstring in LDS, written once per item, and the ranges' sums are added in
// FP64 by a second kernel in a fixed order.
#include <algorithm>
#include <vector>

#include "device_common.hpp"
#include "internal.hpp"

namespace chsim {

namespace {

constexpr int XB = 8;              // bitstrings per wave batch
constexpr int kQ = 64 / XB;        // lanes that share one bitstring in the transposed sum
constexpr int kWaves = 4;          // waves per workgroup
constexpr int kRedStride = 65;     // padded row (in complex elements) of the batch buffer
constexpr uint32_t kXChunk = 512;  // bitstrings per work item

struct AmpConst {
  uint64_t s, nv, vs, glo, ghi;
  uint32_t w, pad;
  double w0r, w0i, w1r, w1i;  // b 2^{-|v|/2} and the same times e^{i pi/4}
};

template <typename T>
struct Cpx {
  T r, i;
};

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

template <typename T>
struct Acc;

// FP32 with a running compensation term per component.
template <>
struct Acc<float> {
  float sr = 0.f, er = 0.f, si = 0.f, ei = 0.f;
  __device__ __forceinline__ void add(float r, float i) {
    float s, e;
    two_sum(sr, r, s, e);
    sr = s;
    er += e;
    two_sum(si, i, s, e);
    si = s;
    ei += e;
  }
  __device__ __forceinline__ void merge_xor(int mask) {
    const float osr = __shfl_xor(sr, mask), oer = __shfl_xor(er, mask);
    const float osi = __shfl_xor(si, mask), oei = __shfl_xor(ei, mask);
    float s, e;
    two_sum(sr, osr, s, e);
    sr = s;
    er = er + oer + e;
    two_sum(si, osi, s, e);
    si = s;
    ei = ei + oei + e;
  }
  __device__ __forceinline__ double2 value() const {
    return make_double2((double)sr + (double)er, (double)si + (double)ei);
  }
};

template <>
struct Acc<double> {
  double sr = 0.0, si = 0.0;
  __device__ __forceinline__ void add(double r, double i) {
    sr += r;
    si += i;
  }
  __device__ __forceinline__ void merge_xor(int mask) {
    sr += __shfl_xor(sr, mask);
    si += __shfl_xor(si, mask);
  }
  __device__ __forceinline__ double2 value() const { return make_double2(sr, si); }
};

template <typename T>
__global__ __launch_bounds__(256) void k_amp(const AmpInst* __restrict__ insts,
                                             const AmpItem* __restrict__ items, uint32_t n_items,
                                             uint32_t* __restrict__ counter, uint32_t n_max) {
  extern __shared__ __align__(16) uint8_t smem[];
  uint4* fm = reinterpret_cast<uint4*>(smem);                                  // [n_max][64]
  AmpConst* ac = reinterpret_cast<AmpConst*>(smem + (size_t)n_max * 64 * 16);  // [64]
  Cpx<T>* red = reinterpret_cast<Cpx<T>*>(ac + 64);                            // [waves][XB][65]
  double2* accx = reinterpret_cast<double2*>(red + (size_t)kWaves * XB * kRedStride);  // [kXChunk]
  __shared__ uint32_t s_item;

  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t wave = uniform32(tid >> 6);
  Cpx<T>* myred = red + (size_t)wave * XB * kRedStride;

  for (;;) {
    // Persistent workgroups pull (instance, tile range, bitstring chunk) items.
    if (tid == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t it = uniform32(s_item);
    __syncthreads();
    if (it >= n_items) break;
    const AmpItem item = items[it];
    const AmpInst& I = insts[item.inst];
    const TermsView& Tv = I.T;
    const uint32_t n = Tv.n;
    const uint64_t chi = Tv.chi;
    const uint64_t xmask = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    const uint32_t nx = item.x1 - item.x0;
    for (uint32_t i = tid; i < nx; i += 256u) accx[i] = make_double2(0.0, 0.0);
    const uint32_t t0 = item.range * I.tiles_per_range;
    const uint32_t tiles = (uint32_t)((chi + kAmpTile - 1) / kAmpTile);
    const uint32_t t1 = min(tiles, t0 + I.tiles_per_range);
    for (uint32_t tile = t0; tile < t1; ++tile) {
      const uint64_t base = (uint64_t)tile * kAmpTile;
      __syncthreads();  // previous tile's readers are done
      for (uint32_t i = tid; i < n * 64u; i += 256u) {
        const uint32_t p = i >> 6, l = i & 63u;
        const uint64_t a = base + l;
        uint64_t F = 0, M = 0;
        if (a < chi) {
          F = Tv.F[(uint64_t)p * chi + a];
          M = Tv.M[(uint64_t)p * chi + a];
        }
        fm[i] = make_uint4((uint32_t)F, (uint32_t)(F >> 32), (uint32_t)M, (uint32_t)(M >> 32));
      }
      if (tid < 64u) {
        const uint64_t a = base + tid;
        AmpConst c;
        c.s = c.nv = c.vs = c.glo = c.ghi = 0;
        c.w = 0;
        c.pad = 0;
        c.w0r = c.w0i = c.w1r = c.w1i = 0.0;
        if (a < chi) {
          const uint64_t v = Tv.v[a], s = Tv.s[a];
          c.s = s;
          c.nv = ~v & xmask;
          c.vs = v & s;
          uint64_t glo = 0, ghi = 0;
          for (uint32_t p = 0; p < n; ++p) {
            const uint32_t g = Tv.gamma[(uint64_t)p * chi + a];
            glo |= (uint64_t)(g & 1u) << p;
            ghi |= (uint64_t)((g >> 1) & 1u) << p;
          }
          c.glo = glo;
          c.ghi = ghi;
          c.w = Tv.omega[a];
          const double2 b = Tv.b[a];
          const int vc = __popcll(v);
          const double h = 0.70710678118654752440;
          const double mag = ldexp(1.0, -(vc >> 1)) * ((vc & 1) ? h : 1.0);
          c.w0r = b.x * mag;
          c.w0i = b.y * mag;
          c.w1r = (c.w0r - c.w0i) * h;
          c.w1i = (c.w0r + c.w0i) * h;
        }
        ac[tid] = c;
      }
      __syncthreads();

      const AmpConst c = ac[lane];
      const T w0r = (T)c.w0r, w0i = (T)c.w0i, w1r = (T)c.w1r, w1i = (T)c.w1i;
      const uint4* fml = fm + lane;
      for (uint32_t xb = wave * XB; xb < nx; xb += kWaves * XB) {
        const uint32_t cnt = min((uint32_t)XB, nx - xb);
        for (uint32_t i = 0; i < cnt; ++i) {
          const uint64_t x = uniform64(I.x[item.x0 + xb + i]) & xmask;  // bits >= n never index a row
          uint64_t u = 0;
          uint32_t cpar = 0;
          uint64_t xm = x;
          while (xm) {
            const uint32_t p = (uint32_t)__builtin_ctzll(xm);
            xm &= xm - 1ull;
            const uint4 r = fml[p * 64u];
            u ^= ((uint64_t)r.y << 32) | r.x;
            const uint64_t Mp = ((uint64_t)r.w << 32) | r.z;
            cpar += (uint32_t)__popcll(u & Mp);
          }
          const bool zero = ((u ^ c.s) & c.nv) != 0ull;
          const uint32_t k = (c.w + 2u * (uint32_t)__popcll(x & c.glo) +
                              4u * ((uint32_t)__popcll(x & c.ghi) + cpar + (uint32_t)__popcll(u & c.vs))) &
                             7u;
          T re = (k & 1u) ? w1r : w0r;
          T im = (k & 1u) ? w1i : w0i;
          const uint32_t m = k >> 1;  // multiply by i^m
          if (m & 1u) {
            const T t = re;
            re = im;
            im = t;
          }
          if ((m ^ (m >> 1)) & 1u) re = -re;
          if (m & 2u) im = -im;
          if (zero) {
            re = (T)0;
            im = (T)0;
          }
          myred[i * kRedStride + lane] = Cpx<T>{re, im};
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // Transposed sum: lane = (bitstring xi, part q); part q adds terms q, q + kQ, ...
        const uint32_t xi = lane / kQ, q = lane % kQ;
        Acc<T> acc;
        if (xi < cnt) {
#pragma unroll
          for (uint32_t k = 0; k < (uint32_t)XB; ++k) {
            const Cpx<T> e = myred[xi * kRedStride + q + kQ * k];
            acc.add(e.r, e.i);
          }
        }
#pragma unroll
        for (int mk = 1; mk < kQ; mk <<= 1) acc.merge_xor(mk);
        if (q == 0u && xi < cnt) {
          // This wave alone owns bitstrings xb .. xb + XB of the chunk.
          const double2 v = acc.value();
          double2 cur = accx[xb + xi];
          cur.x += v.x;
          cur.y += v.y;
          accx[xb + xi] = cur;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __syncthreads();
    for (uint32_t i = tid; i < nx; i += 256u)
      I.partial[(uint64_t)item.range * I.n_x + item.x0 + i] = accx[i];
  }
}

__global__ void k_reset_counter(uint32_t* counter) { *counter = 0u; }

// out[i] = sum over tile ranges of partial[range][i], FP64, fixed order; one
// thread per (request, bitstring) over all requests.
__global__ __launch_bounds__(256) void k_reduce_ranges(const AmpInst* __restrict__ insts,
                                                       const uint64_t* __restrict__ prefix,
                                                       uint32_t n_inst) {
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= prefix[n_inst]) return;
  uint32_t lo = 0, hi = n_inst;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (prefix[mid] <= g) lo = mid;
    else hi = mid;
  }
  const AmpInst& I = insts[lo];
  const uint64_t i = g - prefix[lo];
  double r = 0.0, im = 0.0;
  for (uint32_t t = 0; t < I.n_ranges; ++t) {
    const double2 v = I.partial[(uint64_t)t * I.n_x + i];
    r += v.x;
    im += v.y;
  }
  I.out[i] = make_double2(r, im);
}

template <typename T>
size_t amp_smem(uint32_t n) {
  return (size_t)n * 64 * 16 + 64 * sizeof(AmpConst) +
         (size_t)kWaves * XB * kRedStride * sizeof(Cpx<T>) + (size_t)kXChunk * sizeof(double2);
}

}  // namespace

void amp_plan(const std::vector<AmpRequestPlan>& reqs, uint32_t target_items,
              std::vector<AmpItem>& items, std::vector<uint32_t>& tiles_per_range,
              std::vector<uint32_t>& n_ranges) {
  uint64_t total_tiles = 0;
  for (const auto& r : reqs) total_tiles += (r.chi + kAmpTile - 1) / kAmpTile;
  items.clear();
  tiles_per_range.assign(reqs.size(), 1);
  n_ranges.assign(reqs.size(), 1);
  // Choose one range length for all requests so that the item count reaches
  // the target; at least 1 and at most 64 tiles per range.
  uint64_t chunks_total = 0;
  for (const auto& r : reqs) chunks_total += (r.n_x + kXChunk - 1) / kXChunk;
  uint64_t per = 1;
  if (total_tiles > 0 && chunks_total > 0) {
    const double avg_chunks = (double)chunks_total / (double)reqs.size();
    const double want_ranges = (double)target_items / avg_chunks;
    per = (uint64_t)((double)total_tiles / want_ranges);
    if (per < 1) per = 1;
    if (per > 64) per = 64;
  }
  for (uint32_t q = 0; q < reqs.size(); ++q) {
    const auto& r = reqs[q];
    const uint64_t tiles = (r.chi + kAmpTile - 1) / kAmpTile;
    tiles_per_range[q] = (uint32_t)per;
    n_ranges[q] = (uint32_t)((tiles + per - 1) / per);
    for (uint32_t rg = 0; rg < n_ranges[q]; ++rg)
      for (uint32_t x0 = 0; x0 < r.n_x; x0 += kXChunk)
        items.push_back(AmpItem{q, rg, x0, std::min<uint32_t>(r.n_x, x0 + kXChunk)});
  }
  // Longest first: cost ~ terms x bitstrings x (n / 2 set bits + constant).
  auto cost = [&](const AmpItem& it) {
    const auto& r = reqs[it.inst];
    const uint64_t tiles = (r.chi + kAmpTile - 1) / kAmpTile;
    const uint64_t t0 = (uint64_t)it.range * tiles_per_range[it.inst];
    const uint64_t nt = std::min<uint64_t>(tiles, t0 + tiles_per_range[it.inst]) - t0;
    return (double)nt * (double)(it.x1 - it.x0) * (3.0 * r.n + 20.0);
  };
  std::stable_sort(items.begin(), items.end(),
                   [&](const AmpItem& a, const AmpItem& b) { return cost(a) > cost(b); });
}

hipError_t launch_amp_items(const AmpInst* insts_d, const AmpItem* items_d, uint32_t n_items,
                            uint32_t* counter, uint32_t n_max, bool fp32c, const uint64_t* prefix_d,
                            uint32_t n_inst, uint64_t total_x, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int dev = 0, cus = 256;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t sm = fp32c ? amp_smem<float>(n_max) : amp_smem<double>(n_max);
  const void* fn = fp32c ? (const void*)k_amp<float> : (const void*)k_amp<double>;
  if (sm > 64 * 1024) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
  }
  int per_cu = 1;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, sm);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)n_items, (uint64_t)cus * per_cu);
  if (grid == 0) grid = 1;
  if (fp32c)
    hipLaunchKernelGGL(k_amp<float>, dim3(grid), dim3(256), sm, st, insts_d, items_d, n_items, counter, n_max);
  else
    hipLaunchKernelGGL(k_amp<double>, dim3(grid), dim3(256), sm, st, insts_d, items_d, n_items, counter, n_max);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint32_t blocks = (uint32_t)((total_x + 255) / 256);
  hipLaunchKernelGGL(k_reduce_ranges, dim3(blocks), dim3(256), 0, st, insts_d, prefix_d, n_inst);
  return hipGetLastError();
}

}  // namespace chsim
