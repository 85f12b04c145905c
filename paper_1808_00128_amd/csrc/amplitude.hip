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
// Mapping: a workgroup owns a tile of 64 terms, staged in LDS as
// {F_p, M_p} pairs [p][lane]; lanes run over terms and the bitstring is
// uniform across the wave, so the loop over the set bits of x runs on the
// scalar unit and every lane reads its own term's row p from LDS.  Each wave
// takes a batch of XB bitstrings, parks the per-lane values in a padded LDS
// buffer and sums them transposed (lane = bitstring, sequential over terms)
// with per-lane two-sum compensation in FP32 (or plain FP64), then the tiles'
// partial sums are added in FP64 by a second kernel in a fixed order.
#include "device_common.hpp"
#include "internal.hpp"

namespace chsim {

namespace {

constexpr int XB = 8;              // bitstrings per wave batch
constexpr int kQ = 64 / XB;        // lanes that share one bitstring in the transposed sum
constexpr int kWaves = 4;          // waves per workgroup
constexpr int kRedStride = 65;     // padded row (in complex elements) of the batch buffer

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
__global__ __launch_bounds__(256) void k_amp(TermsView Tv, const uint64_t* __restrict__ xs,
                                             uint32_t n_x, uint32_t x_chunk,
                                             double2* __restrict__ partial) {
  extern __shared__ __align__(16) uint8_t smem[];
  const uint32_t n = Tv.n;
  uint4* fm = reinterpret_cast<uint4*>(smem);                        // [n][64]
  AmpConst* ac = reinterpret_cast<AmpConst*>(smem + (size_t)n * 64 * 16);  // [64]
  Cpx<T>* red = reinterpret_cast<Cpx<T>*>(ac + 64);                  // [waves][XB][65]

  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t wave = uniform32(tid >> 6);
  const uint64_t chi = Tv.chi;
  const uint64_t base = (uint64_t)blockIdx.x * kAmpTile;

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
      const uint64_t nmask = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
      c.s = s;
      c.nv = ~v & nmask;
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
  Cpx<T>* myred = red + (size_t)wave * XB * kRedStride;

  const uint64_t xmask = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
  const uint32_t xbeg = blockIdx.y * x_chunk;
  const uint32_t xend = min(n_x, xbeg + x_chunk);
  for (uint32_t xb = xbeg + wave * XB; xb < xend; xb += kWaves * XB) {
    const uint32_t cnt = min((uint32_t)XB, xend - xb);
    for (uint32_t i = 0; i < cnt; ++i) {
      const uint64_t x = uniform64(xs[xb + i]) & xmask;  // bits >= n never index a row
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
    for (int m = 1; m < kQ; m <<= 1) acc.merge_xor(m);
    if (q == 0u && xi < cnt) partial[(uint64_t)blockIdx.x * n_x + xb + xi] = acc.value();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// out[i] = sum over tiles of partial[tile][i], FP64, fixed order.
__global__ __launch_bounds__(256) void k_reduce_tiles(const double2* __restrict__ partial,
                                                      uint32_t n_tiles, uint32_t n_x,
                                                      double2* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_x) return;
  double r = 0.0, im = 0.0;
  for (uint32_t t = 0; t < n_tiles; ++t) {
    const double2 v = partial[(uint64_t)t * n_x + i];
    r += v.x;
    im += v.y;
  }
  out[i] = make_double2(r, im);
}

template <typename T>
size_t amp_smem(uint32_t n) {
  return (size_t)n * 64 * 16 + 64 * sizeof(AmpConst) + (size_t)kWaves * XB * kRedStride * sizeof(Cpx<T>);
}

}  // namespace

size_t amp_partial_elems(const TermsView& T, uint32_t n_x) {
  const uint64_t tiles = (T.chi + kAmpTile - 1) / kAmpTile;
  return (size_t)tiles * n_x;
}

hipError_t launch_amplitudes(const TermsView& T, const uint64_t* x, uint32_t n_x, bool fp32c,
                             double2* partial, double2* out, hipStream_t st) {
  const uint32_t tiles = (uint32_t)((T.chi + kAmpTile - 1) / kAmpTile);
  // Split the bitstrings so the grid has several workgroups per CU.
  uint32_t chunks = 1;
  while ((uint64_t)tiles * chunks < 4096 && (n_x + chunks * 2 - 1) / (chunks * 2) >= kWaves * XB) chunks *= 2;
  const uint32_t x_chunk = (n_x + chunks - 1) / chunks;
  const dim3 grid(tiles, chunks);
  if (fp32c) {
    const size_t sm = amp_smem<float>(T.n);
    if (sm > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void*)k_amp<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_amp<float>, grid, dim3(256), sm, st, T, x, n_x, x_chunk, partial);
  } else {
    const size_t sm = amp_smem<double>(T.n);
    if (sm > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void*)k_amp<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_amp<double>, grid, dim3(256), sm, st, T, x, n_x, x_chunk, partial);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_tiles, dim3((n_x + 255) / 256), dim3(256), 0, st, partial, tiles, n_x,
                     out);
  return hipGetLastError();
}

}  // namespace chsim
