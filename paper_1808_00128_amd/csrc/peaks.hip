// Microbenchmarks of the roofline peaks on the device the path runs on: the
// int32 VALU issue rate, the HBM copy bandwidth and the LDS read bandwidth.
// They measure the machine, not the method, and give the denominators of the
// roofline fractions next to the chip's published figures.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "chsim.h"

namespace {

constexpr uint32_t kValuIters = 2048;

// 8 independent chains of v_xor_b32 / v_add_u32 per lane (16 VALU
// instructions per iteration, each operating on 64 lanes).
__global__ __launch_bounds__(256) void k_peak_valu(uint32_t* __restrict__ sink, uint32_t iters) {
  uint32_t a0 = threadIdx.x, a1 = a0 + 1u, a2 = a0 + 2u, a3 = a0 + 3u;
  uint32_t a4 = a0 + 4u, a5 = a0 + 5u, a6 = a0 + 6u, a7 = a0 + 7u;
  const uint32_t k = blockIdx.x | 1u;
  for (uint32_t it = 0; it < iters; ++it) {
    asm volatile(
        "v_xor_b32 %0, %0, %8\n\t"
        "v_xor_b32 %1, %1, %8\n\t"
        "v_xor_b32 %2, %2, %8\n\t"
        "v_xor_b32 %3, %3, %8\n\t"
        "v_xor_b32 %4, %4, %8\n\t"
        "v_xor_b32 %5, %5, %8\n\t"
        "v_xor_b32 %6, %6, %8\n\t"
        "v_xor_b32 %7, %7, %8\n\t"
        "v_add_u32 %0, %0, %8\n\t"
        "v_add_u32 %1, %1, %8\n\t"
        "v_add_u32 %2, %2, %8\n\t"
        "v_add_u32 %3, %3, %8\n\t"
        "v_add_u32 %4, %4, %8\n\t"
        "v_add_u32 %5, %5, %8\n\t"
        "v_add_u32 %6, %6, %8\n\t"
        "v_add_u32 %7, %7, %8"
        : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
        : "v"(k));
  }
  const uint32_t r = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
  if (r == 0x9E3779B9u) sink[blockIdx.x] = r;  // keeps the chains live
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Copy in 16-byte elements, four per thread in flight (all loads issued
// before the stores), one contiguous 16 KiB chunk per workgroup and pass.
__global__ __launch_bounds__(256) void k_peak_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                   uint64_t count) {
  const uint64_t chunk = 4ull * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * chunk; base < count; base += (uint64_t)gridDim.x * chunk) {
    u32x4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t i = base + (uint64_t)k * blockDim.x + threadIdx.x;
      if (i < count) v[k] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t i = base + (uint64_t)k * blockDim.x + threadIdx.x;
      if (i < count) __builtin_nontemporal_store(v[k], dst + i);
    }
  }
}

constexpr uint32_t kLdsWords = 8192;  // 64 KiB per workgroup
constexpr uint32_t kLdsIters = 1024;

// 8-byte LDS reads: lane-consecutive words (conflict-free), 8 reads per
// iteration at immediate offsets from one address; a compiler memory barrier
// per iteration makes every iteration read again, with no address arithmetic
// between the reads.
__global__ __launch_bounds__(256) void k_peak_lds(uint64_t* __restrict__ sink, uint32_t iters) {
  __shared__ uint64_t buf[kLdsWords];
  for (uint32_t i = threadIdx.x; i < kLdsWords; i += 256u) buf[i] = (uint64_t)i * 0x9E3779B97F4A7C15ull;
  __syncthreads();
  uint64_t acc = 0;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (uint32_t r = 0; r < 8; ++r) acc ^= buf[threadIdx.x + r * 256u];
    asm volatile("" ::: "memory");  // the next iteration reads LDS again
  }
  if (acc == 0x12345ull) sink[blockIdx.x] = acc;
}

}  // namespace

extern "C" chsim_status chsim_measure_peaks(int device, double out[3]) {
  if (!out) return CHSIM_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CHSIM_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return CHSIM_EDEVICE;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return CHSIM_EDEVICE;
  const uint64_t copy_bytes = uint64_t(1) << 30;  // per buffer
  void *sink = nullptr, *src = nullptr, *dst = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  chsim_status st = CHSIM_OK;
  auto timed = [&](auto&& launch, int reps, float* best) -> bool {
    *best = 1e30f;
    for (int r = 0; r < reps + 1; ++r) {
      if (hipEventRecord(e0, nullptr) != hipSuccess) return false;
      launch();
      if (hipGetLastError() != hipSuccess) return false;
      if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return false;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return false;
      if (r > 0) *best = std::min(*best, ms);  // the first run warms up
    }
    return true;
  };
  do {
    if (hipMalloc(&sink, 1 << 20) != hipSuccess || hipMalloc(&src, copy_bytes) != hipSuccess ||
        hipMalloc(&dst, copy_bytes) != hipSuccess) {
      st = CHSIM_ENOMEM;
      break;
    }
    if (hipMemset(src, 1, copy_bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
      st = CHSIM_EDEVICE;
      break;
    }
    float ms = 0.f;
    // VALU: 32 workgroups of 4 waves per compute unit.
    const uint32_t vblocks = (uint32_t)cus * 32u;
    if (!timed([&] { hipLaunchKernelGGL(k_peak_valu, dim3(vblocks), dim3(256), 0, nullptr, (uint32_t*)sink, kValuIters); },
               3, &ms)) {
      st = CHSIM_EDEVICE;
      break;
    }
    out[0] = (double)vblocks * 256.0 * kValuIters * 16.0 / (ms * 1e-3);
    // HBM: copy 1 GiB (read + write).
    const uint64_t cnt = copy_bytes / sizeof(u32x4);
    if (!timed([&] {
          hipLaunchKernelGGL(k_peak_copy, dim3((uint32_t)cus * 8u), dim3(256), 0, nullptr, (const u32x4*)src,
                             (u32x4*)dst, cnt);
        },
               3, &ms)) {
      st = CHSIM_EDEVICE;
      break;
    }
    out[1] = 2.0 * (double)copy_bytes / (ms * 1e-3);
    // The runtime's own device-to-device copy; the faster of the two counts.
    if (!timed([&] { (void)hipMemcpyAsync(dst, src, copy_bytes, hipMemcpyDeviceToDevice, nullptr); }, 3, &ms)) {
      st = CHSIM_EDEVICE;
      break;
    }
    out[1] = std::max(out[1], 2.0 * (double)copy_bytes / (ms * 1e-3));
    // LDS: 4 workgroups per compute unit (64 KiB each).
    const uint32_t lblocks = (uint32_t)cus * 4u;
    if (!timed([&] { hipLaunchKernelGGL(k_peak_lds, dim3(lblocks), dim3(256), 0, nullptr, (uint64_t*)sink, kLdsIters); },
               3, &ms)) {
      st = CHSIM_EDEVICE;
      break;
    }
    out[2] = (double)lblocks * 256.0 * kLdsIters * 8.0 * 8.0 / (ms * 1e-3);
  } while (false);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (sink) (void)hipFree(sink);
  if (src) (void)hipFree(src);
  if (dst) (void)hipFree(dst);
  return st;
}
