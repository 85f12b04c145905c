// Learned Metropolis proposal: a small MLP n -> H -> H -> n on BF16 matrix
// cores, trained by BCE on flip masks, and the Metropolis-Hastings chain that
// uses it.
//
// The paper's sampler (Sec. "Heuristic Metropolis simulator") proposes single
// bit flips; here the proposal is the mixture
//   q(y|x) = eps [|m| = 1]/n + (1 - eps) prod_j pi_j(x)^{m_j} (1 - pi_j(x))^{1-m_j},
// m = x ^ y, pi_j = clip(sigmoid(f(x)_j), pi_min, pi_max), and a move is
// accepted iff U < P(y) q(x|y) / (P(x) q(y|x)) with the exact amplitude ratio
// of the sum over Cliffords, so the stationary law is unchanged.
//
// Matrix products: v_mfma_f32_16x16x32_bf16 (gfx950: BF16 operands, FP32
// accumulate, K = 32 per instruction), 32x32 output tile per 256-thread
// workgroup (2 x 2 waves, one 16x16 MFMA tile each), operands staged through
// LDS in BF16 with arbitrary source strides, so forward and backward products
// use the same kernel.
#include <algorithm>

#include "device_common.hpp"
#include "internal.hpp"
#include "mlp.hpp"

namespace chsim {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8s __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Eight BF16 values from two 8-byte halves (LDS rows are 8-byte aligned).
__device__ __forceinline__ bf16x8 join8(bf16x4 lo, bf16x4 hi) {
  const bf16x8s v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ bf16x8 lds8(const uint16_t* p) {
  return join8(*reinterpret_cast<const bf16x4*>(p), *reinterpret_cast<const bf16x4*>(p + 4));
}

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return 0x7FC0;  // NaN
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// C[M x N] = A[M x K] B[K x N], BF16 operands, FP32 accumulation.
// A(i, k) = A[i * sai + k * sak], B(k, j) = B[k * sbk + j * sbj].
// Epilogues:
//   EPI_STORE: Cf = acc.
//   EPI_BIAS_RELU: z = acc + bias[j]; Cf = z; Cb = bf16(max(z, 0)).
//   EPI_BIAS: Cf = acc + bias[j]  (no activation; logits).
//   EPI_MASK: v = acc * (mask[i][j] > 0); Cf = v; Cb = bf16(v).
//
// 32 x 32 output tile per 256-thread workgroup (2 x 2 waves, one 16 x 16
// MFMA tile each), K staged 64 at a time through LDS (four MFMAs per wave per
// stage) with the next stage's global loads issued before the MFMAs.  Each
// operand is read with the lanes running along whichever index has unit
// stride.  Products with few output tiles and a long K (the weight gradients,
// K = batch) split K over gridDim.z into FP32 partials that a second kernel
// sums in a fixed order before the epilogue, so results do not depend on
// scheduling.
// ---------------------------------------------------------------------------
enum { EPI_STORE = 0, EPI_BIAS_RELU = 1, EPI_BIAS = 2, EPI_MASK = 3 };

// Small batches (inference in the chain, up to kFusedMaxBatch rows) take one
// fused kernel for the whole network instead of features + three products.
constexpr uint32_t kFusedMaxBatch = 256;

constexpr int kGT = 32;       // output tile edge
constexpr int kGK = 64;       // K per LDS stage
constexpr int kGRow = kGK + 4;  // LDS row pitch (elements)

struct GemmArgs {
  const uint16_t* A;
  const uint16_t* B;
  int64_t sai, sak, sbk, sbj;
  int M, N, K;
  int epi;
  const float* bias;
  const float* mask;  // [M][ldc]
  float* Cf;          // may be null
  uint16_t* Cb;       // may be null
  int ldc;
  int kc;             // K extent of one split (multiple of kGK)
  float* part;        // [splits][M][N] partial sums when gridDim.z > 1
};

__device__ __forceinline__ void gemm_epilogue(const GemmArgs& g, int row, int col, float v) {
  const int64_t o = (int64_t)row * g.ldc + col;
  switch (g.epi) {
    case EPI_BIAS_RELU:
      v += g.bias[col];
      if (g.Cf) g.Cf[o] = v;
      if (g.Cb) g.Cb[o] = f2bf(v > 0.f ? v : 0.f);
      break;
    case EPI_BIAS:
      v += g.bias[col];
      if (g.Cf) g.Cf[o] = v;
      if (g.Cb) g.Cb[o] = f2bf(v);
      break;
    case EPI_MASK:
      v = g.mask[o] > 0.f ? v : 0.f;
      if (g.Cf) g.Cf[o] = v;
      if (g.Cb) g.Cb[o] = f2bf(v);
      break;
    default:
      if (g.Cf) g.Cf[o] = v;
      if (g.Cb) g.Cb[o] = f2bf(v);
      break;
  }
}

// Element q of this thread's share of a [32 rows][64 k] operand stage: with
// k_fast the 64 lanes of a wave cover one row's 64 k; otherwise two k's of
// all 32 rows.
__device__ __forceinline__ void stage_index(int q, bool k_fast, int& i, int& k) {
  const int e = (int)threadIdx.x + 256 * q;
  if (k_fast) {
    i = e >> 6;
    k = e & 63;
  } else {
    k = e >> 5;
    i = e & 31;
  }
}

__device__ __forceinline__ void stage_load(const uint16_t* __restrict__ P, int64_t s_row, int64_t s_k,
                                           int rows, int r0, int k0, int kend, bool k_fast,
                                           uint16_t (&v)[8]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    int i, k;
    stage_index(q, k_fast, i, k);
    const int gi = r0 + i, gk = k0 + k;
    v[q] = (gi < rows && gk < kend) ? P[(int64_t)gi * s_row + (int64_t)gk * s_k] : (uint16_t)0;
  }
}

__device__ __forceinline__ void stage_store(uint16_t (*S)[kGRow], bool k_fast, const uint16_t (&v)[8]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    int i, k;
    stage_index(q, k_fast, i, k);
    S[i][k] = v[q];
  }
}

__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[kGT][kGRow];  // [m][k]
  __shared__ __align__(16) uint16_t Bs[kGT][kGRow];  // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.x * kGT, n0 = blockIdx.y * kGT;
  const int kbeg = blockIdx.z * g.kc;
  const int kend = min(g.K, kbeg + g.kc);
  const bool a_kf = g.sak == 1, b_kf = g.sbk == 1;
  uint16_t va[8], vb[8];
  stage_load(g.A, g.sai, g.sak, g.M, m0, kbeg, kend, a_kf, va);
  stage_load(g.B, g.sbj, g.sbk, g.N, n0, kbeg, kend, b_kf, vb);
  // 16x16x32 operands: lane l holds A[l % 16][k] and B[k][l % 16] for the
  // eight k = 8 (l / 16) .. +7 of each 32-wide step (the same k for both, so
  // the contraction does not depend on their order inside the instruction);
  // the result C[4 (l / 16) + r][l % 16], r = 0..3.
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += kGK) {
    __syncthreads();
    stage_store(As, a_kf, va);
    stage_store(Bs, b_kf, vb);
    __syncthreads();
    if (k0 + kGK < kend) {
      stage_load(g.A, g.sai, g.sak, g.M, m0, k0 + kGK, kend, a_kf, va);
      stage_load(g.B, g.sbj, g.sbk, g.N, n0, k0 + kGK, kend, b_kf, vb);
    }
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 32) {
      const bf16x8 a = lds8(&As[wm * 16 + r16][kk + kq]);
      const bf16x8 b = lds8(&Bs[wn * 16 + r16][kk + kq]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
  }
  const int col = n0 + wn * 16 + (lane & 15);
  for (int r = 0; r < 4; ++r) {
    const int row = m0 + wm * 16 + (lane >> 4) * 4 + r;
    if (row >= g.M || col >= g.N) continue;
    if (gridDim.z == 1)
      gemm_epilogue(g, row, col, acc[r]);
    else
      g.part[((int64_t)blockIdx.z * g.M + row) * g.N + col] = acc[r];
  }
}

// Sum of the K-split partials in split order, then the epilogue.
__global__ __launch_bounds__(256) void k_gemm_splitk(GemmArgs g, int splits) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t mn = (int64_t)g.M * g.N;
  if (e >= mn) return;
  float v = 0.f;
  for (int z = 0; z < splits; ++z) v += g.part[z * mn + e];
  gemm_epilogue(g, (int)(e / g.N), (int)(e % g.N), v);
}

static hipError_t gemm(GemmArgs g, const MLPDev& d, hipStream_t st) {
  const int bm = (g.M + kGT - 1) / kGT, bn = (g.N + kGT - 1) / kGT;
  const int blocks = bm * bn;
  const int n_kt = (g.K + kGK - 1) / kGK;
  int splits = 1;
  if (blocks < 128 && n_kt > 4) {
    splits = std::min((256 + blocks - 1) / blocks, n_kt / 2);
    while (splits > 1 && (uint64_t)splits * g.M * g.N > d.part_cap) --splits;
  }
  const int kt_per = (n_kt + splits - 1) / splits;
  g.kc = kt_per * kGK;
  splits = (n_kt + kt_per - 1) / kt_per;
  g.part = d.part;
  hipLaunchKernelGGL(k_gemm_bf16, dim3(bm, bn, splits), dim3(256), 0, st, g);
  if (splits > 1) {
    const int64_t mn = (int64_t)g.M * g.N;
    hipLaunchKernelGGL(k_gemm_splitk, dim3((uint32_t)((mn + 255) / 256)), dim3(256), 0, st, g, splits);
  }
  return hipGetLastError();
}

// s_j = 1 - 2 x_j as BF16, [B][n].
__global__ __launch_bounds__(256) void k_features(const uint64_t* __restrict__ x, uint32_t B, uint32_t n,
                                                  uint16_t* __restrict__ a0) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * n) return;
  const uint32_t b = i / n, j = i % n;
  a0[i] = ((x[b] >> j) & 1ull) ? (uint16_t)0xBF80 /* -1 */ : (uint16_t)0x3F80 /* +1 */;
}

// g = (sigmoid(l) - t) / (B n); loss partial sums softplus(l) - t l.
__global__ __launch_bounds__(256) void k_bce_grad(const float* __restrict__ logits,
                                                  const uint64_t* __restrict__ t, uint32_t B,
                                                  uint32_t n, float* __restrict__ g,
                                                  uint16_t* __restrict__ gb,
                                                  double* __restrict__ loss_acc) {
  __shared__ double part[256];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  double lv = 0.0;
  if (i < B * n) {
    const uint32_t b = i / n, j = i % n;
    const float l = logits[i];
    const float tv = ((t[b] >> j) & 1ull) ? 1.f : 0.f;
    const float sg = 1.f / (1.f + expf(-l));
    const float gv = (sg - tv) / (float)(B * n);
    g[i] = gv;
    gb[i] = f2bf(gv);
    const double ld = (double)l;
    lv = (ld > 0 ? ld + log1p(exp(-ld)) : log1p(exp(ld))) - (double)tv * ld;
  }
  part[threadIdx.x] = lv;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss_acc, part[0]);
}

// db[j] = sum_b d[b][j] (FP32, fixed order) in two passes: split y of
// k_colsum_part sums rows [y R, (y + 1) R) with 4 row groups of 64 columns per
// workgroup; k_colsum_fin adds the splits in order.
__global__ __launch_bounds__(256) void k_colsum_part(const float* __restrict__ d, uint32_t B, uint32_t N,
                                                     uint32_t R, float* __restrict__ part) {
  __shared__ float red[4][64];
  const uint32_t c = threadIdx.x & 63u, grp = threadIdx.x >> 6;
  const uint32_t j = blockIdx.x * 64u + c;
  const uint32_t b0 = blockIdx.y * R, b1 = min(B, b0 + R);
  float s = 0.f;
  if (j < N)
    for (uint32_t b = b0 + grp; b < b1; b += 4u) s += d[(uint64_t)b * N + j];
  red[grp][c] = s;
  __syncthreads();
  if (grp == 0 && j < N) part[(uint64_t)blockIdx.y * N + j] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

__global__ __launch_bounds__(256) void k_colsum_fin(const float* __restrict__ part, uint32_t splits,
                                                    uint32_t N, float* __restrict__ db) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.f;
  for (uint32_t z = 0; z < splits; ++z) s += part[(uint64_t)z * N + j];
  db[j] = s;
}

static hipError_t colsum(const MLPDev& d, const float* src, uint32_t B, uint32_t N, float* db,
                         hipStream_t st) {
  uint32_t splits = std::min<uint32_t>(32u, (B + 63u) / 64u);
  while (splits > 1 && (uint64_t)splits * N > d.part_cap) --splits;
  const uint32_t R = (B + splits - 1) / splits;
  hipLaunchKernelGGL(k_colsum_part, dim3((N + 63) / 64, splits), dim3(256), 0, st, src, B, N, R, d.part);
  hipLaunchKernelGGL(k_colsum_fin, dim3((N + 255) / 256), dim3(256), 0, st, d.part, splits, N, db);
  return hipGetLastError();
}

// Adam on the packed FP32 parameters, then refresh the BF16 weight copies.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              uint64_t count, float lr, float c1, float c2,
                                              MLPLayout L, uint16_t* __restrict__ wb) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  const float pi = p[i] - lr * mh / (sqrtf(vh) + 1e-8f);
  p[i] = pi;
  const int64_t w = L.weight_index(i);
  if (w >= 0) wb[w] = f2bf(pi);
}

__global__ __launch_bounds__(256) void k_refresh_bf16(const float* __restrict__ p, uint64_t count,
                                                      MLPLayout L, uint16_t* __restrict__ wb) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t w = L.weight_index(i);
  if (w >= 0) wb[w] = f2bf(p[i]);
}

// ---------------------------------------------------------------------------
// Host-side drivers.
// ---------------------------------------------------------------------------
hipError_t mlp_refresh(MLPDev& d, hipStream_t st) {
  const uint64_t cnt = d.L.count();
  hipLaunchKernelGGL(k_refresh_bf16, dim3((uint32_t)((cnt + 255) / 256)), dim3(256), 0, st, d.p, cnt,
                     d.L, d.wb);
  return hipGetLastError();
}

// Forward for `B` inputs already expanded into d.a0.
static hipError_t forward_a0(MLPDev& d, uint32_t B, float* logits, hipStream_t st) {
  const MLPLayout& L = d.L;
  const int n = (int)L.n, H = (int)L.H;
  GemmArgs g{};
  // z1 = a0 W1^T + b1, a1 = bf16(relu(z1))
  g.A = d.a0; g.sai = n; g.sak = 1;
  g.B = d.wb + L.wb_W1(); g.sbk = 1; g.sbj = n;
  g.M = (int)B; g.N = H; g.K = n; g.epi = EPI_BIAS_RELU; g.bias = d.p + L.off_b1();
  g.Cf = d.z1; g.Cb = d.a1; g.ldc = H;
  hipError_t e = gemm(g, d, st);
  if (e != hipSuccess) return e;
  // z2 = a1 W2^T + b2, a2 = bf16(relu(z2))
  g.A = d.a1; g.sai = H; g.sak = 1;
  g.B = d.wb + L.wb_W2(); g.sbk = 1; g.sbj = H;
  g.N = H; g.K = H; g.bias = d.p + L.off_b2(); g.Cf = d.z2; g.Cb = d.a2; g.ldc = H;
  if ((e = gemm(g, d, st)) != hipSuccess) return e;
  // logits = a2 W3^T + b3
  g.A = d.a2; g.sai = H; g.sak = 1;
  g.B = d.wb + L.wb_W3(); g.sbk = 1; g.sbj = H;
  g.N = n; g.K = H; g.epi = EPI_BIAS; g.bias = d.p + L.off_b3(); g.Cf = logits; g.Cb = nullptr;
  g.ldc = n;
  return gemm(g, d, st);
}

static bool fused_ok(const MLPDev& d);
static hipError_t fused_forward(MLPDev& d, const uint64_t* x, uint32_t B, float* logits, hipStream_t st);

hipError_t mlp_forward(MLPDev& d, const uint64_t* x, uint32_t B, float* logits, hipStream_t st) {
  if (fused_ok(d) && B <= kFusedMaxBatch) return fused_forward(d, x, B, logits, st);
  const uint32_t cnt = B * d.L.n;
  hipLaunchKernelGGL(k_features, dim3((cnt + 255) / 256), dim3(256), 0, st, x, B, d.L.n, d.a0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return forward_a0(d, B, logits, st);
}

hipError_t mlp_loss_grad(MLPDev& d, const uint64_t* x, const uint64_t* t, uint32_t B,
                         double* loss_acc, hipStream_t st) {
  const MLPLayout& L = d.L;
  const int n = (int)L.n, H = (int)L.H;
  hipError_t e = mlp_forward(d, x, B, d.logits, st);
  if (e != hipSuccess) return e;
  const uint32_t cnt = B * L.n;
  hipLaunchKernelGGL(k_bce_grad, dim3((cnt + 255) / 256), dim3(256), 0, st, d.logits, t, B, L.n,
                     d.gf, d.gb, loss_acc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  float* G = d.grad;
  GemmArgs g{};
  // dW3[n][H] = gb^T a2
  g.A = d.gb; g.sai = 1; g.sak = n; g.B = d.a2; g.sbk = H; g.sbj = 1;
  g.M = n; g.N = H; g.K = (int)B; g.epi = EPI_STORE; g.Cf = G + L.off_W3(); g.Cb = nullptr; g.ldc = H;
  if ((e = gemm(g, d, st)) != hipSuccess) return e;
  if ((e = colsum(d, d.gf, B, (uint32_t)n, G + L.off_b3(), st)) != hipSuccess) return e;
  // dZ2 = (gb W3) * [z2 > 0]
  g.A = d.gb; g.sai = n; g.sak = 1; g.B = d.wb + L.wb_W3(); g.sbk = H; g.sbj = 1;
  g.M = (int)B; g.N = H; g.K = n; g.epi = EPI_MASK; g.mask = d.z2; g.Cf = d.dz2; g.Cb = d.gz2; g.ldc = H;
  if ((e = gemm(g, d, st)) != hipSuccess) return e;
  // dW2[H][H] = gz2^T a1
  g.A = d.gz2; g.sai = 1; g.sak = H; g.B = d.a1; g.sbk = H; g.sbj = 1;
  g.M = H; g.N = H; g.K = (int)B; g.epi = EPI_STORE; g.Cf = G + L.off_W2(); g.Cb = nullptr; g.ldc = H;
  if ((e = gemm(g, d, st)) != hipSuccess) return e;
  if ((e = colsum(d, d.dz2, B, (uint32_t)H, G + L.off_b2(), st)) != hipSuccess) return e;
  // dZ1 = (gz2 W2) * [z1 > 0]
  g.A = d.gz2; g.sai = H; g.sak = 1; g.B = d.wb + L.wb_W2(); g.sbk = H; g.sbj = 1;
  g.M = (int)B; g.N = H; g.K = H; g.epi = EPI_MASK; g.mask = d.z1; g.Cf = d.dz1; g.Cb = d.gz1; g.ldc = H;
  if ((e = gemm(g, d, st)) != hipSuccess) return e;
  // dW1[H][n] = gz1^T a0
  g.A = d.gz1; g.sai = 1; g.sak = H; g.B = d.a0; g.sbk = n; g.sbj = 1;
  g.M = H; g.N = n; g.K = (int)B; g.epi = EPI_STORE; g.Cf = G + L.off_W1(); g.Cb = nullptr; g.ldc = n;
  if ((e = gemm(g, d, st)) != hipSuccess) return e;
  return colsum(d, d.dz1, B, (uint32_t)H, G + L.off_b1(), st);
}

hipError_t mlp_adam(MLPDev& d, float lr, hipStream_t st) {
  d.step += 1;
  const float c1 = 1.f - powf(0.9f, (float)d.step);
  const float c2 = 1.f - powf(0.999f, (float)d.step);
  const uint64_t cnt = d.L.count();
  hipLaunchKernelGGL(k_adam, dim3((uint32_t)((cnt + 255) / 256)), dim3(256), 0, st, d.p, d.grad,
                     d.adam_m, d.adam_v, cnt, lr, c1, c2, d.L, d.wb);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Learned Metropolis chain kernels.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float clip_sigmoid(float l, float lo, float hi) {
  float p = 1.f / (1.f + expf(-l));
  return fminf(fmaxf(p, lo), hi);
}

// Term j of log prod_j pi_j^{m_j} (1 - pi_j)^{1 - m_j} for logit l.
__device__ __forceinline__ double log_q_bit(float l, bool flip, float lo, float hi) {
  const double p = (double)clip_sigmoid(l, lo, hi);
  return flip ? log(p) : log1p(-p);
}

// log q(y|x) of the mixture eps [|m| = 1] / n + (1 - eps) exp(lp), lp the
// product's log, in the log domain: log(e^A + e^B) = max + log1p(e^{min - max})
// with A = log(eps / n) (only for |m| = 1) and B = log1p(-eps) + lp.  A term
// that is zero (eps = 0, |m| != 1, eps = 1) is -inf and drops out, so exp(lp)
// never underflows to a 0 / 0 ratio.
__device__ __forceinline__ double log_q_mix(double lp, uint64_t m, uint32_t n, float eps) {
  const double e = (double)eps;
  const double ninf = -__builtin_huge_val();
  const double A = (__popcll(m) == 1 && e > 0.0) ? log(e / (double)n) : ninf;
  const double Bt = (e < 1.0) ? log1p(-e) + lp : ninf;
  const double hi = fmax(A, Bt), lo = fmin(A, Bt);
  if (hi == ninf) return ninf;
  return hi + log1p(exp(lo - hi));
}

// Flip mask of chain c at this step, drawn from pi(x); also stores the mask
// and the proposal y = x ^ m.
__device__ __forceinline__ uint64_t draw_mask(const LearnedView& Lv, uint32_t c, uint32_t step) {
  const uint32_t n = Lv.n;
  const uint64_t idx = (uint64_t)c * Lv.n_steps + step;
  uint64_t m = 0;
  if (Lv.u_mix[idx] < (double)Lv.eps) {
    m = 1ull << (Lv.j[idx] % n);
  } else {
    const float* lx = Lv.logit_x + (uint64_t)c * n;
    const double* ub = Lv.u_bits + idx * n;
    for (uint32_t j = 0; j < n; ++j)
      if (ub[j] < (double)clip_sigmoid(lx[j], Lv.pi_min, Lv.pi_max)) m |= 1ull << j;
  }
  const uint64_t y = Lv.x[c] ^ m;
  Lv.mask[c] = m;
  Lv.y[c] = y;
  return y;
}

// One thread per chain: draw the flip mask of this step from pi(x).
__global__ void k_learned_mask(LearnedView Lv, uint32_t step) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Lv.n_chain) return;
  draw_mask(Lv, c, step);
}

// ---------------------------------------------------------------------------
// The whole network for up to 16 rows per 1024-thread workgroup: features,
// then the three layers with the activations in LDS and the BF16 weights
// read from L2.  Each output 16 x 16 tile takes the same MFMAs over the same
// k blocks (to the next multiple of 64, zero-padded) as k_gemm_bf16, and the
// same epilogues, so the values equal the three-product path bit for bit.
// kDraw: the rows are chains; draw their masks first and evaluate the
// network at the proposals y (logits to logit_y).  Otherwise the rows are
// x[0..B) and the activations are also stored for the backward pass.
// ---------------------------------------------------------------------------
constexpr int kFR = 16;                 // rows per workgroup
constexpr int kFWaves = 16;             // waves per workgroup (one 16-column tile each)
constexpr int kFMaxH = 256;             // widest hidden layer of the fused path
constexpr int kFP0 = 64 + 4;            // LDS pitch of the features (elements)
constexpr int kFPH = kFMaxH + 4;        // LDS pitch of a hidden activation

static bool fused_ok(const MLPDev& d) { return d.L.H <= (uint32_t)kFMaxH && d.L.n <= 64; }

// One layer: out[r][j] = act(sum_k A[r][k] W[j][k] + bias[j]) for the
// workgroup's 16 rows; wave w takes the output tiles w, w + kFWaves, ...
__device__ __forceinline__ void fused_layer(const uint16_t* As, int pa, int K,
                                            const uint16_t* __restrict__ W, int N,
                                            const float* __restrict__ bias, int epi, uint16_t* Os,
                                            int po, float* zf, uint16_t* zb, float* out, int ldo,
                                            int rows) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  const int kb_n = ((K + kGK - 1) / kGK) * (kGK / 32);  // 32-wide k blocks
  const bool vec = (K % 4) == 0;                        // rows of W 8-byte aligned
  for (int ct = wave; ct * 16 < N; ct += kFWaves) {
    const int col = ct * 16 + r16;
    bf16x8 b[kFMaxH / 32];
#pragma unroll
    for (int kb = 0; kb < kFMaxH / 32; ++kb) {
      bf16x4 v[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        const int k = kb * 32 + kq + 4 * hf;
        if (kb < kb_n && col < N && k < K) {
          const uint16_t* w = W + (int64_t)col * K + k;
          if (vec) {
            v[hf] = *reinterpret_cast<const bf16x4*>(w);
          } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) v[hf][i] = (k + i < K) ? (short)w[i] : (short)0;
          }
        }
      }
      b[kb] = join8(v[0], v[1]);
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < kFMaxH / 32; ++kb) {
      if (kb < kb_n) {  // kb_n is wave-uniform
        const bf16x8 a = lds8(&As[r16 * pa + kb * 32 + kq]);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[kb], acc, 0, 0, 0);
      }
    }
    if (col >= N) continue;
    const float bj = bias[col];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = (lane >> 4) * 4 + r;
      const float v = acc[r] + bj;
      if (epi == EPI_BIAS_RELU) {
        const uint16_t a = f2bf(v > 0.f ? v : 0.f);
        Os[row * po + col] = a;
        if (row < rows && zf) zf[(int64_t)row * ldo + col] = v;
        if (row < rows && zb) zb[(int64_t)row * ldo + col] = a;
      } else if (row < rows) {
        out[(int64_t)row * ldo + col] = v;
      }
    }
  }
}

template <bool kDraw>
__global__ __launch_bounds__(64 * kFWaves) void k_mlp_fused(MLPDev d, const uint64_t* __restrict__ x,
                                                   uint32_t B, float* __restrict__ logits,
                                                   LearnedView Lv, uint32_t step) {
  __shared__ __align__(16) uint16_t A0[kFR * kFP0];
  __shared__ __align__(16) uint16_t A1[kFR * kFPH];
  __shared__ __align__(16) uint16_t A2[kFR * kFPH];
  __shared__ uint64_t sx[kFR];
  const MLPLayout& L = d.L;
  const int n = (int)L.n, H = (int)L.H;
  const uint32_t r0 = blockIdx.x * kFR;
  const int rows = (int)min((uint32_t)kFR, B - r0);
  const uint32_t tid = threadIdx.x;
  if (kDraw) {
    // Wave r draws the mask of row r: lane j decides bit j (the comparisons
    // of draw_mask), one ballot assembles the mask.
    static_assert(kFWaves == kFR, "one wave per row");
    const uint32_t r = tid >> 6, lane = tid & 63u;
    uint64_t y = 0;
    if ((int)r < rows) {
      const uint32_t c = r0 + r;
      const uint64_t idx = (uint64_t)c * Lv.n_steps + step;
      uint64_t m;
      if (Lv.u_mix[idx] < (double)Lv.eps) {
        m = 1ull << (Lv.j[idx] % (uint32_t)n);
      } else {
        const bool bit = (int)lane < n &&
                         Lv.u_bits[idx * n + lane] <
                             (double)clip_sigmoid(Lv.logit_x[(uint64_t)c * n + lane], Lv.pi_min, Lv.pi_max);
        m = __ballot(bit);
      }
      y = Lv.x[c] ^ m;
      if (lane == 0) {
        Lv.mask[c] = m;
        Lv.y[c] = y;
      }
    }
    if (lane == 0) sx[r] = y;
  } else if (tid < (uint32_t)kFR) {
    sx[tid] = (int)tid < rows ? x[r0 + tid] : 0ull;
  }
  // Zero the hidden activations' padding columns (read as zero k blocks).
  for (uint32_t e = tid; e < (uint32_t)(kFR * kFPH); e += 64u * kFWaves) {
    A1[e] = 0;
    A2[e] = 0;
  }
  __syncthreads();
  for (uint32_t e = tid; e < (uint32_t)(kFR * 64); e += 64u * kFWaves) {
    const int r = (int)(e / 64), k = (int)(e % 64);
    uint16_t f = 0;
    if (k < n && r < rows) f = ((sx[r] >> k) & 1ull) ? (uint16_t)0xBF80 /* -1 */ : (uint16_t)0x3F80;
    A0[r * kFP0 + k] = f;
    if (!kDraw && k < n && r < rows) d.a0[(int64_t)(r0 + r) * n + k] = f;
  }
  __syncthreads();
  const int64_t o = (int64_t)r0 * H;
  fused_layer(A0, kFP0, n, d.wb + L.wb_W1(), H, d.p + L.off_b1(), EPI_BIAS_RELU, A1, kFPH,
              kDraw ? nullptr : d.z1 + o, kDraw ? nullptr : d.a1 + o, nullptr, H, rows);
  __syncthreads();
  fused_layer(A1, kFPH, H, d.wb + L.wb_W2(), H, d.p + L.off_b2(), EPI_BIAS_RELU, A2, kFPH,
              kDraw ? nullptr : d.z2 + o, kDraw ? nullptr : d.a2 + o, nullptr, H, rows);
  __syncthreads();
  float* out = kDraw ? Lv.logit_y + (int64_t)r0 * n : logits + (int64_t)r0 * n;
  fused_layer(A2, kFPH, H, d.wb + L.wb_W3(), n, d.p + L.off_b3(), EPI_BIAS, nullptr, 0, nullptr,
              nullptr, out, n, rows);
}

static hipError_t fused_forward(MLPDev& d, const uint64_t* x, uint32_t B, float* logits, hipStream_t st) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_fused<false>, dim3((B + kFR - 1) / kFR), dim3(64 * kFWaves), 0, st, d, x, B, logits,
                     LearnedView{}, 0u);
  return hipGetLastError();
}

// One thread per term, loop over chains: Q_y = Q_x prod_{j in m} P_j (the
// factors commute), <y|phi_alpha> from (u', mu'), tile sums per chain.
__global__ __launch_bounds__(256) void k_learned_accept(MetroView Mv, LearnedView Lv, uint32_t step) {
  __shared__ double part_r[256], part_i[256];
  const uint32_t ch = blockIdx.x;
  const uint32_t n = Lv.n;
  double ar = 0.0, ai = 0.0;
  for (uint32_t t = threadIdx.x; t < Mv.n_tiles; t += 256u) {
    const double2 v = Mv.partial[(uint64_t)ch * Mv.n_tiles + t];
    ar += v.x;
    ai += v.y;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    ar += __shfl_down(ar, o);
    ai += __shfl_down(ai, o);
  }
  if ((threadIdx.x & 63u) == 0) {
    part_r[threadIdx.x >> 6] = ar;
    part_i[threadIdx.x >> 6] = ai;
  }
  __syncthreads();
  __shared__ uint32_t acc_s;
  if (threadIdx.x < 64) {
    // Wave 0: lane j < n takes bit j of both proposal densities, then lane 0
    // decides.
    const uint32_t lane = threadIdx.x;
    const uint64_t m = Lv.mask[ch];
    double lrev = 0.0, lfwd = 0.0;
    if (m != 0ull && lane < n) {
      const bool f = (m >> lane) & 1ull;
      lrev = log_q_bit(Lv.logit_y[(uint64_t)ch * n + lane], f, Lv.pi_min, Lv.pi_max);
      lfwd = log_q_bit(Lv.logit_x[(uint64_t)ch * n + lane], f, Lv.pi_min, Lv.pi_max);
    }
    for (int o = 32; o >= 1; o >>= 1) {
      lrev += __shfl_xor(lrev, o);
      lfwd += __shfl_xor(lfwd, o);
    }
    if (lane == 0) {
      double yr = 0.0, yi = 0.0;
      for (int q = 0; q < 4; ++q) {
        yr += part_r[q];
        yi += part_i[q];
      }
      const uint64_t idx = (uint64_t)ch * Lv.n_steps + step;
      uint32_t acc = 1u;
      if (m != 0ull) {
        const double2 ax = Mv.amp[ch];
        const double px = ax.x * ax.x + ax.y * ax.y;
        const double py = yr * yr + yi * yi;
        const double lq_rev = log_q_mix(lrev, m, n, Lv.eps);
        const double lq_fwd = log_q_mix(lfwd, m, n, Lv.eps);
        const double r = (py / px) * exp(lq_rev - lq_fwd);
        acc = (px > 0.0) && (Lv.u[idx] < r);
        if (acc) {
          Mv.x[ch] = Lv.y[ch];
          Lv.x[ch] = Lv.y[ch];
          Mv.amp[ch] = make_double2(yr, yi);
        }
      }
      // The chain's cache is brought up to date with an accepted mask by the
      // next proposal step (or the final pass of the call).
      Mv.pmask[ch] = (acc && m != 0ull) ? m : 0ull;
      acc_s = acc && (m != 0ull);
      if (Mv.trace) Mv.trace[idx] = Mv.x[ch];
      if (Mv.accepted) Mv.accepted[idx] = (uint8_t)acc;
      if (Lv.n_flips) Lv.n_flips[idx] = (uint32_t)__popcll(m);
    }
  }
  __syncthreads();
  if (acc_s)
    for (uint32_t j = threadIdx.x; j < n; j += 256u)
      Lv.logit_x[(uint64_t)ch * n + j] = Lv.logit_y[(uint64_t)ch * n + j];
}

hipError_t launch_learned_steps(const TermsView& T, MetroView& Mv, LearnedView& Lv, MLPDev& d,
                                uint32_t n_steps, hipStream_t st) {
  hipError_t e;
  const bool fused = fused_ok(d);
  for (uint32_t t = 0; t < n_steps; ++t) {
    if (fused) {
      // Masks, proposals and the network at the proposals in one kernel.
      hipLaunchKernelGGL(k_mlp_fused<true>, dim3((Lv.n_chain + kFR - 1) / kFR), dim3(64 * kFWaves), 0, st, d,
                         nullptr, Lv.n_chain, nullptr, Lv, t);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
      hipLaunchKernelGGL(k_learned_mask, dim3((Lv.n_chain + 63) / 64), dim3(64), 0, st, Lv, t);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if ((e = mlp_forward(d, Lv.y, Lv.n_chain, Lv.logit_y, st)) != hipSuccess) return e;
    }
    const uint32_t mode = kProposeMasks | (t > 0 ? kProposeApplyPending : 0u);
    if ((e = launch_propose(T, Mv, Lv.mask, mode, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_learned_accept, dim3(Mv.n_chain), dim3(256), 0, st, Mv, Lv, t);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // The last step's accepted masks, so that the caches are up to date when the
  // call returns.
  return n_steps ? launch_propose(T, Mv, Lv.mask, kProposeApplyPending, st) : hipSuccess;
}

}  // namespace chsim
