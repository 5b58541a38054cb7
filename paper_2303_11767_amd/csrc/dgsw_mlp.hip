// Learned right-hand-side correction: a 108 -> 256 -> 256 -> 12 GELU network
// in BF16 with FP32 accumulation on the gfx950 matrix cores (v_mfma 16x16x32
// bf16), its backward pass and Adam, the 3x3-stencil features of an r = 1
// state, and the learned stage (plain r = 1 right-hand side + correction, with
// a per-element trust bound and a global mass correction).
//
// MFMA 16x16x32 bf16 operand layout (lane l of 64): A[row = l%16][k = 8(l/16)+j],
// B[k = 8(l/16)+j][col = l%16], j = 0..7; result C[row = 4(l/16)+i][col = l%16],
// i = 0..3.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "dgsw_ctx.hpp"
#include "dgsw_device.hpp"
#include "dgsw_mlp.hpp"

namespace dgsw {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// GELU(z) = z Phi(z) = (z/2)(1 + erf(z / sqrt 2)) with erf from the rational
// approximation of Abramowitz & Stegun, formula 7.1.26 (Hastings): for x >= 0,
// erf(x) = 1 - P(t) exp(-x^2), t = 1 / (1 + p x),
// P(t) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))), absolute error <= 1.5e-7,
// far below the BF16 rounding the activations then take.  Since erf is odd,
// z erf(z / sqrt 2) = |z| (1 - P exp(-z^2 / 2)), so
//   GELU(z)  = max(z, 0) - |z| P / 2 exp(-z^2 / 2),
//   GELU'(z) = Phi(z) + z phi(z) = [z >= 0] - sgn(z) P / 2 e + z e / sqrt(2 pi),
// e = exp(-z^2 / 2): branch-free, one hardware reciprocal and one hardware
// base-2 exponential each.  The A&S coefficients enter halved (P / 2) and p
// is scaled by 1 / sqrt 2 (t from |z| directly).
namespace gelu_as {
constexpr float kP = 0.3275911f * 0.70710678118654752f;
constexpr float kA1 = 0.5f * 0.254829592f, kA2 = 0.5f * -0.284496736f, kA3 = 0.5f * 1.421413741f,
                kA4 = 0.5f * -1.453152027f, kA5 = 0.5f * 1.061405429f;
constexpr float kHalfLog2e = 0.72134752044448170f;   // log2(e) / 2: exp(-z^2/2) = 2^(-z^2 log2(e)/2)
__device__ __forceinline__ float half_poly(float az) {
  const float t = __builtin_amdgcn_rcpf(fmaf(kP, az, 1.0f));
  return t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, kA5, kA4), kA3), kA2), kA1);
}
__device__ __forceinline__ float gauss(float z) { return __builtin_amdgcn_exp2f(-(z * z) * kHalfLog2e); }
}  // namespace gelu_as

__device__ __forceinline__ float gelu_f(float z) {
  const float az = fabsf(z);
  return fmaf(-az * gelu_as::half_poly(az), gelu_as::gauss(z), fmaxf(z, 0.0f));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
  const float hp = gelu_as::half_poly(fabsf(z));
  return fmaf(gelu_as::gauss(z), fmaf(z, 0.39894228040143268f, -copysignf(hp, z)), z >= 0.0f ? 1.0f : 0.0f);
}

// ------------------------------------------------------------------ GEMM
// C[M][N] = A(m, k) B(k, n) over k < K (K % 32 == 0, N % 32 == 0), with
//   A_KC: A(m, k) = A[m * lda + k]   (else A[k * lda + m])
//   B_KC: B(k, n) = B[n * ldb + k]   (else B[k * ldb + n])
// A workgroup of 4 wavefronts computes a 64 x 64 tile, a wavefront 32 x 32
// (2 x 2 MFMA tiles); rows >= M are read clamped and not written.
template <bool A_KC, bool B_KC, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const __bf16 *__restrict__ A, const __bf16 *__restrict__ B,
                                              int M, int N, int K, int lda, int ldb,
                                              const float *__restrict__ bias,
                                              const float *__restrict__ Zin, float *__restrict__ Zout,
                                              void *__restrict__ C, int ldc) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int m0 = blockIdx.x * 64 + (wv >> 1) * 32;
  const int n0 = blockIdx.y * 64 + (wv & 1) * 32;
  if (n0 >= N) return;
  // split K: workgroup z sums k in [z kc, min(K, (z + 1) kc)) into the z-th
  // partial product C + z M ldc (gridDim.z == 1: the whole K into C)
  const int kc = gridDim.z == 1 ? K : ((K / 32 + gridDim.z - 1) / gridDim.z) * 32;
  const int kb = blockIdx.z * kc, ke = kb + kc < K ? kb + kc : K;
  if (gridDim.z > 1) C = static_cast<float *>(C) + (size_t)blockIdx.z * M * ldc;
  const int r = lane & 15, kq = (lane >> 4) * 8;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  int ma[2], nb[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int m = m0 + 16 * i + r;
    ma[i] = m < M ? m : M - 1;
    nb[i] = n0 + 16 * i + r;
  }
  for (int k0 = kb; k0 < ke; k0 += 32) {
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if constexpr (A_KC) {
        a[i] = *reinterpret_cast<const bf16x8 *>(A + (size_t)ma[i] * lda + k0 + kq);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[i][j] = A[(size_t)(k0 + kq + j) * lda + ma[i]];
      }
      if constexpr (B_KC) {
        b[i] = *reinterpret_cast<const bf16x8 *>(B + (size_t)nb[i] * ldb + k0 + kq);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) b[i][j] = B[(size_t)(k0 + kq + j) * ldb + nb[i]];
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
  // epilogue: lane holds rows 4(l/16)+e of each 16 x 16 tile, column l%16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + 16 * i + (lane >> 4) * 4 + e;
        const int n = n0 + 16 * j + r;
        if (m >= M) continue;
        float z = acc[i][j][e];
        const size_t o = (size_t)m * ldc + n;
        if constexpr (EPI == kEpiBiasGelu) {
          z += bias[n];
          if (Zout) Zout[o] = z;
          static_cast<__bf16 *>(C)[o] = (__bf16)gelu_f(z);
        } else if constexpr (EPI == kEpiBias) {
          static_cast<float *>(C)[o] = z + bias[n];
        } else if constexpr (EPI == kEpiGeluGrad) {
          z *= gelu_grad_f(Zin[o]);
          if (Zout) Zout[o] = z;
          static_cast<__bf16 *>(C)[o] = (__bf16)z;
        } else {
          static_cast<float *>(C)[o] = z;
        }
      }
}

template <bool A_KC, bool B_KC, int EPI>
static hipError_t gemm_t(const GemmArgs &g, hipStream_t s) {
  dim3 grid((g.M + 63) / 64, (g.N + 63) / 64);
  hipLaunchKernelGGL((k_gemm<A_KC, B_KC, EPI>), grid, dim3(256), 0, s, g.A, g.B, g.M, g.N, g.K, g.lda,
                     g.ldb, g.bias, g.Zin, g.Zout, g.C, g.ldc);
  return hipGetLastError();
}

// Sum of nsplit partial products part[z][n] over z in order (deterministic):
// four consecutive outputs per thread, the loads of several z in flight.
__global__ void k_sum_split(const float *__restrict__ part, int nsplit, int n4, float *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n4) return;
  const float4 *p = reinterpret_cast<const float4 *>(part) + i;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 8
  for (int z = 0; z < nsplit; ++z) {
    const float4 v = p[(size_t)z * n4];
    acc.x += v.x;
    acc.y += v.y;
    acc.z += v.z;
    acc.w += v.w;
  }
  reinterpret_cast<float4 *>(out)[i] = acc;
}
// the same one output per thread (n not a multiple of 4, or unaligned)
__global__ void k_sum_split1(const float *__restrict__ part, int nsplit, int n, float *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.f;
  for (int z = 0; z < nsplit; ++z) acc += part[(size_t)z * n + i];
  out[i] = acc;
}

hipError_t launch_sum_split(const float *part, int nsplit, int n, float *out, hipStream_t s) {
  if (n % 4 == 0 && reinterpret_cast<uintptr_t>(part) % 16 == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0)
    hipLaunchKernelGGL(k_sum_split, dim3((n / 4 + 255) / 256), dim3(256), 0, s, part, nsplit, n / 4, out);
  else
    hipLaunchKernelGGL(k_sum_split1, dim3((n + 255) / 256), dim3(256), 0, s, part, nsplit, n, out);
  return hipGetLastError();
}

int gemm_splits(int K) {
  const int s = (K + 255) / 256;
  return s < 1 ? 1 : (s > kMaxSplits ? kMaxSplits : s);
}

hipError_t launch_gemm_splitk(const GemmArgs &g, float *partial, hipStream_t s) {
  if (g.M <= 0) return hipSuccess;
  if (g.K % 32 || g.N % 32) return hipErrorInvalidValue;
  const int z = gemm_splits(g.K);
  GemmArgs p = g;
  p.C = partial;
  dim3 grid((g.M + 63) / 64, (g.N + 63) / 64, z);
  hipLaunchKernelGGL((k_gemm<false, false, kEpiPlain>), grid, dim3(256), 0, s, p.A, p.B, p.M, p.N, p.K, p.lda,
                     p.ldb, p.bias, p.Zin, p.Zout, p.C, p.ldc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_split(partial, z, g.M * g.ldc, static_cast<float *>(g.C), s);
}

hipError_t launch_gemm(bool a_kc, bool b_kc, int epi, const GemmArgs &g, hipStream_t s) {
  if (g.M <= 0) return hipSuccess;
  if (g.K % 32 || g.N % 32) return hipErrorInvalidValue;
#define DGSW_GEMM(AK, BK, E) \
  if (a_kc == AK && b_kc == BK && epi == E) return gemm_t<AK, BK, E>(g, s);
  DGSW_GEMM(true, true, kEpiBiasGelu) DGSW_GEMM(true, true, kEpiBias)
  DGSW_GEMM(true, true, kEpiGeluGrad) DGSW_GEMM(true, true, kEpiPlain)
  DGSW_GEMM(false, false, kEpiPlain)
#undef DGSW_GEMM
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ fused inference
// The whole network in one persistent kernel: one workgroup of 8 wavefronts
// per compute unit, looping over tiles of 64 rows.  Each wavefront loads its
// slice of the two hidden layers' weights into registers once (32 units of
// each, from the fragment order of k_prep_weights: one contiguous kilobyte
// per load) and keeps them for every tile, the output layer's weights are
// copied to LDS, so the weights cross the cache hierarchy once per workgroup
// instead of once per 64 rows.  Per tile the BF16 inputs
// (stencil features computed from an r = 1 state, or given FP32 rows) and
// both hidden layers stay in LDS; only the inputs and the FP32 outputs touch
// global memory.  Each product is computed transposed, out^T = W in^T: the
// weights are the MFMA A operand (row = unit, 8 consecutive k per lane) and
// the LDS rows the B operand, so every lane ends with 4 consecutive units of
// one row and writes them as one 8-byte LDS store.  Same rounding points as
// the unfused path: BF16 inputs, weights and hidden activations, FP32
// accumulation, bias and GELU in FP32.
constexpr int kRows = 64;                 // rows per tile
constexpr int kMlpGrid = 256;             // persistent workgroups: one per MI355X compute unit
template <typename T>
struct MlpCorrection {           // the learned stage's correction step (FROM_Q)
  const T *L1;
  const float *omean, *ostd;
  const double *mass_w;
  float kappa;
  float *C;
  double *partial;
  int64_t *fallback;
};
constexpr int kWaves = 8;                 // wavefronts per workgroup
constexpr int kLd = kHidden + 8;          // LDS row stride in BF16 (+16 B: no bank conflicts)
constexpr int kYs = kRows + 4;            // stride of the network outputs' unit columns in LDS
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// One hidden layer for the 64 rows of a tile: wavefront wv computes units
// [32 wv, 32 wv + 32) of out = gelu(in W^T + b), K inputs per row, from the
// weight fragments w[ks][nt] it holds.
template <int K>
__device__ __forceinline__ void fused_hidden(const bf16x8 (&w)[K / 32][2], const f32x4 (&bv)[2], const __bf16 *in,
                                             __bf16 *out, int wv, int lane) {
  constexpr int NT = 2, MT = kRows / 16, KS = K / 32;
  const int r = lane & 15, kq = (lane >> 4) * 8;
  f32x4 acc[NT][MT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = bv[nt];   // the bias, then the products
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    bf16x8 b[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      b[mt] = *reinterpret_cast<const bf16x8 *>(in + (16 * mt + r) * kLd + 32 * ks + kq);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        acc[nt][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[ks][nt], b[mt], acc[nt][mt], 0, 0, 0);
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int n0 = 32 * wv + 16 * nt + (lane >> 4) * 4;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      bf16x4 h;
#pragma unroll
      for (int i = 0; i < 4; ++i) h[i] = (__bf16)gelu_f(acc[nt][mt][i]);
      *reinterpret_cast<bf16x4 *>(out + (16 * mt + r) * kLd + n0) = h;
    }
  }
}

// This wavefront's weight fragments of a hidden layer (units 32 wv ..), from
// the fragment order Wf (one contiguous kilobyte per load), and the matching
// biases.
template <int K>
__device__ __forceinline__ void load_hidden(const __bf16 *__restrict__ Wf, const float *__restrict__ bias, int wv,
                                            int lane, bf16x8 (&w)[K / 32][2], f32x4 (&bv)[2]) {
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const __bf16 *blk = Wf + (size_t)(2 * wv + nt) * (K / 32) * 512 + lane * 8;
#pragma unroll
    for (int ks = 0; ks < K / 32; ++ks) w[ks][nt] = *reinterpret_cast<const bf16x8 *>(blk + 512 * ks);
    bv[nt] = *reinterpret_cast<const f32x4 *>(bias + 32 * wv + 16 * nt + (lane >> 4) * 4);
  }
}

// Per-element correction from the network output y[12] (standardised), as
// k_correction: c = mean_j + std_j y with c_(h,00) = 0; rejected (c = 0) if
// non-finite or, for a variable, max|c| > kappa max|L1|.  Returns whether it
// fell back and the element's h-mass of the correction.
template <int SY, int SL>
__device__ __forceinline__ bool correction_row(const float *y, const float *L1e, const float *om, const float *os,
                                               float kappa, float *c) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    c[k] = k == 0 ? 0.f : om[k * SL] + os[k * SL] * y[k * SY];
    ok = ok && isfinite(c[k]);
  }
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    float mc = 0.f, ml = 0.f;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      mc = fmaxf(mc, fabsf(c[v * 4 + m]));
      ml = fmaxf(ml, fabsf(L1e[(v * 4 + m) * SL]));
    }
    ok = ok && !(mc > kappa * ml);
  }
  if (!ok) {
#pragma unroll
    for (int k = 0; k < 12; ++k) c[k] = 0.f;
  }
  return !ok;
}

// FROM_Q: features of the r = 1 state q (as k_features), then the correction
// of every element (the learned stage): C[rows][12], the workgroup's h-mass
// of the corrections (summed over its tiles in tile order) in
// partial[blockIdx.x] and the fallback count; else the network on rows of
// X[rows][108], output Y[rows][32].  Tiles blockIdx.x, blockIdx.x + gridDim.x, ..
template <typename T, bool FROM_Q>
__global__ __launch_bounds__(64 * kWaves) void k_mlp_fused(const T *__restrict__ q, int n_lon, int n_lat,
                                                          const float *__restrict__ fmean,
                                                          const float *__restrict__ fistd,
                                                          const float *__restrict__ X, int rows,
                                                          const __bf16 *__restrict__ W1f,
                                                          const __bf16 *__restrict__ W2f,
                                                          const __bf16 *__restrict__ W3t,
                                                          const float *__restrict__ b1, const float *__restrict__ b2,
                                                          const float *__restrict__ b3p, float *__restrict__ Y,
                                                          MlpCorrection<T> cor) {
  __shared__ __attribute__((aligned(16))) __bf16 buf0[kRows * kLd];
  __shared__ __attribute__((aligned(16))) __bf16 buf1[kRows * kLd];
  __shared__ __attribute__((aligned(16))) __bf16 st_w3[kOutPad * kLd];
  // the correction's operands of the tile's rows (FROM_Q): the r = 1
  // right-hand side, the output mean and spread of the row's latitude (value
  // k of row i at k kRows + i: the lane-per-row reads hit distinct banks), the
  // latitude's h-mass weight of mode (0, 1)
  __shared__ float st_l1[FROM_Q ? kRows * 12 : 1], st_om[FROM_Q ? kRows * 12 : 1], st_os[FROM_Q ? kRows * 12 : 1];
  __shared__ double st_mw[FROM_Q ? kRows : 1];
  // the feature standardisation (FROM_Q), once per workgroup
  __shared__ float st_fm[FROM_Q ? kFeatures : 1], st_fi[FROM_Q ? kFeatures : 1];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r = lane & 15, kq = (lane >> 4) * 8;
  // the output layer's weights in LDS (rows padded like the activations):
  // registers held for 8 products per tile would push the kernel into scratch
  for (int c = tid; c < kOutPad * kHidden / 8; c += 64 * kWaves) {
    const int u = c / (kHidden / 8), k8 = c - u * (kHidden / 8);
    *reinterpret_cast<bf16x8 *>(st_w3 + u * kLd + 8 * k8) =
        *reinterpret_cast<const bf16x8 *>(W3t + (size_t)u * kHidden + 8 * k8);
  }
  // the hidden layers' weights in registers, requested after the LDS tables
  // (loads complete in order: the tables' stores wait only for their own
  // loads, and these arrive while the first tile's inputs are fetched)
  bf16x8 w1[kInPad / 32][2], w2[kHidden / 32][2];
  f32x4 bv1[2], bv2[2];
  // output layer: wavefront wv takes rows [16 (wv / 2), +16) and units [16 (wv % 2), +16)
  const int mt = wv >> 1, nt = wv & 1;
  const int n0 = 16 * nt + (lane >> 4) * 4;
  const f32x4 bv3 = *reinterpret_cast<const f32x4 *>(b3p + n0);
  // zero padding of the inputs beyond the 108 features (never overwritten)
  for (int idx = tid; idx < kRows * (kInPad - kFeatures); idx += 64 * kWaves) {
    const int rr = idx / (kInPad - kFeatures);
    buf0[rr * kLd + kFeatures + (idx - rr * (kInPad - kFeatures))] = (__bf16)0.f;
  }
  if constexpr (FROM_Q) {
    for (int k = tid; k < kFeatures; k += 64 * kWaves) {
      st_fm[k] = fmean[k];
      st_fi[k] = fistd[k];
    }
  }
  load_hidden<kInPad>(W1f, b1, wv, lane, w1, bv1);
  load_hidden<kHidden>(W2f, b2, wv, lane, w2, bv2);
  __syncthreads();            // the tables above before their first use
  double mass = 0.0;          // wavefront 0: this workgroup's h-mass of the corrections
  bool any_fell = false;
  unsigned long long fell_count = 0ull;
  // the 12 values of input task (row rr, stencil neighbour sn), raw, and
  // their BF16 features in buf0
  using In = typename std::conditional<FROM_Q, T, float>::type;
  int e0 = 0;
  auto load_task = [&](int task, In (&x)[12]) {
    const int rr = task / 9, sn = task - rr * 9;
    const int e = e0 + rr < rows ? e0 + rr : rows - 1;
    const In *src;
    if constexpr (FROM_Q) {
      const int dj = sn / 3 - 1, di = sn % 3 - 1;
      const int j = e / n_lon, i = e - j * n_lon;
      int jj = j + dj;
      jj = jj < 0 ? 0 : (jj >= n_lat ? n_lat - 1 : jj);
      int ii = i + di;
      ii = ii < 0 ? ii + n_lon : (ii >= n_lon ? ii - n_lon : ii);
      src = q + ((size_t)jj * n_lon + ii) * 12;
    } else {
      src = X + (size_t)e * kFeatures + sn * 12;
    }
#pragma unroll
    for (int vm = 0; vm < 12; ++vm) x[vm] = src[vm];
  };
  auto store_task = [&](int task, const In (&raw)[12]) {
    const int rr = task / 9, sn = task - rr * 9;
    float x[12];
#pragma unroll
    for (int vm = 0; vm < 12; ++vm) x[vm] = (float)raw[vm];
    if constexpr (FROM_Q) {
#pragma unroll
      for (int vm = 0; vm < 12; ++vm) x[vm] = (x[vm] - st_fm[sn * 12 + vm]) * st_fi[sn * 12 + vm];
    }
    bf16x4 *dst = reinterpret_cast<bf16x4 *>(buf0 + rr * kLd + sn * 12);
#pragma unroll
    for (int h4 = 0; h4 < 3; ++h4)
      dst[h4] = bf16x4{(__bf16)x[4 * h4], (__bf16)x[4 * h4 + 1], (__bf16)x[4 * h4 + 2], (__bf16)x[4 * h4 + 3]};
  };
  const int ntiles = (rows + kRows - 1) / kRows;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    e0 = tile * kRows;
    // inputs: one task per (row, stencil neighbour), 12 contiguous values;
    // the 64 tasks beyond one per lane go to wavefront 0, and the correction's
    // operands of the tile's rows are staged in LDS by wavefronts 1 .. 3, all
    // loads issued before any is waited for (one memory round trip per tile)
    constexpr int kTasks = kRows * 9;
    static_assert(kTasks > 64 * kWaves && kTasks <= 64 * kWaves + 64, "one extra task per lane of wavefront 0");
    In raw0[12], raw1[12];
    load_task(tid, raw0);
    if (wv == 0) load_task(tid + 64 * kWaves, raw1);
    if constexpr (FROM_Q) {
      const int e = e0 + lane < rows ? e0 + lane : rows - 1;
      const int j = e / n_lon;
      if (wv == 1) {
        const T *src = cor.L1 + (size_t)e * 12;
        T l1[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) l1[k] = src[k];
#pragma unroll
        for (int k = 0; k < 12; ++k) st_l1[k * kRows + lane] = (float)l1[k];
      } else if (wv == 2) {
        float om[12], os[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          om[k] = cor.omean[j * 12 + k];
          os[k] = cor.ostd[j * 12 + k];
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          st_om[k * kRows + lane] = om[k];
          st_os[k * kRows + lane] = os[k];
        }
      } else if (wv == 3) {
        st_mw[lane] = cor.mass_w[j * 2 + 1];
      }
    }
    store_task(tid, raw0);
    if (wv == 0) store_task(tid + 64 * kWaves, raw1);
    __syncthreads();
    fused_hidden<kInPad>(w1, bv1, buf0, buf1, wv, lane);
    __syncthreads();
    fused_hidden<kHidden>(w2, bv2, buf1, buf0, wv, lane);
    __syncthreads();
    f32x4 acc = bv3;
#pragma unroll
    for (int ks = 0; ks < kHidden / 32; ++ks) {
      const bf16x8 b = *reinterpret_cast<const bf16x8 *>(buf0 + (16 * mt + r) * kLd + 32 * ks + kq);
      const bf16x8 w3 = *reinterpret_cast<const bf16x8 *>(st_w3 + (16 * nt + r) * kLd + 32 * ks + kq);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3, b, acc, 0, 0, 0);
    }
    const f32x4 out = acc;
    if constexpr (!FROM_Q) {
      const int e = e0 + 16 * mt + r;
      if (e < rows) *reinterpret_cast<f32x4 *>(Y + (size_t)e * kOutPad + n0) = out;
    } else {
      // outputs to LDS (the first hidden layer's buffer is free), then one
      // lane per row forms its element's correction (wavefront 0)
      // (unit n of row i at n kYs + i: conflict-free stores and lane-per-row reads)
      float *ys = reinterpret_cast<float *>(buf1);
#pragma unroll
      for (int i = 0; i < 4; ++i) ys[(n0 + i) * kYs + 16 * mt + r] = out[i];
      __syncthreads();
      if (wv == 0) {
        const int e = e0 + lane;
        double m = 0.0;
        bool fell = false;
        if (e < rows) {
          float c[12];
          fell = correction_row<kYs, kRows>(ys + lane, st_l1 + lane, st_om + lane, st_os + lane, cor.kappa, c);
          // h-mass of the correction: modes (a, b) = (0, 0) and (0, 1), i.e. 0 and 2
          m = st_mw[lane] * (double)c[2];
          float4 *cd = reinterpret_cast<float4 *>(cor.C + (size_t)e * 12);
#pragma unroll
          for (int k4 = 0; k4 < 3; ++k4) cd[k4] = make_float4(c[4 * k4], c[4 * k4 + 1], c[4 * k4 + 2], c[4 * k4 + 3]);
        }
        const unsigned long long fb = __ballot(fell);
        fell_count += (unsigned long long)__popcll(fb);
        any_fell = any_fell || fb != 0ull;
        // fixed-order (tree) wavefront sum of the tile's 64 masses, added in tile order
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m += __shfl_down(m, off, 64);
        mass += m;
      }
    }
    __syncthreads();   // the next tile overwrites both buffers
  }
  if constexpr (FROM_Q) {
    if (wv == 0 && lane == 0) {
      cor.partial[blockIdx.x] = mass;
      if (cor.fallback && any_fell)
        atomicAdd(reinterpret_cast<unsigned long long *>(cor.fallback), fell_count);
    }
  }
}

int mlp_fused_blocks(int rows) {
  const int tiles = (rows + kRows - 1) / kRows;
  return tiles < kMlpGrid ? tiles : kMlpGrid;
}

hipError_t launch_mlp_fused(int dtype, const void *q, int n_lon, int n_lat, const float *fmean, const float *fistd,
                            const float *X, int rows, const __bf16 *W1f, const __bf16 *W2f, const __bf16 *W3t,
                            const float *b1, const float *b2, const float *b3p, float *Y, hipStream_t s,
                            const CorrectionArgs *ca) {
  static_assert(kInPad % 32 == 0 && kHidden == 32 * kWaves && kOutPad == 32 && kRows == 8 * kWaves,
                "fused network shape");
  if (rows <= 0) return hipSuccess;
  const dim3 grid(mlp_fused_blocks(rows)), block(64 * kWaves);
  if (!q) {
    hipLaunchKernelGGL((k_mlp_fused<float, false>), grid, block, 0, s, nullptr, 0, 0, nullptr, nullptr, X, rows, W1f,
                       W2f, W3t, b1, b2, b3p, Y, MlpCorrection<float>{});
    return hipGetLastError();
  }
  if (!ca) return hipErrorInvalidValue;
  if (dtype == 0) {
    MlpCorrection<double> c{static_cast<const double *>(ca->L1), ca->omean, ca->ostd, ca->mass_w, ca->kappa, ca->C,
                            ca->partial, ca->fallback};
    hipLaunchKernelGGL((k_mlp_fused<double, true>), grid, block, 0, s, static_cast<const double *>(q), n_lon, n_lat,
                       fmean, fistd, nullptr, rows, W1f, W2f, W3t, b1, b2, b3p, Y, c);
  } else {
    MlpCorrection<float> c{static_cast<const float *>(ca->L1), ca->omean, ca->ostd, ca->mass_w, ca->kappa, ca->C,
                           ca->partial, ca->fallback};
    hipLaunchKernelGGL((k_mlp_fused<float, true>), grid, block, 0, s, static_cast<const float *>(q), n_lon, n_lat,
                       fmean, fistd, nullptr, rows, W1f, W2f, W3t, b1, b2, b3p, Y, c);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ weights
// FP32 parameter vector -> BF16 operand copies: Wt[n][kp] (forward, k
// contiguous, k padded with zeros to kp) and Wr[k][np] (backward, rows padded
// to the next layer's padded width np, columns beyond n zero), and Wf, the
// forward weights in the order the fused kernel's wavefronts read them: for
// units [16 u, 16 u + 16) and inputs [32 c, 32 c + 32) one 1 KB block,
// ((u K/32 + c) 64 + lane) 8 + j holding unit 16 u + lane % 16 and input
// 32 c + 8 (lane / 16) + j (the MFMA A-operand layout), so that each of its
// loads is one contiguous kilobyte (kp % 32 == 0, np % 16 == 0).
__global__ void k_prep_weights(const float *__restrict__ W, int k_in, int n_out, int kp, int np_,
                               __bf16 *__restrict__ Wt, __bf16 *__restrict__ Wr, __bf16 *__restrict__ Wf) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = kp * np_;
  if (idx >= total) return;
  const int k = idx / np_, n = idx - k * np_;
  const float w = (k < k_in && n < n_out) ? W[(size_t)k * n_out + n] : 0.0f;
  if (Wr) Wr[(size_t)k * np_ + n] = (__bf16)w;
  if (Wt) Wt[(size_t)n * kp + k] = (__bf16)w;
  if (Wf) {
    const int lane = n % 16 + 16 * ((k % 32) / 8);
    Wf[((size_t)(n / 16) * (kp / 32) + k / 32) * 512 + lane * 8 + k % 8] = (__bf16)w;
  }
}

hipError_t launch_prep_weights(const float *W, int k_in, int n_out, int kp, int np_, __bf16 *Wt, __bf16 *Wr,
                               __bf16 *Wf, hipStream_t s) {
  if (Wf && (kp % 32 || np_ % 16)) return hipErrorInvalidValue;
  const int total = kp * np_;
  hipLaunchKernelGGL(k_prep_weights, dim3((total + 255) / 256), dim3(256), 0, s, W, k_in, n_out, kp, np_, Wt, Wr,
                     Wf);
  return hipGetLastError();
}

// ------------------------------------------------------------------ loss
// dY = 2 (Y - T) mask / (rows * sum(mask)) as BF16 (padded columns zero) and
// the squared error summed per block into partial[blockIdx.x].  The 0/1 mask
// of the outputs arrives as bits (bit n: output n counts).
__global__ __launch_bounds__(256) void k_mse_grad(const float *__restrict__ Y, const float *__restrict__ T,
                                                  unsigned mask_bits, int rows, int n_out, int ld,
                                                  float scale, __bf16 *__restrict__ dY, float *__restrict__ dYf,
                                                  float *__restrict__ partial) {
  __shared__ float sh[256];
  const int idx = blockIdx.x * 256 + threadIdx.x;
  float se = 0.f;
  if (idx < rows * ld) {
    const int m = idx / ld, n = idx - m * ld;
    float g = 0.f;
    if (n < n_out && ((mask_bits >> n) & 1u)) {
      const float d = Y[(size_t)m * ld + n] - T[(size_t)m * n_out + n];
      se = d * d;
      g = 2.f * d * scale;
    }
    dY[idx] = (__bf16)g;
    dYf[idx] = g;
  }
  sh[threadIdx.x] = se;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

hipError_t launch_mse_grad(const float *Y, const float *T, unsigned mask_bits, int rows, int n_out, int ld,
                           float scale, __bf16 *dY, float *dYf, float *partial, int *nblocks, hipStream_t s) {
  *nblocks = (rows * ld + 255) / 256;
  hipLaunchKernelGGL(k_mse_grad, dim3(*nblocks), dim3(256), 0, s, Y, T, mask_bits, rows, n_out, ld, scale, dY, dYf,
                     partial);
  return hipGetLastError();
}

// Column sums of G[rows][ld] for the first n columns (bias gradients) in two
// deterministic passes: workgroup (column block, chunk) sums its chunk of
// rows for 64 columns (4 row lanes per column, then a fixed tree), and
// launch_sum_split adds the chunks in order.
__global__ __launch_bounds__(256) void k_colsum_part(const float *__restrict__ G, int rows, int n, int ld,
                                                     int chunk, float *__restrict__ part) {
  __shared__ float sh[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), rl = threadIdx.x >> 6;
  const int r0 = blockIdx.y * chunk, r1 = r0 + chunk < rows ? r0 + chunk : rows;
  float acc = 0.f;
  if (c < n)
    for (int m = r0 + rl; m < r1; m += 4) acc += G[(size_t)m * ld + c];
  sh[rl][threadIdx.x & 63] = acc;
  __syncthreads();
  if (rl == 0 && c < n)
    part[(size_t)blockIdx.y * n + c] = (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
}

int colsum_chunks(int rows) {
  const int c = (rows + 63) / 64;
  return c < 1 ? 1 : (c > kMaxColChunks ? kMaxColChunks : c);
}

hipError_t launch_colsum(const float *G, int rows, int n, int ld, float *part, float *out, hipStream_t s) {
  const int chunks = colsum_chunks(rows);
  const int chunk = (rows + chunks - 1) / chunks;
  hipLaunchKernelGGL(k_colsum_part, dim3((n + 63) / 64, chunks), dim3(256), 0, s, G, rows, n, ld, chunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_split(part, chunks, n, out, s);
}

// scale * (sum of `n` partials), single block, fixed order, into *out.
__global__ __launch_bounds__(256) void k_sum(const float *__restrict__ p, int n, float scale,
                                             float *__restrict__ out) {
  __shared__ float sh[256];
  float acc = 0.f;
  for (int k = threadIdx.x; k < n; k += 256) acc += p[k];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = scale * sh[0];
}

hipError_t launch_sum(const float *p, int n, float scale, float *out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, p, n, scale, out);
  return hipGetLastError();
}

// X[rows][n] (FP32) -> Xb[rows][ldx] (BF16, columns >= n zero)
__global__ void k_to_bf16(const float *__restrict__ X, int rows, int n, int ldx, __bf16 *__restrict__ Xb) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)rows * ldx) return;
  const size_t m = idx / ldx;
  const int k = (int)(idx - m * ldx);
  Xb[idx] = (__bf16)(k < n ? X[m * n + k] : 0.0f);
}

hipError_t launch_to_bf16(const float *X, int rows, int n, int ldx, __bf16 *Xb, hipStream_t s) {
  const size_t total = (size_t)rows * ldx;
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, X, rows, n, ldx, Xb);
  return hipGetLastError();
}

// b[n] -> out[np_] with zeros beyond n
__global__ void k_pad(const float *__restrict__ b, int n, int np_, float *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np_) out[i] = i < n ? b[i] : 0.0f;
}

hipError_t launch_pad(const float *b, int n, int np_, float *out, hipStream_t s) {
  hipLaunchKernelGGL(k_pad, dim3((np_ + 63) / 64), dim3(64), 0, s, b, n, np_, out);
  return hipGetLastError();
}

// Gradient of a weight matrix W[k_in][n_out] from the padded GEMM result
// G[kp][np_] (rows/cols beyond the real sizes dropped) into the flat vector.
__global__ void k_unpad(const float *__restrict__ G, int k_in, int n_out, int np_, float *__restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= k_in * n_out) return;
  const int k = idx / n_out, n = idx - k * n_out;
  out[idx] = G[(size_t)k * np_ + n];
}

hipError_t launch_unpad(const float *G, int k_in, int n_out, int np_, float *out, hipStream_t s) {
  const int total = k_in * n_out;
  hipLaunchKernelGGL(k_unpad, dim3((total + 255) / 256), dim3(256), 0, s, G, k_in, n_out, np_, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Adam
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

// ------------------------------------------------------------------ features
// X[e][k] = bf16((q1[nb(e, k)][v][m] - mean[k]) * istd[k]) for the 3 x 3 stencil
// of an r = 1 state (periodic in longitude, pole row repeated across a pole),
// k = ((dj+1)*3 + (di+1))*12 + v*4 + m; columns 108..ldx-1 are zero.
template <typename T>
__global__ void k_features(const T *__restrict__ q, int n_lon, int n_lat, const float *__restrict__ mean,
                           const float *__restrict__ istd, int ldx, __bf16 *__restrict__ X) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t E = (size_t)n_lon * n_lat;
  if (idx >= E * ldx) return;
  const int e = (int)(idx / ldx), k = (int)(idx - (size_t)e * ldx);
  float x = 0.f;
  if (k < kFeatures) {
    const int s = k / 12, vm = k - s * 12;
    const int dj = s / 3 - 1, di = s % 3 - 1;
    const int j = e / n_lon, i = e - j * n_lon;
    int jj = j + dj;
    jj = jj < 0 ? 0 : (jj >= n_lat ? n_lat - 1 : jj);
    int ii = i + di;
    ii = ii < 0 ? ii + n_lon : (ii >= n_lon ? ii - n_lon : ii);
    x = ((float)q[((size_t)jj * n_lon + ii) * 12 + vm] - mean[k]) * istd[k];
  }
  X[idx] = (__bf16)x;
}

// Same features in FP32, [E][108], standardised when mean/istd are given.
template <typename T>
__global__ void k_features_f32(const T *__restrict__ q, int n_lon, int n_lat, const float *__restrict__ mean,
                               const float *__restrict__ istd, float *__restrict__ X) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t E = (size_t)n_lon * n_lat;
  if (idx >= E * kFeatures) return;
  const int e = (int)(idx / kFeatures), k = (int)(idx - (size_t)e * kFeatures);
  const int s = k / 12, vm = k - s * 12;
  const int dj = s / 3 - 1, di = s % 3 - 1;
  const int j = e / n_lon, i = e - j * n_lon;
  int jj = j + dj;
  jj = jj < 0 ? 0 : (jj >= n_lat ? n_lat - 1 : jj);
  int ii = i + di;
  ii = ii < 0 ? ii + n_lon : (ii >= n_lon ? ii - n_lon : ii);
  float x = (float)q[((size_t)jj * n_lon + ii) * 12 + vm];
  if (mean) x = (x - mean[k]) * istd[k];
  X[idx] = x;
}

hipError_t launch_features_f32(int dtype, const void *q, int n_lon, int n_lat, const float *mean, const float *istd,
                               float *X, hipStream_t s) {
  const size_t total = (size_t)n_lon * n_lat * kFeatures;
  const dim3 grid((unsigned)((total + 255) / 256));
  if (dtype == 0)
    hipLaunchKernelGGL(k_features_f32<double>, grid, dim3(256), 0, s, static_cast<const double *>(q), n_lon, n_lat,
                       mean, istd, X);
  else
    hipLaunchKernelGGL(k_features_f32<float>, grid, dim3(256), 0, s, static_cast<const float *>(q), n_lon, n_lat,
                       mean, istd, X);
  return hipGetLastError();
}

hipError_t launch_features(int dtype, const void *q, int n_lon, int n_lat, const float *mean, const float *istd,
                           int ldx, __bf16 *X, hipStream_t s) {
  const size_t total = (size_t)n_lon * n_lat * ldx;
  const dim3 grid((unsigned)((total + 255) / 256));
  if (dtype == 0)
    hipLaunchKernelGGL(k_features<double>, grid, dim3(256), 0, s, static_cast<const double *>(q), n_lon, n_lat, mean,
                       istd, ldx, X);
  else
    hipLaunchKernelGGL(k_features<float>, grid, dim3(256), 0, s, static_cast<const float *>(q), n_lon, n_lat, mean,
                       istd, ldx, X);
  return hipGetLastError();
}

// ------------------------------------------------------------------ learned stage
// delta = -(sum of partials) / (sum over elements of mass_w[j][0]): the mode-00
// h-correction that makes the total h-mass change of the correction zero.
// Every block of the output kernel forms it itself, in the same fixed order.
__device__ __forceinline__ double block_mass_delta(const double *__restrict__ partial, int nparts, double area,
                                                  double *sh) {
  double acc = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 256) acc += partial[k];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  return -sh[0] / area;
}

// out = combine ? c0 q0 + c1 (q + dt (L1 + c)) : L1 + c, with c_(h,00) = delta;
// the combination is evaluated as y + c0 (q0 - y) + ce y, y = q + dt (L1 + c),
// ce = c0 + c1 - 1 formed in FP64, so the weights sum to one exactly.
template <typename T>
__global__ __launch_bounds__(256) void k_learned_out(const T *__restrict__ q, const T *q0, const T *__restrict__ L1,
                                                     const float *__restrict__ C, const double *__restrict__ partial,
                                                     int nparts, double area, int E, int combine, T c0, T ce, T dt,
                                                     T *out) {
  __shared__ double sh[256];
  // the element's operands first, so that their loads are in flight while
  // the block sums the mass partials (the same arithmetic either way)
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const bool live = idx < E * 12;
  const int k = idx % 12;
  T l1v = T(0), qv = T(0), qn = T(0);
  float cv = 0.f;
  if (live) {
    l1v = L1[idx];
    if (k != 0) cv = C[idx];
    if (combine) {
      qv = q[idx];
      if (c0 != T(0)) qn = q0[idx];
    }
  }
  const double delta = block_mass_delta(partial, nparts, area, sh);
  if (!live) return;
  const T corr = k == 0 ? (T)delta : (T)cv;
  const T l = l1v + corr;
  if (combine) {
    const T y = qv + dt * l;
    out[idx] = y + c0 * (qn - y) + ce * y;
  } else {
    out[idx] = l;
  }
}

hipError_t launch_learned_out(int dtype, const LearnedOut &a, hipStream_t s) {
  const int ob = (a.E * 12 + 255) / 256;
  if (dtype == 0)
    hipLaunchKernelGGL(k_learned_out<double>, dim3(ob), dim3(256), 0, s, static_cast<const double *>(a.q),
                       static_cast<const double *>(a.q0), static_cast<const double *>(a.L1), a.C, a.partial, a.nparts,
                       a.area, a.E, a.combine, a.c0, a.c0 + a.c1 - 1.0, a.dt, static_cast<double *>(a.out));
  else
    hipLaunchKernelGGL(k_learned_out<float>, dim3(ob), dim3(256), 0, s, static_cast<const float *>(a.q),
                       static_cast<const float *>(a.q0), static_cast<const float *>(a.L1), a.C, a.partial, a.nparts,
                       a.area, a.E, a.combine, (float)a.c0, (float)(a.c0 + a.c1 - 1.0), (float)a.dt,
                       static_cast<float *>(a.out));
  return hipGetLastError();
}

// ------------------------------------------------------------------ projection
// Cos-weighted L2 projection of an order-r state onto order k on the same
// mesh: the longitude degrees a <= min(k, r) are kept (orthonormal, the mass
// matrix is diagonal in a), the latitude degrees mix through the per-row
// (k+1) x (r+1) matrix Pj[b'][b].  One thread per output value.
template <typename T>
__global__ void k_project(const T *__restrict__ q, int n_lon, int E, int np, int nk,
                          const double *__restrict__ P, T *__restrict__ out) {
  const int per = 3 * nk * nk;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * per) return;
  const int e = (int)(idx / per), k = (int)(idx - (long long)e * per);
  const int v = k / (nk * nk), m = k - v * nk * nk, bp = m / nk, a = m - bp * nk;
  const int j = e / n_lon;
  const T *qe = q + (size_t)e * 3 * np * np + (size_t)v * np * np;
  double acc = 0.0;
  if (a < np)
    for (int b = 0; b < np; ++b) acc += P[((size_t)j * nk + bp) * np + b] * (double)qe[b * np + a];
  out[idx] = (T)acc;
}

hipError_t launch_project(int dtype, const void *q, int n_lon, int E, int np, int nk, const double *P,
                          void *out, hipStream_t s) {
  const long long n = (long long)E * 3 * nk * nk;
  const int blocks = (int)((n + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_project<double>, dim3(blocks), dim3(256), 0, s, static_cast<const double *>(q), n_lon, E,
                       np, nk, P, static_cast<double *>(out));
  else
    hipLaunchKernelGGL(k_project<float>, dim3(blocks), dim3(256), 0, s, static_cast<const float *>(q), n_lon, E,
                       np, nk, P, static_cast<float *>(out));
  return hipGetLastError();
}

}  // namespace dgsw
