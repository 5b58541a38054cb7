// Launchers of the learned-correction kernels (dgsw_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace dgsw {

constexpr int kFeatures = 108;   // 3 x 3 stencil x 3 variables x 4 modes
constexpr int kHidden = 256;
constexpr int kOut = 12;         // 3 variables x 4 modes of r = 1
constexpr int kInPad = 128;      // feature width padded for the K loop
constexpr int kOutPad = 32;      // output width padded for the N tiles

enum { kEpiBiasGelu = 0, kEpiBias = 1, kEpiGeluGrad = 2, kEpiPlain = 3 };

struct GemmArgs {
  const __bf16 *A, *B;
  int M, N, K, lda, ldb;
  const float *bias;   // kEpiBiasGelu, kEpiBias
  const float *Zin;    // kEpiGeluGrad: pre-activations
  float *Zout;         // kEpiBiasGelu: pre-activations out; kEpiGeluGrad: FP32 result out (optional)
  void *C;             // BF16 (gelu variants) or FP32 result
  int ldc;
};
hipError_t launch_gemm(bool a_kc, bool b_kc, int epi, const GemmArgs &g, hipStream_t s);
// Weight gradients C[M][N] = sum over k < K of A[k][m] B[k][n] (both operands
// row-major over k): K split into gemm_splits(K) ranges of workgroups, the
// partial products (partial: gemm_splits(K) * M * ldc floats) summed in order.
constexpr int kMaxSplits = 64;
int gemm_splits(int K);
hipError_t launch_gemm_splitk(const GemmArgs &g, float *partial, hipStream_t s);
// The learned stage's correction step, fused into the network kernel.
struct CorrectionArgs {
  const void *L1;                // plain r = 1 right-hand side [E][12] (state dtype)
  const float *omean, *ostd;     // [n_lat][12]
  const double *mass_w;          // [n_lat][2]
  float kappa;
  float *C;                      // corrections [E][12]
  double *partial;               // one h-mass per workgroup: mlp_fused_blocks(E)
  int64_t *fallback;             // optional device counter (64-bit: never wraps)
};
// workgroups of the persistent network kernel for `rows` rows (at most one
// per compute unit)
int mlp_fused_blocks(int rows);
// Whole-network inference, tiles of 64 rows, activations in LDS.  With q:
// rows = elements of the r = 1 state q (dtype 0/1), features computed from q,
// then the correction of each element (ca required; Y unused).  With q == NULL:
// rows of X[rows][108] (FP32) -> Y[rows][32] FP32 (the first 12 used).  W1f,
// W2f: the hidden layers' weights in fragment order (launch_prep_weights' Wf),
// W3t: the output layer's as Wt.
hipError_t launch_mlp_fused(int dtype, const void *q, int n_lon, int n_lat, const float *fmean, const float *fistd,
                            const float *X, int rows, const __bf16 *W1f, const __bf16 *W2f, const __bf16 *W3t,
                            const float *b1, const float *b2, const float *b3p, float *Y, hipStream_t s,
                            const CorrectionArgs *ca);
hipError_t launch_prep_weights(const float *W, int k_in, int n_out, int kp, int np_, __bf16 *Wt, __bf16 *Wr,
                               __bf16 *Wf, hipStream_t s);
hipError_t launch_mse_grad(const float *Y, const float *T, unsigned mask_bits, int rows, int n_out, int ld,
                           float scale, __bf16 *dY, float *dYf, float *partial, int *nblocks, hipStream_t s);
// column sums over rows (partial: colsum_chunks(rows) * n floats)
constexpr int kMaxColChunks = 256;
int colsum_chunks(int rows);
hipError_t launch_colsum(const float *G, int rows, int n, int ld, float *part, float *out, hipStream_t s);
hipError_t launch_sum(const float *p, int n, float scale, float *out, hipStream_t s);
hipError_t launch_to_bf16(const float *X, int rows, int n, int ldx, __bf16 *Xb, hipStream_t s);
hipError_t launch_pad(const float *b, int n, int np_, float *out, hipStream_t s);
hipError_t launch_unpad(const float *G, int k_in, int n_out, int np_, float *out, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);
hipError_t launch_features(int dtype, const void *q, int n_lon, int n_lat, const float *mean, const float *istd,
                           int ldx, __bf16 *X, hipStream_t s);
hipError_t launch_features_f32(int dtype, const void *q, int n_lon, int n_lat, const float *mean, const float *istd,
                               float *X, hipStream_t s);
hipError_t launch_project(int dtype, const void *q, int n_lon, int E, int np, int nk, const double *P,
                          void *out, hipStream_t s);

// The learned stage's last step: out = L1 + C, the (h, 00) entry replaced by
// the global h-mass delta formed from the per-workgroup partials, or the
// Runge-Kutta combination with it.
struct LearnedOut {
  const void *L1;        // plain r = 1 right-hand side [E][12]
  const float *C;        // corrections [E][12]
  const double *partial; // nparts per-workgroup h-masses of the corrections
  int nparts, E;
  double area;           // sum over elements of mass_w[j][0]
  const void *q, *q0;
  void *out;
  int combine;
  double c0, c1, dt;
};
hipError_t launch_learned_out(int dtype, const LearnedOut &a, hipStream_t s);

}  // namespace dgsw
