// Throughput probe of the volume-integral contraction at r = 5 in FP32 (the
// 360 x 180 configuration's order), in the two forms a stage kernel can use:
//
//   VALU, sum-factorised (what the stage kernels do): per element and flux
//   quantity, Z[p][b] = sum_s x(p, s) M[s][b] over the latitude nodes, then
//   out[a][b] = sum_p D[p][a] Z_F[p][b] + B[p][a] (Z_G + Z_S)[p][b] over the
//   longitude nodes: 2 n^3 multiply-adds per quantity (n = 6).
//
//   MFMA, dense (the form of the paper's volume stencil, phi_grad^T (f w)):
//   out_v = sum_q A_q x_q with the 36 x 36 matrices A_q = (1-D table) x
//   (1-D table) formed once, batched over elements as GEMMs on
//   v_mfma_f32_16x16x4f32 (36 padded to 48): N^2 = n^4 multiply-adds per
//   quantity, on the matrix cores.
//
// Only the contraction is timed: the nodal values x are synthesised in
// registers from the element index (the same values in both forms) and each
// wavefront writes one checksum per lane, so no HBM traffic hides the
// arithmetic.  Both forms compute the same numbers; dgp_contraction_check
// compares them element by element.  Not part of the solver: a measurement
// of a design choice, built as its own library.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

namespace {

constexpr int NP = 6, N = 36, NQ = 8;    // nodes per direction, per element; flux quantities
constexpr int MT = 3, KS = 9;            // 48 / 16 output tiles, 36 / 4 k-steps
constexpr int GPW = 10;                  // VALU form: elements per wavefront (6 lanes each)

typedef float f32x4 __attribute__((ext_vector_type(4)));

// quantity q contributes to variable var(q): F0, F1, F2 -> 0, 1, 2; G0, G1,
// G2 -> 0, 1, 2; S1, S2 -> 1, 2
__host__ __device__ constexpr int qvar(int q) { return q < 3 ? q : (q < 6 ? q - 3 : q - 5); }

// synthetic nodal value of quantity q at node k = s * NP + p of element e
__device__ __forceinline__ float xval(int e, int q, int k) {
  const unsigned h = (unsigned)e * 2654435761u + (unsigned)q * 40503u + (unsigned)k * 977u;
  return (float)((h >> 9) & 1023u) * (1.0f / 1024.0f) - 0.5f;
}

struct Tabs {
  float M[2][NP][NP];     // [BM, DM][s][b]
  float P[2][NP][NP];     // [D, B][p][a]
};

// VALU form: lane t of an element owns longitude node p = t, then output row b = t
__global__ __launch_bounds__(64) void k_contract_valu(const Tabs *__restrict__ tb, int n_elem, float *__restrict__ sum,
                                                      float *__restrict__ out) {
  __shared__ float Z[GPW][NQ][NP][NP];     // [element][quantity][p][b]
  const int lane = threadIdx.x, g = lane / NP, t = lane - g * NP;
  const bool idle = g >= GPW;
  const int e = blockIdx.x * GPW + (idle ? 0 : g);
  float acc_sum = 0.f;
  if (!idle) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int mi = (q >= 3 && q < 6) ? 1 : 0;     // G uses DM, F and S use BM
      float x[NP];
#pragma unroll
      for (int s = 0; s < NP; ++s) x[s] = xval(e, q, s * NP + t);
#pragma unroll
      for (int b = 0; b < NP; ++b) {
        float z = 0.f;
#pragma unroll
        for (int s = 0; s < NP; ++s) z += x[s] * tb->M[mi][s][b];
        Z[g][q][t][b] = z;
      }
    }
  }
  __syncthreads();
  if (!idle) {
#pragma unroll
    for (int v = 0; v < 3; ++v) {
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        float o = 0.f;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          float zg = Z[g][3 + v][p][t];
          if (v > 0) zg += Z[g][5 + v][p][t];
          o += tb->P[0][p][a] * Z[g][v][p][t] + tb->P[1][p][a] * zg;
        }
        if (out && e < n_elem) out[((size_t)e * 3 + v) * N + t * NP + a] = o;
        acc_sum += o;
      }
    }
  }
  sum[blockIdx.x * 64 + lane] = acc_sum;
}

// MFMA form: a wavefront takes 16 elements as the 16 columns of each product;
// lane l supplies A[row l % 16][k = 4 ks + l / 16] and x[k][column l % 16] and
// holds D[4 (l / 16) + i][l % 16].  The dense matrices (48 x 48 per quantity,
// zero padded) sit in LDS in that lane order.
__global__ __launch_bounds__(256) void k_contract_mfma(const float *__restrict__ A, int n_elem, float *__restrict__ sum,
                                                       float *__restrict__ out) {
  __shared__ float As[NQ][MT][KS][64];
  for (int i = threadIdx.x; i < NQ * MT * KS * 64; i += 256) (&As[0][0][0][0])[i] = A[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = lane & 15, gq = lane >> 4;
  const int e0 = (blockIdx.x * 4 + wv) * 16;
  const int e = e0 + c;
  f32x4 acc[3][MT];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[v][m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int v = qvar(q);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const float xb = xval(e, q, 4 * ks + gq);
#pragma unroll
      for (int m = 0; m < MT; ++m)
        acc[v][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(As[q][m][ks][lane], xb, acc[v][m], 0, 0, 0);
    }
  }
  float acc_sum = 0.f;
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * m + 4 * gq + i;     // output mode index (b a order: m = b NP + a)
        if (row < N) {
          acc_sum += acc[v][m][i];
          if (out && e < n_elem) out[((size_t)e * 3 + v) * N + row] = acc[v][m][i];
        }
      }
  sum[(blockIdx.x * 4 + wv) * 64 + lane] = acc_sum;
}

void make_tables(Tabs &t, std::vector<float> &dense) {
  // fixed, well-scaled 1-D tables (the structure, not the values, is what is timed)
  for (int i = 0; i < NP; ++i)
    for (int j = 0; j < NP; ++j) {
      t.M[0][i][j] = std::cos(0.3f * i + 0.7f * j);
      t.M[1][i][j] = std::sin(0.5f * i - 0.2f * j + 0.1f);
      t.P[0][i][j] = std::cos(0.4f * i * j + 0.2f);
      t.P[1][i][j] = std::sin(0.9f * i + 0.3f * j + 0.3f);
    }
  // dense A_q[m][k], m = b NP + a, k = s NP + p: the product of the two 1-D
  // factors of quantity q, laid out [q][mt][ks][lane] in MFMA operand order
  dense.assign((size_t)NQ * MT * KS * 64, 0.f);
  for (int q = 0; q < NQ; ++q) {
    const int mi = (q >= 3 && q < 6) ? 1 : 0;
    const int pi = q < 3 ? 0 : 1;                    // F with D, G and S with B
    for (int mt = 0; mt < MT; ++mt)
      for (int ks = 0; ks < KS; ++ks)
        for (int l = 0; l < 64; ++l) {
          const int m = 16 * mt + (l & 15), k = 4 * ks + (l >> 4);
          float a = 0.f;
          if (m < N && k < N) {
            const int b = m / NP, aa = m % NP, s = k / NP, p = k % NP;
            a = t.P[pi][p][aa] * t.M[mi][s][b];
          }
          dense[(((size_t)q * MT + mt) * KS + ks) * 64 + l] = a;
        }
  }
}

struct Bufs {
  Tabs *d_tabs = nullptr;
  float *d_dense = nullptr, *d_sum = nullptr, *d_out0 = nullptr, *d_out1 = nullptr;
};

int setup(int n_elem, Bufs &b, bool with_out) {
  Tabs t;
  std::vector<float> dense;
  make_tables(t, dense);
  const size_t sum_n = (size_t)(n_elem / GPW + 2) * 64 + (size_t)(n_elem / 16 + 8) * 64;
  if (hipMalloc(&b.d_tabs, sizeof(Tabs)) != hipSuccess || hipMalloc(&b.d_dense, dense.size() * 4) != hipSuccess ||
      hipMalloc(&b.d_sum, sum_n * 4) != hipSuccess)
    return -3;
  if (with_out && (hipMalloc(&b.d_out0, (size_t)n_elem * 3 * N * 4) != hipSuccess ||
                   hipMalloc(&b.d_out1, (size_t)n_elem * 3 * N * 4) != hipSuccess))
    return -3;
  if (hipMemcpy(b.d_tabs, &t, sizeof(Tabs), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b.d_dense, dense.data(), dense.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
    return -4;
  return 0;
}

void release(Bufs &b) {
  if (b.d_tabs) (void)hipFree(b.d_tabs);
  if (b.d_dense) (void)hipFree(b.d_dense);
  if (b.d_sum) (void)hipFree(b.d_sum);
  if (b.d_out0) (void)hipFree(b.d_out0);
  if (b.d_out1) (void)hipFree(b.d_out1);
}

hipError_t launch(int variant, int n_elem, const Bufs &b, float *out) {
  if (variant == 0)
    hipLaunchKernelGGL(k_contract_valu, dim3((n_elem + GPW - 1) / GPW), dim3(64), 0, 0, b.d_tabs, n_elem, b.d_sum,
                       out);
  else
    hipLaunchKernelGGL(k_contract_mfma, dim3((n_elem + 63) / 64), dim3(256), 0, 0, b.d_dense, n_elem, b.d_sum, out);
  return hipGetLastError();
}

}  // namespace

extern "C" {

// Mean time [ms] of one launch of the contraction form `variant` (0: VALU
// sum-factorised, 1: MFMA dense) over n_elem elements, over `reps` launches
// after two warm-ups.  0 on success, < 0 on error.
int dgp_contraction_time(int variant, int n_elem, int reps, double *ms) {
  if (!ms || n_elem < 1 || reps < 1 || (variant != 0 && variant != 1)) return -1;
  Bufs b;
  int rc = setup(n_elem, b, false);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (rc == 0 && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = -4;
  for (int w = 0; rc == 0 && w < 2; ++w)
    if (launch(variant, n_elem, b, nullptr) != hipSuccess) rc = -4;
  if (rc == 0) {
    (void)hipEventRecord(e0, 0);
    for (int r = 0; r < reps && rc == 0; ++r)
      if (launch(variant, n_elem, b, nullptr) != hipSuccess) rc = -4;
    (void)hipEventRecord(e1, 0);
    if (hipEventSynchronize(e1) != hipSuccess) rc = -4;
    float t = 0.f;
    (void)hipEventElapsedTime(&t, e0, e1);
    *ms = (double)t / reps;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  release(b);
  return rc;
}

// Both forms on n_elem elements with their outputs written: the largest
// difference relative to the largest value, into *rel.
int dgp_contraction_check(int n_elem, double *rel) {
  if (!rel || n_elem < 1) return -1;
  Bufs b;
  int rc = setup(n_elem, b, true);
  if (rc == 0 && (launch(0, n_elem, b, b.d_out0) != hipSuccess || launch(1, n_elem, b, b.d_out1) != hipSuccess))
    rc = -4;
  if (rc == 0) {
    const size_t n = (size_t)n_elem * 3 * N;
    std::vector<float> h0(n), h1(n);
    if (hipMemcpy(h0.data(), b.d_out0, n * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(h1.data(), b.d_out1, n * 4, hipMemcpyDeviceToHost) != hipSuccess) {
      rc = -4;
    } else {
      double dmax = 0.0, vmax = 0.0;
      for (size_t i = 0; i < n; ++i) {
        dmax = std::fmax(dmax, std::fabs((double)h0[i] - (double)h1[i]));
        vmax = std::fmax(vmax, std::fabs((double)h0[i]));
      }
      *rel = vmax > 0.0 ? dmax / vmax : dmax;
    }
  }
  release(b);
  return rc;
}

}  // extern "C"
