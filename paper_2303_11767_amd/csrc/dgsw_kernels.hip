// Mesh stage kernels (both layouts), mass diagnostic, launchers and the
// upload of the tables; the stage itself is in dgsw_stage.hpp.
#include "dgsw_stage.hpp"

namespace dgsw {

// PK: wavefront w of a layer takes the GPW consecutive elements from w GPW on,
// across row ends (needs GPW <= n_lon; ceil(E / GPW) wavefronts); otherwise
// row-aligned segments, segs per row.  One wavefront per workgroup (8960
// bytes of LDS at FP64 r = 3: the 16 wavefronts per CU that the registers
// allow fit).  Register budget: four wavefronts per SIMD (128 registers) at
// FP64 r = 3 with the one-state combinations, which fit without spilling (the
// RK4 combination would spill); two (256) elsewhere, which keeps the FP64
// r >= 5 cases, at the edge of 256, from spilling into accumulation registers
// and halving their occupancy.
template <typename T, int NP, int CM>
struct H2Occ {
  static constexpr int value = sizeof(T) == 8 && NP == 4 && CM != 2 ? 4 : 2;
};

template <typename T, int NP, int WPB, int CM, bool PK>
__global__ __attribute__((amdgpu_waves_per_eu(H2Occ<T, NP, CM>::value))) __launch_bounds__(64 * WPB) void k_dg_stage_h2(
    StageArgs<T, NP> A, int segs) {
  using S_ = ShapeH2<T, NP>;
  __shared__ T tab_all[WPB][S_::TB];
  __shared__ T sh_all[WPB][S_::SLOTS * S_::SH];
  const int wv = WPB == 1 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int blk = xcd_block(blockIdx.x, gridDim.x) * WPB + wv;
  const int E = A.n_lon * A.n_lat;
  const int per = PK ? (E + S_::GPW - 1) / S_::GPW : segs * A.n_lat;   // wavefronts of one layer
  if (blk >= per * A.levels) return;
  const int lev = blk / per;
  blk -= lev * per;
  int j0, e0, e_end;
  if (PK) {
    e0 = blk * S_::GPW;
    j0 = e0 / A.n_lon;
    e_end = E;
  } else {
    j0 = blk / segs;
    e0 = j0 * A.n_lon + (blk - j0 * segs) * S_::GPW;
    e_end = (j0 + 1) * A.n_lon;
  }
  stage_wave_h2<T, NP, CM, PK>(layer_args(A, lev), j0, e0, e_end, threadIdx.x & 63, tab_all[wv],
                               sh_all[wv]);
}

template <typename T, int NP, int WPB, int CM>
__global__ __launch_bounds__(64 * WPB) void k_dg_stage(StageArgs<T, NP> A, int segs) {
  using S_ = Shape<T, NP>;
  // WPB independent wavefronts per workgroup (fewer workgroups to dispatch on
  // large meshes); each wavefront has its own LDS slice and never waits for
  // another one
  __shared__ T tab_all[WPB][S_::TB];
  __shared__ T sh_all[WPB][(S_::GPW + 1) * S_::SH];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int blk = xcd_block(blockIdx.x, gridDim.x) * WPB + wv;
  const int per = segs * A.n_lat;            // wavefronts of one layer
  if (blk >= per * A.levels) return;         // spare wavefront of the last workgroup
  const int lev = blk / per;
  blk -= lev * per;
  const int j = blk / segs;
  stage_wave<T, NP, CM>(layer_args(A, lev), j, blk - j * segs, threadIdx.x & 63, tab_all[wv],
                        sh_all[wv]);
}

// ------------------------------------------------------------------ mass
constexpr int kMassThreads = 256;
constexpr int kMassBlocks = 512;

int mass_blocks() { return kMassBlocks; }

int waves_per_row(int np, int n_lon) {
  const int gpw = 64 / np;
  return (n_lon + gpw - 1) / gpw;
}

template <int NT>
__device__ __forceinline__ void block_sum4(double v[4], double *sh) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 4; ++k) sh[k * NT + tid] = v[k];
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if (tid < off)
#pragma unroll
      for (int k = 0; k < 4; ++k) sh[k * NT + tid] += sh[k * NT + tid + off];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = sh[k * NT];
}

template <typename T, int NP>
__global__ __launch_bounds__(kMassThreads) void k_mass_partial(const T *__restrict__ q,
                                                               const double *__restrict__ mw,
                                                               int n_lon, int E, long long E_all,
                                                               double *__restrict__ partial) {
  constexpr int N = NP * NP;
  __shared__ double sh[4 * kMassThreads];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // E_all = layers x E elements; the row of element e of any layer
  for (long long e = blockIdx.x * kMassThreads + threadIdx.x; e < E_all;
       e += (long long)gridDim.x * kMassThreads) {
    const int j = (int)(e % E) / n_lon;
    const T *qe = q + (size_t)e * 3 * N;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
#pragma unroll
      for (int b = 0; b < NP; ++b) acc[v] += mw[j * NP + b] * (double)qe[v * N + b * NP];
    }
    for (int k = 0; k < 3 * N; ++k)
      if (!isfinite((double)qe[k])) acc[3] += 1.0;
  }
  block_sum4<kMassThreads>(acc, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) partial[blockIdx.x * 4 + k] = acc[k];
}

__global__ __launch_bounds__(kMassThreads) void k_mass_final(const double *__restrict__ partial,
                                                             int nblocks, double *__restrict__ out4) {
  __shared__ double sh[4 * kMassThreads];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kMassThreads)
    for (int k = 0; k < 4; ++k) acc[k] += partial[b * 4 + k];
  block_sum4<kMassThreads>(acc, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) out4[k] = acc[k];
}

// ------------------------------------------------------------------ dispatch
template <typename T, int NP>
static StageArgs<T, NP> stage_args(const StageLaunch &a) {
  StageArgs<T, NP> A;
  A.q = static_cast<const T *>(a.q);
  A.q0 = static_cast<const T *>(a.q0);
  A.out = static_cast<T *>(a.out);
  A.forcing = static_cast<const T *>(a.forcing);
  A.qa = static_cast<const T *>(a.qa);
  A.qb = static_cast<const T *>(a.qb);
  A.ca = T(a.ca);
  A.cb = T(a.cb);
  A.gt = static_cast<const GlobTab<T, NP> *>(a.glob);
  A.rows = static_cast<const RowTab<T, NP> *>(a.rows);
  A.n_lon = a.n_lon;
  A.n_lat = a.n_lat;
  A.alpha_global = a.alpha_global;
  A.periodic_y = a.periodic_y;
  A.combine = a.combine;
  A.c0 = T(a.c0);
  A.c1 = T(a.c1);
  A.ce = T(a.c0 + a.c1 - 1.0);
  A.dt = T(a.dt);
  A.levels = a.levels;
  A.lstride = (long long)a.E * 3 * NP * NP;
  return A;
}

template <typename T, int NP>
static hipError_t launch_stage_t(const StageLaunch &a, hipStream_t s) {
  if (a.levels < 1) return hipErrorInvalidValue;
  const StageArgs<T, NP> A = stage_args<T, NP>(a);
  if (a.variant == 1) {
    constexpr int GPW = ShapeH2<T, NP>::GPW;
    const int segs = (a.n_lon + GPW - 1) / GPW;
    // rows that end in a partly filled wavefront: pack the elements across
    // row ends instead (a wavefront then spans at most two rows)
    const bool packed = GPW <= a.n_lon && a.n_lon % GPW != 0;
    const int per = packed ? (a.n_lon * a.n_lat + GPW - 1) / GPW : segs * a.n_lat;
    const int waves = per * a.levels;
    const dim3 grid(waves), block(64);
#define DGSW_H2(CM_)                                                                      \
  do {                                                                                    \
    if (packed) hipLaunchKernelGGL((k_dg_stage_h2<T, NP, 1, CM_, true>), grid, block, 0, s, A, segs); \
    else hipLaunchKernelGGL((k_dg_stage_h2<T, NP, 1, CM_, false>), grid, block, 0, s, A, segs);      \
  } while (0)
    switch (a.combine) {
      case 0: DGSW_H2(0); break;
      case 1: DGSW_H2(1); break;
      case 2: DGSW_H2(2); break;
      default:
        return hipErrorInvalidValue;
    }
#undef DGSW_H2
    return hipGetLastError();
  }
  constexpr int GPW = Shape<T, NP>::GPW;
  const int segs = (a.n_lon + GPW - 1) / GPW;
  const int waves = segs * a.n_lat * a.levels;
  const bool big = waves >= 4096;
  const dim3 grid(big ? (waves + 3) / 4 : waves), block(big ? 256 : 64);
  switch (a.combine) {
    case 0:
      if (big) hipLaunchKernelGGL((k_dg_stage<T, NP, 4, 0>), grid, block, 0, s, A, segs);
      else hipLaunchKernelGGL((k_dg_stage<T, NP, 1, 0>), grid, block, 0, s, A, segs);
      break;
    case 1:
      if (big) hipLaunchKernelGGL((k_dg_stage<T, NP, 4, 1>), grid, block, 0, s, A, segs);
      else hipLaunchKernelGGL((k_dg_stage<T, NP, 1, 1>), grid, block, 0, s, A, segs);
      break;
    case 2:
      if (big) hipLaunchKernelGGL((k_dg_stage<T, NP, 4, 2>), grid, block, 0, s, A, segs);
      else hipLaunchKernelGGL((k_dg_stage<T, NP, 1, 2>), grid, block, 0, s, A, segs);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int NP>
static hipError_t launch_mass_t(const void *q, const double *mw, int n_lon, int E, int levels,
                                double *partial, double *out4, hipStream_t s) {
  hipLaunchKernelGGL((k_mass_partial<T, NP>), dim3(kMassBlocks), dim3(kMassThreads), 0, s,
                     static_cast<const T *>(q), mw, n_lon, E, (long long)E * levels, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(kMassThreads), 0, s, partial, kMassBlocks, out4);
  return hipGetLastError();
}

hipError_t launch_stage(int dtype, int np, const StageLaunch &a, hipStream_t s) {
  DGSW_DISPATCH(dtype, np, launch_stage_t, a, s)
  return hipErrorInvalidValue;
}

hipError_t launch_mass(int dtype, int np, const void *q, const double *mw, int n_lon, int E,
                       int levels, double *partial, double *out4, hipStream_t s) {
  DGSW_DISPATCH(dtype, np, launch_mass_t, q, mw, n_lon, E, levels, partial, out4, s)
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ tables
template <typename T, int NP>
static void fill_glob_t(const HostTables &t, double g, double radius, double omega, double href,
                        double alpha, void *dst) {
  GlobTab<T, NP> G;
  std::memset(&G, 0, sizeof(G));
  for (int p = 0; p < NP; ++p)
    for (int a = 0; a < NP; ++a) { G.B[p][a] = T(t.B[p * NP + a]); G.D[p][a] = T(t.D[p * NP + a]); }
  for (int a = 0; a < NP; ++a) { G.Pp[a] = T(t.Pp[a]); G.Pm[a] = T(t.Pm[a]); G.w[a] = T(t.w[a]); }
  G.cF = T(2.0 / t.dlam);
  G.cG = T(2.0 / t.dth);
  G.g = T(g);
  G.invR = T(1.0 / radius);
  (void)omega;   // enters through the per-row source factors
  G.href = T(href);
  G.two_href = T(2.0 * href);
  G.alpha = T(alpha);
  std::memcpy(dst, &G, sizeof(G));
}

template <typename T, int NP>
static void fill_rows_t(const HostTables &t, void *dst) {
  RowTab<T, NP> *R = static_cast<RowTab<T, NP> *>(dst);
  for (int j = 0; j < t.n_lat; ++j) {
    RowTab<T, NP> r;
    std::memset(&r, 0, sizeof(r));
    for (int s = 0; s < NP; ++s) {
      r.cosn[s] = T(t.cosn[j * NP + s]);
      r.fc[s] = T(t.fc[j * NP + s]);
      r.snR[s] = T(t.snR[j * NP + s]);
      r.stR[s] = T(t.stR[j * NP + s]);
      for (int b = 0; b < NP; ++b) {
        r.BM[s][b] = T(t.BM[(j * NP + s) * NP + b]);
        r.DM[s][b] = T(t.DM[(j * NP + s) * NP + b]);
      }
      r.MN[s] = T(t.MN[j * NP + s]);
      r.MS[s] = T(t.MS[j * NP + s]);
    }
    r.ctop = T(t.ctop[j]);
    r.cbot = T(t.cbot[j]);
    std::memcpy(&R[j], &r, sizeof(r));
  }
}

template <typename T, int NP>
static size_t glob_bytes_t() { return sizeof(GlobTab<T, NP>); }
template <typename T, int NP>
static size_t rows_bytes_t(int n_lat) { return sizeof(RowTab<T, NP>) * (size_t)n_lat; }
template <typename T, int NP>
static int fill_glob_d(const HostTables &t, double g, double radius, double omega, double href,
                       double alpha, void *dst) {
  fill_glob_t<T, NP>(t, g, radius, omega, href, alpha, dst);
  return 0;
}
template <typename T, int NP>
static int fill_rows_d(const HostTables &t, void *dst) {
  fill_rows_t<T, NP>(t, dst);
  return 0;
}

size_t glob_bytes(int dtype, int np) {
  DGSW_DISPATCH(dtype, np, glob_bytes_t)
  return 0;
}

size_t rows_bytes(int dtype, int np, int n_lat) {
  DGSW_DISPATCH(dtype, np, rows_bytes_t, n_lat)
  return 0;
}

static int fill_glob_i(int dtype, int np, const HostTables &t, double g, double radius,
                       double omega, double href, double alpha, void *dst) {
  DGSW_DISPATCH(dtype, np, fill_glob_d, t, g, radius, omega, href, alpha, dst)
  return -1;
}

static int fill_rows_i(int dtype, int np, const HostTables &t, void *dst) {
  DGSW_DISPATCH(dtype, np, fill_rows_d, t, dst)
  return -1;
}

void fill_glob(int dtype, int np, const HostTables &t, double g, double radius, double omega,
               double href, double alpha, void *dst) {
  (void)fill_glob_i(dtype, np, t, g, radius, omega, href, alpha, dst);
}

void fill_rows(int dtype, int np, const HostTables &t, void *dst) {
  (void)fill_rows_i(dtype, np, t, dst);
}

}  // namespace dgsw
