// Ensemble stage kernels: many meshes of different size and order in one
// launch per stage (or one per order); the stage itself is in dgsw_stage.hpp.
#include "dgsw_stage.hpp"

namespace dgsw {

// ------------------------------------------------------------------ ensemble
// LDS of one wavefront for any order up to NPMAX
constexpr int lds_tab(int k) { return (2 * k * k + k + 63) / 64 * 64; }   // Shape<T, k>::TB
constexpr int lds_sh(int k) {
  return (64 / k + 1) * ((3 * (k + 2) * k + 12 * k) > (6 * k * k + 6 * k) ? (3 * (k + 2) * k + 12 * k)
                                                                           : (6 * k * k + 6 * k));
}
constexpr int lds_max_tab(int npmax) { return npmax == 0 ? 0 : (lds_tab(npmax) > lds_max_tab(npmax - 1) ? lds_tab(npmax) : lds_max_tab(npmax - 1)); }
constexpr int lds_max_sh(int npmax) { return npmax == 0 ? 0 : (lds_sh(npmax) > lds_max_sh(npmax - 1) ? lds_sh(npmax) : lds_max_sh(npmax - 1)); }

template <typename T, int NP, int CM>
__device__ __forceinline__ void ens_case(const EnsItem &m, const unsigned char *__restrict__ tabs, const T *q,
                                         const T *q0, T *out, int combine, T c0, T ce, int lane, T *tab, T *sh) {
  static_assert(Shape<T, NP>::TB <= lds_tab(NP) && (Shape<T, NP>::GPW + 1) * Shape<T, NP>::SH <= lds_sh(NP),
                "the fused kernel's LDS slices hold this order's");
  StageArgs<T, NP> A;
  A.q = q + m.off;
  A.q0 = q0 ? q0 + m.off : nullptr;
  A.out = out + m.off;
  A.forcing = nullptr;
  A.qa = A.qb = nullptr;
  A.ca = A.cb = T(0);
  A.gt = reinterpret_cast<const GlobTab<T, NP> *>(tabs + m.glob);
  A.rows = reinterpret_cast<const RowTab<T, NP> *>(tabs + m.rows);
  A.n_lon = m.n_lon;
  A.n_lat = m.n_lat;
  A.alpha_global = m.alpha_global;
  A.periodic_y = 0;
  A.combine = combine;
  A.c0 = c0;
  A.c1 = T(0);
  A.ce = ce;
  A.dt = T(m.dt);
  stage_wave<T, NP, CM>(A, m.j, m.seg, lane, tab, sh);
}

// One launch per Runge-Kutta stage for a whole ensemble of meshes of different
// size and order, packed back to back in q / q0 / out.  Work unit: one
// wavefront of one member (items[k] = {member, wave index}).  Workgroup b
// (renumbered so each XCD gets a contiguous range) works through the
// contiguous item range [bounds[b], bounds[b+1]), balanced by cost on the host;
// its WPB wavefronts take every WPB-th item.  The order of each member is a
// wave-uniform switch.
template <typename T, int NPMAX, int WPB, int CM>
__global__ __launch_bounds__(64 * WPB) void k_ens_stage(const T *__restrict__ q, const T *q0, T *out,
                                                        const unsigned char *__restrict__ tabs,
                                                        const EnsItem *__restrict__ items,
                                                        const int *__restrict__ bounds, int combine,
                                                        T c0, T ce) {
  __shared__ T tab_all[WPB][lds_max_tab(NPMAX)];
  __shared__ T sh_all[WPB][lds_max_sh(NPMAX)];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  T *tab = tab_all[wv], *sh = sh_all[wv];
  const int part = xcd_block(blockIdx.x, gridDim.x);
  const int end = bounds[part + 1];
  for (int it = bounds[part] + wv; it < end; it += WPB) {
    const EnsItem m = items[it];
    switch (m.np) {
      case 1: ens_case<T, 1, CM>(m, tabs, q, q0, out, combine, c0, ce, lane, tab, sh); break;
      case 2: ens_case<T, 2, CM>(m, tabs, q, q0, out, combine, c0, ce, lane, tab, sh); break;
      case 3: ens_case<T, 3, CM>(m, tabs, q, q0, out, combine, c0, ce, lane, tab, sh); break;
      case 4: ens_case<T, 4, CM>(m, tabs, q, q0, out, combine, c0, ce, lane, tab, sh); break;
      case 5: ens_case<T, 5, CM>(m, tabs, q, q0, out, combine, c0, ce, lane, tab, sh); break;
      default:
        if constexpr (NPMAX > 5) {
          switch (m.np) {
            case 6: ens_case<T, (NPMAX > 5 ? 6 : 1), CM>(m, tabs, q, q0, out, combine, c0, ce, lane, tab, sh); break;
            case 7: ens_case<T, (NPMAX > 6 ? 7 : 1), CM>(m, tabs, q, q0, out, combine, c0, ce, lane, tab, sh); break;
            case 8: ens_case<T, (NPMAX > 7 ? 8 : 1), CM>(m, tabs, q, q0, out, combine, c0, ce, lane, tab, sh); break;
            default: break;
          }
        }
        break;
    }
  }
}

// The same for the half layout (2 NP lanes per element); items give their
// element range.
template <typename T, int NP>
__device__ __forceinline__ StageArgs<T, NP> ens_args(const EnsItem &m, const unsigned char *__restrict__ tabs,
                                                     const T *q, const T *q0, T *out, int combine, T c0, T ce) {
  StageArgs<T, NP> A;
  A.q = q + m.off;
  A.q0 = q0 ? q0 + m.off : nullptr;
  A.out = out + m.off;
  A.forcing = nullptr;
  A.qa = A.qb = nullptr;
  A.ca = A.cb = T(0);
  A.gt = reinterpret_cast<const GlobTab<T, NP> *>(tabs + m.glob);
  A.rows = reinterpret_cast<const RowTab<T, NP> *>(tabs + m.rows);
  A.n_lon = m.n_lon;
  A.n_lat = m.n_lat;
  A.alpha_global = m.alpha_global;
  A.periodic_y = 0;
  A.combine = combine;
  A.c0 = c0;
  A.c1 = T(0);
  A.ce = ce;
  A.dt = T(m.dt);
  A.levels = 1;
  A.lstride = 0;
  return A;
}

// LDS of one wavefront per layout: the line and half variants
template <typename T, int NP, int LAY>
struct EnsLds {
  static constexpr int TB = LAY == 0 ? Shape<T, NP>::TB : ShapeH2<T, NP>::TB;
  static constexpr int SH = LAY == 0 ? (Shape<T, NP>::GPW + 1) * Shape<T, NP>::SH
                                     : ShapeH2<T, NP>::SLOTS * ShapeH2<T, NP>::SH;
};

template <typename T, int NP, int LAY, int CM>
__device__ __forceinline__ void ens_item(const EnsItem &m, const unsigned char *__restrict__ tabs, const T *q,
                                         const T *q0, T *out, int combine, T c0, T ce, int lane, T *tab, T *sh) {
  if constexpr (LAY == 0) {
    ens_case<T, NP, CM>(m, tabs, q, q0, out, combine, c0, ce, lane, tab, sh);
  } else {
    stage_wave_h2<T, NP, CM, true>(ens_args<T, NP>(m, tabs, q, q0, out, combine, c0, ce), m.j, m.seg, m.e_end, lane,
                                   tab, sh);
  }
}

// Ensemble stage restricted to the members of one order and layout (the work
// list is sorted by both; bounds cover this group's items): the kernel is
// compiled for that order and layout alone, so it keeps their register
// budget and occupancy.
template <typename T, int NP, int LAY, int WPB, int CM>
__global__ __launch_bounds__(64 * WPB) void k_ens_stage_np(const T *__restrict__ q, const T *q0, T *out,
                                                           const unsigned char *__restrict__ tabs,
                                                           const EnsItem *__restrict__ items,
                                                           const int *__restrict__ bounds, int combine,
                                                           T c0, T ce) {
  __shared__ T tab_all[WPB][EnsLds<T, NP, LAY>::TB];
  __shared__ T sh_all[WPB][EnsLds<T, NP, LAY>::SH];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int part = xcd_block(blockIdx.x, gridDim.x);
  const int end = bounds[part + 1];
  for (int it = bounds[part] + wv; it < end; it += WPB) {
    const EnsItem m = items[it];
    ens_item<T, NP, LAY, CM>(m, tabs, q, q0, out, combine, c0, ce, lane, tab_all[wv], sh_all[wv]);
  }
}

// Flat form: workgroup b takes items begin + b*WPB + wv, one item per
// wavefront, so the hardware schedules the ensemble like an ordinary grid
// (no loop: same register budget as the single-mesh kernel).
template <typename T, int NP, int LAY, int WPB, int CM>
__global__ __launch_bounds__(64 * WPB) void k_ens_stage_flat(const T *__restrict__ q, const T *q0, T *out,
                                                             const unsigned char *__restrict__ tabs,
                                                             const EnsItem *__restrict__ items,
                                                             int begin, int end, int combine, T c0, T ce) {
  __shared__ T tab_all[WPB][EnsLds<T, NP, LAY>::TB];
  __shared__ T sh_all[WPB][EnsLds<T, NP, LAY>::SH];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int it = begin + xcd_block(blockIdx.x, gridDim.x) * WPB + wv;
  if (it >= end) return;
  const EnsItem m = items[it];
  ens_item<T, NP, LAY, CM>(m, tabs, q, q0, out, combine, c0, ce, lane, tab_all[wv], sh_all[wv]);
}

// the combination mode is a template parameter of the ensemble kernels too:
// 0 (right-hand side) or 1 (Shu-Osher stage)
template <typename T, int NP, int LAY, int WPB>
static hipError_t launch_ens_flat_t(const EnsLaunch &a, hipStream_t s) {
  const int n = a.end - a.begin;
  const dim3 grid((n + WPB - 1) / WPB), block(64 * WPB);
  if (a.combine)
    hipLaunchKernelGGL((k_ens_stage_flat<T, NP, LAY, WPB, 1>), grid, block, 0, s, static_cast<const T *>(a.q),
                       static_cast<const T *>(a.q0), static_cast<T *>(a.out),
                       static_cast<const unsigned char *>(a.tabs), a.items, a.begin, a.end, 1, T(a.c0),
                       T(a.c0 + a.c1 - 1.0));
  else
    hipLaunchKernelGGL((k_ens_stage_flat<T, NP, LAY, WPB, 0>), grid, block, 0, s, static_cast<const T *>(a.q),
                       static_cast<const T *>(a.q0), static_cast<T *>(a.out),
                       static_cast<const unsigned char *>(a.tabs), a.items, a.begin, a.end, 0, T(a.c0),
                       T(a.c0 + a.c1 - 1.0));
  return hipGetLastError();
}

template <typename T, int NP, int LAY, int WPB>
static hipError_t launch_ens_np_t(const EnsLaunch &a, hipStream_t s) {
  if (a.combine)
    hipLaunchKernelGGL((k_ens_stage_np<T, NP, LAY, WPB, 1>), dim3(a.parts), dim3(64 * WPB), 0, s,
                       static_cast<const T *>(a.q), static_cast<const T *>(a.q0), static_cast<T *>(a.out),
                       static_cast<const unsigned char *>(a.tabs), a.items,
                       a.bounds, 1, T(a.c0), T(a.c0 + a.c1 - 1.0));
  else
    hipLaunchKernelGGL((k_ens_stage_np<T, NP, LAY, WPB, 0>), dim3(a.parts), dim3(64 * WPB), 0, s,
                       static_cast<const T *>(a.q), static_cast<const T *>(a.q0), static_cast<T *>(a.out),
                       static_cast<const unsigned char *>(a.tabs), a.items,
                       a.bounds, 0, T(a.c0), T(a.c0 + a.c1 - 1.0));
  return hipGetLastError();
}

template <typename T, int NP, int LAY>
static hipError_t launch_ens_np_l(int wpb, const EnsLaunch &a, hipStream_t s) {
  if (a.flat) {
    switch (wpb) {
      case 1: return launch_ens_flat_t<T, NP, LAY, 1>(a, s);
      case 2: return launch_ens_flat_t<T, NP, LAY, 2>(a, s);
      case 4: return launch_ens_flat_t<T, NP, LAY, 4>(a, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (wpb) {
    case 1: return launch_ens_np_t<T, NP, LAY, 1>(a, s);
    case 2: return launch_ens_np_t<T, NP, LAY, 2>(a, s);
    case 4: return launch_ens_np_t<T, NP, LAY, 4>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int NP>
static hipError_t launch_ens_np_w(int layout, int wpb, const EnsLaunch &a, hipStream_t s) {
  switch (layout) {
    case 0: return launch_ens_np_l<T, NP, 0>(wpb, a, s);
    case 1: return launch_ens_np_l<T, NP, 1>(wpb, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ens_stage_np(int dtype, int np, int layout, int wpb, const EnsLaunch &a, hipStream_t s) {
  DGSW_DISPATCH(dtype, np, launch_ens_np_w, layout, wpb, a, s)
  return hipErrorInvalidValue;
}

template <typename T, int NPMAX, int WPB>
static hipError_t launch_ens_t(const EnsLaunch &a, hipStream_t s) {
  if (a.combine)
    hipLaunchKernelGGL((k_ens_stage<T, NPMAX, WPB, 1>), dim3(a.parts), dim3(64 * WPB), 0, s,
                       static_cast<const T *>(a.q), static_cast<const T *>(a.q0), static_cast<T *>(a.out),
                       static_cast<const unsigned char *>(a.tabs), a.items,
                       a.bounds, 1, T(a.c0), T(a.c0 + a.c1 - 1.0));
  else
    hipLaunchKernelGGL((k_ens_stage<T, NPMAX, WPB, 0>), dim3(a.parts), dim3(64 * WPB), 0, s,
                       static_cast<const T *>(a.q), static_cast<const T *>(a.q0), static_cast<T *>(a.out),
                       static_cast<const unsigned char *>(a.tabs), a.items,
                       a.bounds, 0, T(a.c0), T(a.c0 + a.c1 - 1.0));
  return hipGetLastError();
}

hipError_t launch_ens_stage(int dtype, int npmax, int wpb, const EnsLaunch &a, hipStream_t s) {
#define DGSW_ENS(NPM, W)                                                                  \
  if (npmax <= NPM && wpb == W)                                                           \
    return dtype == 0 ? launch_ens_t<double, NPM, W>(a, s) : launch_ens_t<float, NPM, W>(a, s);
  DGSW_ENS(5, 1) DGSW_ENS(5, 2) DGSW_ENS(5, 4) DGSW_ENS(8, 1) DGSW_ENS(8, 2) DGSW_ENS(8, 4)
#undef DGSW_ENS
  return hipErrorInvalidValue;
}

}  // namespace dgsw
