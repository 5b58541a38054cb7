// Planar linear advection du/dt + div(beta u) = 0 on the periodic rectangle
// (section 4.1's convergence test; equation "lin_adv"), C ABI declared in
// include/dgsw.h.
//
// The discretisation is the shallow-water one with a linear flux: orthonormal
// Legendre tensor basis, (r+1)-point Gauss-Legendre volume and edge rules,
// the weak form of equation "dg_parts", the Rusanov flux of equation
// "rusanov" (for f(u) = b u it is the upwind flux) and the mass matrix
// (dx dy / 4) I.  Because the operator is linear and the mesh uniform, the host
// assembles it once into five N x N matrices, one per stencil slot (the
// element and its east, west, north and south neighbours); a stage is then
// dq_e/dt = sum_k A_k q_{neighbour k of e}, a dense contraction of length 5N
// per output mode.  Work unit: one (element, mode) per lane; the matrices
// and the workgroup's stencil rows are staged in LDS.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "dgsw.h"
#include "dgsw_ctx.hpp"
#include "dgsw_tables.hpp"

using dgsw::aligned16;
using dgsw::fail;
using dgsw::hip_fail;

struct dg_adv {
  dg_adv_desc d;
  int np = 0, N = 0, E = 0;
  int64_t state_n = 0;
  size_t elem_bytes = 0;
  void *d_ops = nullptr;     // [5][N][N] in the state dtype
};

namespace {

constexpr int kSlots = 5;    // self, east, west, north, south

// Residual contribution, to every output mode of one element, of a single
// unit coefficient n in stencil slot `slot` (so column n of A_slot): the
// volume term for the element itself and the upwind surface terms of the edge
// shared with that neighbour.  Host FP64; M^-1 = 4 / (dx dy) applied at the end.
void assemble(int np, double dx, double dy, double bx, double by, std::vector<double> &A) {
  const int N = np * np;
  std::vector<double> x, w;
  dgsw::gauss_legendre(np, x, w);
  std::vector<double> P(np * np), D(np * np), Pp(np), Pm(np);
  double pv[dgsw::kMaxNP], dv[dgsw::kMaxNP];
  for (int p = 0; p < np; ++p) {
    dgsw::legendre_onb(np - 1, x[p], pv, dv);
    for (int a = 0; a < np; ++a) { P[p * np + a] = pv[a]; D[p * np + a] = dv[a]; }
  }
  dgsw::legendre_onb(np - 1, 1.0, pv, dv);
  for (int a = 0; a < np; ++a) Pp[a] = pv[a];
  dgsw::legendre_onb(np - 1, -1.0, pv, dv);
  for (int a = 0; a < np; ++a) Pm[a] = pv[a];
  A.assign((size_t)kSlots * N * N, 0.0);
  auto at = [&](int slot, int m, int n) -> double & { return A[((size_t)slot * N + m) * N + n]; };
  const double minv = 4.0 / (dx * dy);
  for (int m = 0; m < N; ++m) {
    const int am = m % np, bm = m / np;
    for (int n = 0; n < N; ++n) {
      const int an = n % np, bn = n / np;
      // volume: (dy/2) int bx u dphi/dxi + (dx/2) int by u dphi/deta, by quadrature
      double vol = 0.0;
      for (int s = 0; s < np; ++s)
        for (int p = 0; p < np; ++p) {
          const double u = P[p * np + an] * P[s * np + bn];
          vol += w[p] * w[s] * u *
                 (0.5 * dy * bx * D[p * np + am] * P[s * np + bm] + 0.5 * dx * by * P[p * np + am] * D[s * np + bm]);
        }
      at(0, m, n) += minv * vol;
      // x edges: flux bx u_upwind at the edge nodes eta_s, weight (dy/2) w_s
      for (int s = 0; s < np; ++s) {
        const double ws = 0.5 * dy * w[s] * P[s * np + bm] * P[s * np + bn];
        // east edge (xi = +1 of this element, -1 of the east neighbour): - F^ phi_m(+1)
        if (bx >= 0.0) at(0, m, n) -= minv * ws * bx * Pp[an] * Pp[am];
        else at(1, m, n) -= minv * ws * bx * Pm[an] * Pp[am];
        // west edge (xi = -1 of this element, +1 of the west neighbour): + F^ phi_m(-1)
        if (bx >= 0.0) at(2, m, n) += minv * ws * bx * Pp[an] * Pm[am];
        else at(0, m, n) += minv * ws * bx * Pm[an] * Pm[am];
      }
      // y edges, the same with by, dx and eta
      for (int p = 0; p < np; ++p) {
        const double wp = 0.5 * dx * w[p] * P[p * np + am] * P[p * np + an];
        if (by >= 0.0) at(0, m, n) -= minv * wp * by * Pp[bn] * Pp[bm];
        else at(3, m, n) -= minv * wp * by * Pm[bn] * Pp[bm];
        if (by >= 0.0) at(4, m, n) += minv * wp * by * Pp[bn] * Pm[bm];
        else at(0, m, n) += minv * wp * by * Pm[bn] * Pm[bm];
      }
    }
  }
}

struct AdvArgs {
  const void *q, *q0, *qa, *qb;
  void *out;
  int nx, ny, N, combine;          // combine: 0 rhs, 1 Shu-Osher, 2 general (as the SWE stages)
  double c0, c1, ce, dt, ca, cb;
};

// One lane per (element, output mode), G = 256 / N consecutive elements per
// workgroup.  The five matrices and the G elements' five stencil rows are
// staged in LDS (the rows with coalesced loads, one value per lane per slot),
// then every lane contracts its output row of each matrix with its element's
// rows: 5N multiply-adds from LDS.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_adv_stage(const T *__restrict__ ops, const T *__restrict__ q,
                                                   const T *q0, const T *qa, const T *qb, T *out, int nx, int ny,
                                                   int combine, T c0, T c1, T ce, T dt, T ca, T cb) {
  constexpr int G = 256 / N;
  // padded strides: rows of different output modes / elements start in
  // different LDS banks
  constexpr int LA = N + 1, LQ = kSlots * N + 1;
  __shared__ T sA[kSlots * N * LA];
  __shared__ T sQ[G * LQ];
  for (int k = threadIdx.x; k < kSlots * N * N; k += 256) sA[(k / N) * LA + k % N] = ops[k];
  const int64_t E = (int64_t)nx * ny;
  const int g = threadIdx.x / N, m = threadIdx.x - g * N;
  const int64_t e64 = (int64_t)blockIdx.x * G + g;
  const bool live = g < G && e64 < E;
  const int e = live ? (int)e64 : 0;
  const int j = e / nx, i = e - j * nx;
  if (g < G) {
    const int nb[kSlots] = {e, j * nx + (i + 1 == nx ? 0 : i + 1), j * nx + (i == 0 ? nx - 1 : i - 1),
                            (j + 1 == ny ? 0 : j + 1) * nx + i, (j == 0 ? ny - 1 : j - 1) * nx + i};
#pragma unroll
    for (int k = 0; k < kSlots; ++k) sQ[g * LQ + k * N + m] = q[(size_t)nb[k] * N + m];
  }
  __syncthreads();
  if (!live) return;
  T acc = T(0);
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    const T *row = sA + (k * N + m) * LA;
    const T *src = sQ + g * LQ + k * N;
#pragma unroll
    for (int n = 0; n < N; ++n) acc += row[n] * src[n];
  }
  const size_t o = (size_t)e * N + m;
  const T qo = sQ[g * LQ + m];
  T res;
  if (combine == 2) {
    const T b0 = q0[o];
    res = b0 + dt * acc + (c1 * (qo - b0) + ((qa ? ca * (qa[o] - b0) : T(0)) + (qb ? cb * (qb[o] - b0) : T(0))));
  } else if (combine == 1) {
    const T y = qo + dt * acc;
    res = y + c0 * ((c0 != T(0) ? q0[o] : T(0)) - y) + ce * y;
  } else {
    res = acc;
  }
  out[o] = res;
}

template <typename T, int N>
hipError_t launch_adv_t(const dg_adv *a, const AdvArgs &g, hipStream_t s) {
  constexpr int G = 256 / N;
  const int64_t E = (int64_t)g.nx * g.ny;
  const dim3 grid((unsigned)((E + G - 1) / G)), block(256);
  hipLaunchKernelGGL((k_adv_stage<T, N>), grid, block, 0, s, static_cast<const T *>(a->d_ops),
                     static_cast<const T *>(g.q), static_cast<const T *>(g.q0), static_cast<const T *>(g.qa),
                     static_cast<const T *>(g.qb), static_cast<T *>(g.out), g.nx, g.ny, g.combine, T(g.c0), T(g.c1),
                     T(g.ce), T(g.dt), T(g.ca), T(g.cb));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adv_d(const dg_adv *a, const AdvArgs &g, hipStream_t s) {
  switch (a->np) {
    case 1: return launch_adv_t<T, 1>(a, g, s);
    case 2: return launch_adv_t<T, 4>(a, g, s);
    case 3: return launch_adv_t<T, 9>(a, g, s);
    case 4: return launch_adv_t<T, 16>(a, g, s);
    case 5: return launch_adv_t<T, 25>(a, g, s);
    case 6: return launch_adv_t<T, 36>(a, g, s);
    case 7: return launch_adv_t<T, 49>(a, g, s);
    default: return hipErrorInvalidValue;
  }
}

int adv_stage(dg_adv *a, const void *q, const void *q0, void *out, int combine, double c0, double c1, double dt,
              const void *qa, double ca, const void *qb, double cb, hipStream_t s) {
  AdvArgs g;
  g.q = q; g.q0 = q0; g.qa = qa; g.qb = qb; g.out = out;
  g.nx = a->d.nx; g.ny = a->d.ny; g.N = a->N; g.combine = combine;
  g.c0 = c0; g.c1 = c1; g.ce = c0 + c1 - 1.0; g.dt = dt; g.ca = ca; g.cb = cb;
  hipError_t e = a->d.dtype == DG_F64 ? launch_adv_d<double>(a, g, s) : launch_adv_d<float>(a, g, s);
  if (e != hipSuccess) return hip_fail(e, "advection stage launch");
  return DG_OK;
}

}  // namespace

extern "C" {

int dg_adv_init(const dg_adv_desc *d, void *hip_stream, dg_adv **out) {
  if (!out) return fail(DG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d) return fail(DG_EINVAL, "desc is NULL");
  if (d->abi_version != DG_ABI_VERSION) return fail(DG_EINVAL, "abi_version mismatch");
  if (d->nx < 1 || d->ny < 1) return fail(DG_EINVAL, "nx and ny must be >= 1");
  if (d->order < 0) return fail(DG_EINVAL, "order must be >= 0");
  if (d->order > 6) return fail(DG_EUNSUPPORTED, "order > 6 is not supported for advection");
  if (d->reserved != 0) return fail(DG_EINVAL, "reserved must be 0");
  if (d->dtype != DG_F64 && d->dtype != DG_F32) return fail(DG_EDTYPE, "dtype must be DG_F64 or DG_F32");
  if (!(d->lx > 0.0) || !std::isfinite(d->lx) || !(d->ly > 0.0) || !std::isfinite(d->ly))
    return fail(DG_EINVAL, "lx and ly must be > 0");
  if (!std::isfinite(d->bx) || !std::isfinite(d->by)) return fail(DG_EINVAL, "beta must be finite");
  const int64_t np = d->order + 1;
  if ((int64_t)d->nx * d->ny * np * np >= (int64_t(1) << 31)) return fail(DG_EINVAL, "state exceeds 2^31 values");
  dg_adv *a = new dg_adv();
  a->d = *d;
  a->np = (int)np;
  a->N = (int)(np * np);
  a->E = d->nx * d->ny;
  a->state_n = (int64_t)a->E * a->N;
  a->elem_bytes = d->dtype == DG_F64 ? 8 : 4;
  std::vector<double> A;
  assemble(a->np, d->lx / d->nx, d->ly / d->ny, d->bx, d->by, A);
  std::vector<unsigned char> h(A.size() * a->elem_bytes);
  if (d->dtype == DG_F64) {
    std::memcpy(h.data(), A.data(), h.size());
  } else {
    for (size_t k = 0; k < A.size(); ++k) {
      const float f = (float)A[k];
      std::memcpy(h.data() + 4 * k, &f, 4);
    }
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e;
  if ((e = hipMalloc(&a->d_ops, h.size())) != hipSuccess) {
    delete a;
    return fail(DG_ENOMEM, "hipMalloc of the advection operator");
  }
  if ((e = hipMemcpyAsync(a->d_ops, h.data(), h.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess) {
    (void)hipFree(a->d_ops);
    delete a;
    return hip_fail(e, "upload of the advection operator");
  }
  *out = a;
  return DG_OK;
}

int dg_adv_free(dg_adv *a) {
  if (!a) return DG_OK;
  if (a->d_ops) (void)hipFree(a->d_ops);
  delete a;
  return DG_OK;
}

int dg_adv_state_size(const dg_adv *a, int64_t *n_values) {
  if (!a || !n_values) return fail(DG_EINVAL, "NULL argument");
  *n_values = a->state_n;
  return DG_OK;
}

int dg_adv_rhs(dg_adv *a, const void *q, void *dqdt, void *hip_stream) {
  if (!a || !q || !dqdt) return fail(DG_EINVAL, "NULL argument");
  if (!aligned16(q) || !aligned16(dqdt)) return fail(DG_EINVAL, "state pointers must be 16-byte aligned");
  const size_t bytes = a->state_n * a->elem_bytes;
  const char *x = static_cast<const char *>(q), *y = static_cast<const char *>(dqdt);
  if (x < y + bytes && y < x + bytes) return fail(DG_EINVAL, "q and dqdt overlap");
  return adv_stage(a, q, nullptr, dqdt, 0, 0.0, 1.0, 0.0, nullptr, 0.0, nullptr, 0.0,
                   static_cast<hipStream_t>(hip_stream));
}

int dg_adv_rk_step(dg_adv *a, void *q, void *work, double dt, int32_t scheme, int32_t nsteps, void *hip_stream) {
  if (!a || !q || !work) return fail(DG_EINVAL, "NULL argument");
  if (!aligned16(q) || !aligned16(work)) return fail(DG_EINVAL, "state pointers must be 16-byte aligned");
  if (nsteps < 0 || !std::isfinite(dt)) return fail(DG_EINVAL, "bad nsteps or dt");
  int nwork;
  switch (scheme) {
    case DG_SSP_RK1: nwork = 1; break;
    case DG_SSP_RK2:
    case DG_SSP_RK3: nwork = 2; break;
    case DG_RK4: nwork = 3; break;
    default: return fail(DG_EINVAL, "unknown scheme");
  }
  const size_t bytes = a->state_n * a->elem_bytes;
  {
    const char *x = static_cast<const char *>(q), *y = static_cast<const char *>(work);
    if (x < y + nwork * bytes && y < x + bytes) return fail(DG_EINVAL, "q and work overlap");
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  char *w0 = static_cast<char *>(work), *w1 = w0 + bytes, *w2 = w1 + bytes;
  int rc;
  for (int n = 0; n < nsteps; ++n) {
    switch (scheme) {
      case DG_SSP_RK1: {
        if ((rc = adv_stage(a, q, nullptr, w0, 1, 0.0, 1.0, dt, nullptr, 0, nullptr, 0, s)) != DG_OK) return rc;
        hipError_t e = hipMemcpyAsync(q, w0, bytes, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "RK1 copy-back");
        break;
      }
      case DG_SSP_RK2:
        if ((rc = adv_stage(a, q, nullptr, w0, 1, 0.0, 1.0, dt, nullptr, 0, nullptr, 0, s)) != DG_OK) return rc;
        if ((rc = adv_stage(a, w0, q, q, 1, 0.5, 0.5, dt, nullptr, 0, nullptr, 0, s)) != DG_OK) return rc;
        break;
      case DG_SSP_RK3:
        if ((rc = adv_stage(a, q, nullptr, w0, 1, 0.0, 1.0, dt, nullptr, 0, nullptr, 0, s)) != DG_OK) return rc;
        if ((rc = adv_stage(a, w0, q, w1, 1, 0.75, 0.25, dt, nullptr, 0, nullptr, 0, s)) != DG_OK) return rc;
        if ((rc = adv_stage(a, w1, q, q, 1, 1.0 / 3.0, 2.0 / 3.0, dt, nullptr, 0, nullptr, 0, s)) != DG_OK) return rc;
        break;
      case DG_RK4:
        if ((rc = adv_stage(a, q, nullptr, w0, 1, 0.0, 1.0, 0.5 * dt, nullptr, 0, nullptr, 0, s)) != DG_OK) return rc;
        if ((rc = adv_stage(a, w0, q, w1, 2, 1.0, 0.0, 0.5 * dt, nullptr, 0, nullptr, 0, s)) != DG_OK) return rc;
        if ((rc = adv_stage(a, w1, q, w2, 2, 1.0, 0.0, dt, nullptr, 0, nullptr, 0, s)) != DG_OK) return rc;
        if ((rc = adv_stage(a, w2, q, q, 2, 0.0, 1.0 / 3.0, dt / 6.0, w0, 1.0 / 3.0, w1, 2.0 / 3.0, s)) != DG_OK)
          return rc;
        break;
    }
  }
  return DG_OK;
}

}  // extern "C"
