// C ABI of libdgsw (declared in include/dgsw.h).
#include "dgsw.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dgsw_ctx.hpp"
#include "dgsw_device.hpp"
#include "dgsw_tables.hpp"

namespace dgsw {

static thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(DG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

const char *last_error() { return g_err.c_str(); }

}  // namespace dgsw

using dgsw::aligned16;
using dgsw::fail;
using dgsw::hip_fail;

namespace {

void release(dg_ctx *c) {
  if (!c) return;
  if (c->d_glob) (void)hipFree(c->d_glob);
  if (c->d_rows) (void)hipFree(c->d_rows);
  if (c->d_mass_w) (void)hipFree(c->d_mass_w);
  if (c->d_partial) (void)hipFree(c->d_partial);
  if (c->d_out4) (void)hipFree(c->d_out4);
  if (c->d_proj) (void)hipFree(c->d_proj);
  delete c;
}

int validate(const dg_mesh_desc *d) {
  if (!d) return fail(DG_EINVAL, "desc is NULL");
  if (d->abi_version != DG_ABI_VERSION) return fail(DG_EINVAL, "abi_version mismatch");
  if (d->n_lon < 1 || d->n_lat < 1) return fail(DG_EINVAL, "n_lon and n_lat must be >= 1");
  if (d->order < 0) return fail(DG_EINVAL, "order must be >= 0");
  if (d->order > dgsw::kMaxOrder) return fail(DG_EUNSUPPORTED, "order > 7 is not supported");
  if (d->dtype != DG_F64 && d->dtype != DG_F32) return fail(DG_EDTYPE, "dtype must be DG_F64 or DG_F32");
  if (d->metric != DG_METRIC_BALANCED && d->metric != DG_METRIC_POINTWISE)
    return fail(DG_EINVAL, "unknown metric");
  if (d->alpha_mode != DG_ALPHA_LOCAL && d->alpha_mode != DG_ALPHA_GLOBAL)
    return fail(DG_EINVAL, "unknown alpha_mode");
  if (d->reserved != 0) return fail(DG_EINVAL, "reserved must be 0");
  if (!(d->radius > 0.0) || !std::isfinite(d->radius)) return fail(DG_EINVAL, "radius must be > 0");
  if (!(d->gravity > 0.0) || !std::isfinite(d->gravity)) return fail(DG_EINVAL, "gravity must be > 0");
  if (!std::isfinite(d->omega)) return fail(DG_EINVAL, "omega must be finite");
  if (!(d->h_ref >= 0.0) || !std::isfinite(d->h_ref)) return fail(DG_EINVAL, "h_ref must be >= 0");
  if (d->h_ref != 0.0 && d->metric != DG_METRIC_BALANCED)
    return fail(DG_EINVAL, "h_ref > 0 requires DG_METRIC_BALANCED");
  if (d->alpha_mode == DG_ALPHA_GLOBAL && (!(d->alpha >= 0.0) || !std::isfinite(d->alpha)))
    return fail(DG_EINVAL, "alpha must be >= 0 with DG_ALPHA_GLOBAL");
  const int64_t np = d->order + 1;
  const int64_t vals = (int64_t)d->n_lon * d->n_lat * 3 * np * np;
  if (vals >= (int64_t(1) << 31)) return fail(DG_EINVAL, "state exceeds 2^31 values");
  return DG_OK;
}

}  // namespace

extern "C" {

const char *dg_last_error(void) { return dgsw::last_error(); }

}  // extern "C"

namespace {

// Context from validated parameters and the host tables of its geometry.
int make_ctx(const dg_mesh_desc *desc, const dgsw::HostTables &t, hipStream_t s, dg_ctx **out) {
  dg_ctx *c = new dg_ctx();
  c->d = *desc;
  c->periodic_y = t.periodic_y ? 1 : 0;
  // kernel layout, chosen from MI355X stage timings of both layouts over
  // r = 1..5, 90x45 .. 720x360 and both precisions: the half-line layout at
  // r = 1 (its 4 lanes per element against the line layout's 2), for FP64 at
  // r >= 5, where the line layout's registers allow only one wavefront per
  // SIMD, for FP64 at r = 3, where it holds four wavefronts per SIMD against
  // the line layout's two, and where the line layout leaves the GPU
  // latency-bound (at most 2048 wavefronts, about two per SIMD; at r >= 4,
  // where the work the two halves duplicate costs more, at most 512); the
  // line layout otherwise (dg_autotune measures instead)
  {
    const int waves_line = dgsw::waves_per_row(desc->order + 1, desc->n_lon) * desc->n_lat;
    const bool half = desc->order == 1 ||
                      (desc->dtype == DG_F64 && (desc->order >= 5 || desc->order == 3)) ||
                      waves_line <= (desc->order >= 4 ? 512 : 2048);
    c->kernel = half ? DG_KERNEL_HALF : DG_KERNEL_LINE;
  }
  c->np = desc->order + 1;
  c->N = c->np * c->np;
  c->E = desc->n_lon * desc->n_lat;
  c->state_n = (int64_t)c->E * 3 * c->N;
  c->level_n = c->state_n;
  c->levels = 1;
  c->elem_bytes = desc->dtype == DG_F64 ? 8 : 4;
  {
    double cmin = 1.0;
    for (double cv : t.cosn) cmin = cv < cmin ? cv : cmin;
    const double wl = t.dlam * cmin;
    c->min_width = desc->radius * (t.dth < wl ? t.dth : wl);
  }

  const int dt = desc->dtype == DG_F64 ? 0 : 1;
  const size_t gb = dgsw::glob_bytes(dt, c->np);
  const size_t rb = dgsw::rows_bytes(dt, c->np, desc->n_lat);
  std::vector<unsigned char> hg(gb), hr(rb);
  dgsw::fill_glob(dt, c->np, t, desc->gravity, desc->radius, desc->omega, desc->h_ref,
                  desc->alpha_mode == DG_ALPHA_GLOBAL ? desc->alpha : 0.0, hg.data());
  dgsw::fill_rows(dt, c->np, t, hr.data());

  // cos-weighted projection onto every order k = 0..7 on the same mesh, per
  // latitude row j: P_kj = Mk_j^-1 Mth_j[0..k][:], Mk_j the leading (k+1)^2
  // block of the latitude mass matrix (k <= r); for k > r the state already
  // lies in the target space and the rows are the identity (embedding)
  const int npp = c->np;
  std::vector<double> proj((size_t)desc->n_lat * npp * dgsw::proj_rows_total(), 0.0);
  for (int j = 0; j < desc->n_lat; ++j) {
    const double *Mj = &t.Mth[(size_t)j * npp * npp];
    c->mass_area += desc->n_lon * t.mass_w[(size_t)j * npp + 0];
    for (int k = 0; k <= dgsw::kMaxOrder; ++k) {
      const int nk = k + 1;
      double *Pk = &proj[dgsw::proj_offset(k, desc->n_lat, npp) + (size_t)j * nk * npp];
      if (k >= npp - 1) {
        for (int b = 0; b < npp; ++b) Pk[b * npp + b] = 1.0;
        continue;
      }
      // Gauss-Jordan on [Mk | Mth rows 0..k]: the left block is symmetric
      // positive definite (a Gram matrix), so no pivoting is needed
      double A[dgsw::kMaxNP][dgsw::kMaxNP], X[dgsw::kMaxNP][dgsw::kMaxNP];
      for (int r = 0; r < nk; ++r)
        for (int cc = 0; cc < nk; ++cc) A[r][cc] = Mj[r * npp + cc];
      for (int r = 0; r < nk; ++r)
        for (int b = 0; b < npp; ++b) X[r][b] = Mj[r * npp + b];
      for (int piv = 0; piv < nk; ++piv) {
        const double d = 1.0 / A[piv][piv];
        for (int cc = 0; cc < nk; ++cc) A[piv][cc] *= d;
        for (int b = 0; b < npp; ++b) X[piv][b] *= d;
        for (int r = 0; r < nk; ++r) {
          if (r == piv) continue;
          const double f = A[r][piv];
          for (int cc = 0; cc < nk; ++cc) A[r][cc] -= f * A[piv][cc];
          for (int b = 0; b < npp; ++b) X[r][b] -= f * X[piv][b];
        }
      }
      for (int r = 0; r < nk; ++r)
        for (int b = 0; b < npp; ++b) Pk[r * npp + b] = X[r][b];
    }
  }

  hipError_t e;
  c->glob_bytes = gb;
  c->rows_bytes = rb;
  if ((e = hipMalloc(&c->d_glob, gb)) != hipSuccess ||
      (e = hipMalloc(&c->d_rows, rb)) != hipSuccess ||
      (e = hipMalloc(reinterpret_cast<void **>(&c->d_mass_w), t.mass_w.size() * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(reinterpret_cast<void **>(&c->d_partial), dgsw::mass_blocks() * 4 * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(reinterpret_cast<void **>(&c->d_out4), 4 * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(reinterpret_cast<void **>(&c->d_proj), proj.size() * sizeof(double))) != hipSuccess) {
    release(c);
    return fail(DG_ENOMEM, std::string("hipMalloc of context tables: ") + hipGetErrorString(e));
  }
  if ((e = hipMemcpyAsync(c->d_glob, hg.data(), gb, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(c->d_rows, hr.data(), rb, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(c->d_mass_w, t.mass_w.data(), t.mass_w.size() * sizeof(double),
                          hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(c->d_proj, proj.data(), proj.size() * sizeof(double), hipMemcpyHostToDevice,
                          s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess) {
    release(c);
    return hip_fail(e, "upload of context tables");
  }
  *out = c;
  return DG_OK;
}

}  // namespace

extern "C" {

int dg_init_mesh(const dg_mesh_desc *desc, void *hip_stream, dg_ctx **out) {
  if (!out) return fail(DG_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(desc);
  if (rc != DG_OK) return rc;
  dgsw::HostTables t;
  const char *msg = "";
  if (!dgsw::build_tables(desc->n_lon, desc->n_lat, desc->order,
                          desc->metric == DG_METRIC_BALANCED ? 0 : 1, desc->radius, desc->omega,
                          t, &msg))
    return fail(DG_EINVAL, msg);
  return make_ctx(desc, t, static_cast<hipStream_t>(hip_stream), out);
}

int dg_init_plane(const dg_plane_desc *p, void *hip_stream, dg_ctx **out) {
  if (!out) return fail(DG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p) return fail(DG_EINVAL, "desc is NULL");
  if (p->abi_version != DG_ABI_VERSION) return fail(DG_EINVAL, "abi_version mismatch");
  if (!(p->lx > 0.0) || !std::isfinite(p->lx) || !(p->ly > 0.0) || !std::isfinite(p->ly))
    return fail(DG_EINVAL, "lx and ly must be > 0");
  if (!std::isfinite(p->f)) return fail(DG_EINVAL, "f must be finite");
  // the sphere descriptor with the plane's values: validated by the same rules
  dg_mesh_desc d{};
  d.abi_version = p->abi_version;
  d.n_lon = p->nx;
  d.n_lat = p->ny;
  d.order = p->order;
  d.dtype = p->dtype;
  d.metric = DG_METRIC_BALANCED;
  d.alpha_mode = p->alpha_mode;
  d.reserved = 0;
  d.alpha = p->alpha;
  d.radius = 1.0;
  d.gravity = p->gravity;
  d.omega = 0.0;
  d.h_ref = p->h_ref;
  int rc = validate(&d);
  if (rc != DG_OK) return rc;
  dgsw::HostTables t;
  const char *msg = "";
  if (!dgsw::build_tables_plane(p->nx, p->ny, p->order, p->lx, p->ly, p->f, t, &msg))
    return fail(DG_EINVAL, msg);
  return make_ctx(&d, t, static_cast<hipStream_t>(hip_stream), out);
}

int dg_set_kernel(dg_ctx *ctx, int32_t kernel) {
  if (!ctx) return fail(DG_EINVAL, "ctx is NULL");
  if (kernel != DG_KERNEL_LINE && kernel != DG_KERNEL_HALF) return fail(DG_EINVAL, "unknown kernel");
  ctx->kernel = kernel;
  return DG_OK;
}

int dg_get_kernel(const dg_ctx *ctx, int32_t *kernel) {
  if (!ctx || !kernel) return fail(DG_EINVAL, "NULL argument");
  *kernel = ctx->kernel;
  return DG_OK;
}

static int stage(dg_ctx *c, const void *q, const void *q0, void *out, int combine, double c0,
                 double c1, double dt, hipStream_t s);

int dg_autotune(dg_ctx *ctx, const void *q, void *work, int32_t *chosen, void *hip_stream) {
  if (!ctx || !q || !work) return fail(DG_EINVAL, "NULL argument");
  if (!aligned16(q) || !aligned16(work)) return fail(DG_EINVAL, "state pointers must be 16-byte aligned");
  const size_t bytes = ctx->state_n * ctx->elem_bytes;
  {
    const char *a = static_cast<const char *>(q);
    const char *b = static_cast<const char *>(work);
    if (a < b + 2 * bytes && b < a + bytes) return fail(DG_EINVAL, "q and work overlap");
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  char *w0 = static_cast<char *>(work);
  char *w1 = w0 + bytes;
  hipEvent_t ev[2];
  if (hipEventCreate(&ev[0]) != hipSuccess) return fail(DG_EHIP, "hipEventCreate");
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return fail(DG_EHIP, "hipEventCreate");
  }
  const int keep = ctx->kernel;
  float best = 1e30f;
  int best_k = keep, rc = DG_OK;
  for (int k : {DG_KERNEL_LINE, DG_KERNEL_HALF}) {
    ctx->kernel = k;
    float t_best = 1e30f;
    for (int rep = 0; rep < 4 && rc == DG_OK; ++rep) {
      hipError_t e = hipEventRecord(ev[0], s);
      if (e != hipSuccess) { rc = hip_fail(e, "hipEventRecord"); break; }
      if ((rc = stage(ctx, q, nullptr, w0, 1, 0.0, 1.0, 0.0, s)) != DG_OK) break;
      if ((rc = stage(ctx, w0, q, w1, 1, 0.75, 0.25, 0.0, s)) != DG_OK) break;
      if ((e = hipEventRecord(ev[1], s)) != hipSuccess || (e = hipEventSynchronize(ev[1])) != hipSuccess) {
        rc = hip_fail(e, "autotune timing");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
      if (rep > 0) t_best = std::min(t_best, ms);   // the first repetition warms up
    }
    if (rc != DG_OK) break;
    if (t_best < best) {
      best = t_best;
      best_k = k;
    }
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  ctx->kernel = rc == DG_OK ? best_k : keep;
  if (rc == DG_OK && chosen) *chosen = best_k;
  return rc;
}

int dg_set_levels(dg_ctx *ctx, int32_t n_levels) {
  if (!ctx) return fail(DG_EINVAL, "ctx is NULL");
  if (n_levels < 1 || n_levels > 65535) return fail(DG_EINVAL, "n_levels must be in 1..65535");
  if (ctx->member && n_levels != 1)
    return fail(DG_EUNSUPPORTED, "an ensemble member holds one layer");
  // wavefronts of one layer in either layout (the half-line layout row-aligned
  // or packed across rows), bounded so that all layers fit one launch
  const int64_t gh = 64 / (2 * ctx->np);
  const int64_t E = (int64_t)ctx->d.n_lon * ctx->d.n_lat;
  int64_t per = (int64_t)dgsw::waves_per_row(ctx->np, ctx->d.n_lon) * ctx->d.n_lat;
  per = std::max(per, (ctx->d.n_lon + gh - 1) / gh * ctx->d.n_lat);
  per = std::max(per, (E + gh - 1) / gh);
  if (per * n_levels >= ((int64_t)1 << 31)) return fail(DG_EINVAL, "too many layers for one launch");
  ctx->levels = n_levels;
  ctx->state_n = ctx->level_n * n_levels;
  return DG_OK;
}

int dg_get_levels(const dg_ctx *ctx, int32_t *n_levels) {
  if (!ctx || !n_levels) return fail(DG_EINVAL, "NULL argument");
  *n_levels = ctx->levels;
  return DG_OK;
}

int dg_free(dg_ctx *ctx) {
  if (!ctx) return DG_OK;
  // a captured graph reads the context's device tables: keep them until the
  // last such graph is freed (dg_graph_free completes the release)
  if (ctx->graphs > 0) {
    ctx->freed = 1;
    return DG_OK;
  }
  release(ctx);
  return DG_OK;
}

int dg_state_size(const dg_ctx *ctx, int64_t *n_values) {
  if (!ctx || !n_values) return fail(DG_EINVAL, "NULL argument");
  *n_values = ctx->state_n;
  return DG_OK;
}

int dg_min_width(const dg_ctx *ctx, double *meters) {
  if (!ctx || !meters) return fail(DG_EINVAL, "NULL argument");
  *meters = ctx->min_width;
  return DG_OK;
}

int dg_work_size(const dg_ctx *ctx, int32_t scheme, int64_t *n_values) {
  if (!ctx || !n_values) return fail(DG_EINVAL, "NULL argument");
  switch (scheme) {
    case DG_SSP_RK1: *n_values = ctx->state_n; return DG_OK;
    case DG_SSP_RK2:
    case DG_SSP_RK3: *n_values = 2 * ctx->state_n; return DG_OK;
    case DG_RK4: *n_values = 3 * ctx->state_n; return DG_OK;
    default: return fail(DG_EINVAL, "unknown scheme");
  }
}

int dg_set_forcing(dg_ctx *ctx, const void *fhat) {
  if (!ctx) return fail(DG_EINVAL, "ctx is NULL");
  if (fhat && !aligned16(fhat)) return fail(DG_EINVAL, "fhat must be 16-byte aligned");
  ctx->forcing = fhat;
  return DG_OK;
}

static int stage(dg_ctx *c, const void *q, const void *q0, void *out, int combine, double c0,
                 double c1, double dt, hipStream_t s) {
  dgsw::StageLaunch a;
  a.q = q;
  a.q0 = q0;
  a.out = out;
  a.forcing = c->forcing;
  a.glob = c->d_glob;
  a.rows = c->d_rows;
  a.n_lon = c->d.n_lon;
  a.n_lat = c->d.n_lat;
  a.E = c->E;
  a.alpha_global = c->d.alpha_mode == DG_ALPHA_GLOBAL;
  a.periodic_y = c->periodic_y;
  a.variant = c->kernel;
  a.levels = c->levels;
  a.combine = combine;
  a.c0 = c0;
  a.c1 = c1;
  a.dt = dt;
  hipError_t e = dgsw::launch_stage(c->d.dtype == DG_F64 ? 0 : 1, c->np, a, s);
  if (e != hipSuccess) return hip_fail(e, "stage kernel launch");
  return DG_OK;
}

// General stage: out = q0 + c1 (q - q0) + ca (qa - q0) + cb (qb - q0) + dt L(q)
// (q0, qa, qb read at the element itself only, so any of them may be the same
// buffer as out).
static int stage_general(dg_ctx *c, const void *q, const void *q0, void *out, double c1,
                         double dt, const void *qa, double ca, const void *qb, double cb,
                         hipStream_t s) {
  dgsw::StageLaunch a;
  a.q = q;
  a.q0 = q0;
  a.out = out;
  a.forcing = c->forcing;
  a.glob = c->d_glob;
  a.rows = c->d_rows;
  a.n_lon = c->d.n_lon;
  a.n_lat = c->d.n_lat;
  a.E = c->E;
  a.alpha_global = c->d.alpha_mode == DG_ALPHA_GLOBAL;
  a.periodic_y = c->periodic_y;
  a.variant = c->kernel;
  a.levels = c->levels;
  a.combine = 2;
  a.c0 = 1.0 - c1 - ca - cb;
  a.c1 = c1;
  a.dt = dt;
  a.qa = qa;
  a.qb = qb;
  a.ca = ca;
  a.cb = cb;
  hipError_t e = dgsw::launch_stage(c->d.dtype == DG_F64 ? 0 : 1, c->np, a, s);
  if (e != hipSuccess) return hip_fail(e, "stage kernel launch");
  return DG_OK;
}

int dg_rhs(dg_ctx *ctx, const void *q, void *dqdt, void *hip_stream) {
  if (!ctx || !q || !dqdt) return fail(DG_EINVAL, "NULL argument");
  if (!aligned16(q) || !aligned16(dqdt)) return fail(DG_EINVAL, "state pointers must be 16-byte aligned");
  const size_t bytes = ctx->state_n * ctx->elem_bytes;
  const char *a = static_cast<const char *>(q);
  const char *b = static_cast<const char *>(dqdt);
  if (a < b + bytes && b < a + bytes) return fail(DG_EINVAL, "q and dqdt overlap");
  return stage(ctx, q, nullptr, dqdt, 0, 0.0, 1.0, 0.0, static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"

// nsteps steps of the scheme on q with the stage states in work (already
// checked: dg_work_size values, not overlapping q); shared by dg_rk_step and
// dg_rk_step_noalloc.
static int rk_steps(dg_ctx *ctx, void *q, void *work, double dt, int32_t scheme, int32_t nsteps,
                    hipStream_t s) {
  int rc = DG_OK;
  const size_t bytes = ctx->state_n * ctx->elem_bytes;
  char *w0 = static_cast<char *>(work);
  char *w1 = w0 + bytes;
  for (int n = 0; n < nsteps; ++n) {
    switch (scheme) {
      case DG_SSP_RK1:
        if ((rc = stage(ctx, q, nullptr, w0, 1, 0.0, 1.0, dt, s)) != DG_OK) return rc;
        {
          hipError_t e = hipMemcpyAsync(q, w0, bytes, hipMemcpyDeviceToDevice, s);
          if (e != hipSuccess) return hip_fail(e, "RK1 copy-back");
        }
        break;
      case DG_SSP_RK2:
        if ((rc = stage(ctx, q, nullptr, w0, 1, 0.0, 1.0, dt, s)) != DG_OK) return rc;
        if ((rc = stage(ctx, w0, q, q, 1, 0.5, 0.5, dt, s)) != DG_OK) return rc;
        break;
      case DG_SSP_RK3:
        if ((rc = stage(ctx, q, nullptr, w0, 1, 0.0, 1.0, dt, s)) != DG_OK) return rc;
        if ((rc = stage(ctx, w0, q, w1, 1, 0.75, 0.25, dt, s)) != DG_OK) return rc;
        if ((rc = stage(ctx, w1, q, q, 1, 1.0 / 3.0, 2.0 / 3.0, dt, s)) != DG_OK) return rc;
        break;
      case DG_RK4: {
        char *w2 = w1 + bytes;
        if ((rc = stage(ctx, q, nullptr, w0, 1, 0.0, 1.0, 0.5 * dt, s)) != DG_OK) return rc;
        if ((rc = stage_general(ctx, w0, q, w1, 0.0, 0.5 * dt, nullptr, 0.0, nullptr, 0.0, s)) !=
            DG_OK)
          return rc;
        if ((rc = stage_general(ctx, w1, q, w2, 0.0, dt, nullptr, 0.0, nullptr, 0.0, s)) != DG_OK)
          return rc;
        if ((rc = stage_general(ctx, w2, q, q, 1.0 / 3.0, dt / 6.0, w0, 1.0 / 3.0, w1, 2.0 / 3.0,
                                s)) != DG_OK)
          return rc;
        break;
      }
      default:
        return fail(DG_EINVAL, "unknown scheme");
    }
  }
  return DG_OK;
}

// Argument checks of an RK step on q; wn receives the work values the scheme needs.
static int rk_check(dg_ctx *ctx, const void *q, double dt, int32_t scheme, int32_t nsteps,
                    int64_t *wn) {
  if (!ctx || !q) return fail(DG_EINVAL, "NULL argument");
  if (!aligned16(q)) return fail(DG_EINVAL, "state pointers must be 16-byte aligned");
  if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(dt)) return fail(DG_EINVAL, "dt must be finite");
  return dg_work_size(ctx, scheme, wn);
}

extern "C" {

int dg_rk_step(dg_ctx *ctx, void *q, void *work, double dt, int32_t scheme, int32_t nsteps,
               void *hip_stream) {
  if (!work) return fail(DG_EINVAL, "NULL argument");
  if (!aligned16(work)) return fail(DG_EINVAL, "state pointers must be 16-byte aligned");
  int64_t wn = 0;
  int rc = rk_check(ctx, q, dt, scheme, nsteps, &wn);
  if (rc != DG_OK) return rc;
  const size_t bytes = ctx->state_n * ctx->elem_bytes;
  {
    const char *a = static_cast<const char *>(q);
    const char *b = static_cast<const char *>(work);
    if (a < b + wn * ctx->elem_bytes && b < a + bytes) return fail(DG_EINVAL, "q and work overlap");
  }
  return rk_steps(ctx, q, work, dt, scheme, nsteps, static_cast<hipStream_t>(hip_stream));
}

int dg_rk_stage(dg_ctx *ctx, const void *q, const void *q0, void *out, double c0, double c1,
                double dt, void *hip_stream) {
  if (!ctx || !q || !out) return fail(DG_EINVAL, "NULL argument");
  if (!q0 && c0 != 0.0) return fail(DG_EINVAL, "q0 is NULL but c0 != 0");
  if (!aligned16(q) || !aligned16(out) || (q0 && !aligned16(q0)))
    return fail(DG_EINVAL, "state pointers must be 16-byte aligned");
  if (!std::isfinite(c0) || !std::isfinite(c1) || !std::isfinite(dt))
    return fail(DG_EINVAL, "c0, c1 and dt must be finite");
  const size_t bytes = ctx->state_n * ctx->elem_bytes;
  const char *a = static_cast<const char *>(q);
  const char *o = static_cast<const char *>(out);
  if (a < o + bytes && o < a + bytes) return fail(DG_EINVAL, "q and out overlap");
  if (q0) {
    const char *b = static_cast<const char *>(q0);
    if (b != o && b < o + bytes && o < b + bytes) return fail(DG_EINVAL, "q0 partially overlaps out");
  }
  return stage(ctx, q, q0, out, 1, c0, c1, dt, static_cast<hipStream_t>(hip_stream));
}

int dg_mass(dg_ctx *ctx, const void *q, double out[3], void *hip_stream) {
  if (!ctx || !q || !out) return fail(DG_EINVAL, "NULL argument");
  if (!aligned16(q)) return fail(DG_EINVAL, "q must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = dgsw::launch_mass(ctx->d.dtype == DG_F64 ? 0 : 1, ctx->np, q, ctx->d_mass_w,
                                   ctx->d.n_lon, ctx->E, ctx->levels, ctx->d_partial,
                                   ctx->d_out4, s);
  if (e != hipSuccess) return hip_fail(e, "mass kernel launch");
  double h4[4];
  if ((e = hipMemcpyAsync(h4, ctx->d_out4, sizeof(h4), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(e, "mass copy-out");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "mass synchronise");
  out[0] = h4[0];
  out[1] = h4[1];
  out[2] = h4[2];
  if (h4[3] != 0.0 || !std::isfinite(h4[0]) || !std::isfinite(h4[1]) || !std::isfinite(h4[2]))
    return fail(DG_ENONFINITE, "state holds " + std::to_string((long long)h4[3]) + " non-finite values");
  return DG_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ no-allocation RK step
// Stage states of dg_rk_step_noalloc: one array per GPU, loaded with the
// library and held until the process ends.  Host code never uses the array's
// name as an address: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[DG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up on the first call on
// the device), or an error code.
int scratch_ptr(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(DG_EUNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress of the no-allocation scratch");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return DG_OK;
}
}  // namespace

extern "C" {

int dg_rk_step_noalloc(dg_ctx *ctx, void *q, double dt, int32_t scheme, int32_t nsteps,
                       void *hip_stream) {
  int64_t wn = 0;
  int rc = rk_check(ctx, q, dt, scheme, nsteps, &wn);
  if (rc != DG_OK) return rc;
  const uint64_t need = (uint64_t)wn * ctx->elem_bytes;
  if (need > (uint64_t)DG_NOALLOC_SCRATCH_BYTES)
    return fail(DG_EINVAL, "dg_rk_step_noalloc: the scheme's stage states need " + std::to_string(need) +
                               " bytes, more than the " + std::to_string((long long)DG_NOALLOC_SCRATCH_BYTES) +
                               "-byte scratch; use dg_rk_step with a caller work buffer");
  void *work = nullptr;
  if ((rc = scratch_ptr(&work)) != DG_OK) return rc;
  return rk_steps(ctx, q, work, dt, scheme, nsteps, static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"
