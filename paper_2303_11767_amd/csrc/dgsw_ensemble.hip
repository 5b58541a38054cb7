// C ABI of ensembles and HIP graphs (declared in include/dgsw.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <sstream>
#include <string>
#include <vector>

#include "dgsw.h"
#include "dgsw_ctx.hpp"
#include "dgsw_device.hpp"

using dgsw::aligned16;
using dgsw::fail;
using dgsw::hip_fail;

struct dg_ens {
  int n = 0, dtype = 0, npmax = 0;
  size_t elem_bytes = 0;
  std::vector<dg_ctx *> members;
  std::vector<int64_t> off;              // n + 1 packed offsets (values)
  std::vector<dgsw::EnsMember> hmem;
  std::vector<int2> items;               // {member, wave}
  std::vector<double> cost;              // per item
  dgsw::EnsMember *d_mem = nullptr;
  int2 *d_items = nullptr;
  int *d_bounds = nullptr;
  int bounds_cap = 0;
  int wpb = 4, parts = 0;
};

struct dg_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void ens_release(dg_ens *e) {
  if (!e) return;
  for (dg_ctx *c : e->members) dg_free(c);
  if (e->d_mem) (void)hipFree(e->d_mem);
  if (e->d_items) (void)hipFree(e->d_items);
  if (e->d_bounds) (void)hipFree(e->d_bounds);
  delete e;
}

// Contiguous cost-balanced ranges of the work list, one per workgroup.
int upload_schedule(dg_ens *e, int wpb, int parts) {
  const int n_items = (int)e->items.size();
  if (parts < 1) parts = 1;
  double total = 0.0;
  for (double c : e->cost) total += c;
  std::vector<int> b(parts + 1, n_items);
  b[0] = 0;
  double acc = 0.0;
  int k = 1;
  for (int it = 0; it < n_items && k < parts; ++it) {
    acc += e->cost[it];
    while (k < parts && acc >= total * k / parts) b[k++] = it + 1;
  }
  for (int p = 1; p <= parts; ++p) b[p] = std::max(b[p], b[p - 1]);
  if (parts + 1 > e->bounds_cap) {
    if (e->d_bounds) (void)hipFree(e->d_bounds);
    e->d_bounds = nullptr;
    hipError_t err = hipMalloc(reinterpret_cast<void **>(&e->d_bounds), (parts + 1) * sizeof(int));
    if (err != hipSuccess) return fail(DG_ENOMEM, "hipMalloc of ensemble schedule");
    e->bounds_cap = parts + 1;
  }
  hipError_t err = hipMemcpy(e->d_bounds, b.data(), (parts + 1) * sizeof(int), hipMemcpyHostToDevice);
  if (err != hipSuccess) return hip_fail(err, "upload of ensemble schedule");
  e->wpb = wpb;
  e->parts = parts;
  return DG_OK;
}

int ens_stage(dg_ens *e, const void *q, const void *q0, void *out, int combine, double c0,
              double c1, hipStream_t s) {
  dgsw::EnsLaunch a;
  a.q = q;
  a.q0 = q0;
  a.out = out;
  a.mem = e->d_mem;
  a.items = e->d_items;
  a.bounds = e->d_bounds;
  a.parts = e->parts;
  a.combine = combine;
  a.c0 = c0;
  a.c1 = c1;
  hipError_t err = dgsw::launch_ens_stage(e->dtype, e->npmax, e->wpb, a, s);
  if (err != hipSuccess) return hip_fail(err, "ensemble stage launch");
  return DG_OK;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
  const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
  return x < y + nb && y < x + na;
}

std::string ens_key(const dg_ens *e) {
  hipDeviceProp_t prop;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  std::ostringstream k;
  k << arch << "|" << (e->dtype == 0 ? "f64" : "f32") << "|" << e->n;
  for (const dg_ctx *c : e->members) k << "|" << c->d.n_lon << "x" << c->d.n_lat << "r" << c->d.order;
  return k.str();
}

}  // namespace

extern "C" {

int dg_ens_init(const dg_mesh_desc *members, int32_t n_members, void *hip_stream, dg_ens **out) {
  if (!out) return fail(DG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!members || n_members < 1) return fail(DG_EINVAL, "need at least one member");
  const int dtype = members[0].dtype;
  for (int m = 0; m < n_members; ++m)
    if (members[m].dtype != dtype) return fail(DG_EINVAL, "ensemble members must share the dtype");
  dg_ens *e = new dg_ens();
  e->n = n_members;
  e->dtype = dtype == DG_F64 ? 0 : 1;
  e->elem_bytes = dtype == DG_F64 ? 8 : 4;
  const int64_t align = 16 / (int64_t)e->elem_bytes;
  e->off.assign(n_members + 1, 0);
  for (int m = 0; m < n_members; ++m) {
    dg_ctx *c = nullptr;
    int rc = dg_init_mesh(&members[m], hip_stream, &c);
    if (rc != DG_OK) {
      ens_release(e);
      return rc;
    }
    e->members.push_back(c);
    e->npmax = std::max(e->npmax, c->np);
    e->off[m + 1] = e->off[m] + (c->state_n + align - 1) / align * align;
    dgsw::EnsMember hm;
    std::memset(&hm, 0, sizeof(hm));
    hm.glob = c->d_glob;
    hm.rows = c->d_rows;
    hm.off = e->off[m];
    hm.n_lon = c->d.n_lon;
    hm.n_lat = c->d.n_lat;
    hm.np = c->np;
    hm.segs = dgsw::waves_per_row(c->np, c->d.n_lon);
    hm.alpha_global = c->d.alpha_mode == DG_ALPHA_GLOBAL;
    hm.dt = 0.0;
    e->hmem.push_back(hm);
    // work items of this member in row-major wave order; cost ~ lanes busy x work per lane
    const int waves = hm.segs * hm.n_lat;
    const double cost = (double)c->np * c->np * c->np;
    for (int w = 0; w < waves; ++w) {
      e->items.push_back(make_int2(m, w));
      e->cost.push_back(cost);
    }
  }
  if (e->off[n_members] >= (int64_t(1) << 31)) {
    ens_release(e);
    return fail(DG_EINVAL, "packed ensemble state exceeds 2^31 values");
  }
  hipError_t err;
  if ((err = hipMalloc(reinterpret_cast<void **>(&e->d_mem), n_members * sizeof(dgsw::EnsMember))) != hipSuccess ||
      (err = hipMalloc(reinterpret_cast<void **>(&e->d_items), e->items.size() * sizeof(int2))) != hipSuccess) {
    ens_release(e);
    return fail(DG_ENOMEM, "hipMalloc of the ensemble work list");
  }
  if ((err = hipMemcpy(e->d_mem, e->hmem.data(), n_members * sizeof(dgsw::EnsMember),
                       hipMemcpyHostToDevice)) != hipSuccess ||
      (err = hipMemcpy(e->d_items, e->items.data(), e->items.size() * sizeof(int2),
                       hipMemcpyHostToDevice)) != hipSuccess) {
    ens_release(e);
    return hip_fail(err, "upload of the ensemble work list");
  }
  const int default_parts = std::max(1, std::min((int)e->items.size() / 4, 2048));
  int rc = upload_schedule(e, 4, default_parts);
  if (rc != DG_OK) {
    ens_release(e);
    return rc;
  }
  *out = e;
  return DG_OK;
}

int dg_ens_free(dg_ens *ens) {
  ens_release(ens);
  return DG_OK;
}

int dg_ens_state_size(const dg_ens *ens, int64_t *n_values) {
  if (!ens || !n_values) return fail(DG_EINVAL, "NULL argument");
  *n_values = ens->off[ens->n];
  return DG_OK;
}

int dg_ens_offsets(const dg_ens *ens, int64_t *offsets) {
  if (!ens || !offsets) return fail(DG_EINVAL, "NULL argument");
  for (int m = 0; m <= ens->n; ++m) offsets[m] = ens->off[m];
  return DG_OK;
}

int dg_ens_member(dg_ens *ens, int32_t m, dg_ctx **ctx) {
  if (!ens || !ctx) return fail(DG_EINVAL, "NULL argument");
  if (m < 0 || m >= ens->n) return fail(DG_EINVAL, "member index out of range");
  *ctx = ens->members[m];
  return DG_OK;
}

int dg_ens_set_dt(dg_ens *ens, const double *dt) {
  if (!ens || !dt) return fail(DG_EINVAL, "NULL argument");
  for (int m = 0; m < ens->n; ++m) {
    if (!std::isfinite(dt[m])) return fail(DG_EINVAL, "dt must be finite");
    ens->hmem[m].dt = dt[m];
  }
  hipError_t err = hipMemcpy(ens->d_mem, ens->hmem.data(), ens->n * sizeof(dgsw::EnsMember),
                             hipMemcpyHostToDevice);
  if (err != hipSuccess) return hip_fail(err, "upload of ensemble time steps");
  return DG_OK;
}

int dg_ens_rhs(dg_ens *ens, const void *q, void *dqdt, void *hip_stream) {
  if (!ens || !q || !dqdt) return fail(DG_EINVAL, "NULL argument");
  if (!aligned16(q) || !aligned16(dqdt)) return fail(DG_EINVAL, "state pointers must be 16-byte aligned");
  const size_t bytes = ens->off[ens->n] * ens->elem_bytes;
  if (overlaps(q, bytes, dqdt, bytes)) return fail(DG_EINVAL, "q and dqdt overlap");
  return ens_stage(ens, q, nullptr, dqdt, 0, 0.0, 1.0, static_cast<hipStream_t>(hip_stream));
}

int dg_ens_rk_stage(dg_ens *ens, const void *q, const void *q0, void *out, double c0, double c1,
                    void *hip_stream) {
  if (!ens || !q || !out) return fail(DG_EINVAL, "NULL argument");
  if (!q0 && c0 != 0.0) return fail(DG_EINVAL, "q0 is NULL but c0 != 0");
  if (!aligned16(q) || !aligned16(out) || (q0 && !aligned16(q0)))
    return fail(DG_EINVAL, "state pointers must be 16-byte aligned");
  if (!std::isfinite(c0) || !std::isfinite(c1)) return fail(DG_EINVAL, "c0 and c1 must be finite");
  const size_t bytes = ens->off[ens->n] * ens->elem_bytes;
  if (overlaps(q, bytes, out, bytes)) return fail(DG_EINVAL, "q and out overlap");
  if (q0 && q0 != out && overlaps(q0, bytes, out, bytes)) return fail(DG_EINVAL, "q0 partially overlaps out");
  return ens_stage(ens, q, q0, out, 1, c0, c1, static_cast<hipStream_t>(hip_stream));
}

int dg_ens_rk_step(dg_ens *ens, void *q, void *work, int32_t nsteps, void *hip_stream) {
  if (!ens || !q || !work) return fail(DG_EINVAL, "NULL argument");
  if (!aligned16(q) || !aligned16(work)) return fail(DG_EINVAL, "state pointers must be 16-byte aligned");
  if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
  const size_t bytes = ens->off[ens->n] * ens->elem_bytes;
  if (overlaps(q, bytes, work, 2 * bytes)) return fail(DG_EINVAL, "q and work overlap");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  char *w0 = static_cast<char *>(work);
  char *w1 = w0 + bytes;
  int rc;
  for (int k = 0; k < nsteps; ++k) {
    if ((rc = ens_stage(ens, q, nullptr, w0, 1, 0.0, 1.0, s)) != DG_OK) return rc;
    if ((rc = ens_stage(ens, w0, q, w1, 1, 0.75, 0.25, s)) != DG_OK) return rc;
    if ((rc = ens_stage(ens, w1, q, q, 1, 1.0 / 3.0, 2.0 / 3.0, s)) != DG_OK) return rc;
  }
  return DG_OK;
}

int dg_ens_set_schedule(dg_ens *ens, int32_t waves_per_group, int32_t groups) {
  if (!ens) return fail(DG_EINVAL, "ens is NULL");
  if (waves_per_group != 1 && waves_per_group != 2 && waves_per_group != 4)
    return fail(DG_EINVAL, "waves_per_group must be 1, 2 or 4");
  if (groups < 1 || groups > (1 << 20)) return fail(DG_EINVAL, "groups out of range");
  return upload_schedule(ens, waves_per_group, groups);
}

int dg_ens_get_schedule(const dg_ens *ens, int32_t *waves_per_group, int32_t *groups) {
  if (!ens || !waves_per_group || !groups) return fail(DG_EINVAL, "NULL argument");
  *waves_per_group = ens->wpb;
  *groups = ens->parts;
  return DG_OK;
}

int dg_ens_autotune(dg_ens *ens, const void *q, void *work, const char *cache_path, void *hip_stream) {
  if (!ens || !q || !work) return fail(DG_EINVAL, "NULL argument");
  const std::string key = ens_key(ens);
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      int w = 0, p = 0;
      if (ls >> k >> w >> p && k == key) return dg_ens_set_schedule(ens, w, p);
    }
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const size_t bytes = ens->off[ens->n] * ens->elem_bytes;
  char *w0 = static_cast<char *>(work);
  char *w1 = w0 + bytes;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return fail(DG_EHIP, "hipEventCreate");
  const int n_items = (int)ens->items.size();
  float best = 1e30f;
  int best_w = ens->wpb, best_p = ens->parts;
  int rc = DG_OK;
  for (int w : {1, 2, 4}) {
    for (int p : {256, 512, 1024, 2048, 4096, 8192, 16384}) {
      if (p * w > 4 * n_items && p > 256) continue;
      if ((rc = upload_schedule(ens, w, p)) != DG_OK) break;
      float t_best = 1e30f;
      for (int rep = 0; rep < 4 && rc == DG_OK; ++rep) {
        (void)hipEventRecord(a, s);
        if ((rc = ens_stage(ens, q, nullptr, w0, 1, 0.0, 1.0, s)) != DG_OK) break;
        if ((rc = ens_stage(ens, w0, q, w1, 1, 0.75, 0.25, s)) != DG_OK) break;
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        if (rep > 0) t_best = std::min(t_best, ms);   // first repetition warms up
      }
      if (rc != DG_OK) break;
      if (t_best < best) {
        best = t_best;
        best_w = w;
        best_p = p;
      }
    }
    if (rc != DG_OK) break;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != DG_OK) return rc;
  rc = upload_schedule(ens, best_w, best_p);
  if (rc == DG_OK && cache_path) {
    std::ofstream o(cache_path, std::ios::app);
    o << key << " " << best_w << " " << best_p << "\n";
  }
  return rc;
}

// ------------------------------------------------------------------ graphs
static int capture(dg_graph **out, const std::function<int(hipStream_t)> &body);

int dg_graph_rk(dg_ctx *ctx, void *q, void *work, double dt, int32_t scheme, int32_t nsteps,
                dg_graph **out) {
  if (!ctx || !out) return fail(DG_EINVAL, "NULL argument");
  return capture(out, [&](hipStream_t s) { return dg_rk_step(ctx, q, work, dt, scheme, nsteps, s); });
}

int dg_graph_ens(dg_ens *ens, void *q, void *work, int32_t nsteps, dg_graph **out) {
  if (!ens || !out) return fail(DG_EINVAL, "NULL argument");
  return capture(out, [&](hipStream_t s) { return dg_ens_rk_step(ens, q, work, nsteps, s); });
}

int dg_graph_launch(dg_graph *graph, void *hip_stream) {
  if (!graph || !graph->exec) return fail(DG_EINVAL, "graph is NULL");
  hipError_t err = hipGraphLaunch(graph->exec, static_cast<hipStream_t>(hip_stream));
  if (err != hipSuccess) return hip_fail(err, "hipGraphLaunch");
  return DG_OK;
}

int dg_graph_free(dg_graph *graph) {
  if (!graph) return DG_OK;
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  delete graph;
  return DG_OK;
}

}  // extern "C"

// Record the launches of `body` on a private stream (capture cannot run on the
// legacy null stream a caller may use) and instantiate them.
static int capture(dg_graph **out, const std::function<int(hipStream_t)> &body) {
  *out = nullptr;
  hipStream_t s;
  hipError_t err = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (err != hipSuccess) return hip_fail(err, "hipStreamCreate");
  dg_graph *g = new dg_graph();
  err = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (err != hipSuccess) {
    delete g;
    (void)hipStreamDestroy(s);
    return hip_fail(err, "hipStreamBeginCapture");
  }
  const int rc = body(s);
  err = hipStreamEndCapture(s, &g->graph);
  (void)hipStreamDestroy(s);
  if (rc != DG_OK) {
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return rc;
  }
  if (err != hipSuccess) {
    delete g;
    return hip_fail(err, "hipStreamEndCapture");
  }
  err = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (err != hipSuccess) {
    (void)hipGraphDestroy(g->graph);
    delete g;
    return hip_fail(err, "hipGraphInstantiate");
  }
  *out = g;
  return DG_OK;
}
