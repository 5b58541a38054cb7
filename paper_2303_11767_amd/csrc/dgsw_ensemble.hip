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
  std::vector<dgsw::EnsItem> items;      // one wavefront of one member each
  std::vector<double> cost;              // per item
  std::vector<double> dt;                // per member
  dgsw::EnsItem *d_items = nullptr;
  int *d_bounds = nullptr;
  // every member's GlobTab and RowTab array copied into one buffer, so the
  // kernels reach them from a kernel argument (scalar loads of the uniform
  // table reads) through the byte offsets in the work items
  unsigned char *d_tabs = nullptr;
  std::vector<long long> tab_glob, tab_rows;   // per member
  int bounds_cap = 0;
  int wpb = 4, parts = 0, fused = 0, flat = 1;
  std::vector<int> layout;               // per member: DG_KERNEL_LINE or DG_KERNEL_HALF
  // members of one order and layout form one contiguous group of the sorted work list
  struct Group { int np, lay, begin, end, parts, bounds_off; double cost; };
  std::vector<Group> groups;
  int graphs = 0;   // live dg_graph objects captured on this ensemble
  int freed = 0;    // dg_ens_free called while graphs were live: release deferred
};

// A captured graph holds the device addresses of its context's or ensemble's
// tables and schedule, so it pins that object: frees are deferred until the
// last graph is gone, and the ensemble schedule cannot change meanwhile.
struct dg_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  dg_ctx *ctx = nullptr;
  dg_ens *ens = nullptr;
};

namespace {

void ens_release(dg_ens *e) {
  if (!e) return;
  for (dg_ctx *c : e->members) dg_free(c);
  if (e->d_items) (void)hipFree(e->d_items);
  if (e->d_bounds) (void)hipFree(e->d_bounds);
  if (e->d_tabs) (void)hipFree(e->d_tabs);
  delete e;
}

// The work list: every member's wavefronts in its layout (row-major), sorted
// by (order, layout), stable so members and rows keep their order; one group
// per (order, layout); uploaded to the device.
int build_items(dg_ens *e) {
  std::vector<dgsw::EnsItem> items;
  std::vector<double> cost;
  std::vector<std::pair<int, int>> key;
  for (int m = 0; m < e->n; ++m) {
    const dg_ctx *c = e->members[m];
    const int lay = e->layout[m];
    dgsw::EnsItem it;
    std::memset(&it, 0, sizeof(it));
    it.glob = e->tab_glob[m];
    it.rows = e->tab_rows[m];
    it.off = e->off[m];
    it.dt = e->dt.empty() ? 0.0 : e->dt[m];
    it.n_lon = c->d.n_lon;
    it.n_lat = c->d.n_lat;
    it.np = c->np;
    it.alpha_global = c->d.alpha_mode == DG_ALPHA_GLOBAL;
    it.member = m;
    const int n_lon = c->d.n_lon, n_lat = c->d.n_lat, E = c->E;
    // cost ~ the work of one wavefront: elements per wavefront times the work
    // per element (~np^3 per line of np lanes)
    const double np3 = (double)c->np * c->np * c->np;
    auto add = [&](int j, int seg, int e_end, double w) {
      it.j = j;
      it.seg = seg;
      it.e_end = e_end;
      items.push_back(it);
      cost.push_back(w);
      key.emplace_back(c->np, lay);
    };
    if (lay == DG_KERNEL_LINE) {
      const int segs = dgsw::waves_per_row(c->np, n_lon);
      for (int j = 0; j < n_lat; ++j)
        for (int sg = 0; sg < segs; ++sg) add(j, sg, 0, np3);
    } else {
      const int gpw = 64 / (2 * c->np);
      const double w = np3 * 0.5;
      if (gpw <= n_lon && n_lon % gpw != 0) {      // packed across row ends
        for (int e0 = 0; e0 < E; e0 += gpw) add(e0 / n_lon, e0, E, w);
      } else {
        const int segs = (n_lon + gpw - 1) / gpw;
        for (int j = 0; j < n_lat; ++j)
          for (int sg = 0; sg < segs; ++sg) add(j, j * n_lon + sg * gpw, (j + 1) * n_lon, w);
      }
    }
  }
  std::vector<int> idx(items.size());
  for (size_t k = 0; k < idx.size(); ++k) idx[k] = (int)k;
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return key[x] < key[y]; });
  e->items.resize(items.size());
  e->cost.resize(items.size());
  for (size_t k = 0; k < idx.size(); ++k) {
    e->items[k] = items[idx[k]];
    e->cost[k] = cost[idx[k]];
  }
  e->groups.clear();
  for (int k = 0; k < (int)e->items.size();) {
    const std::pair<int, int> g0 = key[idx[k]];
    dg_ens::Group g{g0.first, g0.second, k, k, 0, 0, 0.0};
    while (k < (int)e->items.size() && key[idx[k]] == g0) g.cost += e->cost[k++];
    g.end = k;
    e->groups.push_back(g);
  }
  if (e->d_items) (void)hipFree(e->d_items);
  e->d_items = nullptr;
  hipError_t err;
  if ((err = hipMalloc(reinterpret_cast<void **>(&e->d_items), e->items.size() * sizeof(dgsw::EnsItem))) !=
      hipSuccess)
    return fail(DG_ENOMEM, "hipMalloc of the ensemble work list");
  if ((err = hipMemcpy(e->d_items, e->items.data(), e->items.size() * sizeof(dgsw::EnsItem),
                       hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(err, "upload of the ensemble work list");
  return DG_OK;
}

bool all_line(const dg_ens *e) {
  for (int l : e->layout)
    if (l != DG_KERNEL_LINE) return false;
  return true;
}

// Split items [begin, end) into `parts` contiguous ranges of about equal cost;
// appends parts + 1 absolute item offsets to b.
void balanced_ranges(const dg_ens *e, int begin, int end, int parts, std::vector<int> &b) {
  double total = 0.0;
  for (int it = begin; it < end; ++it) total += e->cost[it];
  const size_t b0 = b.size();
  b.push_back(begin);
  double acc = 0.0;
  int k = 1;
  for (int it = begin; it < end && k < parts; ++it) {
    acc += e->cost[it];
    while (k < parts && acc >= total * k / parts) {
      b.push_back(it + 1);
      ++k;
    }
  }
  while ((int)(b.size() - b0) < parts + 1) b.push_back(end);
}

// Schedule: `parts` workgroups in total, each taking one contiguous,
// cost-balanced range of the work list.  fused: one launch over all orders;
// otherwise one launch per order with the workgroups shared out by cost.
int upload_schedule(dg_ens *e, int wpb, int parts, int fused) {
  if (fused && !all_line(e))
    return fail(DG_EINVAL, "the single fused launch runs line-layout members only: "
                           "set every order's layout to DG_KERNEL_LINE first (dg_ens_set_kernel)");
  // parts == 0: "flat", one workgroup per wpb consecutive items, scheduled by
  // the hardware like an ordinary grid
  const bool flat = parts == 0;
  std::vector<int> b;
  if (fused) {
    const int n = (int)e->items.size();
    const int p = flat ? (n + wpb - 1) / wpb : parts;
    balanced_ranges(e, 0, n, p, b);
  } else {
    double total = 0.0;
    for (const auto &g : e->groups) total += g.cost;
    for (auto &g : e->groups) {
      g.parts = flat ? (g.end - g.begin + wpb - 1) / wpb
                     : std::max(1, (int)std::llround(parts * g.cost / total));
      g.bounds_off = (int)b.size();
      balanced_ranges(e, g.begin, g.end, g.parts, b);
    }
  }
  if (fused && flat) parts = (int)b.size() - 1;
  if ((int)b.size() > e->bounds_cap) {
    if (e->d_bounds) (void)hipFree(e->d_bounds);
    e->d_bounds = nullptr;
    e->bounds_cap = 0;
    hipError_t err = hipMalloc(reinterpret_cast<void **>(&e->d_bounds), b.size() * sizeof(int));
    if (err != hipSuccess) return fail(DG_ENOMEM, "hipMalloc of ensemble schedule");
    e->bounds_cap = (int)b.size();
  }
  hipError_t err = hipMemcpy(e->d_bounds, b.data(), b.size() * sizeof(int), hipMemcpyHostToDevice);
  if (err != hipSuccess) return hip_fail(err, "upload of ensemble schedule");
  e->wpb = wpb;
  e->parts = parts;
  e->fused = fused;
  e->flat = flat ? 1 : 0;
  return DG_OK;
}

int ens_stage(dg_ens *e, const void *q, const void *q0, void *out, int combine, double c0,
              double c1, hipStream_t s) {
  dgsw::EnsLaunch a;
  a.q = q;
  a.q0 = q0;
  a.out = out;
  a.tabs = e->d_tabs;
  a.items = e->d_items;
  a.combine = combine;
  a.c0 = c0;
  a.c1 = c1;
  a.flat = 0;
  a.begin = a.end = 0;
  if (e->fused) {
    a.bounds = e->d_bounds;
    a.parts = e->parts;
    hipError_t err = dgsw::launch_ens_stage(e->dtype, e->npmax, e->wpb, a, s);
    if (err != hipSuccess) return hip_fail(err, "ensemble stage launch");
    return DG_OK;
  }
  for (const auto &g : e->groups) {
    a.bounds = e->d_bounds + g.bounds_off;
    a.parts = g.parts;
    a.flat = e->flat;
    a.begin = g.begin;
    a.end = g.end;
    hipError_t err = dgsw::launch_ens_stage_np(e->dtype, g.np, g.lay, e->wpb, a, s);
    if (err != hipSuccess) return hip_fail(err, "ensemble stage launch");
  }
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
    c->member = 1;
    e->members.push_back(c);
    e->npmax = std::max(e->npmax, c->np);
    e->off[m + 1] = e->off[m] + (c->state_n + align - 1) / align * align;
    // the member's layout as a single mesh of its size and order would take it
    e->layout.push_back(c->kernel);
  }
  e->dt.assign(n_members, 0.0);
  if (e->off[n_members] >= (int64_t(1) << 31)) {
    ens_release(e);
    return fail(DG_EINVAL, "packed ensemble state exceeds 2^31 values");
  }
  {
    // the members' tables, each at a 256-byte aligned offset of one buffer
    auto up = [](size_t b) { return (long long)((b + 255) / 256 * 256); };
    long long total = 0;
    for (const dg_ctx *c : e->members) {
      e->tab_glob.push_back(total);
      total += up(c->glob_bytes);
      e->tab_rows.push_back(total);
      total += up(c->rows_bytes);
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipError_t err = hipMalloc(reinterpret_cast<void **>(&e->d_tabs), (size_t)total);
    if (err != hipSuccess) {
      ens_release(e);
      return fail(DG_ENOMEM, "hipMalloc of the ensemble's table copy");
    }
    for (int m = 0; m < n_members && err == hipSuccess; ++m) {
      const dg_ctx *c = e->members[m];
      err = hipMemcpyAsync(e->d_tabs + e->tab_glob[m], c->d_glob, c->glob_bytes, hipMemcpyDeviceToDevice, s);
      if (err == hipSuccess)
        err = hipMemcpyAsync(e->d_tabs + e->tab_rows[m], c->d_rows, c->rows_bytes, hipMemcpyDeviceToDevice, s);
    }
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err != hipSuccess) {
      ens_release(e);
      return hip_fail(err, "copy of the members' tables");
    }
  }
  {
    const int rc = build_items(e);
    if (rc != DG_OK) {
      ens_release(e);
      return rc;
    }
  }
  int rc = upload_schedule(e, 4, 0, 0);
  if (rc != DG_OK) {
    ens_release(e);
    return rc;
  }
  *out = e;
  return DG_OK;
}

int dg_ens_free(dg_ens *ens) {
  if (ens && ens->graphs > 0) {
    ens->freed = 1;
    return DG_OK;
  }
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
  for (int m = 0; m < ens->n; ++m)
    if (!std::isfinite(dt[m])) return fail(DG_EINVAL, "dt must be finite");
  for (int m = 0; m < ens->n; ++m) ens->dt[m] = dt[m];
  for (auto &it : ens->items) it.dt = dt[it.member];
  hipError_t err = hipMemcpy(ens->d_items, ens->items.data(), ens->items.size() * sizeof(dgsw::EnsItem),
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

int dg_ens_set_schedule(dg_ens *ens, int32_t waves_per_group, int32_t groups, int32_t fused) {
  if (!ens) return fail(DG_EINVAL, "ens is NULL");
  if (waves_per_group != 1 && waves_per_group != 2 && waves_per_group != 4)
    return fail(DG_EINVAL, "waves_per_group must be 1, 2 or 4");
  if (groups < 0 || groups > (1 << 20)) return fail(DG_EINVAL, "groups out of range");
  if (fused != 0 && fused != 1) return fail(DG_EINVAL, "fused must be 0 or 1");
  if (ens->graphs > 0)
    return fail(DG_EINVAL, "the schedule is baked into live graphs of this ensemble: free them first");
  return upload_schedule(ens, waves_per_group, groups, fused);
}

int dg_ens_set_kernel(dg_ens *ens, int32_t order, int32_t kernel) {
  if (!ens) return fail(DG_EINVAL, "ens is NULL");
  if (kernel != DG_KERNEL_LINE && kernel != DG_KERNEL_HALF) return fail(DG_EINVAL, "unknown kernel");
  if (ens->graphs > 0)
    return fail(DG_EINVAL, "the work list is baked into live graphs of this ensemble: free them first");
  bool any = false;
  for (int m = 0; m < ens->n; ++m)
    if (ens->members[m]->np == order + 1) any = true;
  if (!any) return fail(DG_EINVAL, "no member of this order");
  if (kernel != DG_KERNEL_LINE && ens->fused)
    return fail(DG_EINVAL, "the single fused launch runs line-layout members only: choose a per-order schedule first");
  for (int m = 0; m < ens->n; ++m)
    if (ens->members[m]->np == order + 1) ens->layout[m] = kernel;
  int rc = build_items(ens);
  if (rc != DG_OK) return rc;
  return upload_schedule(ens, ens->wpb, ens->flat ? 0 : ens->parts, ens->fused);
}

int dg_ens_get_kernel(const dg_ens *ens, int32_t order, int32_t *kernel) {
  if (!ens || !kernel) return fail(DG_EINVAL, "NULL argument");
  for (int m = 0; m < ens->n; ++m)
    if (ens->members[m]->np == order + 1) {
      *kernel = ens->layout[m];
      return DG_OK;
    }
  return fail(DG_EINVAL, "no member of this order");
}

int dg_ens_get_schedule(const dg_ens *ens, int32_t *waves_per_group, int32_t *groups,
                        int32_t *fused) {
  if (!ens || !waves_per_group || !groups || !fused) return fail(DG_EINVAL, "NULL argument");
  *waves_per_group = ens->wpb;
  *groups = ens->parts;
  *fused = ens->fused;
  return DG_OK;
}

int dg_ens_autotune(dg_ens *ens, const void *q, void *work, const char *cache_path, void *hip_stream) {
  if (!ens || !q || !work) return fail(DG_EINVAL, "NULL argument");
  if (ens->graphs > 0)
    return fail(DG_EINVAL, "the schedule is baked into live graphs of this ensemble: free them first");
  const std::string key = ens_key(ens);
  std::vector<int> orders;
  for (const dg_ctx *c : ens->members)
    if (std::find(orders.begin(), orders.end(), c->np - 1) == orders.end()) orders.push_back(c->np - 1);
  std::sort(orders.begin(), orders.end());
  auto set_layouts = [&](const std::vector<int> &lay) -> int {
    for (int m = 0; m < ens->n; ++m) ens->layout[m] = lay[ens->members[m]->np - 1];
    return build_items(ens);
  };
  if (cache_path) {
    // line: key waves_per_group groups fused layout(order 0) .. layout(order 7)
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      int w = 0, p = 0, f = 0;
      std::vector<int> lay(dgsw::kMaxNP, DG_KERNEL_LINE);
      if (!(ls >> k >> w >> p >> f) || k != key) continue;
      bool ok = true;
      for (int o = 0; o < dgsw::kMaxNP && ok; ++o) ok = (bool)(ls >> lay[o]);
      if (!ok) continue;
      int rc = set_layouts(lay);
      if (rc != DG_OK) return rc;
      return dg_ens_set_schedule(ens, w, p, f);
    }
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const size_t bytes = ens->off[ens->n] * ens->elem_bytes;
  char *w0 = static_cast<char *>(work);
  char *w1 = w0 + bytes;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return fail(DG_EHIP, "hipEventCreate");
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(DG_EHIP, "hipEventCreate");
  }
  int rc = DG_OK;
  // two stages on the caller's state (read only: q is input, work output),
  // the best of three after a warm-up
  auto time_two_stages = [&](float *out_ms) -> int {
    float t_best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      (void)hipEventRecord(a, s);
      int r = ens_stage(ens, q, nullptr, w0, 1, 0.0, 1.0, s);
      if (r == DG_OK) r = ens_stage(ens, w0, q, w1, 1, 0.75, 0.25, s);
      if (r != DG_OK) return r;
      (void)hipEventRecord(b, s);
      (void)hipEventSynchronize(b);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, a, b);
      if (rep > 0) t_best = std::min(t_best, ms);
    }
    *out_ms = t_best;
    return DG_OK;
  };
  // 1. the layout of each order (flat per-order launches, 4 wavefronts per
  //    workgroup), one order at a time with the others unchanged
  std::vector<int> lay(dgsw::kMaxNP, DG_KERNEL_LINE);
  for (int m = 0; m < ens->n; ++m) lay[ens->members[m]->np - 1] = ens->layout[m];
  for (int o : orders) {
    float best = 1e30f;
    int best_l = lay[o];
    for (int l : {DG_KERNEL_LINE, DG_KERNEL_HALF}) {
      lay[o] = l;
      float ms = 0.f;
      if ((rc = set_layouts(lay)) != DG_OK || (rc = upload_schedule(ens, 4, 0, 0)) != DG_OK ||
          (rc = time_two_stages(&ms)) != DG_OK)
        break;
      if (ms < best) {
        best = ms;
        best_l = l;
      }
    }
    if (rc != DG_OK) break;
    lay[o] = best_l;
  }
  if (rc == DG_OK) rc = set_layouts(lay);
  // 2. the schedule: per-order or (line layouts only) one fused launch;
  //    persistent with 256 .. 16384 cost-balanced workgroups, or flat; 1, 2
  //    or 4 wavefronts per workgroup
  const int n_items = (int)ens->items.size();
  float best = 1e30f;
  int best_w = 4, best_p = 0, best_f = 0;
  for (int f : {0, 1}) {
    if (rc != DG_OK) break;
    if (f == 1 && !all_line(ens)) continue;
    for (int w : {1, 2, 4}) {
      if (rc != DG_OK) break;
      for (int p : {0, 256, 1024, 4096, 16384}) {
        if (p * w > 4 * n_items && p > 256) continue;
        float ms = 0.f;
        if ((rc = upload_schedule(ens, w, p, f)) != DG_OK || (rc = time_two_stages(&ms)) != DG_OK) break;
        if (ms < best) {
          best = ms;
          best_w = w;
          best_p = p;
          best_f = f;
        }
      }
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != DG_OK) return rc;
  rc = upload_schedule(ens, best_w, best_p, best_f);
  if (rc == DG_OK && cache_path) {
    std::ofstream o(cache_path, std::ios::app);
    o << key << " " << best_w << " " << best_p << " " << best_f;
    for (int l : lay) o << " " << l;
    o << "\n";
  }
  return rc;
}

// ------------------------------------------------------------------ graphs
static int capture(dg_graph **out, const std::function<int(hipStream_t)> &body);

int dg_graph_rk(dg_ctx *ctx, void *q, void *work, double dt, int32_t scheme, int32_t nsteps,
                dg_graph **out) {
  if (!ctx || !out) return fail(DG_EINVAL, "NULL argument");
  if (ctx->freed) return fail(DG_EINVAL, "context already freed");
  const int rc = capture(out, [&](hipStream_t s) { return dg_rk_step(ctx, q, work, dt, scheme, nsteps, s); });
  if (rc == DG_OK) {
    (*out)->ctx = ctx;
    ++ctx->graphs;
  }
  return rc;
}

int dg_graph_ens(dg_ens *ens, void *q, void *work, int32_t nsteps, dg_graph **out) {
  if (!ens || !out) return fail(DG_EINVAL, "NULL argument");
  if (ens->freed) return fail(DG_EINVAL, "ensemble already freed");
  const int rc = capture(out, [&](hipStream_t s) { return dg_ens_rk_step(ens, q, work, nsteps, s); });
  if (rc == DG_OK) {
    (*out)->ens = ens;
    ++ens->graphs;
  }
  return rc;
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
  if (graph->ctx && --graph->ctx->graphs == 0 && graph->ctx->freed) dg_free(graph->ctx);
  if (graph->ens && --graph->ens->graphs == 0 && graph->ens->freed) dg_ens_free(graph->ens);
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
