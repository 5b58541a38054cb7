// Context of one mesh and the error helpers shared by the C ABI sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "dgsw.h"

struct dg_ctx {
  dg_mesh_desc d;
  int np = 0, N = 0, E = 0;
  int64_t state_n = 0;
  size_t elem_bytes = 0;
  void *d_glob = nullptr;      // GlobTab<T, np>
  void *d_rows = nullptr;      // RowTab<T, np>[n_lat]
  size_t glob_bytes = 0, rows_bytes = 0;   // sizes of the two
  double *d_mass_w = nullptr;  // mass diagnostic weights [n_lat][np]
  double *d_partial = nullptr; // mass partial sums
  double *d_out4 = nullptr;    // mass result
  const void *forcing = nullptr;
  double min_width = 0.0;
  double *d_proj = nullptr;    // cos-weighted projection onto order k = 0..7: blocks
                               // [n_lat][k+1][np] at dgsw::proj_offset(k, n_lat, np)
  double mass_area = 0.0;      // sum over elements of mass_w[j][0]
  int periodic_y = 0;          // 1: the doubly periodic plane
  int kernel = 0;              // DG_KERNEL_LINE or DG_KERNEL_HALF
  int levels = 1;              // identical layers held by every state buffer
  int64_t level_n = 0;         // values of one layer, E * 3 * N
  int member = 0;              // 1: owned by an ensemble (one layer only)
  int graphs = 0;              // live dg_graph objects captured on this context
  int freed = 0;               // dg_free called while graphs were live: release deferred
};

namespace dgsw {
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
bool aligned16(const void *p);
}  // namespace dgsw
