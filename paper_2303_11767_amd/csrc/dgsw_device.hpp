// Device-side table layouts and the host-callable launchers of the DG kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dgsw_tables.hpp"

namespace dgsw {

// Tables shared by every element (uploaded once per context, read by
// wave-uniform addresses, so they arrive through the scalar cache).
template <typename T, int NP>
struct GlobTab {
  T B[NP][NP];   // P~_a(xi_p), [p][a]
  T D[NP][NP];   // P~'_a(xi_p), [p][a]
  T Pp[NP];      // P~_a(+1)
  T Pm[NP];      // P~_a(-1)
  T w[NP];       // Gauss-Legendre weights
  T cF;          // 2 / dlambda: longitude volume and edge terms after M^-1
  T cG;          // 2 / dtheta:  latitude volume and edge terms after M^-1
  T g;           // gravity
  T invR;        // 1 / radius (1 on the plane)
  T href;        // reference depth H (0: off)
  T two_href;    // 2 H: the (h, mode 00) coefficient of the constant H
  T alpha;       // fixed Rusanov speed when alpha_global
};

// Tables of one latitude row (the mass matrix depends on latitude only).
template <typename T, int NP>
struct RowTab {
  T cosn[NP];     // cos(theta) at the row's latitude nodes (1 on the plane)
  T fc[NP];       // Coriolis part of the source factor: 2 Omega sin cos (f on the plane)
  T snR[NP];      // sin(theta) / R: the metric part u sin / R (0 on the plane)
  T stR[NP];      // pressure-metric factor (balanced s~ or sin) / R (0 on the plane)
  T BM[NP][NP];   // w_s sum_b' Minv[b][b'] P~_b'(eta_s), [s][b]
  T DM[NP][NP];   // w_s sum_b' Minv[b][b'] P~'_b'(eta_s), [s][b]
  T MN[NP];       // sum_b' Minv[b][b'] P~_b'(+1)
  T MS[NP];       // sum_b' Minv[b][b'] P~_b'(-1)
  T ctop;         // cos(theta) at the north edge (0 at the pole)
  T cbot;         // cos(theta) at the south edge (0 at the pole)
};

struct StageLaunch {
  const void *q;        // state L is evaluated on
  const void *q0;       // q^n of the stage combination (may alias out)
  void *out;            // result
  const void *forcing;  // optional modal forcing (may be null)
  const void *glob;     // GlobTab<T, NP> on the device
  const void *rows;     // RowTab<T, NP>[n_lat] on the device
  int n_lon, n_lat, E;
  int alpha_global;
  int periodic_y = 0;   // 1: rows wrap (plane); 0: pole rows (sphere)
  int variant = 0;      // 0: NP lanes per element; 1: 2 NP lanes (half lines)
  int combine;          // 0: out = L(q); 1: out = c0 q0 + c1 (q + dt L(q));
                        // 2: out = q0 + c1 (q - q0) + ca (qa - q0) + cb (qb - q0) + dt L(q)
  double c0, c1, dt;
  const void *qa = nullptr, *qb = nullptr;   // extra operands of combine == 2
  double ca = 0.0, cb = 0.0;
  int levels = 1;       // identical layers, each E * 3 * N values after the previous one
};

// dtype 0 = double, 1 = float; np = order + 1.  Returns a hipError_t.
hipError_t launch_stage(int dtype, int np, const StageLaunch &a, hipStream_t s);

// One work item of the ensemble kernels: one wavefront of one member, with
// everything the wavefront needs (a single 64-byte scalar load).
// One wavefront of one member.  Line layout: row j, segment seg.  Half
// layout: the elements seg .. e_end - 1 from row j on (packed across a row
// end, or one row's segment when e_end is that row's end).
struct alignas(16) EnsItem {
  long long glob;     // byte offset of the member's GlobTab<T, np> in the ensemble's table copy
  long long rows;     // byte offset of its RowTab<T, np>[n_lat] there
  long long off;      // offset of the member's state in the packed buffers (values)
  double dt;
  int n_lon, n_lat, np, j;
  int seg, alpha_global, member, e_end;
};

struct EnsLaunch {
  const void *q, *q0;
  void *out;
  const void *tabs;     // every member's tables, one device buffer (EnsItem offsets)
  const EnsItem *items;
  const int *bounds;    // parts + 1 item offsets, one contiguous range per workgroup
  int parts, combine;
  int flat;             // one item per wavefront over [begin, end) (per-order launches)
  int begin, end;
  double c0, c1;
};

// Ensemble stage, all orders in one launch: npmax = largest member order + 1
// (<= 8), wpb in {1, 2, 4}.
hipError_t launch_ens_stage(int dtype, int npmax, int wpb, const EnsLaunch &a, hipStream_t s);
// Ensemble stage over the members of one order np and one stage-kernel layout
// (0 line, 1 half; the items and bounds of that group).
hipError_t launch_ens_stage_np(int dtype, int np, int layout, int wpb, const EnsLaunch &a, hipStream_t s);

// Wavefronts (work items) of one member, and elements per wavefront.
int waves_per_row(int np, int n_lon);

// Upload helpers: convert FP64 host tables to the device layouts.
// Returns the number of bytes of each table for (dtype, np).
size_t glob_bytes(int dtype, int np);
size_t rows_bytes(int dtype, int np, int n_lat);
void fill_glob(int dtype, int np, const HostTables &t, double g, double radius,
               double omega, double href, double alpha, void *dst);
void fill_rows(int dtype, int np, const HostTables &t, void *dst);

// Mass diagnostic: partial sums per block, then one ordered final sum.
// out4 (device) = (mass_h, mass_hu, mass_hv, count of non-finite values),
// summed over the layers.
int mass_blocks();
hipError_t launch_mass(int dtype, int np, const void *q, const double *mass_w,
                       int n_lon, int E, int levels, double *partial, double *out4,
                       hipStream_t s);

}  // namespace dgsw
