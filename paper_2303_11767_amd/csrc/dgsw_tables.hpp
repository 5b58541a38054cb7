// Host precompute of the DG tables, in FP64 (section 3.2, "DG solver:
// precomputation": quadrature, Vandermonde-type basis tables and the inverse
// mass matrix are computed once on the CPU).  Pure C++: no HIP types, so it
// also builds and runs on its own for host-side checks.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace dgsw {

constexpr int kMaxOrder = 7;
constexpr int kMaxNP = kMaxOrder + 1;

// Layout of a context's projection tables: for each target order k = 0..7 a
// block [n_lat][k+1][np]; the blocks are stored one after the other.
constexpr int proj_rows_total() { return (kMaxNP * (kMaxNP + 1)) / 2; }
inline size_t proj_offset(int k, int n_lat, int np) {
  return (size_t)n_lat * np * (size_t)((k * (k + 1)) / 2);
}

// n-point Gauss-Legendre rule on [-1, 1] by Newton iteration on P_n from
// Chebyshev initial guesses; nodes ascending.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);

// Orthonormal Legendre P~_a(x) = sqrt((2a+1)/2) P_a(x) and derivative,
// a = 0..nmax, at one point (Bonnet recurrence).
void legendre_onb(int nmax, double x, double *p, double *dp);

// Everything the kernels need for one mesh, in FP64, laid out as the device
// tables (converted to the state dtype when uploaded).
struct HostTables {
  int n_lon = 0, n_lat = 0, order = 0, np = 0;
  double dlam = 0, dth = 0;
  // global 1-D tables (np x np row-major [p][a]) and edge values
  std::vector<double> B, D, Pp, Pm, w;
  // per latitude row j, node s: cos, sin, balanced or pointwise metric factor
  std::vector<double> cosn, sinn, stil;           // [j][s]
  // source factors per row node: S_hu = (fc + u snR) hv,
  // S_hv = -p stR - (fc + u snR) hu with p the pressure g h^2/2.  Sphere:
  // fc = 2 Omega sin cos, snR = sin / R, stR = (s~ or sin) / R; plane: fc = f.
  std::vector<double> fc, snR, stR;               // [j][s]
  bool periodic_y = false;                        // plane: rows wrap, no poles
  std::vector<double> ctop, cbot;                 // cos at the north/south edge of row j (0 at poles)
  // per row, the inverse latitude mass matrix folded with quadrature tables:
  //   BM[j][s][b] = w_s sum_b' Minv_j[b][b'] P~_b'(eta_s)
  //   DM[j][s][b] = w_s sum_b' Minv_j[b][b'] P~'_b'(eta_s)
  //   MN[j][b]    = sum_b' Minv_j[b][b'] P~_b'(+1),  MS[j][b] likewise at -1
  std::vector<double> BM, DM, MN, MS;
  // latitude mass matrix M_j[b][b'] = int P~_b P~_b' cos(theta_j(eta)) deta
  std::vector<double> Mth;                        // [j][b][b']
  // mass diagnostic weights: R^2 (dlam dth / 2) M_j[0][b]
  std::vector<double> mass_w;                     // [j][b]
};

// metric: 0 balanced, 1 pointwise.  Returns false (with msg) on failure.
bool build_tables(int n_lon, int n_lat, int order, int metric, double radius, double omega,
                  HostTables &t, const char **msg);

// Doubly periodic plane [0, lx] x [0, ly] with nx x ny elements and constant
// Coriolis parameter f (section 4.2, the planar shallow-water setting): the
// same tables with dlam = dx, dth = dy, cos = 1, no metric source and an
// identity latitude mass matrix (radius 1).
bool build_tables_plane(int nx, int ny, int order, double lx, double ly, double f,
                        HostTables &t, const char **msg);

}  // namespace dgsw
