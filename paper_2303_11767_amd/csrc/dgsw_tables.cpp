// Host precompute of the DG tables in FP64; see dgsw_tables.hpp.
#include "dgsw_tables.hpp"

#include <cmath>

namespace dgsw {

static const double kPi = 3.14159265358979323846;

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  if (n == 1) { x[0] = 0.0; w[0] = 2.0; return; }
  for (int k = 0; k < (n + 1) / 2; ++k) {
    // k-th largest root of P_n, refined by Newton on the standard P_n
    double z = std::cos(kPi * (k + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int m = 1; m < n; ++m) {
        double p2 = ((2.0 * m + 1.0) * z * p1 - m * p0) / (m + 1.0);
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    {  // final derivative at the converged root
      double p0 = 1.0, p1 = z;
      for (int m = 1; m < n; ++m) {
        double p2 = ((2.0 * m + 1.0) * z * p1 - m * p0) / (m + 1.0);
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    double wk = 2.0 / ((1.0 - z * z) * dp * dp);
    x[n - 1 - k] = z;
    x[k] = -z;
    w[n - 1 - k] = wk;
    w[k] = wk;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

void legendre_onb(int nmax, double x, double *p, double *dp) {
  double P[kMaxNP + 2], dP[kMaxNP + 2];
  P[0] = 1.0;
  dP[0] = 0.0;
  if (nmax >= 1) { P[1] = x; dP[1] = 1.0; }
  for (int k = 1; k < nmax; ++k) {
    P[k + 1] = ((2.0 * k + 1.0) * x * P[k] - k * P[k - 1]) / (k + 1.0);
    dP[k + 1] = dP[k - 1] + (2.0 * k + 1.0) * P[k];
  }
  for (int a = 0; a <= nmax; ++a) {
    double s = std::sqrt((2.0 * a + 1.0) / 2.0);
    p[a] = s * P[a];
    dp[a] = s * dP[a];
  }
}

// In-place inverse of a small SPD matrix by Gauss-Jordan with partial pivoting.
static bool invert(int n, std::vector<double> &A) {
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) { std::swap(A[c * n + k], A[piv * n + k]); std::swap(I[c * n + k], I[piv * n + k]); }
    double d = 1.0 / A[c * n + c];
    for (int k = 0; k < n; ++k) { A[c * n + k] *= d; I[c * n + k] *= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) { A[r * n + k] -= f * A[c * n + k]; I[r * n + k] -= f * I[c * n + k]; }
    }
  }
  A.swap(I);
  return true;
}

namespace {

// Everything that depends on the row geometry only through cos(theta) of the
// nodes, the row edges and the mass-matrix weight function: the 1-D basis
// tables, the latitude mass matrix, its inverse folded into the quadrature
// tables, and the mass diagnostic weights.  plane: cos = 1 everywhere.
bool build_common(int n_lon, int n_lat, int order, double dlam, double dth, bool plane,
                  double radius, HostTables &t, const char **msg) {
  const int np = order + 1;
  t.n_lon = n_lon;
  t.n_lat = n_lat;
  t.order = order;
  t.np = np;
  t.dlam = dlam;
  t.dth = dth;
  t.periodic_y = plane;

  std::vector<double> x, w;
  gauss_legendre(np, x, w);
  t.w = w;
  t.B.assign(np * np, 0.0);
  t.D.assign(np * np, 0.0);
  t.Pp.assign(np, 0.0);
  t.Pm.assign(np, 0.0);
  double pv[kMaxNP], dv[kMaxNP];
  for (int p = 0; p < np; ++p) {
    legendre_onb(order, x[p], pv, dv);
    for (int a = 0; a < np; ++a) { t.B[p * np + a] = pv[a]; t.D[p * np + a] = dv[a]; }
  }
  legendre_onb(order, 1.0, pv, dv);
  for (int a = 0; a < np; ++a) t.Pp[a] = pv[a];
  legendre_onb(order, -1.0, pv, dv);
  for (int a = 0; a < np; ++a) t.Pm[a] = pv[a];

  // 32-point rule in latitude for the mass matrix (exact to roundoff for
  // degree-2r polynomials times the analytic cos over one row)
  std::vector<double> xq, wq;
  const int nq = 32;
  gauss_legendre(nq, xq, wq);
  std::vector<double> Pq(nq * np);
  for (int q = 0; q < nq; ++q) {
    legendre_onb(order, xq[q], pv, dv);
    for (int b = 0; b < np; ++b) Pq[q * np + b] = pv[b];
  }

  t.cosn.assign(n_lat * np, 0.0);
  t.sinn.assign(n_lat * np, 0.0);
  t.stil.assign(n_lat * np, 0.0);
  t.ctop.assign(n_lat, 0.0);
  t.cbot.assign(n_lat, 0.0);
  t.BM.assign(n_lat * np * np, 0.0);
  t.DM.assign(n_lat * np * np, 0.0);
  t.MN.assign(n_lat * np, 0.0);
  t.MS.assign(n_lat * np, 0.0);
  t.Mth.assign(n_lat * np * np, 0.0);
  t.mass_w.assign(n_lat * np, 0.0);

  for (int j = 0; j < n_lat; ++j) {
    const double tb = -0.5 * kPi + j * t.dth;
    const double cb = plane ? 1.0 : (j == 0) ? 0.0 : std::cos(tb);
    const double ct = plane ? 1.0 : (j == n_lat - 1) ? 0.0 : std::cos(tb + t.dth);
    t.cbot[j] = cb;
    t.ctop[j] = ct;
    for (int s = 0; s < np; ++s) {
      double th = tb + 0.5 * (1.0 + x[s]) * t.dth;
      t.cosn[j * np + s] = plane ? 1.0 : std::cos(th);
      t.sinn[j * np + s] = plane ? 0.0 : std::sin(th);
    }
    // latitude mass matrix
    std::vector<double> M(np * np, 0.0);
    for (int q = 0; q < nq; ++q) {
      double wc = wq[q] * (plane ? 1.0 : std::cos(tb + 0.5 * (1.0 + xq[q]) * t.dth));
      for (int b = 0; b < np; ++b)
        for (int c = 0; c < np; ++c) M[b * np + c] += wc * Pq[q * np + b] * Pq[q * np + c];
    }
    for (int k = 0; k < np * np; ++k) t.Mth[j * np * np + k] = M[k];
    for (int b = 0; b < np; ++b)
      t.mass_w[j * np + b] = radius * radius * 0.5 * t.dlam * t.dth * M[0 * np + b];
    std::vector<double> Mi = M;
    if (!invert(np, Mi)) { *msg = "singular latitude mass matrix"; return false; }
    // folded tables
    for (int s = 0; s < np; ++s)
      for (int b = 0; b < np; ++b) {
        double bm = 0.0, dm = 0.0;
        for (int c = 0; c < np; ++c) {
          bm += Mi[b * np + c] * t.B[s * np + c];
          dm += Mi[b * np + c] * t.D[s * np + c];
        }
        t.BM[(j * np + s) * np + b] = w[s] * bm;
        t.DM[(j * np + s) * np + b] = w[s] * dm;
      }
    for (int b = 0; b < np; ++b) {
      double mn = 0.0, ms = 0.0;
      for (int c = 0; c < np; ++c) { mn += Mi[b * np + c] * t.Pp[c]; ms += Mi[b * np + c] * t.Pm[c]; }
      t.MN[j * np + b] = mn;
      t.MS[j * np + b] = ms;
    }
  }
  return true;
}

}  // namespace

bool build_tables(int n_lon, int n_lat, int order, int metric, double radius, double omega,
                  HostTables &t, const char **msg) {
  if (!build_common(n_lon, n_lat, order, 2.0 * kPi / n_lon, kPi / n_lat, false, radius, t, msg))
    return false;
  const int np = order + 1;
  const std::vector<double> &w = t.w;
  t.fc.assign(n_lat * np, 0.0);
  t.snR.assign(n_lat * np, 0.0);
  t.stR.assign(n_lat * np, 0.0);
  for (int j = 0; j < n_lat; ++j) {
    const double cb = t.cbot[j], ct = t.ctop[j];
    // metric factor of the pressure source
    if (metric == 0) {
      // beta_b = sum_s w_s cos(theta_s) P~'_b(eta_s) - (c_t P~_b(1) - c_b P~_b(-1));
      // s~_s = (2/dth) sum_b P~_b(eta_s) beta_b
      double beta[kMaxNP];
      for (int b = 0; b < np; ++b) {
        double acc = 0.0;
        for (int s = 0; s < np; ++s) acc += w[s] * t.cosn[j * np + s] * t.D[s * np + b];
        beta[b] = acc - (ct * t.Pp[b] - cb * t.Pm[b]);
      }
      for (int s = 0; s < np; ++s) {
        double acc = 0.0;
        for (int b = 0; b < np; ++b) acc += t.B[s * np + b] * beta[b];
        t.stil[j * np + s] = (2.0 / t.dth) * acc;
      }
    } else {
      for (int s = 0; s < np; ++s) t.stil[j * np + s] = t.sinn[j * np + s];
    }
    for (int s = 0; s < np; ++s) {
      const int k = j * np + s;
      t.fc[k] = 2.0 * omega * t.sinn[k] * t.cosn[k];
      t.snR[k] = t.sinn[k] / radius;
      t.stR[k] = t.stil[k] / radius;
    }
  }
  return true;
}

bool build_tables_plane(int nx, int ny, int order, double lx, double ly, double f,
                        HostTables &t, const char **msg) {
  if (!build_common(nx, ny, order, lx / nx, ly / ny, true, 1.0, t, msg)) return false;
  const size_t n = (size_t)ny * (order + 1);
  t.stil.assign(n, 0.0);
  t.fc.assign(n, f);
  t.snR.assign(n, 0.0);
  t.stR.assign(n, 0.0);
  return true;
}

}  // namespace dgsw
