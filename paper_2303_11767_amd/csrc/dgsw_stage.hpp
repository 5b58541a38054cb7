// Device code of one stage of the DG right-hand side, shared by the mesh
// kernels (dgsw_kernels.hip) and the ensemble kernels (dgsw_ens_kernels.hip).
//
// HIP kernels of the modal DG shallow-water right-hand side on the sphere,
// for gfx950 (64-wide wavefronts).  The same kernels run the doubly periodic
// plane of section 4.2 (cos = 1, radius 1, constant f, rows that wrap), which
// differs from the sphere only in its tables and the row wrap.
//
// One fused kernel per Runge-Kutta stage.  Work unit: one element, handled by
// NP = r+1 lanes ("line lanes"); a 64-lane wavefront holds 64/NP elements and
// is one workgroup.  Lane t of an element owns line t of the element's data in
// every phase and the phases are joined by transposes through LDS:
//
//   load      lane t holds modal row b = t of h, hu, hv (n contiguous values:
//             coalesced 16-byte loads across the element's lanes)
//   xi pass   A[p][b=t] = sum_a q[a][t] P~_a(xi_p), and the same at xi = +-1
//   --- LDS transpose ---
//   eta pass  lane t = node column p: nodal values Q[t][s] (modal -> quadrature
//             of h, hu, hv, eq. "basis_expansion") and the north/south traces;
//             lane t = edge node s: the east/west traces
//   halo      traces of the four neighbours at the shared edges, each from one
//             row or column of the neighbour's coefficients (periodic in
//             longitude, none across a pole; periodic in y on the plane)
//   edges     Rusanov flux (eq. "rusanov") at edge node t of all four edges
//   volume    fluxes F, G and sources S at the n nodes of column t, contracted
//             over the latitude nodes with the inverse mass matrix folded in
//             (per-row tables BM, DM, MN, MS), north/south surface terms added
//   --- LDS transpose ---
//   xi pass   lane t = latitude degree b: contraction over the longitude nodes
//             with P~' (F term) and P~ (G and S terms), east/west surface
//             terms, giving row b of dq/dt = M^-1 h(q) (eq. "ode")
//   epilogue  optional forcing, then either dq/dt, the Shu-Osher stage
//             combination c0 q^n + c1 (q + dt dq/dt), or the general one
//             q^n + c1 (q - q^n) + ca (qa - q^n) + cb (qb - q^n) + dt dq/dt
//             (classical RK4); both written so that the weights of the states
//             sum to one exactly in the working precision (no systematic
//             mass drift from rounded coefficients such as 1/3), stored
//             as row b.
//
// The weak form is that of eq. "dg_parts": volume term of F . grad(phi) plus
// the source, minus the surface term of the Rusanov flux times phi.  Integrals
// are in (lambda, theta) coordinates: the longitude volume and edge terms
// carry dtheta/2, the latitude ones dlambda/2, the source dlambda dtheta/4, and
// the mass matrix dlambda dtheta/4 times the latitude matrix
// int P~_b P~_b' cos(theta) deta, whose inverse is folded into the tables
// (hence the constants 2/dlambda and 2/dtheta).
#pragma once

#include "dgsw_device.hpp"

#include <cstddef>
#include <cstring>
#include <type_traits>

namespace dgsw {


template <typename T, int NP>
struct Shape {
  static constexpr int N = NP * NP;
  static constexpr int GPW = 64 / NP;  // elements per wavefront
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  // per-element LDS, two phases sharing one region:
  //   A/B: the xi-pass rows (n+2 per variable) and the neighbour partial sums
  //   C/D: the second transpose (two n x n per variable) and the E/W edge fluxes
  static constexpr int NB = 3 * (NP + 2) * NP;
  static constexpr int SH = cmax(NB + 12 * NP, 6 * NP * NP + 6 * NP);
  // tables read with a lane-dependent index, copied to LDS per wavefront:
  // P~(xi_p) [p][a], weights, and the row's BM [s][b] (TBU values), the
  // region rounded up to whole 64-lane rounds of the copy
  static constexpr int TBU = NP * NP + NP + NP * NP;
  static constexpr int TB = (TBU + 63) / 64 * 64;
  // byte alignment of one modal row (NP values) given a 16-byte aligned base
  static constexpr int gcd(int a, int b) { return b == 0 ? a : gcd(b, a % b); }
  static constexpr int ROWALIGN = gcd(16, NP * (int)sizeof(T));
};

// Reciprocal and square root from the hardware approximations.  FP64: v_rcp_f64
// refined by two Newton steps, and v_rsq_f64 refined by a Goldschmidt step (both
// within an ulp or two for the normal, positive depths used here); FP32: v_rcp_f32
// and v_sqrt_f32 (1 ulp).  The square root only enters the Rusanov speed estimate.
template <typename T>
__device__ __forceinline__ T dg_rcp(T x);
template <>
__device__ __forceinline__ double dg_rcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
template <>
__device__ __forceinline__ float dg_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename T>
__device__ __forceinline__ T dg_sqrt(T x);
template <>
__device__ __forceinline__ double dg_sqrt<double>(double x) {
  // One Goldschmidt step from the hardware reciprocal square root (about 29
  // correct bits): with g = x y and h = y / 2, r = 1/2 - g h and g + g r has a
  // relative error of about 3/2 of the square of y's, i.e. within an ulp or two;
  // enough for the wave-speed estimate, the only use of this square root.
  const double y = __builtin_amdgcn_rsq(x);
  const double g = x * y;
  const double r = __builtin_fma(-g, 0.5 * y, 0.5);
  return __builtin_fma(g, r, g);
}
template <>
__device__ __forceinline__ float dg_sqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

// LDS ordering between the lanes of one wavefront (a workgroup is one
// wavefront): LDS requests of a wave complete in order, so a wave-scope fence
// around a scheduling barrier is enough.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroups are dispatched round-robin over the 8 XCDs; renumber them so that
// each XCD gets one contiguous range of rows (its L2 then holds the rows and
// their north/south neighbours).  Bijective for any count.
__device__ __forceinline__ int xcd_block(int w, int nb) {
  const int xcd = w & 7, k = w >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return xcd < rem ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

template <typename T, int NP>
__device__ __forceinline__ void load_row(const T *p, T (&r)[NP]) {
  const T *pa = static_cast<const T *>(__builtin_assume_aligned(p, Shape<T, NP>::ROWALIGN));
#pragma unroll
  for (int a = 0; a < NP; ++a) r[a] = pa[a];
}

template <typename T, int NP>
__device__ __forceinline__ void store_row(T *p, const T (&r)[NP]) {
  T *pa = static_cast<T *>(__builtin_assume_aligned(p, Shape<T, NP>::ROWALIGN));
#pragma unroll
  for (int a = 0; a < NP; ++a) pa[a] = r[a];
}

// One side of a Rusanov edge: velocity along the edge normal and sqrt(g h).
// Variable 0 of a trace is h - H; the pressure is g (h^2 - H^2) / 2.
template <typename T>
struct Side {
  T h, rh, u, v, p, c;
  __device__ __forceinline__ Side(const T q[3], T H, T g) {
    h = q[0] + H;
    rh = dg_rcp(h);
    u = q[1] * rh;
    v = q[2] * rh;
    p = T(0.5) * g * q[0] * (h + H);
    c = dg_sqrt(g * h);
  }
};

// Rusanov bracket on a constant-longitude edge, without the 1/R factor:
// (f(q-) + f(q+))/2 - alpha/2 (q+ - q-), f = (hu, hu u + p, hu v).  The
// bracket is symmetric in its two states except for the jump, so the caller
// may pass them in either order: sgn = 1 for (q-, q+), -1 for (q+, q-) (the
// result is the same to the last bit: only signs change).
template <typename T>
__device__ __forceinline__ void rusanov_lambda(const T qm[3], const T qp[3], T H, T g,
                                               bool fixed, T alpha_fixed, T out[3], T sgn = T(1)) {
  const Side<T> m(qm, H, g), p(qp, H, g);
  T a = alpha_fixed;
  if (!fixed) {
    const T sm = fabs(m.u) + m.c, sp = fabs(p.u) + p.c;
    a = fmax(sm, sp);
  }
  a *= sgn;
  out[0] = T(0.5) * (qm[1] + qp[1]) - T(0.5) * a * (qp[0] - qm[0]);
  out[1] = T(0.5) * ((qm[1] * m.u + m.p) + (qp[1] * p.u + p.p)) - T(0.5) * a * (qp[1] - qm[1]);
  out[2] = T(0.5) * (qm[1] * m.v + qp[1] * p.v) - T(0.5) * a * (qp[2] - qm[2]);
}

// Same on a constant-latitude edge, g-flux = (hv, hv u, hv v + p), without
// the cos(theta_edge)/R factor.
template <typename T>
__device__ __forceinline__ void rusanov_theta(const T qm[3], const T qp[3], T H, T g,
                                              bool fixed, T alpha_fixed, T out[3], T sgn = T(1)) {
  const Side<T> m(qm, H, g), p(qp, H, g);
  T a = alpha_fixed;
  if (!fixed) {
    const T sm = fabs(m.v) + m.c, sp = fabs(p.v) + p.c;
    a = fmax(sm, sp);
  }
  a *= sgn;
  out[0] = T(0.5) * (qm[2] + qp[2]) - T(0.5) * a * (qp[0] - qm[0]);
  out[1] = T(0.5) * (qm[2] * m.u + qp[2] * p.u) - T(0.5) * a * (qp[1] - qm[1]);
  out[2] = T(0.5) * ((qm[2] * m.v + m.p) + (qp[2] * p.v + p.p)) - T(0.5) * a * (qp[2] - qm[2]);
}

// Arguments of one stage on one mesh.
template <typename T, int NP>
struct StageArgs {
  const T *q;            // state L is evaluated on
  const T *q0;           // q^n of the combination (may alias out)
  T *out;
  const T *forcing;      // optional modal forcing
  const T *qa, *qb;      // extra states of the general combination (may be null)
  const GlobTab<T, NP> *gt;
  const RowTab<T, NP> *rows;
  int n_lon, n_lat, alpha_global, combine, periodic_y;
  T c0, c1, dt, ca, cb;
  T ce;                  // c0 + c1 - 1, formed in FP64 on the host (0 for the schemes here)
  int levels;            // identical layers, one after the other in every state buffer
  long long lstride;     // values of one layer (E * 3 * N)
};

// The arguments of layer `lev`: every state-shaped pointer moved to the layer.
template <typename T, int NP>
__device__ __forceinline__ StageArgs<T, NP> layer_args(const StageArgs<T, NP> &A, int lev) {
  StageArgs<T, NP> B = A;
  const long long off = (long long)lev * A.lstride;
  B.q = A.q + off;
  B.q0 = A.q0 ? A.q0 + off : nullptr;
  B.out = A.out + off;
  B.forcing = A.forcing ? A.forcing + off : nullptr;
  B.qa = A.qa ? A.qa + off : nullptr;
  B.qb = A.qb ? A.qb + off : nullptr;
  return B;
}

// One wavefront's share of a stage: GPW elements of one latitude row
// (segment `seg` of row j), so the row's tables are wave-uniform (scalar
// loads) and the pole tests are uniform branches.  tab and sh are this
// wavefront's LDS slices (TB and (GPW+1)*SH values).
// CM: the stage combination as a compile-time mode (0: dq/dt, 1: Shu-Osher,
// 2: general) so each launch carries only its own epilogue, or CM_RUNTIME to
// take 0 or 1 from A.combine (the ensemble kernels).
constexpr int CM_RUNTIME = 3;

template <typename T, int NP, int CM>
__device__ __forceinline__ void stage_wave(const StageArgs<T, NP> &A, const int j, const int seg,
                                           const int lane, T *tab, T *sh) {
  using S_ = Shape<T, NP>;
  constexpr int N = S_::N, GPW = S_::GPW, SH = S_::SH, NB = S_::NB;
  const T *__restrict__ q = A.q;
  const T *q0 = A.q0;
  T *out = A.out;
  const T *__restrict__ forcing = A.forcing;
  const GlobTab<T, NP> *__restrict__ gt = A.gt;
  const RowTab<T, NP> *__restrict__ rows = A.rows;
  const int n_lon = A.n_lon, n_lat = A.n_lat;
  const int combine = CM == CM_RUNTIME ? (A.combine != 0 ? 1 : 0) : CM;
  const T c0 = A.c0, c1 = A.c1, dt = A.dt;
  int g = lane / NP, t = lane - g * NP;
  const bool idle = g >= GPW;          // the 64 mod NP spare lanes: a dummy LDS slot
  if (idle) { g = GPW; t = lane - GPW * NP; }
  const int i_raw = seg * GPW + g;
  const bool active = !idle && i_raw < n_lon;
  const int i = i_raw < n_lon ? i_raw : n_lon - 1;   // tail lanes work on a valid element
  const int e = j * n_lon + i;
  T *S = sh + g * SH;
  const RowTab<T, NP> *rt = rows + j;
  const bool periodic = A.periodic_y != 0;
  const bool hasN = periodic || j < n_lat - 1, hasS = periodic || j > 0;
  // north / south neighbours (rows wrap on the plane)
  const int eN = j < n_lat - 1 ? e + n_lon : i;
  const int eS = j > 0 ? e - n_lon : (n_lat - 1) * n_lon + i;
  const T H = gt->href, H2 = gt->two_href, grav = gt->g, invR = gt->invR;
  const bool fixed = A.alpha_global != 0;
  const T alpha = gt->alpha;

  // ---- every global load of the stage, issued up front
  const size_t row_off = (size_t)t * NP;
  const size_t base = (size_t)e * 3 * N + row_off;
  const int eE = (i + 1 == n_lon) ? e + 1 - n_lon : e + 1;
  const int eW = (i == 0) ? e - 1 + n_lon : e - 1;
  T qr[3][NP], xE[3][NP], xW[3][NP], xN[3][NP], xS[3][NP];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    load_row<T, NP>(q + base + v * N, qr[v]);
    load_row<T, NP>(q + (size_t)eE * 3 * N + row_off + v * N, xE[v]);   // row b = t
    load_row<T, NP>(q + (size_t)eW * 3 * N + row_off + v * N, xW[v]);
  }
  if (hasN) {
    const T *c = q + (size_t)eN * 3 * N + t;                             // column a = t
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int k = 0; k < NP; ++k) xN[v][k] = c[v * N + k * NP];
  } else {
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int k = 0; k < NP; ++k) xN[v][k] = T(0);
  }
  if (hasS) {
    const T *c = q + (size_t)eS * 3 * N + t;
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int k = 0; k < NP; ++k) xS[v][k] = c[v * N + k * NP];
  } else {
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int k = 0; k < NP; ++k) xS[v][k] = T(0);
  }
  {
    // one round of 64 lanes up to r = 4 (a single wait, which the state
    // loads need anyway); the registers of a two-phase copy would push the
    // FP64 r >= 4 kernels into scratch
    const T *gB = &gt->B[0][0], *gw = &gt->w[0], *rBM = &rt->BM[0][0];
    for (int k = lane; k < S_::TBU; k += 64)
      tab[k] = k < NP * NP ? gB[k] : (k < NP * NP + NP ? gw[k - NP * NP] : rBM[k - NP * NP - NP]);
  }

  // ---- xi pass: A[v][p][b=t] and the xi = +1/-1 rows; neighbour partial sums
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    T qa[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) qa[a] = qr[v][a];
    if (v == 0 && t == 0) qa[0] -= H2;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      T acc = T(0);
#pragma unroll
      for (int a = 0; a < NP; ++a) acc += qa[a] * gt->B[p][a];
      S[(v * (NP + 2) + p) * NP + t] = acc;
    }
    T ae = T(0), aw = T(0);
#pragma unroll
    for (int a = 0; a < NP; ++a) { ae += qa[a] * gt->Pp[a]; aw += qa[a] * gt->Pm[a]; }
    S[(v * (NP + 2) + NP) * NP + t] = ae;
    S[(v * (NP + 2) + NP + 1) * NP + t] = aw;

    T ue = T(0), uw = T(0), vn = T(0), vs = T(0);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      T ye = xE[v][k], yw = xW[v][k], yn = xN[v][k], ys = xS[v][k];
      if (v == 0 && t == 0 && k == 0) { ye -= H2; yw -= H2; yn -= H2; ys -= H2; }
      ue += ye * gt->Pm[k];   // east neighbour seen from its west edge
      uw += yw * gt->Pp[k];   // west neighbour seen from its east edge
      vn += yn * gt->Pm[k];   // north neighbour seen from its south edge
      vs += ys * gt->Pp[k];   // south neighbour seen from its north edge
    }
    S[NB + (0 * 3 + v) * NP + t] = ue;
    S[NB + (1 * 3 + v) * NP + t] = uw;
    S[NB + (2 * 3 + v) * NP + t] = vn;
    S[NB + (3 * 3 + v) * NP + t] = vs;
  }
  wave_sync();

  // ---- eta pass: nodal values of column p = t, own and neighbour traces at node t
  T nd[3][NP], trN[3], trS[3], trE[3], trW[3], nbE[3], nbW[3], nbN[3], nbS[3];
  T bt[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) bt[k] = tab[t * NP + k];          // P~_k(xi_t)
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    T col[NP];
#pragma unroll
    for (int b = 0; b < NP; ++b) col[b] = S[(v * (NP + 2) + t) * NP + b];
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      T acc = T(0);
#pragma unroll
      for (int b = 0; b < NP; ++b) acc += col[b] * gt->B[s][b];
      nd[v][s] = acc;
    }
    T an = T(0), as = T(0), ae = T(0), aw = T(0);
    T ne = T(0), nw = T(0), nn = T(0), ns = T(0);
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      an += col[b] * gt->Pp[b];
      as += col[b] * gt->Pm[b];
      ae += S[(v * (NP + 2) + NP) * NP + b] * bt[b];
      aw += S[(v * (NP + 2) + NP + 1) * NP + b] * bt[b];
      ne += S[NB + (0 * 3 + v) * NP + b] * bt[b];
      nw += S[NB + (1 * 3 + v) * NP + b] * bt[b];
      nn += S[NB + (2 * 3 + v) * NP + b] * bt[b];
      ns += S[NB + (3 * 3 + v) * NP + b] * bt[b];
    }
    trN[v] = an; trS[v] = as; trE[v] = ae; trW[v] = aw;
    nbE[v] = ne; nbW[v] = nw; nbN[v] = nn; nbS[v] = ns;
  }
  wave_sync();

  // ---- Rusanov fluxes at edge node t of the four edges (minus = west/south)
  T FhE[3], FhW[3], GhN[3], GhS[3];
  rusanov_lambda<T>(trE, nbE, H, grav, fixed, alpha, FhE);
  rusanov_lambda<T>(nbW, trW, H, grav, fixed, alpha, FhW);
  if (hasN) {
    rusanov_theta<T>(trN, nbN, H, grav, fixed, alpha, GhN);
  }
  if (hasS) {
    rusanov_theta<T>(nbS, trS, H, grav, fixed, alpha, GhS);
  }
  const T fN = hasN ? rt->ctop * invR : T(0);   // zero flux through a pole (sphere)
  const T fS = hasS ? rt->cbot * invR : T(0);
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    FhE[v] *= invR;
    FhW[v] *= invR;
    GhN[v] = hasN ? GhN[v] * fN : T(0);
    GhS[v] = hasS ? GhS[v] * fS : T(0);
  }

  // ---- volume: fluxes and sources at the nodes (p = t, s), contracted over s
  T ZD[3][NP], ZG[3][NP], ZS[2][NP];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int b = 0; b < NP; ++b) { ZD[v][b] = T(0); ZG[v][b] = T(0); }
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int b = 0; b < NP; ++b) ZS[v][b] = T(0);
#pragma unroll
  for (int s = 0; s < NP; ++s) {
    const T dh = nd[0][s], hu = nd[1][s], hv = nd[2][s];
    const T h = dh + H;
    const T rh = dg_rcp(h);
    const T u = hu * rh, vv = hv * rh;
    const T pr = T(0.5) * grav * dh * (h + H);
    const T c = rt->cosn[s];
    const T F0 = hu * invR, F1 = (hu * u + pr) * invR, F2 = hu * vv * invR;
    const T cR = c * invR;
    const T G0 = hv * cR, G1 = hv * u * cR, G2 = (hv * vv + pr) * cR;
    const T C = rt->fc[s] + u * rt->snR[s];       // f cos + u sin / R (f on the plane)
    const T S1 = C * hv, S2 = -pr * rt->stR[s] - C * hu;
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      const T bm = rt->BM[s][b], dm = rt->DM[s][b];
      ZD[0][b] += F0 * bm; ZD[1][b] += F1 * bm; ZD[2][b] += F2 * bm;
      ZG[0][b] += G0 * dm; ZG[1][b] += G1 * dm; ZG[2][b] += G2 * dm;
      ZS[0][b] += S1 * bm; ZS[1][b] += S2 * bm;
    }
  }
  const T wt = tab[NP * NP + t], cF = gt->cF, cG = gt->cG;
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      T zg = ZG[v][b];
      zg -= GhN[v] * rt->MN[b];
      zg += GhS[v] * rt->MS[b];
      const T zs = v == 0 ? T(0) : ZS[v - 1][b];
      S[((v * 2 + 0) * NP + t) * NP + b] = cF * wt * ZD[v][b];
      S[((v * 2 + 1) * NP + t) * NP + b] = wt * (cG * zg + zs);
    }
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    S[6 * NP * NP + (v * 2 + 0) * NP + t] = FhE[v];
    S[6 * NP * NP + (v * 2 + 1) * NP + t] = FhW[v];
  }
  wave_sync();

  // ---- the epilogue's operands, loaded late to keep registers free: q (again,
  // from cache), q^n and the forcing
  const bool use_q0 = combine == 2 || (combine == 1 && c0 != T(0));
  T q0r[3][NP], fr[3][NP];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    if (combine) load_row<T, NP>(q + base + v * N, qr[v]);
    if (use_q0) {
      load_row<T, NP>(q0 + base + v * N, q0r[v]);
    } else {
#pragma unroll
      for (int a = 0; a < NP; ++a) q0r[v][a] = T(0);
    }
    if (forcing) {
      load_row<T, NP>(forcing + base + v * N, fr[v]);
    } else {
#pragma unroll
      for (int a = 0; a < NP; ++a) fr[v][a] = T(0);
    }
  }

  // ---- xi pass back to modes: lane t = latitude degree b
  T bmt[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) bmt[p] = tab[NP * NP + NP + p * NP + t];   // BM[p][t]
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    T zd[NP], zb[NP];
    T XE = T(0), XW = T(0);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      zd[p] = S[((v * 2 + 0) * NP + p) * NP + t];
      zb[p] = S[((v * 2 + 1) * NP + p) * NP + t];
      XE += S[6 * NP * NP + (v * 2 + 0) * NP + p] * bmt[p];
      XW += S[6 * NP * NP + (v * 2 + 1) * NP + p] * bmt[p];
    }
    // general combination (combine == 2, classical RK4): its two extra
    // operands, loaded one variable at a time
    T xa[NP], xb[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) xa[a] = xb[a] = T(0);
    if (combine == 2 && A.qa) load_row<T, NP>(A.qa + base + v * N, xa);
    if (combine == 2 && A.qb) load_row<T, NP>(A.qb + base + v * N, xb);
    T res[NP];
    const T cXE = cF * XE, cXW = cF * XW;
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      // the forcing, then chained FMAs (a sum of products first costs a third instruction)
      T acc = fr[v][a];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        acc += gt->D[p][a] * zd[p];
        acc += gt->B[p][a] * zb[p];
      }
      acc -= gt->Pp[a] * cXE;
      acc += gt->Pm[a] * cXW;
      if (combine == 2) {
        const T b0 = q0r[v][a];
        res[a] = b0 + dt * acc + (c1 * (qr[v][a] - b0) + (A.ca * (xa[a] - b0) + A.cb * (xb[a] - b0)));
      } else if (combine) {
        // c0 q0 + c1 y = y + c0 (q0 - y) + (c0 + c1 - 1) y, y = q + dt L
        const T y = qr[v][a] + dt * acc;
        res[a] = y + c0 * (q0r[v][a] - y) + A.ce * y;
      } else {
        res[a] = acc;
      }
    }
    if (active) store_row<T, NP>(out + base + v * N, res);
  }
}

// ------------------------------------------------------------------ half-line variant
// Same stage with 2 NP lanes per element: lane (h, t), h = 0 or 1, owns line t
// as above but only half of each line's outputs (indices h K0 .. h K0 + K0 - 1,
// K0 = ceil(NP / 2)), and half of the edge work: h = 0 the east and north
// edges, h = 1 the west and south edges (traces, neighbour loads and Rusanov
// fluxes).  In the volume both halves evaluate the fluxes at all NP nodes of
// column t and each contracts them for its own K0 outputs, so no partial
// sums cross between the halves (only the latitude edge fluxes, through
// LDS).  Twice the wavefronts with about 0.6x the instructions and 0.7x the
// registers each: more latency hiding where one wavefront per SIMD is all a
// mesh provides, and higher occupancy on large meshes.
template <typename T, int NP>
struct ShapeH2 {
  static constexpr int N = NP * NP;
  static constexpr int GPW = 64 / (2 * NP);            // elements per wavefront
  static constexpr bool SPARE = GPW * 2 * NP < 64;      // lanes left over: a dummy slot
  static constexpr int K0 = (NP + 1) / 2;
  static constexpr int NB = 3 * (NP + 2) * NP;
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  // SPLIT: each half evaluates the node terms at its own NP / 2 nodes of a
  // column and hands them to the other half (FP64 with an even r + 1 >= 4)
  static constexpr bool SPLIT = sizeof(T) == 8 && NP % 2 == 0 && NP >= 4;
  // second phase: the volume outputs [3][2][NP][NP], the longitude edge
  // fluxes of both halves [3][2][NP], and the latitude ones [3][2][NP] (oGY).
  // With SPLIT the latitude ones and then the node terms, XQ quantities
  // [XQ][NP][NP] at a time, use the region of the volume outputs first (both
  // are read before those are written), which keeps FP64 r = 3 within the LDS
  // of 16 wavefronts per CU.
  static constexpr int oFX = 6 * NP * NP, oGY = SPLIT ? 0 : oFX + 6 * NP, XQ = 4;
  static constexpr int SH = cmax(NB + 12 * NP, oFX + (SPLIT ? 6 : 12) * NP);
  static constexpr int SLOTS = GPW + (SPARE ? 1 : 0);
  // LDS copy of the tables: the GlobTab prefix (B, D, Pp, Pm, w), then the
  // whole RowTab of the wavefront's first row and of the row after it (a
  // wavefront of consecutive elements may end in the next row)
  static constexpr int oB = 0, oD = N, oPp = 2 * N, oPm = 2 * N + NP, oW = 2 * N + 2 * NP;
  static constexpr int G1 = 2 * N + 3 * NP;
  static constexpr int rCos = 0, rFc = NP, rSnR = 2 * NP, rStR = 3 * NP;
  static constexpr int rBM = 4 * NP, rDM = rBM + N, rMN = rDM + N, rMS = rMN + NP;
  static constexpr int rTop = rMS + NP, rBot = rTop + 1;
  static constexpr int RP = rBot + 1;                   // values of one RowTab
  // rounded up to whole 64-lane rounds: the copy stores every lane's value
  // (those past the tables are clamped duplicates, never read)
  static constexpr int TB = (G1 + 2 * RP + 63) / 64 * 64;
  static constexpr int gcd(int a, int b) { return b == 0 ? a : gcd(b, a % b); }
  static constexpr int ROWALIGN = gcd(16, NP * (int)sizeof(T));
  // alignment of a half row starting at h K0 (even NP only; odd NP: element)
  static constexpr int HALFALIGN = NP % 2 == 0 ? gcd(ROWALIGN, K0 * (int)sizeof(T)) : (int)sizeof(T);
};

// K0 values of a modal row starting at index h K0 (clamped to the row for the
// odd-NP tail, whose value is then unused)
template <typename T, int NP>
__device__ __forceinline__ void load_half(const T *row, int h, T (&r)[ShapeH2<T, NP>::K0]) {
  using S_ = ShapeH2<T, NP>;
  if (NP % 2 == 0) {
    const T *p = static_cast<const T *>(__builtin_assume_aligned(row + h * S_::K0, S_::HALFALIGN));
#pragma unroll
    for (int k = 0; k < S_::K0; ++k) r[k] = p[k];
  } else {
#pragma unroll
    for (int k = 0; k < S_::K0; ++k) {
      const int a = h * S_::K0 + k;
      r[k] = row[a < NP ? a : NP - 1];
    }
  }
}

template <typename T, int NP>
__device__ __forceinline__ void store_half(T *row, int h, const T (&r)[ShapeH2<T, NP>::K0]) {
  using S_ = ShapeH2<T, NP>;
  if (NP % 2 == 0) {
    T *p = static_cast<T *>(__builtin_assume_aligned(row + h * S_::K0, S_::HALFALIGN));
#pragma unroll
    for (int k = 0; k < S_::K0; ++k) p[k] = r[k];
  } else {
#pragma unroll
    for (int k = 0; k < S_::K0; ++k)
      if (h * S_::K0 + k < NP) row[h * S_::K0 + k] = r[k];
  }
}

// An integer the compiler must treat as unknown: values derived from it are
// recomputed rather than reused from earlier in the kernel (no instruction).
__device__ __forceinline__ int opaque_int(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// The state offset of lane `lane`'s element and modal row in the half layout
// (tail and spare lanes on the last valid element).
template <int NP, int GPW>
__device__ __forceinline__ size_t h2_row_offset(int lane, int e0, int e_end) {
  int g = lane / (2 * NP), r = lane - g * 2 * NP;
  if (g >= GPW) { g = GPW; r = lane - GPW * 2 * NP; }
  const int t = r >= NP ? r - NP : r;
  const int e = e0 + g < e_end ? e0 + g : e_end - 1;
  return (size_t)e * 3 * NP * NP + (size_t)t * NP;
}

// The wavefront takes the GPW consecutive elements e0 .. e0 + GPW - 1 below
// e_end (lanes past it idle), starting in row j0.  PK = false: a row-aligned
// segment (e_end = the end of row j0); PK = true: elements packed across
// row ends (e_end = E, needs GPW <= n_lon), so the last ones may lie in row
// j0 + 1 and each lane picks its row's tables.
template <typename T, int NP, int CM, bool PK>
__device__ __forceinline__ void stage_wave_h2(const StageArgs<T, NP> &A, const int j0, const int e0,
                                              const int e_end, const int lane, T *tab, T *sh) {
  using S_ = ShapeH2<T, NP>;
  constexpr int N = S_::N, GPW = S_::GPW, SH = S_::SH, NB = S_::NB, K0 = S_::K0;
  // SPLIT: each half evaluates the node terms at its own K0 nodes of the
  // column and takes the other half's through LDS (FP64 with an even r + 1 >= 4,
  // where the node terms dominate and it measured faster); otherwise both
  // halves evaluate all r + 1 nodes (faster at r = 2 and 4 and in FP32)
  constexpr bool SPLIT = S_::SPLIT;
  static_assert(sizeof(GlobTab<T, NP>) >= sizeof(T) * S_::G1, "GlobTab prefix");
  using RT_ = RowTab<T, NP>;
  static_assert(offsetof(RT_, MS) == sizeof(T) * S_::rMS, "RowTab layout");
  static_assert(sizeof(RT_) == sizeof(T) * S_::RP, "RowTab layout");
  const T *__restrict__ q = A.q;
  const T *q0 = A.q0;
  T *out = A.out;
  const T *__restrict__ forcing = A.forcing;
  const GlobTab<T, NP> *__restrict__ gt = A.gt;
  const int n_lon = A.n_lon, n_lat = A.n_lat;
  const int combine = CM == CM_RUNTIME ? (A.combine != 0 ? 1 : 0) : CM;
  const T c0 = A.c0, c1 = A.c1, dt = A.dt;
  int g = lane / (2 * NP), r = lane - g * 2 * NP;
  const bool idle = g >= GPW;
  if (idle) { g = GPW; r = lane - GPW * 2 * NP; }
  const int h = r >= NP ? 1 : 0;
  const int t = r - h * NP;
  const int e_raw = e0 + g;
  // lanes that store, as a wavefront mask (scalar registers: nothing per lane
  // stays live until the stores)
  const unsigned long long store_mask = __builtin_amdgcn_ballot_w64(!idle && e_raw < e_end);
  const int e = e_raw < e_end ? e_raw : e_end - 1;      // tail lanes work on a valid element
  const int rsel = PK && e >= (j0 + 1) * n_lon ? 1 : 0;  // 1: the element is in row j0 + 1
  const int j = j0 + rsel;
  const int i = e - j * n_lon;
  const int ro = S_::G1 + rsel * S_::RP;                 // this lane's row tables in LDS
  T *S = sh + g * SH;
  // neighbours; across a pole (sphere) the latitude neighbour is the element
  // of the row at the other end of the grid (the plane's periodic neighbour),
  // read but weighted by the pole edge's zero cosine
  const int eE = (i + 1 == n_lon) ? e + 1 - n_lon : e + 1;
  const int eW = (i == 0) ? e - 1 + n_lon : e - 1;
  const int eN = j < n_lat - 1 ? e + n_lon : i;
  const int eS = j > 0 ? e - n_lon : (n_lat - 1) * n_lon + i;
  const int eX = h ? eW : eE, eY = h ? eS : eN;
  const T H = gt->href, H2 = gt->two_href, grav = gt->g, invR = gt->invR;
  const bool fixed = A.alpha_global != 0;
  const T alpha = gt->alpha;

  // the tables read with lane-dependent indices: loaded first and stored to LDS
  // once the state loads are in flight (a load-store loop would wait for every
  // load, and for all the state loads issued before it)
  constexpr int TBU = PK ? S_::TB : S_::G1 + S_::RP;     // the second row only when packed
  constexpr int TIT = (TBU + 63) / 64;
  static_assert(TIT * 64 <= S_::TB, "table copy rounds");
  T tv[TIT];
  {
    const T *g0 = &gt->B[0][0], *ra = &A.rows[j0].cosn[0];
    const T *rb = &A.rows[j0 + 1 < n_lat ? j0 + 1 : j0].cosn[0];
#pragma unroll
    for (int it = 0; it < TIT; ++it) {
      const int k = lane + 64 * it < TBU ? lane + 64 * it : TBU - 1;   // clamped: read, not stored
      const T *p = k < S_::G1 ? g0 + k : (k < S_::G1 + S_::RP ? ra + (k - S_::G1) : rb + (k - S_::G1 - S_::RP));
      tv[it] = *p;
    }
  }
  // ---- global loads: own row b = t, this half's longitude neighbour row and
  // latitude neighbour column
  const size_t row_off = (size_t)t * NP;
  const size_t base = (size_t)e * 3 * N + row_off;
  T qr[3][NP], xX[3][NP], xY[3][NP];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    load_row<T, NP>(q + base + v * N, qr[v]);
    load_row<T, NP>(q + (size_t)eX * 3 * N + row_off + v * N, xX[v]);
  }
  {
    // eY is a valid element at a pole edge too (the row across the grid),
    // whose trace the zero pole flux then discards: no branch, no zero fill
    const T *c = q + (size_t)eY * 3 * N + t;
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int k = 0; k < NP; ++k) xY[v][k] = c[v * N + k * NP];
  }
#pragma unroll
  for (int it = 0; it < TIT; ++it) tab[lane + 64 * it] = tv[it];
  // per-lane coefficients: rows h K0 + k of B (clamped), this half's own edge
  // (h = 0: +1, h = 1: -1) and the facing edge of its neighbours; from the
  // LDS tables where the registers are tight (SPLIT), else selected from the
  // scalar-loaded tables
  T BP[K0][NP], PE[NP], PF[NP];
  if (SPLIT) {
    wave_sync();
#pragma unroll
    for (int k = 0; k < K0; ++k) {
      const int p = h * K0 + k < NP ? h * K0 + k : NP - 1;
#pragma unroll
      for (int a = 0; a < NP; ++a) BP[k][a] = tab[S_::oB + p * NP + a];
    }
    const int oE = h ? S_::oPm : S_::oPp, oF = h ? S_::oPp : S_::oPm;
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      PE[a] = tab[oE + a];
      PF[a] = tab[oF + a];
    }
  } else {
#pragma unroll
    for (int k = 0; k < K0; ++k)
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        const int p1 = K0 + k < NP ? K0 + k : NP - 1;
        BP[k][a] = h ? gt->B[p1][a] : gt->B[k][a];
      }
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      PE[a] = h ? gt->Pm[a] : gt->Pp[a];
      PF[a] = h ? gt->Pp[a] : gt->Pm[a];
    }
  }

  // ---- xi pass: A[v][p][b=t] for this half's p, the own edge row, the
  // neighbour partial sums
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    T qa[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) qa[a] = qr[v][a];
    if (v == 0 && t == 0) qa[0] -= H2;
#pragma unroll
    for (int k = 0; k < K0; ++k) {
      T acc = T(0);
#pragma unroll
      for (int a = 0; a < NP; ++a) acc += qa[a] * BP[k][a];
      const int p = h * K0 + k;
      if (NP % 2 == 0 || p < NP) S[(v * (NP + 2) + p) * NP + t] = acc;
    }
    T ae = T(0);
#pragma unroll
    for (int a = 0; a < NP; ++a) ae += qa[a] * PE[a];
    S[(v * (NP + 2) + NP + h) * NP + t] = ae;
    T ux = T(0), uy = T(0);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      T yx = xX[v][k], yy = xY[v][k];
      if (v == 0 && t == 0 && k == 0) { yx -= H2; yy -= H2; }
      ux += yx * PF[k];
      uy += yy * PF[k];
    }
    S[NB + (h * 3 + v) * NP + t] = ux;          // slot 0: east, 1: west
    S[NB + ((2 + h) * 3 + v) * NP + t] = uy;    // slot 2: north, 3: south
  }
  wave_sync();

  // ---- eta pass: nodal values of column p = t at the nodes s this lane
  // evaluates (SPLIT: this half's s = h K0 + k, clamped like the xi pass's
  // rows; else all s), own and neighbour traces of this half's two edges
  constexpr int NDN = SPLIT ? K0 : NP;
  T nd[3][NDN], trX[3], trY[3], nbX[3], nbY[3];
  T bt[NP], Bs[NDN][NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) bt[k] = tab[S_::oB + t * NP + k];          // P~_k(xi_t)
#pragma unroll
  for (int k = 0; k < NDN; ++k) {
    const int sk = !SPLIT ? k : (h * K0 + k < NP ? h * K0 + k : NP - 1);
#pragma unroll
    for (int b = 0; b < NP; ++b) Bs[k][b] = SPLIT ? tab[S_::oB + sk * NP + b] : gt->B[k][b];  // P~_b(eta_s)
  }
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    T col[NP];
#pragma unroll
    for (int b = 0; b < NP; ++b) col[b] = S[(v * (NP + 2) + t) * NP + b];
#pragma unroll
    for (int k = 0; k < NDN; ++k) {
      T acc = T(0);
#pragma unroll
      for (int b = 0; b < NP; ++b) acc += col[b] * Bs[k][b];
      nd[v][k] = acc;
    }
    T ay = T(0), ax = T(0), nx = T(0), ny = T(0);
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      ay += col[b] * PE[b];
      ax += S[(v * (NP + 2) + NP + h) * NP + b] * bt[b];
      nx += S[NB + (h * 3 + v) * NP + b] * bt[b];
      ny += S[NB + ((2 + h) * 3 + v) * NP + b] * bt[b];
    }
    trX[v] = ax; trY[v] = ay; nbX[v] = nx; nbY[v] = ny;
  }
  wave_sync();

  // ---- Rusanov fluxes at edge node t of this half's two edges (minus side =
  // west / south: the own trace for h = 0, the neighbour's for h = 1; the
  // states go in as (own, neighbour) with the jump's sign set by h)
  T FhX[3], GhY[3];
  {
    const T sgn = h ? T(-1) : T(1);
    rusanov_lambda<T>(trX, nbX, H, grav, fixed, alpha, FhX, sgn);
    rusanov_theta<T>(trY, nbY, H, grav, fixed, alpha, GhY, sgn);
  }
  // the edge cosine is exactly 0 at a pole edge: zero flux through the pole
  const T fY = tab[ro + (h ? S_::rBot : S_::rTop)] * invR;
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    FhX[v] *= invR;
    GhY[v] *= fY;
    S[S_::oFX + (v * 2 + h) * NP + t] = FhX[v];   // read back in the last xi pass
    S[S_::oGY + (v * 2 + h) * NP + t] = GhY[v];   // the other half's latitude edge
  }
  wave_sync();
  T GhN[3], GhS[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const T other = S[S_::oGY + (v * 2 + 1 - h) * NP + t];
    GhN[v] = h ? other : GhY[v];
    GhS[v] = h ? GhY[v] : other;
  }
  if (SPLIT) wave_sync();   // the node terms below reuse the region of oGY

  // ---- volume: fluxes and sources at the nodes (t, s) of column t,
  // contracted over s for this half's outputs b = h K0 + kb.  SPLIT: this
  // lane evaluates its half's nodes and the other half's arrive through LDS,
  // XQ of the eight node terms at a time; else it evaluates all s.
  T ZD[3][K0], ZG[3][K0], ZS[2][K0];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int kb = 0; kb < K0; ++kb) { ZD[v][kb] = T(0); ZG[v][kb] = T(0); }
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int kb = 0; kb < K0; ++kb) ZS[v][kb] = T(0);
  int bh[K0];
#pragma unroll
  for (int kb = 0; kb < K0; ++kb) bh[kb] = h * K0 + kb < NP ? h * K0 + kb : NP - 1;
  // node terms: F (x 1/R), G (x cos/R) and the two momentum sources
  auto node_terms = [&](int s, const T dh, const T hu, const T hv, T (&f)[8]) {
    const T hh = dh + H;
    const T rh = dg_rcp(hh);
    const T u = hu * rh, vv = hv * rh;
    const T pr = T(0.5) * grav * dh * (hh + H);
    const T c = tab[ro + S_::rCos + s];
    const T cR = c * invR;
    f[0] = hu * invR; f[1] = (hu * u + pr) * invR; f[2] = hu * vv * invR;
    f[3] = hv * cR; f[4] = hv * u * cR; f[5] = (hv * vv + pr) * cR;
    const T C = tab[ro + S_::rFc + s] + u * tab[ro + S_::rSnR + s];
    f[6] = C * hv; f[7] = -pr * tab[ro + S_::rStR + s] - C * hu;
  };
  // add terms q0 .. q1-1 of node s to this half's outputs
  auto contract = [&](int s, const T *f, int q0, int q1) {
#pragma unroll
    for (int kb = 0; kb < K0; ++kb) {
      const T bm = tab[ro + S_::rBM + s * NP + bh[kb]], dm = tab[ro + S_::rDM + s * NP + bh[kb]];
#pragma unroll
      for (int q = q0; q < q1; ++q) {
        if (q < 3) ZD[q][kb] += f[q - q0] * bm;
        else if (q < 6) ZG[q - 3][kb] += f[q - q0] * dm;
        else ZS[q - 6][kb] += f[q - q0] * bm;
      }
    }
  };
  constexpr int XQ = S_::XQ;
  static_assert(!SPLIT || (8 % XQ == 0 && XQ * NP * NP <= S_::oFX && S_::oGY + 6 * NP <= S_::oFX),
                "half-layout LDS regions");
  if constexpr (!SPLIT) {
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      T f[8];
      node_terms(s, nd[0][s], nd[1][s], nd[2][s], f);
      contract(s, f, 0, 8);
    }
  } else {
    static_assert(NP % 2 == 0, "SPLIT halves own K0 = NP / 2 nodes each");
    // own nodes s = h K0 + k: contracted at once; the first XQ terms go to
    // LDS right away, the rest wait in registers for their round
    T own[K0][8];
#pragma unroll
    for (int k = 0; k < K0; ++k) {
      const int s = h * K0 + k;
      node_terms(s, nd[0][k], nd[1][k], nd[2][k], own[k]);
      contract(s, own[k], 0, 8);
#pragma unroll
      for (int q = 0; q < XQ; ++q) S[(q * NP + t) * NP + s] = own[k][q];
    }
#pragma unroll
    for (int q0 = 0; q0 < 8; q0 += XQ) {
      if (q0 > 0) {
#pragma unroll
        for (int k = 0; k < K0; ++k)
#pragma unroll
          for (int q = 0; q < XQ; ++q) S[(q * NP + t) * NP + h * K0 + k] = own[k][q0 + q];
      }
      wave_sync();
#pragma unroll
      for (int k = 0; k < K0; ++k) {     // the other half's nodes
        const int s = (1 - h) * K0 + k;
        T f[XQ];
#pragma unroll
        for (int q = 0; q < XQ; ++q) f[q] = S[(q * NP + t) * NP + s];
        contract(s, f, q0, q0 + XQ);
      }
      wave_sync();
    }
  }
  const T wt = tab[S_::oW + t], cF = gt->cF, cG = gt->cG;
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int kb = 0; kb < K0; ++kb) {
      if (NP % 2 != 0 && h * K0 + kb >= NP) continue;   // the odd-order tail slot
      const int b = bh[kb];
      T zg = ZG[v][kb];
      zg -= GhN[v] * tab[ro + S_::rMN + b];
      zg += GhS[v] * tab[ro + S_::rMS + b];
      const T zs = v == 0 ? T(0) : ZS[v - 1][kb];
      S[((v * 2 + 0) * NP + t) * NP + b] = cF * wt * ZD[v][kb];
      S[((v * 2 + 1) * NP + t) * NP + b] = wt * (cG * zg + zs);
    }
  wave_sync();

  // ---- epilogue operands for this half's modes a = h K0 + k of row b = t
  // (their offset recomputed from the lane index instead of held in registers
  // through the stage)
  const size_t ebase = h2_row_offset<NP, GPW>(opaque_int(lane), e0, e_end);
  const bool use_q0 = combine == 2 || (combine == 1 && c0 != T(0));
  T qh[3][K0], q0h[3][K0], fh[3][K0];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
#pragma unroll
    for (int k = 0; k < K0; ++k) { qh[v][k] = T(0); q0h[v][k] = T(0); fh[v][k] = T(0); }
    if (combine) load_half<T, NP>(q + ebase + v * N, h, qh[v]);
    if (use_q0) load_half<T, NP>(q0 + ebase + v * N, h, q0h[v]);
    if (forcing) load_half<T, NP>(forcing + ebase + v * N, h, fh[v]);
  }

  // ---- xi pass back to modes: lane t = latitude degree b, this half's a
  T bmt[NP], DA[NP][K0], BA[NP][K0], PpA[K0], PmA[K0];
#pragma unroll
  for (int p = 0; p < NP; ++p) bmt[p] = tab[ro + S_::rBM + p * NP + t];   // BM[p][t]
#pragma unroll
  for (int k = 0; k < K0; ++k) {
    const int a_raw = h * K0 + k;
    const int a = a_raw < NP ? a_raw : NP - 1;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      DA[p][k] = tab[S_::oD + p * NP + a];
      BA[p][k] = tab[S_::oB + p * NP + a];
    }
    PpA[k] = tab[S_::oPp + a];
    PmA[k] = tab[S_::oPm + a];
  }
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    T zd[NP], zb[NP];
    T XE = T(0), XW = T(0);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      zd[p] = S[((v * 2 + 0) * NP + p) * NP + t];
      zb[p] = S[((v * 2 + 1) * NP + p) * NP + t];
      XE += S[6 * NP * NP + (v * 2 + 0) * NP + p] * bmt[p];
      XW += S[6 * NP * NP + (v * 2 + 1) * NP + p] * bmt[p];
    }
    T xa[K0], xb[K0];
#pragma unroll
    for (int k = 0; k < K0; ++k) xa[k] = xb[k] = T(0);
    if (combine == 2 && A.qa) load_half<T, NP>(A.qa + ebase + v * N, h, xa);
    if (combine == 2 && A.qb) load_half<T, NP>(A.qb + ebase + v * N, h, xb);
    T res[K0];
    const T cXE = cF * XE, cXW = cF * XW;
#pragma unroll
    for (int k = 0; k < K0; ++k) {
      // the forcing, then chained FMAs (a sum of products first costs a third instruction)
      T acc = fh[v][k];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        acc += DA[p][k] * zd[p];
        acc += BA[p][k] * zb[p];
      }
      acc -= PpA[k] * cXE;
      acc += PmA[k] * cXW;
      if (combine == 2) {
        const T b0 = q0h[v][k];
        res[k] = b0 + dt * acc + (c1 * (qh[v][k] - b0) + (A.ca * (xa[k] - b0) + A.cb * (xb[k] - b0)));
      } else if (combine) {
        const T y = qh[v][k] + dt * acc;
        res[k] = y + c0 * (q0h[v][k] - y) + A.ce * y;
      } else {
        res[k] = acc;
      }
    }
    if ((store_mask >> lane) & 1ull) store_half<T, NP>(out + ebase + v * N, h, res);
  }
}

// expands to a switch over the runtime (dtype, np) that returns FN<T, NP>(args)
#define DGSW_DISPATCH(dtype, np, FN, ...)                                              \
  switch (np) {                                                                       \
    case 1: return (dtype) == 0 ? FN<double, 1>(__VA_ARGS__) : FN<float, 1>(__VA_ARGS__); \
    case 2: return (dtype) == 0 ? FN<double, 2>(__VA_ARGS__) : FN<float, 2>(__VA_ARGS__); \
    case 3: return (dtype) == 0 ? FN<double, 3>(__VA_ARGS__) : FN<float, 3>(__VA_ARGS__); \
    case 4: return (dtype) == 0 ? FN<double, 4>(__VA_ARGS__) : FN<float, 4>(__VA_ARGS__); \
    case 5: return (dtype) == 0 ? FN<double, 5>(__VA_ARGS__) : FN<float, 5>(__VA_ARGS__); \
    case 6: return (dtype) == 0 ? FN<double, 6>(__VA_ARGS__) : FN<float, 6>(__VA_ARGS__); \
    case 7: return (dtype) == 0 ? FN<double, 7>(__VA_ARGS__) : FN<float, 7>(__VA_ARGS__); \
    case 8: return (dtype) == 0 ? FN<double, 8>(__VA_ARGS__) : FN<float, 8>(__VA_ARGS__); \
    default: break;                                                                   \
  }

}  // namespace dgsw
