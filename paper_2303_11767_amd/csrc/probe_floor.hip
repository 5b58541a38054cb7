// The launch and memory floor under one stage of the benchmark-sized grid: a
// kernel that does nothing, one that moves the stage's own bytes (reads q and
// q^n, writes the new state), and one that also reads the neighbour rows and
// columns the stage reads, each with the FP64 r = 3 half layout's wavefronts
// (8 elements of 8 lanes each); timed back to back on one stream and as the
// nodes of one HIP graph.  A measurement beside the solver (libdgsw_probe.so),
// not part of it.
#include <hip/hip_runtime.h>

#include <cstddef>

namespace {

constexpr int NP = 4, N = NP * NP, GPW = 8;

__global__ __launch_bounds__(64) void k_floor_empty(double *out) {
  if (threadIdx.x >= 64) out[0] = 1.0;   // never taken: a launch with no memory traffic
}

// lane (g, h, t): element g of the wavefront, half h, modal row t; every index
// below stays in [0, E) (e < E is checked, the neighbours wrap like the stage's)
template <bool NBR>
__global__ __launch_bounds__(64) void k_floor_stream(const double *__restrict__ q, const double *__restrict__ q0,
                                                     double *__restrict__ out, int n_lon, int n_lat) {
  const int lane = threadIdx.x;
  const int g = lane / (2 * NP), r = lane % (2 * NP), h = r / NP, t = r % NP;
  const int E = n_lon * n_lat;
  const int e = blockIdx.x * GPW + g;
  if (e >= E) return;
  const int j = e / n_lon, i = e % n_lon;
  double acc[3][2];
  for (int v = 0; v < 3; ++v) {
    const double *row = q + (size_t)e * 3 * N + v * N + t * NP + h * 2;
    acc[v][0] = row[0];
    acc[v][1] = row[1];
  }
  if (NBR) {
    const int eX = h ? (i == 0 ? e - 1 + n_lon : e - 1) : (i + 1 == n_lon ? e + 1 - n_lon : e + 1);
    const int eY = h ? (j > 0 ? e - n_lon : (n_lat - 1) * n_lon + i) : (j < n_lat - 1 ? e + n_lon : i);
    for (int v = 0; v < 3; ++v) {
      const double *rx = q + (size_t)eX * 3 * N + v * N + t * NP;
      const double *cy = q + (size_t)eY * 3 * N + v * N + t;
      double sx = 0.0, sy = 0.0;
      for (int k = 0; k < NP; ++k) {
        sx += rx[k];
        sy += cy[k * NP];
      }
      acc[v][0] += 1e-30 * sx;
      acc[v][1] += 1e-30 * sy;
    }
  }
  for (int v = 0; v < 3; ++v) {
    const size_t o = (size_t)e * 3 * N + v * N + t * NP + h * 2;
    out[o] = acc[v][0] + q0[o];
    out[o + 1] = acc[v][1] + q0[o + 1];
  }
}

hipError_t floor_launch(int variant, int waves, const double *q, const double *q0, double *out, int n_lon,
                        int n_lat, hipStream_t s) {
  switch (variant) {
    case 0: hipLaunchKernelGGL(k_floor_empty, dim3(waves), dim3(64), 0, s, out); break;
    case 1: hipLaunchKernelGGL(k_floor_stream<false>, dim3(waves), dim3(64), 0, s, q, q0, out, n_lon, n_lat); break;
    case 2: hipLaunchKernelGGL(k_floor_stream<true>, dim3(waves), dim3(64), 0, s, q, q0, out, n_lon, n_lat); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

extern "C" {

// Mean time [us] per launch of floor kernel `variant` (0: empty, 1: the
// stage's own bytes, 2: plus its neighbour reads) over an n_lon x n_lat r = 3
// FP64 state: `reps` launches back to back on one stream (graph = 0) or the
// `reps` nodes of one captured graph (graph = 1), after a warm-up.  The
// buffers (three states) are allocated and freed inside.  0 on success, < 0
// on error (-1 arguments, -2 allocation, -3 HIP).
int dgp_floor_time(int variant, int n_lon, int n_lat, int graph, int reps, double *us) {
  if (!us || variant < 0 || variant > 2 || n_lon < 1 || n_lat < 1 || reps < 1 || reps > 100000 ||
      (graph != 0 && graph != 1) || (long long)n_lon * n_lat > (1 << 22))
    return -1;
  const int E = n_lon * n_lat;
  const size_t n = (size_t)E * 3 * N;
  const int waves = (E + GPW - 1) / GPW;
  double *q = nullptr, *q0 = nullptr, *out = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipGraph_t gr = nullptr;
  hipGraphExec_t ge = nullptr;
  int rc = 0;
  if (hipMalloc(&q, n * sizeof(double)) != hipSuccess || hipMalloc(&q0, n * sizeof(double)) != hipSuccess ||
      hipMalloc(&out, n * sizeof(double)) != hipSuccess)
    rc = -2;
  if (rc == 0 && (hipMemset(q, 0, n * sizeof(double)) != hipSuccess ||
                  hipMemset(q0, 0, n * sizeof(double)) != hipSuccess ||
                  hipStreamCreate(&s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
                  hipEventCreate(&e1) != hipSuccess))
    rc = -3;
  for (int w = 0; rc == 0 && w < 20; ++w)
    if (floor_launch(variant, waves, q, q0, out, n_lon, n_lat, s) != hipSuccess) rc = -3;
  if (rc == 0 && graph) {
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = -3;
    for (int k = 0; rc == 0 && k < reps; ++k)
      if (floor_launch(variant, waves, q, q0, out, n_lon, n_lat, s) != hipSuccess) rc = -3;
    if (hipStreamEndCapture(s, &gr) != hipSuccess) rc = -3;
    if (rc == 0 && (hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0) != hipSuccess ||
                    hipGraphLaunch(ge, s) != hipSuccess))
      rc = -3;
  }
  if (rc == 0 && hipStreamSynchronize(s) != hipSuccess) rc = -3;
  if (rc == 0) {
    if (hipEventRecord(e0, s) != hipSuccess) rc = -3;
    if (graph) {
      if (rc == 0 && hipGraphLaunch(ge, s) != hipSuccess) rc = -3;
    } else {
      for (int k = 0; rc == 0 && k < reps; ++k)
        if (floor_launch(variant, waves, q, q0, out, n_lon, n_lat, s) != hipSuccess) rc = -3;
    }
    float ms = 0.f;
    if (rc == 0 && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = -3;
    if (rc == 0) *us = (double)ms * 1e3 / reps;
  }
  if (ge) (void)hipGraphExecDestroy(ge);
  if (gr) (void)hipGraphDestroy(gr);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  if (q) (void)hipFree(q);
  if (q0) (void)hipFree(q0);
  if (out) (void)hipFree(out);
  return rc;
}

}  // extern "C"
