// C ABI of the learned right-hand-side correction (declared in include/dgsw.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "dgsw.h"
#include "dgsw_ctx.hpp"
#include "dgsw_device.hpp"
#include "dgsw_mlp.hpp"

using dgsw::aligned16;
using dgsw::fail;
using dgsw::hip_fail;

namespace {

using dgsw::kFeatures;
using dgsw::kHidden;
using dgsw::kInPad;
using dgsw::kOut;
using dgsw::kOutPad;

constexpr int64_t kParams = (int64_t)kFeatures * kHidden + kHidden + (int64_t)kHidden * kHidden + kHidden +
                            (int64_t)kHidden * kOut + kOut;

// offsets into the flat FP32 parameter vector
constexpr int64_t oW1 = 0, ob1 = oW1 + (int64_t)kFeatures * kHidden, oW2 = ob1 + kHidden,
                  ob2 = oW2 + (int64_t)kHidden * kHidden, oW3 = ob2 + kHidden,
                  ob3 = oW3 + (int64_t)kHidden * kOut;

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// Carves a caller-provided workspace into 256-byte aligned pieces.
struct Carve {
  char *base;
  size_t off = 0;
  explicit Carve(void *p) : base(static_cast<char *>(p)) {}
  template <typename T>
  T *take(size_t n) {
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += al(n * sizeof(T));
    return p;
  }
};

// BF16 weights for the forward pass (and the backward pass when Wr != null);
// the hidden layers' also in the fused network kernel's fragment order
struct Weights {
  __bf16 *W1t, *W2t, *W3t, *W1r, *W2r, *W3r, *W1f, *W2f;
  float *b3p;
};

Weights carve_weights(Carve &c, bool backward) {
  Weights w;
  w.W1t = c.take<__bf16>((size_t)kHidden * kInPad);
  w.W2t = c.take<__bf16>((size_t)kHidden * kHidden);
  w.W3t = c.take<__bf16>((size_t)kOutPad * kHidden);
  w.W1r = backward ? c.take<__bf16>((size_t)kInPad * kHidden) : nullptr;
  w.W2r = backward ? c.take<__bf16>((size_t)kHidden * kHidden) : nullptr;
  w.W3r = backward ? c.take<__bf16>((size_t)kHidden * kOutPad) : nullptr;
  w.W1f = c.take<__bf16>((size_t)kHidden * kInPad);
  w.W2f = c.take<__bf16>((size_t)kHidden * kHidden);
  w.b3p = c.take<float>(kOutPad);
  return w;
}

hipError_t prep(const float *P, const Weights &w, hipStream_t s) {
  hipError_t e;
  if ((e = dgsw::launch_prep_weights(P + oW1, kFeatures, kHidden, kInPad, kHidden, w.W1t, w.W1r, w.W1f, s)) != hipSuccess)
    return e;
  if ((e = dgsw::launch_prep_weights(P + oW2, kHidden, kHidden, kHidden, kHidden, w.W2t, w.W2r, w.W2f, s)) != hipSuccess)
    return e;
  if ((e = dgsw::launch_prep_weights(P + oW3, kHidden, kOut, kHidden, kOutPad, w.W3t, w.W3r, nullptr, s)) != hipSuccess)
    return e;
  return dgsw::launch_pad(P + ob3, kOut, kOutPad, w.b3p, s);
}

// Forward pass on Xb[rows][kInPad] -> Y[rows][kOutPad] (FP32), keeping the
// pre-activations when Z1/Z2 are given.
hipError_t forward(const float *P, const Weights &w, const __bf16 *Xb, int rows, float *Z1, __bf16 *H1, float *Z2,
                   __bf16 *H2, float *Y, hipStream_t s) {
  dgsw::GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.A = Xb; g.B = w.W1t; g.M = rows; g.N = kHidden; g.K = kInPad; g.lda = kInPad; g.ldb = kInPad;
  g.bias = P + ob1; g.Zout = Z1; g.C = H1; g.ldc = kHidden;
  hipError_t e = dgsw::launch_gemm(true, true, dgsw::kEpiBiasGelu, g, s);
  if (e != hipSuccess) return e;
  g.A = H1; g.B = w.W2t; g.K = kHidden; g.lda = kHidden; g.ldb = kHidden; g.bias = P + ob2; g.Zout = Z2; g.C = H2;
  if ((e = dgsw::launch_gemm(true, true, dgsw::kEpiBiasGelu, g, s)) != hipSuccess) return e;
  g.A = H2; g.B = w.W3t; g.N = kOutPad; g.bias = w.b3p; g.Zout = nullptr; g.C = Y; g.ldc = kOutPad;
  return dgsw::launch_gemm(true, true, dgsw::kEpiBias, g, s);
}

struct TrainWs {
  Weights w;
  __bf16 *Xb, *H1, *H2, *dY, *dZ2, *dZ1;
  float *Z1, *Z2, *Y, *dYf, *dZ2f, *dZ1f, *G1, *G2, *G3, *grad, *partial, *split, *csum;
};

TrainWs carve_train(void *ws, int64_t rows, size_t *bytes) {
  Carve c(ws);
  TrainWs t;
  t.w = carve_weights(c, true);
  t.Xb = c.take<__bf16>(rows * kInPad);
  t.Z1 = c.take<float>(rows * kHidden);
  t.H1 = c.take<__bf16>(rows * kHidden);
  t.Z2 = c.take<float>(rows * kHidden);
  t.H2 = c.take<__bf16>(rows * kHidden);
  t.Y = c.take<float>(rows * kOutPad);
  t.dY = c.take<__bf16>(rows * kOutPad);
  t.dYf = c.take<float>(rows * kOutPad);
  t.dZ2 = c.take<__bf16>(rows * kHidden);
  t.dZ2f = c.take<float>(rows * kHidden);
  t.dZ1 = c.take<__bf16>(rows * kHidden);
  t.dZ1f = c.take<float>(rows * kHidden);
  t.G1 = c.take<float>((size_t)kInPad * kHidden);
  t.G2 = c.take<float>((size_t)kHidden * kHidden);
  t.G3 = c.take<float>((size_t)kHidden * kOutPad);
  t.grad = c.take<float>(kParams);
  t.partial = c.take<float>((rows * kOutPad + 255) / 256 + 1);
  t.split = c.take<float>((size_t)dgsw::gemm_splits((int)rows) * kHidden * kHidden);
  t.csum = c.take<float>((size_t)dgsw::colsum_chunks((int)rows) * kHidden);
  if (bytes) *bytes = c.off;
  return t;
}

struct LearnWs {
  Weights w;
  void *L1;
  float *C;
  double *partial;
};

LearnWs carve_learn(void *ws, const dg_ctx *ctx, size_t *bytes) {
  Carve c(ws);
  LearnWs t;
  const int64_t E = ctx->E;
  t.w = carve_weights(c, false);
  t.L1 = c.take<char>(E * 12 * ctx->elem_bytes);
  t.C = c.take<float>(E * 12);
  t.partial = c.take<double>(dgsw::mlp_fused_blocks((int)E));
  if (bytes) *bytes = c.off;
  return t;
}

int check_ptrs(std::initializer_list<const void *> ps) {
  for (const void *p : ps)
    if (!p) return fail(DG_EINVAL, "NULL argument");
  return DG_OK;
}

}  // namespace

extern "C" {

int dg_mlp_param_count(int64_t *n) {
  if (!n) return fail(DG_EINVAL, "NULL argument");
  *n = kParams;
  return DG_OK;
}

int dg_mlp_workspace_size(int64_t rows, int64_t *bytes) {
  if (!bytes || rows < 1) return fail(DG_EINVAL, "bad argument");
  size_t b = 0;
  carve_train(nullptr, rows, &b);
  *bytes = (int64_t)b;
  return DG_OK;
}

int dg_mlp_forward(const float *params, const float *X, int64_t rows, float *Y, void *workspace,
                   void *hip_stream) {
  int rc = check_ptrs({params, X, Y, workspace});
  if (rc != DG_OK) return rc;
  if (rows < 1 || rows >= (int64_t(1) << 26)) return fail(DG_EINVAL, "rows out of range");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  TrainWs t = carve_train(workspace, rows, nullptr);
  hipError_t e;
  if ((e = prep(params, t.w, s)) != hipSuccess) return hip_fail(e, "weight preparation");
  if ((e = dgsw::launch_mlp_fused(0, nullptr, 0, 0, nullptr, nullptr, X, (int)rows, t.w.W1f, t.w.W2f, t.w.W3t,
                                  params + ob1, params + ob2, t.w.b3p, t.Y, s, nullptr)) != hipSuccess)
    return hip_fail(e, "forward");
  if ((e = dgsw::launch_unpad(t.Y, (int)rows, kOut, kOutPad, Y, s)) != hipSuccess) return hip_fail(e, "output");
  return DG_OK;
}

int dg_mlp_train_step(float *params, float *adam_m, float *adam_v, int32_t step, float lr, const float *X,
                      const float *T, const float *mask, int64_t rows, float *grads, float *loss,
                      void *workspace, void *hip_stream) {
  int rc = check_ptrs({params, X, T, mask, workspace});
  if (rc != DG_OK) return rc;
  if (rows < 32 || rows % 32 != 0 || rows >= (int64_t(1) << 26))
    return fail(DG_EINVAL, "rows must be a positive multiple of 32");
  if (lr > 0.f && (!adam_m || !adam_v || step < 1)) return fail(DG_EINVAL, "Adam needs m, v and step >= 1");
  // the output mask (host, read here): weights 0 or 1, at least one 1
  unsigned bits = 0;
  int msum = 0;
  for (int n = 0; n < kOut; ++n) {
    if (mask[n] == 1.0f) {
      bits |= 1u << n;
      ++msum;
    } else if (mask[n] != 0.0f) {
      return fail(DG_EINVAL, "mask values must be 0 or 1");
    }
  }
  if (msum == 0) return fail(DG_EINVAL, "mask selects no output");
  const float scale = 1.0f / ((float)rows * (float)msum);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  TrainWs t = carve_train(workspace, rows, nullptr);
  const int R = (int)rows;
  hipError_t e;
  if ((e = prep(params, t.w, s)) != hipSuccess) return hip_fail(e, "weight preparation");
  if ((e = dgsw::launch_to_bf16(X, R, kFeatures, kInPad, t.Xb, s)) != hipSuccess) return hip_fail(e, "features");
  if ((e = forward(params, t.w, t.Xb, R, t.Z1, t.H1, t.Z2, t.H2, t.Y, s)) != hipSuccess) return hip_fail(e, "forward");
  // mean squared error over the unmasked outputs
  int nb = 0;
  if ((e = dgsw::launch_mse_grad(t.Y, T, bits, R, kOut, kOutPad, scale, t.dY, t.dYf, t.partial, &nb, s)) != hipSuccess)
    return hip_fail(e, "loss");
  if (loss && (e = dgsw::launch_sum(t.partial, nb, scale, loss, s)) != hipSuccess) return hip_fail(e, "loss sum");
  dgsw::GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  // dZ2 = (dY W3^T) * gelu'(Z2)
  g.A = t.dY; g.B = t.w.W3r; g.M = R; g.N = kHidden; g.K = kOutPad; g.lda = kOutPad; g.ldb = kOutPad;
  g.Zin = t.Z2; g.Zout = t.dZ2f; g.C = t.dZ2; g.ldc = kHidden;
  if ((e = dgsw::launch_gemm(true, true, dgsw::kEpiGeluGrad, g, s)) != hipSuccess) return hip_fail(e, "backward 3");
  // dZ1 = (dZ2 W2^T) * gelu'(Z1)
  g.A = t.dZ2; g.B = t.w.W2r; g.K = kHidden; g.lda = kHidden; g.ldb = kHidden; g.Zin = t.Z1; g.Zout = t.dZ1f;
  g.C = t.dZ1;
  if ((e = dgsw::launch_gemm(true, true, dgsw::kEpiGeluGrad, g, s)) != hipSuccess) return hip_fail(e, "backward 2");
  // weight gradients: sums over the rows of activation x gradient
  dgsw::GemmArgs w;
  std::memset(&w, 0, sizeof(w));
  w.K = R;
  w.A = t.H2; w.lda = kHidden; w.M = kHidden; w.B = t.dY; w.ldb = kOutPad; w.N = kOutPad; w.C = t.G3; w.ldc = kOutPad;
  if ((e = dgsw::launch_gemm_splitk(w, t.split, s)) != hipSuccess) return hip_fail(e, "dW3");
  w.A = t.H1; w.M = kHidden; w.B = t.dZ2; w.ldb = kHidden; w.N = kHidden; w.C = t.G2; w.ldc = kHidden;
  if ((e = dgsw::launch_gemm_splitk(w, t.split, s)) != hipSuccess) return hip_fail(e, "dW2");
  w.A = t.Xb; w.lda = kInPad; w.M = kInPad; w.B = t.dZ1; w.C = t.G1;
  if ((e = dgsw::launch_gemm_splitk(w, t.split, s)) != hipSuccess) return hip_fail(e, "dW1");
  float *gr = t.grad;
  if ((e = dgsw::launch_unpad(t.G1, kFeatures, kHidden, kHidden, gr + oW1, s)) != hipSuccess ||
      (e = dgsw::launch_colsum(t.dZ1f, R, kHidden, kHidden, t.csum, gr + ob1, s)) != hipSuccess ||
      (e = dgsw::launch_unpad(t.G2, kHidden, kHidden, kHidden, gr + oW2, s)) != hipSuccess ||
      (e = dgsw::launch_colsum(t.dZ2f, R, kHidden, kHidden, t.csum, gr + ob2, s)) != hipSuccess ||
      (e = dgsw::launch_unpad(t.G3, kHidden, kOut, kOutPad, gr + oW3, s)) != hipSuccess ||
      (e = dgsw::launch_colsum(t.dYf, R, kOut, kOutPad, t.csum, gr + ob3, s)) != hipSuccess)
    return hip_fail(e, "gradients");
  if (grads && (e = hipMemcpyAsync(grads, gr, kParams * sizeof(float), hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(e, "gradient copy");
  if (lr > 0.f &&
      (e = dgsw::launch_adam(params, gr, adam_m, adam_v, (int)kParams, lr, 0.9f, 0.999f, 1e-8f, step, s)) != hipSuccess)
    return hip_fail(e, "Adam");
  return DG_OK;
}

int dg_project(const dg_ctx *src, const dg_ctx *dst, const void *q_src, void *q_dst, void *hip_stream) {
  int rc = check_ptrs({src, dst, q_src, q_dst});
  if (rc != DG_OK) return rc;
  if (src->levels != 1 || dst->levels != 1) return fail(DG_EUNSUPPORTED, "projection takes one layer");
  if (src->d.n_lon != dst->d.n_lon || src->d.n_lat != dst->d.n_lat || src->d.dtype != dst->d.dtype ||
      src->periodic_y != dst->periodic_y)
    return fail(DG_EINVAL, "source and target must share the mesh and dtype");
  if (q_src == q_dst) return fail(DG_EINVAL, "q_src and q_dst must be different buffers");
  const int k = dst->np - 1;
  hipError_t e = dgsw::launch_project(src->d.dtype == DG_F64 ? 0 : 1, q_src, src->d.n_lon, src->E, src->np,
                                      dst->np, src->d_proj + dgsw::proj_offset(k, src->d.n_lat, src->np), q_dst,
                                      static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "projection launch");
  return DG_OK;
}

int dg_features(const dg_ctx *ctx, const void *q, const float *feat_mean, const float *feat_istd, float *X,
                void *hip_stream) {
  int rc = check_ptrs({ctx, q, X});
  if (rc != DG_OK) return rc;
  if (ctx->np != 2) return fail(DG_EUNSUPPORTED, "features are defined for order 1");
  if (ctx->levels != 1) return fail(DG_EUNSUPPORTED, "features take one layer");
  if ((feat_mean == nullptr) != (feat_istd == nullptr)) return fail(DG_EINVAL, "give both mean and istd, or neither");
  hipError_t e = dgsw::launch_features_f32(ctx->d.dtype == DG_F64 ? 0 : 1, q, ctx->d.n_lon, ctx->d.n_lat, feat_mean,
                                           feat_istd, X, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "features launch");
  return DG_OK;
}

int dg_learned_workspace_size(const dg_ctx *ctx, int64_t *bytes) {
  if (!ctx || !bytes) return fail(DG_EINVAL, "NULL argument");
  size_t b = 0;
  carve_learn(nullptr, ctx, &b);
  *bytes = (int64_t)b;
  return DG_OK;
}

}  // extern "C"

namespace {

int learned_stage(dg_ctx *ctx, const dg_learned *net, const LearnWs &t, const void *q, const void *q0, void *out,
                  int combine, double c0, double c1, double dt, int64_t *fallbacks, hipStream_t s) {
  const int dt_ = ctx->d.dtype == DG_F64 ? 0 : 1;
  // plain r = 1 right-hand side into the workspace
  dgsw::StageLaunch a;
  std::memset(&a, 0, sizeof(a));
  a.q = q; a.q0 = nullptr; a.out = t.L1; a.forcing = ctx->forcing; a.glob = ctx->d_glob; a.rows = ctx->d_rows;
  a.n_lon = ctx->d.n_lon; a.n_lat = ctx->d.n_lat; a.E = ctx->E;
  a.alpha_global = ctx->d.alpha_mode == DG_ALPHA_GLOBAL; a.combine = 0; a.c0 = 0.0; a.c1 = 1.0; a.dt = 0.0;
  a.periodic_y = ctx->periodic_y;
  a.variant = ctx->kernel;        // the same kernel layout as dg_rhs on this context
  a.levels = 1;
  hipError_t e = dgsw::launch_stage(dt_, ctx->np, a, s);
  if (e != hipSuccess) return hip_fail(e, "r = 1 stage launch");
  // features, the whole network (hidden layers in LDS) and the per-element
  // correction with its trust bound, in one launch
  dgsw::CorrectionArgs ca;
  ca.L1 = t.L1; ca.omean = net->out_mean; ca.ostd = net->out_std; ca.mass_w = ctx->d_mass_w;
  ca.kappa = (float)net->kappa; ca.C = t.C; ca.partial = t.partial; ca.fallback = fallbacks;
  if ((e = dgsw::launch_mlp_fused(dt_, q, ctx->d.n_lon, ctx->d.n_lat, net->feat_mean, net->feat_istd, nullptr,
                                  ctx->E, t.w.W1f, t.w.W2f, t.w.W3t, net->params + ob1, net->params + ob2, t.w.b3p,
                                  nullptr, s, &ca)) != hipSuccess)
    return hip_fail(e, "network launch");
  dgsw::LearnedOut l;
  l.L1 = t.L1; l.C = t.C; l.partial = t.partial; l.nparts = dgsw::mlp_fused_blocks(ctx->E); l.E = ctx->E;
  l.area = ctx->mass_area; l.q = q; l.q0 = q0; l.out = out; l.combine = combine; l.c0 = c0; l.c1 = c1; l.dt = dt;
  if ((e = dgsw::launch_learned_out(dt_, l, s)) != hipSuccess) return hip_fail(e, "output launch");
  return DG_OK;
}

int check_learned(const dg_ctx *ctx, const dg_learned *net, const void *workspace) {
  if (!ctx || !net || !workspace) return fail(DG_EINVAL, "NULL argument");
  if (ctx->np != 2) return fail(DG_EUNSUPPORTED, "the learned correction is defined for order 1");
  if (ctx->periodic_y) return fail(DG_EUNSUPPORTED, "the learned correction is defined on the sphere");
  if (ctx->levels != 1) return fail(DG_EUNSUPPORTED, "the learned correction takes one layer");
  if (!net->params || !net->feat_mean || !net->feat_istd || !net->out_mean || !net->out_std)
    return fail(DG_EINVAL, "dg_learned has a NULL table");
  if (!(net->kappa >= 0.0)) return fail(DG_EINVAL, "kappa must be >= 0");
  if (!aligned16(workspace)) return fail(DG_EINVAL, "workspace must be 16-byte aligned");
  return DG_OK;
}

}  // namespace

extern "C" {

int dg_rhs_learned(dg_ctx *ctx, const dg_learned *net, const void *q, void *dqdt, void *workspace,
                   int64_t *fallbacks, void *hip_stream) {
  int rc = check_learned(ctx, net, workspace);
  if (rc != DG_OK) return rc;
  if (!q || !dqdt) return fail(DG_EINVAL, "NULL argument");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  LearnWs t = carve_learn(workspace, ctx, nullptr);
  hipError_t e = prep(net->params, t.w, s);
  if (e != hipSuccess) return hip_fail(e, "weight preparation");
  return learned_stage(ctx, net, t, q, nullptr, dqdt, 0, 0.0, 1.0, 0.0, fallbacks, s);
}

int dg_rk_step_learned(dg_ctx *ctx, const dg_learned *net, void *q, void *work, void *workspace, double dt,
                       int32_t nsteps, int64_t *fallbacks, void *hip_stream) {
  int rc = check_learned(ctx, net, workspace);
  if (rc != DG_OK) return rc;
  if (!q || !work) return fail(DG_EINVAL, "NULL argument");
  if (nsteps < 0 || !std::isfinite(dt)) return fail(DG_EINVAL, "bad nsteps or dt");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  LearnWs t = carve_learn(workspace, ctx, nullptr);
  hipError_t e = prep(net->params, t.w, s);
  if (e != hipSuccess) return hip_fail(e, "weight preparation");
  const size_t bytes = ctx->state_n * ctx->elem_bytes;
  char *w0 = static_cast<char *>(work);
  char *w1 = w0 + bytes;
  for (int n = 0; n < nsteps; ++n) {
    if ((rc = learned_stage(ctx, net, t, q, nullptr, w0, 1, 0.0, 1.0, dt, fallbacks, s)) != DG_OK) return rc;
    if ((rc = learned_stage(ctx, net, t, w0, q, w1, 1, 0.75, 0.25, dt, fallbacks, s)) != DG_OK) return rc;
    if ((rc = learned_stage(ctx, net, t, w1, q, q, 1, 1.0 / 3.0, 2.0 / 3.0, dt, fallbacks, s)) != DG_OK) return rc;
  }
  return DG_OK;
}

}  // extern "C"
