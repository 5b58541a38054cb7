"""Binding of the learned right-hand-side correction (dg_mlp_*, dg_project,
dg_features, dg_*_learned of the C ABI): argument marshalling only.

The network, its training step, the stencil features, the projection onto
order 1 and the learned stage all run in the library's HIP kernels.
"""
import ctypes

from ._lib import Learned, check, load
from . import _stream_handle

N_IN, N_HID, N_OUT = 108, 256, 12


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("need a contiguous GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


def _f32(t, numel, name):
    import torch
    if t.dtype != torch.float32 or t.numel() != numel:
        raise ValueError(f"{name}: need {numel} float32 values")
    return _ptr(t)


def param_count():
    n = ctypes.c_int64()
    check(load().dg_mlp_param_count(ctypes.byref(n)))
    return n.value


class _Workspace:
    def __init__(self):
        self._buf = None

    def get(self, nbytes, device):
        import torch
        if self._buf is None or self._buf.numel() < nbytes:
            self._buf = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        return self._buf


_ws = _Workspace()


def _mlp_ws(rows, device):
    b = ctypes.c_int64()
    check(load().dg_mlp_workspace_size(int(rows), ctypes.byref(b)))
    return _ws.get(b.value, device)


def mlp_forward(params, X, out=None, stream=None):
    """Y[rows][12] = net(X[rows][108]), all FP32 on the GPU."""
    import torch
    rows = X.shape[0]
    if out is None:
        out = torch.empty((rows, N_OUT), dtype=torch.float32, device=X.device)
    ws = _mlp_ws(rows, X.device)
    check(load().dg_mlp_forward(_f32(params, param_count(), "params"), _f32(X, rows * N_IN, "X"),
                                rows, _f32(out, rows * N_OUT, "Y"), _ptr(ws), _stream_handle(stream)))
    return out


def mlp_train_step(params, X, T, mask, adam_m=None, adam_v=None, step=0, lr=0.0, grads=None,
                   loss=None, stream=None):
    """Forward + backward (+ Adam when lr > 0) on one batch (rows % 32 == 0).
    mask: 12 host values, 0 or 1 (a sequence or a CPU array)."""
    rows = X.shape[0]
    P = param_count()
    ws = _mlp_ws(rows, X.device)
    m = [float(v) for v in mask]
    if len(m) != N_OUT:
        raise ValueError(f"mask needs {N_OUT} values")
    mask_h = (ctypes.c_float * N_OUT)(*m)
    check(load().dg_mlp_train_step(
        _f32(params, P, "params"), _ptr(adam_m), _ptr(adam_v), int(step), float(lr),
        _f32(X, rows * N_IN, "X"), _f32(T, rows * N_OUT, "T"), mask_h, rows,
        _ptr(grads), _ptr(loss), _ptr(ws), _stream_handle(stream)))


def project(src, dst, q_src, q_dst=None, stream=None):
    """Cos-weighted projection of src's state onto dst's basis (dst's order,
    same mesh; a target order at or above src's embeds the state)."""
    if q_dst is None:
        q_dst = dst.empty_state(q_src.device)
    check(load().dg_project(src._ctx, dst._ctx, src._ptr(q_src, "q_src"), dst._ptr(q_dst, "q_dst"),
                            _stream_handle(stream)))
    return q_dst


def features(mesh, q, mean=None, istd=None, out=None, stream=None):
    """X[E][108] stencil features of an order-1 state (standardised if given)."""
    import torch
    if out is None:
        out = torch.empty((mesh.E, N_IN), dtype=torch.float32, device=q.device)
    check(load().dg_features(mesh._ctx, mesh._ptr(q, "q"), _ptr(mean), _ptr(istd),
                             _f32(out, mesh.E * N_IN, "X"), _stream_handle(stream)))
    return out


class LearnedRHS:
    """The learned right-hand side on an order-1 mesh (dg_rhs_learned)."""

    def __init__(self, mesh, params, feat_mean, feat_istd, out_mean, out_std, kappa=1.0):
        import torch
        self.mesh = mesh
        self.tensors = (params, feat_mean, feat_istd, out_mean, out_std)   # kept alive
        self.net = Learned(_f32(params, param_count(), "params").value,
                           _f32(feat_mean, N_IN, "feat_mean").value,
                           _f32(feat_istd, N_IN, "feat_istd").value,
                           _f32(out_mean, mesh.n_lat * N_OUT, "out_mean").value,
                           _f32(out_std, mesh.n_lat * N_OUT, "out_std").value, float(kappa))
        b = ctypes.c_int64()
        check(load().dg_learned_workspace_size(mesh._ctx, ctypes.byref(b)))
        self.workspace = torch.empty(b.value, dtype=torch.uint8, device=params.device)
        self.fallbacks = torch.zeros(1, dtype=torch.int64, device=params.device)

    def rhs(self, q, out=None, stream=None):
        if out is None:
            out = self.mesh.empty_state(q.device)
        check(load().dg_rhs_learned(self.mesh._ctx, ctypes.byref(self.net), self.mesh._ptr(q, "q"),
                                    self.mesh._ptr(out, "out"), _ptr(self.workspace),
                                    _ptr(self.fallbacks), _stream_handle(stream)))
        return out

    def rk_step(self, q, work, dt, nsteps=1, stream=None):
        check(load().dg_rk_step_learned(self.mesh._ctx, ctypes.byref(self.net),
                                        self.mesh._ptr(q, "q"),
                                        self.mesh._ptr(work, "work", self.mesh.work_size()),
                                        _ptr(self.workspace), float(dt), int(nsteps),
                                        _ptr(self.fallbacks), _stream_handle(stream)))
        return q
