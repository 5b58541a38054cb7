"""MI355X-native modal DG shallow-water solver on the sphere.

Python binding of libdgsw (include/dgsw.h): argument marshalling only.  The
state lives in caller-owned torch tensors on the GPU; every step of the
right-hand side and the Runge-Kutta loop runs in the library's HIP kernels
on the caller's current torch stream.
"""
import ctypes
import math

from ._lib import (DG_ALPHA_GLOBAL, DG_ALPHA_LOCAL, DG_F32, DG_F64, DG_METRIC_BALANCED,
                   DG_METRIC_POINTWISE, DG_SSP_RK1, DG_SSP_RK2, DG_SSP_RK3, DGError,
                   MeshDesc, check, load)

__all__ = ["Mesh", "DGError", "cfl_time_step", "DG_SSP_RK1", "DG_SSP_RK2", "DG_SSP_RK3"]

RADIUS, GRAVITY, OMEGA = 6.371e6, 9.80616, 7.292e-5


def cfl_time_step(mesh, cmax, cfl):
    """dt = cfl * H / (max(r, 1) * c_max), the DG Courant number p c dt / H of
    section 2, with H the mesh's smallest element width (dg_min_width)."""
    return cfl * mesh.min_width() / (max(mesh.order, 1) * cmax)


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Mesh:
    """One mesh and basis: a dg_ctx of the C library."""

    def __init__(self, n_lon, n_lat, order, dtype="f64", metric="balanced",
                 alpha_mode="local", alpha=0.0, radius=RADIUS, gravity=GRAVITY,
                 omega=OMEGA, h_ref=0.0, stream=None):
        import torch
        self._lib = load()
        self.dtype = {"f64": torch.float64, "f32": torch.float32,
                      torch.float64: torch.float64, torch.float32: torch.float32}[dtype]
        d = MeshDesc()
        d.abi_version = 1
        d.n_lon, d.n_lat, d.order = int(n_lon), int(n_lat), int(order)
        d.dtype = DG_F64 if self.dtype == torch.float64 else DG_F32
        d.metric = {"balanced": DG_METRIC_BALANCED, "pointwise": DG_METRIC_POINTWISE}[metric]
        d.alpha_mode = {"local": DG_ALPHA_LOCAL, "global": DG_ALPHA_GLOBAL}[alpha_mode]
        d.reserved = 0
        d.alpha, d.radius, d.gravity, d.omega, d.h_ref = alpha, radius, gravity, omega, h_ref
        self.desc = d
        self.n_lon, self.n_lat, self.order = d.n_lon, d.n_lat, d.order
        self.n = self.order + 1
        self.N = self.n * self.n
        self.E = self.n_lon * self.n_lat
        self.shape = (self.E, 3, self.N)
        ctx = ctypes.c_void_p()
        check(self._lib.dg_init_mesh(ctypes.byref(d), _stream_handle(stream), ctypes.byref(ctx)))
        self._ctx = ctx
        self._forcing = None

    # -- sizes
    def state_size(self):
        n = ctypes.c_int64()
        check(self._lib.dg_state_size(self._ctx, ctypes.byref(n)))
        return n.value

    def min_width(self):
        w = ctypes.c_double()
        check(self._lib.dg_min_width(self._ctx, ctypes.byref(w)))
        return w.value

    def work_size(self, scheme=DG_SSP_RK3):
        n = ctypes.c_int64()
        check(self._lib.dg_work_size(self._ctx, scheme, ctypes.byref(n)))
        return n.value

    def empty_state(self, device="cuda"):
        import torch
        return torch.empty(self.shape, dtype=self.dtype, device=device)

    def empty_work(self, scheme=DG_SSP_RK3, device="cuda"):
        import torch
        return torch.empty(self.work_size(scheme), dtype=self.dtype, device=device)

    def _ptr(self, t, name, numel=None):
        if not t.is_cuda:
            raise ValueError(f"{name} must be a GPU tensor")
        if t.dtype != self.dtype:
            raise ValueError(f"{name} has dtype {t.dtype}, the mesh uses {self.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != (numel if numel is not None else self.state_size()):
            raise ValueError(f"{name} has {t.numel()} values, expected {numel or self.state_size()}")
        return ctypes.c_void_p(t.data_ptr())

    # -- calls
    def rhs(self, q, out=None, stream=None):
        """out = M^-1 h(q) (+ forcing)."""
        if out is None:
            out = self.empty_state(q.device)
        check(self._lib.dg_rhs(self._ctx, self._ptr(q, "q"), self._ptr(out, "out"),
                               _stream_handle(stream)))
        return out

    def rk_stage(self, q, q0, out, c0, c1, dt, stream=None):
        """out = c0 q0 + c1 (q + dt L(q)); q0 may be None iff c0 == 0."""
        p0 = self._ptr(q0, "q0") if q0 is not None else None
        check(self._lib.dg_rk_stage(self._ctx, self._ptr(q, "q"), p0, self._ptr(out, "out"),
                                    float(c0), float(c1), float(dt), _stream_handle(stream)))
        return out

    def rk_step(self, q, work, dt, scheme=DG_SSP_RK3, nsteps=1, stream=None):
        """Advance q in place by nsteps steps of the scheme."""
        check(self._lib.dg_rk_step(self._ctx, self._ptr(q, "q"),
                                   self._ptr(work, "work", self.work_size(scheme)),
                                   float(dt), int(scheme), int(nsteps), _stream_handle(stream)))
        return q

    def mass(self, q, stream=None):
        """(h, hu, hv) integrals times R^2; synchronises the stream."""
        out = (ctypes.c_double * 3)()
        check(self._lib.dg_mass(self._ctx, self._ptr(q, "q"), out, _stream_handle(stream)))
        return [out[0], out[1], out[2]]

    def set_forcing(self, fhat):
        """Modal forcing added to every right-hand side (None clears).  The
        tensor is kept alive by the mesh while it is set."""
        if fhat is None:
            check(self._lib.dg_set_forcing(self._ctx, None))
        else:
            check(self._lib.dg_set_forcing(self._ctx, self._ptr(fhat, "fhat")))
        self._forcing = fhat

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.dg_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
