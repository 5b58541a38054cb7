"""MI355X-native modal DG shallow-water solver on the sphere.

Python binding of libdgsw (include/dgsw.h): argument marshalling only.  The
state lives in caller-owned torch tensors on the GPU; every step of the
right-hand side and the Runge-Kutta loop runs in the library's HIP kernels
on the caller's current torch stream.
"""
import ctypes
import math

from ._lib import (DG_ABI_VERSION, DG_ALPHA_GLOBAL, DG_ALPHA_LOCAL, DG_F32, DG_F64,
                   DG_METRIC_BALANCED, DG_METRIC_POINTWISE, DG_SSP_RK1, DG_SSP_RK2, DG_SSP_RK3,
                   DG_RK4, AdvDesc, DGError, MeshDesc, PlaneDesc, check, load)

__all__ = ["Mesh", "Plane", "Advection", "Ensemble", "Graph", "DGError", "cfl_time_step", "DG_SSP_RK1",
           "DG_SSP_RK2", "DG_SSP_RK3", "DG_RK4"]

RADIUS, GRAVITY, OMEGA = 6.371e6, 9.80616, 7.292e-5


def cfl_time_step(mesh, cmax, cfl):
    """dt = cfl * H / (max(r, 1) * c_max), the DG Courant number p c dt / H of
    section 2, with H the mesh's smallest element width (dg_min_width)."""
    return cfl * mesh.min_width() / (max(mesh.order, 1) * cmax)


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_desc(n_lon, n_lat, order, dtype="f64", metric="balanced", alpha_mode="local",
              alpha=0.0, radius=RADIUS, gravity=GRAVITY, omega=OMEGA, h_ref=0.0):
    d = MeshDesc()
    d.abi_version = 1
    d.n_lon, d.n_lat, d.order = int(n_lon), int(n_lat), int(order)
    d.dtype = {"f64": DG_F64, "f32": DG_F32}[_dtype_name(dtype)]
    d.metric = {"balanced": DG_METRIC_BALANCED, "pointwise": DG_METRIC_POINTWISE}[metric]
    d.alpha_mode = {"local": DG_ALPHA_LOCAL, "global": DG_ALPHA_GLOBAL}[alpha_mode]
    d.reserved = 0
    d.alpha, d.radius, d.gravity, d.omega, d.h_ref = alpha, radius, gravity, omega, h_ref
    return d


def _dtype_name(dtype):
    if dtype in ("f64", "f32"):
        return dtype
    import torch
    return {torch.float64: "f64", torch.float32: "f32"}[dtype]


class Graph:
    """A captured, instantiated sequence of steps; launch() replays it."""

    def __init__(self, lib, handle, keep):
        self._lib, self._g, self._keep = lib, handle, keep

    def launch(self, stream=None):
        check(self._lib.dg_graph_launch(self._g, _stream_handle(stream)))

    def close(self):
        if getattr(self, "_g", None):
            self._lib.dg_graph_free(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    """One mesh and basis: a dg_ctx of the C library."""

    def __init__(self, n_lon, n_lat, order, dtype="f64", metric="balanced",
                 alpha_mode="local", alpha=0.0, radius=RADIUS, gravity=GRAVITY,
                 omega=OMEGA, h_ref=0.0, stream=None):
        self._lib = load()
        d = make_desc(n_lon, n_lat, order, dtype, metric, alpha_mode, alpha, radius, gravity,
                      omega, h_ref)
        ctx = ctypes.c_void_p()
        check(self._lib.dg_init_mesh(ctypes.byref(d), _stream_handle(stream), ctypes.byref(ctx)))
        self._setup(d, ctx, owns=True)

    @classmethod
    def _borrowed(cls, desc, ctx):
        """A view of a context owned elsewhere (an ensemble member)."""
        m = cls.__new__(cls)
        m._lib = load()
        m._setup(desc, ctx, owns=False)
        return m

    def _setup(self, d, ctx, owns):
        import torch
        self.desc = d
        self.dtype = torch.float64 if d.dtype == DG_F64 else torch.float32
        self.n_lon, self.n_lat, self.order = d.n_lon, d.n_lat, d.order
        self.n = self.order + 1
        self.N = self.n * self.n
        self.E = self.n_lon * self.n_lat
        self.shape = (self.E, 3, self.N)
        self._ctx = ctx
        self._owns = owns
        self._forcing = None

    # -- stage-kernel layout
    _KERNELS = ("line", "half")

    @property
    def kernel(self):
        """"line" (r+1 lanes per element) or "half" (2(r+1) lanes)."""
        k = ctypes.c_int32()
        check(self._lib.dg_get_kernel(self._ctx, ctypes.byref(k)))
        return self._KERNELS[k.value]

    @kernel.setter
    def kernel(self, name):
        check(self._lib.dg_set_kernel(self._ctx, self._KERNELS.index(name)))

    def autotune(self, q, stream=None):
        """Time the stage-kernel layouts on q (read only) and keep the
        fastest (dg_autotune); returns its name.  Synchronises the stream."""
        work = self.empty_work(DG_SSP_RK3, q.device)
        k = ctypes.c_int32()
        check(self._lib.dg_autotune(self._ctx, self._ptr(q, "q"), self._ptr(work, "work", self.work_size()),
                                    ctypes.byref(k), _stream_handle(stream)))
        return self._KERNELS[k.value]

    # -- identical vertical layers (dg_set_levels)
    @property
    def levels(self):
        """Independent copies of the mesh state held by every state buffer."""
        k = ctypes.c_int32()
        check(self._lib.dg_get_levels(self._ctx, ctypes.byref(k)))
        return k.value

    @levels.setter
    def levels(self, n):
        check(self._lib.dg_set_levels(self._ctx, int(n)))
        self.shape = (self.E, 3, self.N) if int(n) == 1 else (int(n), self.E, 3, self.N)

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

    def rk_step_noalloc(self, q, dt, scheme=DG_SSP_RK3, nsteps=1, stream=None):
        """rk_step with the stage states in the library's per-GPU scratch
        array (no work argument, nothing allocated)."""
        check(self._lib.dg_rk_step_noalloc(self._ctx, self._ptr(q, "q"), float(dt), int(scheme),
                                           int(nsteps), _stream_handle(stream)))
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

    def graph(self, q, work, dt, scheme=DG_SSP_RK3, nsteps=1):
        """Capture nsteps steps on q/work as a HIP graph (pointers baked in)."""
        g = ctypes.c_void_p()
        check(self._lib.dg_graph_rk(self._ctx, self._ptr(q, "q"),
                                    self._ptr(work, "work", self.work_size(scheme)), float(dt),
                                    int(scheme), int(nsteps), ctypes.byref(g)))
        return Graph(self._lib, g, (q, work, self))

    def close(self):
        if getattr(self, "_ctx", None) and getattr(self, "_owns", False):
            self._lib.dg_free(self._ctx)
        self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass



class Plane(Mesh):
    """The doubly periodic f-plane [0, lx] x [0, ly] (section 4.2): a dg_ctx
    built by dg_init_plane; every Mesh method applies.  n_lon / n_lat are the
    element counts along x / y."""

    def __init__(self, nx, ny, order, lx, ly, dtype="f64", f=1.0e-4, gravity=9.81,
                 alpha_mode="local", alpha=0.0, h_ref=0.0, stream=None):
        self._lib = load()
        d = PlaneDesc()
        d.abi_version, d.nx, d.ny, d.order = DG_ABI_VERSION, int(nx), int(ny), int(order)
        d.dtype = {"f64": DG_F64, "f32": DG_F32}[dtype]
        d.alpha_mode = {"local": DG_ALPHA_LOCAL, "global": DG_ALPHA_GLOBAL}[alpha_mode]
        d.alpha, d.lx, d.ly = float(alpha), float(lx), float(ly)
        d.gravity, d.f, d.h_ref = float(gravity), float(f), float(h_ref)
        ctx = ctypes.c_void_p()
        check(self._lib.dg_init_plane(ctypes.byref(d), _stream_handle(stream), ctypes.byref(ctx)))
        self.plane = d
        md = MeshDesc()
        md.abi_version, md.n_lon, md.n_lat, md.order, md.dtype = DG_ABI_VERSION, d.nx, d.ny, d.order, d.dtype
        md.alpha_mode, md.alpha, md.radius, md.gravity, md.h_ref = d.alpha_mode, d.alpha, 1.0, d.gravity, d.h_ref
        self._setup(md, ctx, owns=True)


class Advection:
    """Planar linear advection du/dt + div(beta u) = 0 on the periodic
    rectangle (section 4.1's test): a dg_adv of the C library; state u[E][N]."""

    _WORK = {DG_SSP_RK1: 1, DG_SSP_RK2: 2, DG_SSP_RK3: 2, DG_RK4: 3}

    def __init__(self, nx, ny, order, lx=1.0, ly=1.0, beta=(1.0, 1.0), dtype="f64", stream=None):
        import torch
        self._lib = load()
        d = AdvDesc()
        d.abi_version, d.nx, d.ny, d.order = DG_ABI_VERSION, int(nx), int(ny), int(order)
        d.dtype = {"f64": DG_F64, "f32": DG_F32}[dtype]
        d.reserved = 0
        d.lx, d.ly, d.bx, d.by = float(lx), float(ly), float(beta[0]), float(beta[1])
        h = ctypes.c_void_p()
        check(self._lib.dg_adv_init(ctypes.byref(d), _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self.desc = d
        self.nx, self.ny, self.order = d.nx, d.ny, d.order
        self.n = self.order + 1
        self.N = self.n * self.n
        self.E = self.nx * self.ny
        self.shape = (self.E, self.N)
        self.dtype = torch.float64 if dtype == "f64" else torch.float32
        self.dx, self.dy = float(lx) / nx, float(ly) / ny

    def _ptr(self, t, name, numel=None):
        if not t.is_cuda or t.dtype != self.dtype or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous GPU tensor of {self.dtype}")
        if t.numel() != (numel if numel is not None else self.E * self.N):
            raise ValueError(f"{name} has {t.numel()} values")
        return ctypes.c_void_p(t.data_ptr())

    def empty_state(self, device="cuda"):
        import torch
        return torch.empty(self.shape, dtype=self.dtype, device=device)

    def empty_work(self, scheme=DG_RK4, device="cuda"):
        import torch
        return torch.empty(self._WORK[scheme] * self.E * self.N, dtype=self.dtype, device=device)

    def rhs(self, q, out=None, stream=None):
        if out is None:
            out = self.empty_state(q.device)
        check(self._lib.dg_adv_rhs(self._h, self._ptr(q, "q"), self._ptr(out, "out"), _stream_handle(stream)))
        return out

    def rk_step(self, q, work, dt, scheme=DG_RK4, nsteps=1, stream=None):
        check(self._lib.dg_adv_rk_step(self._h, self._ptr(q, "q"),
                                       self._ptr(work, "work", self._WORK[scheme] * self.E * self.N),
                                       float(dt), int(scheme), int(nsteps), _stream_handle(stream)))
        return q

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dg_adv_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

class Ensemble:
    """Independent meshes of different size and order advanced together: one
    persistent kernel launch per Runge-Kutta stage (dg_ens_* of the C ABI).

    members: list of dicts with n_lon, n_lat, order (and optionally metric,
    alpha_mode, alpha, h_ref).  The state is one packed tensor; views() gives
    each member's (E, 3, N) slice."""

    def __init__(self, members, dtype="f32", stream=None, **common):
        self._lib = load()
        descs = (MeshDesc * len(members))()
        for k, m in enumerate(members):
            kw = dict(common)
            kw.update({key: v for key, v in m.items()
                       if key in ("metric", "alpha_mode", "alpha", "h_ref", "radius", "gravity",
                                  "omega")})
            descs[k] = make_desc(m["n_lon"], m["n_lat"], m["order"], dtype, **kw)
        e = ctypes.c_void_p()
        check(self._lib.dg_ens_init(descs, len(members), _stream_handle(stream), ctypes.byref(e)))
        self._e = e
        self._descs = descs
        self.n = len(members)
        n = ctypes.c_int64()
        check(self._lib.dg_ens_state_size(e, ctypes.byref(n)))
        self.size = n.value
        offs = (ctypes.c_int64 * (self.n + 1))()
        check(self._lib.dg_ens_offsets(e, offs))
        self.offsets = [offs[k] for k in range(self.n + 1)]
        self.members = []
        for k in range(self.n):
            c = ctypes.c_void_p()
            check(self._lib.dg_ens_member(e, k, ctypes.byref(c)))
            self.members.append(Mesh._borrowed(descs[k], c))
        self.dtype = self.members[0].dtype

    def empty_state(self, device="cuda"):
        import torch
        return torch.zeros(self.size, dtype=self.dtype, device=device)

    def empty_work(self, device="cuda"):
        import torch
        return torch.zeros(2 * self.size, dtype=self.dtype, device=device)

    def views(self, q):
        """Per-member (E, 3, N) views into a packed state."""
        return [q[self.offsets[k]:self.offsets[k] + m.state_size()].view(m.shape)
                for k, m in enumerate(self.members)]

    def _ptr(self, t, name, numel):
        if not t.is_cuda or t.dtype != self.dtype or not t.is_contiguous() or t.numel() != numel:
            raise ValueError(f"{name}: need a contiguous {self.dtype} GPU tensor of {numel} values")
        return ctypes.c_void_p(t.data_ptr())

    def set_dt(self, dts):
        arr = (ctypes.c_double * self.n)(*[float(x) for x in dts])
        check(self._lib.dg_ens_set_dt(self._e, arr))

    def rhs(self, q, out=None, stream=None):
        if out is None:
            out = self.empty_state(q.device)
        check(self._lib.dg_ens_rhs(self._e, self._ptr(q, "q", self.size),
                                   self._ptr(out, "out", self.size), _stream_handle(stream)))
        return out

    def rk_stage(self, q, q0, out, c0, c1, stream=None):
        p0 = self._ptr(q0, "q0", self.size) if q0 is not None else None
        check(self._lib.dg_ens_rk_stage(self._e, self._ptr(q, "q", self.size), p0,
                                        self._ptr(out, "out", self.size), float(c0), float(c1),
                                        _stream_handle(stream)))
        return out

    def rk_step(self, q, work, nsteps=1, stream=None):
        check(self._lib.dg_ens_rk_step(self._e, self._ptr(q, "q", self.size),
                                       self._ptr(work, "work", 2 * self.size), int(nsteps),
                                       _stream_handle(stream)))
        return q

    def set_schedule(self, waves_per_group, groups, fused=False):
        check(self._lib.dg_ens_set_schedule(self._e, int(waves_per_group), int(groups),
                                            int(bool(fused))))

    def set_kernel(self, order, name):
        """Stage-kernel layout ("line" or "half") of every member of `order`."""
        check(self._lib.dg_ens_set_kernel(self._e, int(order), Mesh._KERNELS.index(name)))

    def kernel(self, order):
        k = ctypes.c_int32()
        check(self._lib.dg_ens_get_kernel(self._e, int(order), ctypes.byref(k)))
        return Mesh._KERNELS[k.value]

    def schedule(self):
        """(waves per workgroup, workgroups, fused)."""
        w, g, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(self._lib.dg_ens_get_schedule(self._e, ctypes.byref(w), ctypes.byref(g),
                                            ctypes.byref(f)))
        return w.value, g.value, bool(f.value)

    def autotune(self, q, work, cache_path=None, stream=None):
        path = cache_path.encode() if cache_path else None
        check(self._lib.dg_ens_autotune(self._e, self._ptr(q, "q", self.size),
                                        self._ptr(work, "work", 2 * self.size), path,
                                        _stream_handle(stream)))
        return self.schedule()

    def graph(self, q, work, nsteps=1):
        g = ctypes.c_void_p()
        check(self._lib.dg_graph_ens(self._e, self._ptr(q, "q", self.size),
                                     self._ptr(work, "work", 2 * self.size), int(nsteps),
                                     ctypes.byref(g)))
        return Graph(self._lib, g, (q, work, self))

    def close(self):
        for m in getattr(self, "members", []):
            m._ctx = None
        if getattr(self, "_e", None):
            self._lib.dg_ens_free(self._e)
            self._e = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
