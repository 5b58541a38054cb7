"""ctypes loader of libdgsw.so and the C structures of include/dgsw.h.

Argument marshalling only: every computation runs in the library's HIP
kernels.  A missing library is an error, never a fallback.
"""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdgsw.so")

DG_ABI_VERSION = 1
DG_F64, DG_F32 = 0, 1
DG_METRIC_BALANCED, DG_METRIC_POINTWISE = 0, 1
DG_ALPHA_LOCAL, DG_ALPHA_GLOBAL = 0, 1
DG_SSP_RK1, DG_SSP_RK2, DG_SSP_RK3, DG_RK4 = 1, 2, 3, 4
DG_KERNEL_LINE, DG_KERNEL_HALF = 0, 1
DG_OK, DG_EINVAL, DG_EDTYPE, DG_ENOMEM, DG_EHIP, DG_ENONFINITE, DG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6

ERROR_NAMES = {
    DG_EINVAL: "DG_EINVAL", DG_EDTYPE: "DG_EDTYPE", DG_ENOMEM: "DG_ENOMEM",
    DG_EHIP: "DG_EHIP", DG_ENONFINITE: "DG_ENONFINITE", DG_EUNSUPPORTED: "DG_EUNSUPPORTED",
}

# every symbol include/dgsw.h declares
EXPORTS = ("dg_init_mesh", "dg_init_plane", "dg_set_kernel", "dg_get_kernel", "dg_autotune",
           "dg_set_levels",
           "dg_get_levels", "dg_free", "dg_state_size", "dg_work_size", "dg_min_width", "dg_rhs",
           "dg_rk_stage", "dg_rk_step", "dg_mass", "dg_set_forcing", "dg_last_error",
           "dg_ens_init", "dg_ens_free", "dg_ens_state_size", "dg_ens_offsets", "dg_ens_member",
           "dg_ens_set_dt", "dg_ens_rhs", "dg_ens_rk_stage", "dg_ens_rk_step", "dg_ens_set_schedule",
           "dg_ens_set_kernel", "dg_ens_get_kernel",
           "dg_ens_get_schedule", "dg_ens_autotune", "dg_graph_rk", "dg_graph_ens",
           "dg_graph_launch", "dg_graph_free", "dg_mlp_param_count", "dg_mlp_workspace_size",
           "dg_mlp_forward", "dg_mlp_train_step", "dg_project", "dg_features",
           "dg_learned_workspace_size", "dg_rhs_learned", "dg_rk_step_learned",
           "dg_adv_init", "dg_adv_free", "dg_adv_state_size", "dg_adv_rhs", "dg_adv_rk_step",
           "dg_rk_step_noalloc")


class Learned(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("feat_mean", ctypes.c_void_p),
                ("feat_istd", ctypes.c_void_p), ("out_mean", ctypes.c_void_p),
                ("out_std", ctypes.c_void_p), ("kappa", ctypes.c_double)]


class DGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("n_lon", ctypes.c_int32),
                ("n_lat", ctypes.c_int32), ("order", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("metric", ctypes.c_int32),
                ("alpha_mode", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("radius", ctypes.c_double),
                ("gravity", ctypes.c_double), ("omega", ctypes.c_double),
                ("h_ref", ctypes.c_double)]


class PlaneDesc(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("order", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("alpha_mode", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("gravity", ctypes.c_double), ("f", ctypes.c_double), ("h_ref", ctypes.c_double)]


class AdvDesc(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("order", ctypes.c_int32), ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("bx", ctypes.c_double),
                ("by", ctypes.c_double)]


_lib = None


def load():
    """Load libdgsw.so (once) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2303_11767_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
    lib.dg_init_mesh.argtypes = [ctypes.POINTER(MeshDesc), vp, ctypes.POINTER(vp)]
    lib.dg_init_plane.argtypes = [ctypes.POINTER(PlaneDesc), vp, ctypes.POINTER(vp)]
    lib.dg_set_kernel.argtypes = [vp, i32]
    lib.dg_get_kernel.argtypes = [vp, ctypes.POINTER(i32)]
    lib.dg_free.argtypes = [vp]
    lib.dg_state_size.argtypes = [vp, i64p]
    lib.dg_work_size.argtypes = [vp, i32, i64p]
    lib.dg_min_width.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.dg_rhs.argtypes = [vp, vp, vp, vp]
    lib.dg_rk_stage.argtypes = [vp, vp, vp, vp, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, vp]
    lib.dg_rk_step.argtypes = [vp, vp, vp, ctypes.c_double, i32, i32, vp]
    lib.dg_rk_step_noalloc.argtypes = [vp, vp, ctypes.c_double, i32, i32, vp]
    lib.dg_mass.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.dg_set_forcing.argtypes = [vp, vp]
    dp = ctypes.POINTER(ctypes.c_double)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.dg_ens_init.argtypes = [ctypes.POINTER(MeshDesc), i32, vp, ctypes.POINTER(vp)]
    lib.dg_ens_free.argtypes = [vp]
    lib.dg_ens_state_size.argtypes = [vp, i64p]
    lib.dg_ens_offsets.argtypes = [vp, i64p]
    lib.dg_ens_member.argtypes = [vp, i32, ctypes.POINTER(vp)]
    lib.dg_ens_set_dt.argtypes = [vp, dp]
    lib.dg_ens_rhs.argtypes = [vp, vp, vp, vp]
    lib.dg_ens_rk_stage.argtypes = [vp, vp, vp, vp, ctypes.c_double, ctypes.c_double, vp]
    lib.dg_ens_rk_step.argtypes = [vp, vp, vp, i32, vp]
    lib.dg_ens_set_schedule.argtypes = [vp, i32, i32, i32]
    lib.dg_ens_get_schedule.argtypes = [vp, i32p, i32p, i32p]
    lib.dg_ens_set_kernel.argtypes = [vp, i32, i32]
    lib.dg_ens_get_kernel.argtypes = [vp, i32, i32p]
    lib.dg_ens_autotune.argtypes = [vp, vp, vp, ctypes.c_char_p, vp]
    lib.dg_graph_rk.argtypes = [vp, vp, vp, ctypes.c_double, i32, i32, ctypes.POINTER(vp)]
    lib.dg_graph_ens.argtypes = [vp, vp, vp, i32, ctypes.POINTER(vp)]
    lib.dg_graph_launch.argtypes = [vp, vp]
    lib.dg_graph_free.argtypes = [vp]
    lib.dg_mlp_param_count.argtypes = [i64p]
    lib.dg_mlp_workspace_size.argtypes = [ctypes.c_int64, i64p]
    lib.dg_mlp_forward.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp]
    lib.dg_mlp_train_step.argtypes = [vp, vp, vp, i32, ctypes.c_float, vp, vp, vp, ctypes.c_int64,
                                      vp, vp, vp, vp]
    lib.dg_project.argtypes = [vp, vp, vp, vp, vp]
    lib.dg_features.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.dg_learned_workspace_size.argtypes = [vp, i64p]
    lib.dg_rhs_learned.argtypes = [vp, ctypes.POINTER(Learned), vp, vp, vp, vp, vp]
    lib.dg_rk_step_learned.argtypes = [vp, ctypes.POINTER(Learned), vp, vp, vp, ctypes.c_double, i32,
                                       vp, vp]
    lib.dg_adv_init.argtypes = [ctypes.POINTER(AdvDesc), vp, ctypes.POINTER(vp)]
    lib.dg_adv_free.argtypes = [vp]
    lib.dg_adv_state_size.argtypes = [vp, i64p]
    lib.dg_adv_rhs.argtypes = [vp, vp, vp, vp]
    lib.dg_adv_rk_step.argtypes = [vp, vp, vp, ctypes.c_double, i32, i32, vp]
    lib.dg_last_error.argtypes = []
    lib.dg_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "dg_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(rc):
    if rc != DG_OK:
        msg = load().dg_last_error().decode(errors="replace")
        raise DGError(rc, msg)
    return rc
