"""ctypes binding of libmpf (include/mpf.h).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.  Arrays are torch
tensors on the current HIP device; pointers and the current stream are passed
through unchanged.  If the library is not built this module raises at import:
there is no fallback path."""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_INC = os.path.join(os.path.dirname(_HERE), "include")
SO_PATH = os.path.join(_HERE, "libmpf.so")
SOURCES = ["weights.hip", "acm.hip", "lbm.hip", "reduce.hip", "mlp.hip", "mlp_fused.hip", "knn.hip", "tiles.hip"]

MPF_F64, MPF_F32, MPF_MIXED, MPF_F32_KAHAN = 0, 1, 2, 3
MPF_ERR_DIVERGED = -4
MPF_FLAG_NONFINITE, MPF_FLAG_LIMIT = 1, 2
SOLVE_FP64, SOLVE_FP32_IR = 0, 1
OP = {"dx": 0, "dy": 1, "dz": 2, "lap": 3, "dir": 4, "shift": 5, "dn": 6, "shift_row": 7, "taylor": 8}
UNKNOWN_RULE = {"normal": 0, "solid": 1}


class MPFError(RuntimeError):
    pass


class MPFDiverged(MPFError, FloatingPointError):
    """A run's flags word was set: a non-finite state or a stability limit."""


HIPCC_FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build() -> str:
    """Compile libmpf.so for gfx950 in-tree (hipcc cross-compiles without a
    GPU): each source to an object in parallel, then one link."""
    import tempfile
    with tempfile.TemporaryDirectory() as tmpd:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpd, src + ".o")
            cmd = ["/opt/rocm/bin/hipcc", *HIPCC_FLAGS, "-I" + _INC, "-I" + os.path.join(_HERE, "csrc"), "-c",
                   os.path.join(_HERE, "csrc", src), "-o", obj]
            procs.append((src, subprocess.Popen(cmd)))
            objs.append(obj)
        for src, p in procs:
            if p.wait() != 0:
                raise RuntimeError(f"hipcc failed on {src}")
        tmp = SO_PATH + ".tmp"
        subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-shared", *objs, "-o", tmp])
        os.replace(tmp, SO_PATH)
    return SO_PATH


class MlpDesc(ctypes.Structure):
    _fields_ = [("in_dim", ctypes.c_int32), ("width", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("out_dim", ctypes.c_int32)]


class _Op(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("vec", ctypes.c_double * 3)]


class WGeom(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("n_nodes", ctypes.c_int64), ("sten", ctypes.c_void_p),
                ("m", ctypes.c_int64), ("rowvec", ctypes.c_void_p), ("w64", ctypes.c_void_p),
                ("w32", ctypes.c_void_p), ("info", ctypes.c_void_p)]


class WTune(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_int32), ("rows_per_wave", ctypes.c_int32)]


class AcmParams(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("rho", ctypes.c_double), ("dt", ctypes.c_double),
                ("beta", ctypes.c_double), ("v_ref", ctypes.c_double), ("g", ctypes.c_double * 3),
                ("n_p", ctypes.c_int32), ("precision", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("edac", ctypes.c_int32), ("h_min", ctypes.c_double)]


class LbmParams(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("precision", ctypes.c_int32), ("tau_plus", ctypes.c_double),
                ("tau_minus", ctypes.c_double), ("g_lb", ctypes.c_double * 3)]


class Tiles(ctypes.Structure):
    _fields_ = [("count", ctypes.c_void_p), ("halo", ctypes.c_void_p), ("lidx", ctypes.c_void_p),
                ("h_cap", ctypes.c_int32), ("h_max", ctypes.c_int32), ("tile", ctypes.c_int32)]


class LbmUnits(ctypes.Structure):
    _fields_ = [("dx", ctypes.c_double), ("dt", ctypes.c_double), ("nu_lb", ctypes.c_double),
                ("tau_minus", ctypes.c_double), ("vel_scale", ctypes.c_double), ("g_lb", ctypes.c_double * 3)]


def _load():
    if not os.path.exists(SO_PATH):
        raise MPFError(f"libmpf.so is not built ({SO_PATH}); run __graft_entry__.build()")
    lib = ctypes.CDLL(SO_PATH)
    vp, i64, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    flt = ctypes.c_float
    sig = {
        "mpf_strerror": (ctypes.c_char_p, [i32]),
        "mpf_version": (i32, []),
        "mpf_sc_cell": (i32, [dbl, vp, vp]),
        "mpf_weights_workspace": (sz, []),
        "mpf_rbffd_weights": (i32, [vp, i64, vp, i64, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp]),
        "mpf_create": (i32, [vp, i32]),
        "mpf_destroy": (i32, [vp]),
        "mpf_rbffd_weights_batched": (i32, [vp, i32, vp, i32, i32, vp, i32, vp, vp, sz, vp]),
        "mpf_weights_autotune": (i32, [vp, i32, i32, vp, i32, vp, i64, vp, vp, sz]),
        "mpf_acm_dt": (i32, [dbl, dbl, vp]),
        "mpf_acm_workspace": (sz, [i64, i32]),
        "mpf_acm_run": (i32, [vp, i64, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp, sz, vp]),
        "mpf_lbm_init": (i32, [vp, i64, dbl, vp, vp, vp]),
        "mpf_lbm_init_fields": (i32, [vp, i64, vp, vp, dbl, vp, vp]),
        "mpf_lbm_run": (i32, [vp, i64, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp]),
        "mpf_tile_count": (i64, [i64]),
        "mpf_tile_plan": (i32, [i64, i32, vp, i32, vp, vp, vp, vp, vp]),
        "mpf_tile_count_sized": (i64, [i64, i32]),
        "mpf_tile_plan_sized": (i32, [i64, i32, vp, i32, i32, vp, vp, vp, vp, vp]),
        "mpf_lbm_units_of": (i32, [dbl, dbl, dbl, dbl, vp, vp]),
        "mpf_permeability": (i32, [dbl, dbl, vp, dbl, vp]),
        "mpf_drag_coefficient": (i32, [dbl, dbl, dbl, dbl, dbl, vp]),
        "mpf_residual": (i32, [i64, i64, i32, vp, vp, vp, vp, i32, vp, vp, sz, vp]),
        "mpf_pointwise": (i32, [i64, vp, i32, vp, i32, vp, vp, i64, i32, vp, vp, vp]),
        "mpf_flux_planes_noalloc_max": (i64, []),
        "mpf_flux_planes_noalloc": (i32, [i64, i32, vp, vp, vp, i32, i64, vp, vp]),
        "mpf_lbm_unknown": (i32, [i32, i64, i64, vp, vp, i32, dbl, dbl, vp, vp]),
        "mpf_knn_workspace": (ctypes.c_size_t, [i64]),
        "mpf_knn": (i32, [vp, i64, i64, vp, i64, i64, i32, vp, i64, vp, ctypes.c_size_t, vp]),
        "mpf_solver_stencils": (i32, [vp, i64, i64, i32, vp, vp, ctypes.c_size_t, vp]),
        "mpf_lbm_moments": (i32, [vp, i64, vp, vp, dbl, vp, vp, vp]),
        "mpf_reduce_workspace": (sz, [i64]),
        "mpf_flux_planes": (i32, [i64, i32, vp, vp, vp, i32, i64, vp, vp, sz, vp]),
        "mpf_drag": (i32, [i64, vp, vp, i32, i64, i32, vp, vp, vp, dbl, dbl, dbl, vp, vp, sz, vp]),
        "mpf_traction": (i32, [i64, vp, vp, i32, i64, i32, vp, vp, vp, dbl, dbl, vp, vp, vp, sz, vp]),
        "mpf_mlp_param_count": (i64, [vp]),
        "mpf_mlp_packed_count": (i64, [vp]),
        "mpf_mlp_workspace": (sz, [vp, i64, i32]),
        "mpf_mlp_pack": (i32, [vp, vp, vp, vp]),
        "mpf_mlp_forward": (i32, [vp, vp, vp, vp, vp, vp, i64, i32, vp, sz, vp]),
        "mpf_mlp_backward": (i32, [vp, vp, vp, vp, i64, vp, sz, vp]),
        "mpf_mlp_mse": (i32, [i64, vp, vp, vp, vp, vp, vp, sz, vp]),
        "mpf_adam_step": (i32, [i64, vp, vp, vp, vp, i32, flt, flt, flt, flt, vp]),
        "mpf_mlp_features": (i32, [i64, vp, dbl, dbl, vp, vp]),
        "mpf_mlp_to_state": (i32, [i64, i64, vp, dbl, dbl, i32, vp, vp, vp, vp, sz, vp]),
        "mpf_gemm_bf16": (i32, [i64, i32, i64, vp, i64, vp, i64, vp, i64, vp]),
        "mpf_mlp_train_workspace": (sz, [vp, i64]),
        "mpf_shuffle_rows": (i32, [i64, i64, ctypes.c_uint64, vp, vp]),
        "mpf_mlp_fused_workspace": (sz, [vp, i64]),
        "mpf_mlp_grad_fused": (i32, [vp, vp, vp, vp, vp, vp, i64, vp, vp, vp, sz, vp]),
        "mpf_mlp_train_fused": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, i64, i32, flt, flt, flt, flt, flt, vp,
                                      vp, sz, vp]),
        "mpf_scale": (i32, [i64, vp, i32, dbl, vp]),
        "mpf_mlp_train": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, i64, i32, flt, flt, flt, flt, flt, vp, vp,
                                sz, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_LIB = None


def lib():
    """The loaded library; raises MPFError if it has not been built."""
    global _LIB
    if _LIB is None:
        _LIB = _load()
    return _LIB


EXPORTED = ["mpf_strerror", "mpf_version", "mpf_create", "mpf_destroy", "mpf_acm_dt", "mpf_lbm_units_of",
            "mpf_permeability", "mpf_drag_coefficient", "mpf_residual", "mpf_flux_planes_noalloc", "mpf_pointwise",
            "mpf_tile_count", "mpf_tile_plan", "mpf_tile_count_sized", "mpf_tile_plan_sized",
            "mpf_flux_planes_noalloc_max",
            "mpf_sc_cell", "mpf_weights_workspace", "mpf_rbffd_weights",
            "mpf_rbffd_weights_batched", "mpf_weights_autotune", "mpf_acm_workspace", "mpf_acm_run",
            "mpf_lbm_init", "mpf_lbm_init_fields", "mpf_lbm_run", "mpf_lbm_unknown", "mpf_lbm_moments",
            "mpf_knn_workspace", "mpf_knn", "mpf_solver_stencils", "mpf_reduce_workspace",
            "mpf_flux_planes", "mpf_drag", "mpf_traction", "mpf_mlp_param_count", "mpf_mlp_packed_count", "mpf_mlp_workspace",
            "mpf_mlp_pack", "mpf_mlp_forward", "mpf_mlp_backward", "mpf_mlp_mse", "mpf_adam_step",
            "mpf_mlp_features", "mpf_mlp_to_state", "mpf_gemm_bf16", "mpf_mlp_train_workspace", "mpf_mlp_train",
            "mpf_shuffle_rows", "mpf_scale", "mpf_mlp_fused_workspace", "mpf_mlp_grad_fused", "mpf_mlp_train_fused"]


def check(rc: int, what: str):
    if rc != 0:
        cls = MPFDiverged if rc == MPF_ERR_DIVERGED else MPFError
        raise cls(f"{what}: {lib().mpf_strerror(rc).decode()} ({rc})")


_CTX = {}


def ctx(device: int | None = None) -> ctypes.c_void_p:
    """The library context of a HIP device (default: the current one),
    created on first use and kept for the life of the process; it holds the
    weight solve's autotune cache."""
    if device is None:
        import torch
        device = torch.cuda.current_device()
    if device not in _CTX:
        c = ctypes.c_void_p()
        check(lib().mpf_create(ctypes.byref(c), int(device)), "mpf_create")
        _CTX[device] = c
    return _CTX[device]


def make_ops(ops):
    arr = (_Op * len(ops))()
    for i, o in enumerate(ops):
        arr[i].kind = OP[o[0]]
        vec = o[1] if len(o) > 1 and o[1] is not None else (0.0, 0.0, 0.0)
        for t in range(3):
            arr[i].vec[t] = float(vec[t])
    return arr
