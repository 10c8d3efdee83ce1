"""ctypes binding of libfdlb (include/fdlb.h).  Argument marshalling only:
every step of the method runs in the library's HIP kernels.  PyTorch is used
for device memory and streams.  If the library is missing, importing this
module raises: there is no CPU fallback."""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdlb.so")

OK, ENOTCONVERGED, EINVAL, EUNSTABLE, EHIP, EDIVERGED, ESTATE, ENOMEM = 0, 1, -1, -2, -3, -4, -5, -6
HALF, FULL = 0, 1
FP64, FP32, MIXED = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "mixed": MIXED}
PRECISION_NAMES = {v: k for k, v in PRECISIONS.items()}
BOTTOM, TOP, LEFT, RIGHT = 0, 1, 2, 3


class FdlbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libfdlb error {code}: {msg}")
        self.code = code


class ProblemDesc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("lx", C.c_double), ("ly", C.c_double),
        ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("wall_u", C.c_double * 4),
        ("kn", C.c_double), ("cfl", C.c_double),
        ("qx_kind", C.c_int32), ("qx_n", C.c_int32),
        ("qy_kind", C.c_int32), ("qy_n", C.c_int32),
        ("precision", C.c_int32), ("allow_unstable", C.c_int32),
    ]


class Report(C.Structure):
    _fields_ = [
        ("steps", C.c_int64), ("first_below", C.c_int64),
        ("residual", C.c_double), ("wall_s", C.c_double),
        ("updates_per_s", C.c_double), ("bytes_per_s", C.c_double),
        ("status", C.c_int32), ("history_len", C.c_int32), ("history_cap", C.c_int32),
        ("pad_", C.c_int32), ("history", C.POINTER(C.c_double)),
        ("steps_fp32", C.c_int64),
    ]


class HybridDesc(C.Structure):
    _fields_ = [
        ("ny", C.c_int32), ("layer", C.c_int32),
        ("kn", C.c_double), ("u_bottom", C.c_double), ("u_top", C.c_double), ("cfl", C.c_double),
        ("qx_kind", C.c_int32), ("qx_n", C.c_int32),
        ("n_half", C.c_int32), ("n_full", C.c_int32),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python paper_1308_0692_amd/build.py")
    # torch first: the library then binds to the HIP runtime torch has loaded, so that one
    # runtime (one view of the devices, streams and allocations) serves the process.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    dp, vp, i64, i32 = C.POINTER(C.c_double), C.c_void_p, C.c_int64, C.c_int32
    fp = C.POINTER(C.c_float)
    sig = {
        "fdlb_quad_half_range": (C.c_int, [C.c_int, dp, dp]),
        "fdlb_quad_full_range": (C.c_int, [C.c_int, dp, dp]),
        "fdlb_problem_create": (C.c_int, [C.POINTER(ProblemDesc), C.POINTER(vp)]),
        "fdlb_problem_destroy": (None, [vp]),
        "fdlb_problem_q": (C.c_int, [vp]),
        "fdlb_problem_dt": (C.c_double, [vp]),
        "fdlb_problem_omega": (C.c_double, [vp]),
        "fdlb_problem_velocities": (C.c_int, [vp, dp, dp, dp]),
        "fdlb_state_bytes": (C.c_size_t, [vp]),
        "fdlb_workspace_bytes": (C.c_size_t, [vp]),
        "fdlb_bind": (C.c_int, [vp, vp, vp, vp]),
        "fdlb_init_equilibrium": (C.c_int, [vp, dp, dp, dp, C.c_int]),
        "fdlb_init_equilibrium_dev": (C.c_int, [vp, fp, fp, fp, C.c_int]),
        "fdlb_state_upload": (C.c_int, [vp, dp]),
        "fdlb_state_download": (C.c_int, [vp, dp]),
        "fdlb_checkpoint_bytes": (C.c_size_t, [vp]),
        "fdlb_checkpoint_save": (C.c_int, [vp, vp]),
        "fdlb_checkpoint_load": (C.c_int, [vp, vp]),
        "fdlb_step": (C.c_int, [vp, i64]),
        "fdlb_step_static": (C.c_int, [vp, vp, i64, vp]),
        "fdlb_set_pseudo_time": (C.c_int, [vp, C.c_int]),
        "fdlb_problem_pseudo_weights": (C.c_int, [vp, dp]),
        "fdlb_batch_set_pseudo_time": (C.c_int, [vp, C.c_int]),
        "fdlb_step_timed": (C.c_int, [vp, i64, dp, dp]),
        "fdlb_last_residual": (C.c_int, [vp, dp, C.POINTER(i64)]),
        "fdlb_solve_steady": (C.c_int, [vp, C.c_double, i64, i32, i32, C.POINTER(Report)]),
        "fdlb_moments": (C.c_int, [vp, dp, dp, dp, dp]),
        "fdlb_wall_profile": (C.c_int, [vp, C.c_int, dp, dp, dp]),
        "fdlb_tile_count": (C.c_int, [C.c_int]),
        "fdlb_tile_describe": (C.c_int, [C.c_int, C.c_int, C.c_char_p, C.c_size_t]),
        "fdlb_problem_set_tile": (C.c_int, [vp, C.c_int]),
        "fdlb_problem_get_tile": (C.c_int, [vp]),
        "fdlb_autotune": (C.c_int, [vp, C.c_int, dp]),
        "fdlb_problem_active_precision": (C.c_int, [vp]),
        "fdlb_promote": (C.c_int, [vp]),
        "fdlb_stream_copy": (C.c_int, [vp, vp, C.c_size_t, vp]),
        "fdlb_set_tune_cache": (C.c_int, [C.c_char_p]),
        "fdlb_stream_probe": (C.c_int, [vp, vp, C.c_size_t, C.c_int, vp]),
        "fdlb_batch_create": (C.c_int, [C.POINTER(ProblemDesc), C.c_int, C.POINTER(vp)]),
        "fdlb_batch_destroy": (None, [vp]),
        "fdlb_batch_state_bytes": (C.c_size_t, [vp]),
        "fdlb_batch_workspace_bytes": (C.c_size_t, [vp]),
        "fdlb_batch_bind": (C.c_int, [vp, vp, vp, vp]),
        "fdlb_batch_init_equilibrium": (C.c_int, [vp, C.c_int, dp, dp, dp, C.c_int]),
        "fdlb_batch_init_equilibrium_dev": (C.c_int, [vp, C.c_int, fp, fp, fp, C.c_int]),
        "fdlb_batch_solve": (C.c_int, [vp, C.c_double, i64, i32, i32, C.POINTER(Report)]),
        "fdlb_batch_moments": (C.c_int, [vp, C.c_int, dp, dp, dp, dp]),
        "fdlb_batch_wall_profile": (C.c_int, [vp, C.c_int, C.c_int, dp, dp, dp]),
        "fdlb_batch_state_download": (C.c_int, [vp, C.c_int, dp]),
        "fdlb_batch_state_upload": (C.c_int, [vp, C.c_int, dp]),
        "fdlb_batch_problem_q": (C.c_int, [vp, C.c_int]),
        "fdlb_batch_set_tile": (C.c_int, [vp, C.c_int]),
        "fdlb_batch_get_tile": (C.c_int, [vp]),
        "fdlb_batch_autotune": (C.c_int, [vp, C.c_int, dp]),
        "fdlb_batch_active_precision": (C.c_int, [vp, C.c_int]),
        "fdlb_batch_set_retile": (C.c_int, [vp, C.c_int]),
        "fdlb_mlp_create": (C.c_int, [C.c_int, i64, C.POINTER(vp)]),
        "fdlb_mlp_destroy": (None, [vp]),
        "fdlb_mlp_param_count": (i64, [vp]),
        "fdlb_mlp_workspace_bytes": (C.c_size_t, [vp]),
        "fdlb_mlp_init_params": (C.c_int, [vp, C.c_uint64, fp]),
        "fdlb_mlp_bind": (C.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "fdlb_mlp_forward": (C.c_int, [vp, vp, i64, vp]),
        "fdlb_mlp_backward": (C.c_int, [vp, vp, vp, vp, i64]),
        "fdlb_mlp_last_loss": (C.c_int, [vp, dp]),
        "fdlb_mlp_adam_step": (C.c_int, [vp, C.c_double, C.c_double, C.c_double, C.c_double, i64]),
        "fdlb_mlp_train": (C.c_int, [vp, vp, vp, vp, C.c_int64, C.c_int64, C.c_int64, dp, C.c_double, C.c_double,
                                    C.c_double, C.c_int64]),
        "fdlb_mlp_predict_fields": (C.c_int, [vp, C.c_double, C.c_int, C.c_int, C.c_double, vp, vp, vp]),
        "fdlb_field_samples": (C.c_int, [vp, vp, vp]),
        "fdlb_batch_field_samples": (C.c_int, [vp, C.c_int, vp, vp]),
        "fdlb_hybrid_create": (C.c_int, [C.POINTER(HybridDesc), C.c_int, C.POINTER(vp)]),
        "fdlb_hybrid_destroy": (None, [vp]),
        "fdlb_hybrid_state_bytes": (C.c_size_t, [vp]),
        "fdlb_hybrid_workspace_bytes": (C.c_size_t, [vp]),
        "fdlb_hybrid_info": (C.c_int, [vp, C.c_int, C.POINTER(i32), C.POINTER(i32), C.POINTER(i64), dp, dp]),
        "fdlb_hybrid_bind": (C.c_int, [vp, vp, vp, vp]),
        "fdlb_hybrid_init_equilibrium": (C.c_int, [vp, C.c_int, dp, dp, dp]),
        "fdlb_hybrid_set_state": (C.c_int, [vp, C.c_int, dp]),
        "fdlb_hybrid_get_state": (C.c_int, [vp, C.c_int, dp]),
        "fdlb_hybrid_step": (C.c_int, [vp, i64]),
        "fdlb_hybrid_solve": (C.c_int, [vp, C.c_double, i64, i64, C.POINTER(Report)]),
        "fdlb_hybrid_moments": (C.c_int, [vp, C.c_int, dp, dp, dp, dp]),
        "fdlb_hybrid_faces": (C.c_int, [vp, C.c_int, dp]),
        "fdlb_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


def check(code: int, allow=(OK,)) -> int:
    if code in allow:
        return code
    raise FdlbError(code, lib.fdlb_last_error().decode())


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def quad_half_range(n: int):
    x, w = np.empty(2 * n), np.empty(2 * n)
    check(lib.fdlb_quad_half_range(n, _dp(x), _dp(w)))
    return x, w


def quad_full_range(n: int):
    x, w = np.empty(n), np.empty(n)
    check(lib.fdlb_quad_full_range(n, _dp(x), _dp(w)))
    return x, w


def make_desc(nx, ny, periodic_x, periodic_y, wall_u, kn, qx, qy, cfl=0.9, precision="fp32",
              allow_unstable=False, lx=1.0, ly=1.0) -> ProblemDesc:
    kinds = {"half": HALF, "full": FULL}
    d = ProblemDesc()
    d.nx, d.ny = int(nx), int(ny)
    d.lx, d.ly = float(lx), float(ly)
    d.periodic_x, d.periodic_y = int(bool(periodic_x)), int(bool(periodic_y))
    d.wall_u = (C.c_double * 4)(*[float(v) for v in wall_u])
    d.kn = float(kn)
    d.cfl = float(cfl)
    d.qx_kind, d.qx_n = kinds[qx[0]], int(qx[1])
    d.qy_kind, d.qy_n = kinds[qy[0]], int(qy[1])
    d.precision = PRECISIONS[precision]
    d.allow_unstable = int(bool(allow_unstable))
    return d


def make_hybrid_desc(ny, layer, kn, u_w=(-0.01, 0.01), n_half=4, n_full=None, qx=("full", 3),
                     cfl=0.9) -> HybridDesc:
    kinds = {"half": HALF, "full": FULL}
    d = HybridDesc()
    d.ny, d.layer = int(ny), int(layer)
    d.kn = float(kn)
    d.u_bottom, d.u_top = float(u_w[0]), float(u_w[1])
    d.cfl = float(cfl)
    d.qx_kind, d.qx_n = kinds[qx[0]], int(qx[1])
    d.n_half = int(n_half)
    d.n_full = int(n_half if n_full is None else n_full)
    return d


def desc_from_case(case, precision: Optional[str] = None, allow_unstable=False) -> ProblemDesc:
    return make_desc(case.nx, case.ny, case.periodic_x, case.periodic_y, case.wall_u, case.kn,
                     case.qx, case.qy, case.cfl, precision or case.precision, allow_unstable,
                     getattr(case, "lx", 1.0), getattr(case, "ly", 1.0))


def tile_count(precision: str) -> int:
    return check(lib.fdlb_tile_count(FP32 if precision == "fp32" else FP64), allow=range(0, 1 << 20))


def tile_describe(precision: str, tile: int) -> str:
    buf = C.create_string_buffer(128)
    check(lib.fdlb_tile_describe(FP32 if precision == "fp32" else FP64, tile, buf, 128))
    return buf.value.decode()
