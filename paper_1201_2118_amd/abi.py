"""ctypes binding of libns.so with the C ABI's names (include/ns.h).

Argument marshalling only: every stage of the step runs in the HIP library.
If the library cannot be loaded, every call raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libns.so")

NS_OK, NS_E_INVALID, NS_E_OOM, NS_E_DEVICE, NS_E_NONFINITE, NS_E_UNSTABLE, NS_E_STATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "NS_OK", -1: "NS_E_INVALID", -2: "NS_E_OOM", -3: "NS_E_DEVICE",
                -4: "NS_E_NONFINITE", -5: "NS_E_UNSTABLE", -6: "NS_E_STATE"}
NS_U, NS_V, NS_W, NS_P, NS_FX, NS_FY, NS_FZ, NS_F, NS_G, NS_H, NS_RHS = range(11)
FIELD_IDS = {"u": NS_U, "v": NS_V, "w": NS_W, "p": NS_P, "fx": NS_FX, "fy": NS_FY, "fz": NS_FZ,
             "F": NS_F, "G": NS_G, "H": NS_H, "rhs": NS_RHS}
NS_BC_WALL, NS_BC_PERIODIC = 0, 1
NS_FP64, NS_MIXED = 0, 1
NS_ALLOW_UNSTABLE, NS_TIMING, NS_BATCH_LAUNCHES, NS_GENERATED, NS_ADVECTIVE, NS_RK2 = 1, 2, 4, 8, 16, 32
NS_T_BC, NS_T_FGH, NS_T_RHS, NS_T_SOR, NS_T_DEFECT, NS_T_PROJECT, NS_T_OTHER, NS_T_COUNT = 0, 1, 2, 3, 4, 5, 6, 8
EXPORTED = ("ns_params_default", "ns_create", "ns_set_state", "ns_step", "ns_get_state",
            "ns_backward", "ns_get_timing", "ns_destroy", "ns_last_error", "ns_step_noalloc", "ns_guard_check")


class ns_params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
        ("re", ctypes.c_double), ("dt", ctypes.c_double), ("tau", ctypes.c_double),
        ("gamma", ctypes.c_double), ("omega", ctypes.c_double), ("tol", ctypes.c_double),
        ("itermax", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 3),
        ("wall_vel", (ctypes.c_double * 3) * 6),
        ("g", ctypes.c_double * 3),
        ("eta", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("checkpoint_every", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("tile", ctypes.c_int32 * 2),
    ]


class ns_stats(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double), ("dt_last", ctypes.c_double), ("res_last", ctypes.c_double),
        ("sweeps_total", ctypes.c_int64),
        ("steps", ctypes.c_int32), ("sweeps_max", ctypes.c_int32),
        ("steps_unconverged", ctypes.c_int32), ("outer_max", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ns_timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * NS_T_COUNT), ("launches", ctypes.c_int64 * NS_T_COUNT),
                ("sor_bytes", ctypes.c_int64), ("sor_tile", ctypes.c_int32 * 2)]


class NSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libns.so (building it first only when no library exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        from . import build as _build
        _build.build()
    # torch ships its own HIP runtime under the soname the library needs; when
    # torch is installed, load it first so that the process holds one HIP
    # runtime (with the system runtime loaded first, torch maps a second one
    # and finds no GPU)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    P = ctypes.POINTER
    sig = {
        "ns_params_default": (ctypes.c_int, [P(ns_params)]),
        "ns_create": (ctypes.c_int, [P(ns_params), ctypes.c_int32, vp, P(vp)]),
        "ns_set_state": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int32]),
        "ns_step": (ctypes.c_int, [vp, ctypes.c_int32, P(ns_stats)]),
        "ns_get_state": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int32]),
        "ns_backward": (ctypes.c_int, [vp, ctypes.c_int32, P(vp), P(vp), ctypes.c_int32]),
        "ns_get_timing": (ctypes.c_int, [vp, P(ns_timing)]),
        "ns_destroy": (None, [vp]),
        "ns_last_error": (ctypes.c_char_p, [vp]),
        "ns_step_noalloc": (ctypes.c_int, [P(ns_params), vp, vp, vp, vp, ctypes.c_int32, vp, P(ns_stats)]),
        "ns_guard_check": (ctypes.c_int64, [ctypes.c_int32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(code, handle=None):
    if code != NS_OK:
        msg = load().ns_last_error(handle)
        raise NSError(code, msg.decode() if msg else "")
    return code


# -- the C ABI, one Python function per entry point ---------------------------

def ns_params_default(p: ns_params) -> int:
    return load().ns_params_default(ctypes.byref(p))


def ns_create(params, n_instances: int, hip_stream: int | None, out: ctypes.c_void_p) -> int:
    return load().ns_create(params, n_instances, hip_stream, ctypes.byref(out))


def ns_set_state(handle, inst: int, field: int, src_ptr: int, on_device: int) -> int:
    return load().ns_set_state(handle, inst, field, src_ptr, on_device)


def ns_step(handle, nsteps: int, stats) -> int:
    return load().ns_step(handle, nsteps, stats)


def ns_get_state(handle, inst: int, field: int, dst_ptr: int, on_device: int) -> int:
    return load().ns_get_state(handle, inst, field, dst_ptr, on_device)


def ns_backward(handle, inst: int, g_final_ptrs, g_init_ptrs, on_device: int) -> int:
    a = (ctypes.c_void_p * 3)(*g_final_ptrs)
    b = (ctypes.c_void_p * 3)(*g_init_ptrs)
    return load().ns_backward(handle, inst, a, b, on_device)


def ns_get_timing(handle, out: ns_timing) -> int:
    return load().ns_get_timing(handle, ctypes.byref(out))


def ns_destroy(handle) -> None:
    load().ns_destroy(handle)


def ns_step_noalloc(params: ns_params, u_ptr: int, v_ptr: int, w_ptr: int, p_ptr: int, nsteps: int,
                    hip_stream: int | None, stats) -> int:
    return load().ns_step_noalloc(ctypes.byref(params), u_ptr, v_ptr, w_ptr, p_ptr, nsteps, hip_stream,
                                  None if stats is None else ctypes.byref(stats))


def ns_guard_check(self_test: int = 0) -> int:
    """Guard-band count (include/ns.h)."""
    return int(load().ns_guard_check(int(self_test)))


def ns_last_error(handle=None) -> str:
    r = load().ns_last_error(handle)
    return r.decode() if r else ""
