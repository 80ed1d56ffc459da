"""ctypes declarations of the libl1alm C ABI (include/l1_alm.h).

Loading fails loudly when the shared library has not been built: there is no
fallback implementation of any step.

Teardown: every live plan is registered here and destroyed by an ``atexit``
hook, so the library releases its device memory while the HIP runtime and
any profiler attached to it are still fully alive; a plan's ``__del__`` does
nothing once the interpreter is finalizing.
"""
import atexit
import ctypes
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libl1alm.so")

L1_OK, L1_EINVAL, L1_ENOTSPD, L1_ENOMEM, L1_EHIP, L1_ENODEVICE, L1_ENOTAPE = 0, -1, -2, -3, -4, -5, -6
ERROR_NAMES = {L1_EINVAL: "L1_EINVAL", L1_ENOTSPD: "L1_ENOTSPD", L1_ENOMEM: "L1_ENOMEM",
               L1_EHIP: "L1_EHIP", L1_ENODEVICE: "L1_ENODEVICE", L1_ENOTAPE: "L1_ENOTAPE"}
EXPORTED = ("l1_alm_plan", "l1_alm_solve", "l1_alm_backward", "l1_alm_kkt", "l1_alm_classify",
            "l1_alm_class_residuals", "l1_alm_align", "l1_alm_set_ksplit", "l1_alm_tune_ksplit", "l1_alm_last_stats", "l1_alm_kkt_noalloc",
            "l1_alm_destroy", "l1_alm_last_error")


class l1_alm_desc(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int), ("n_dict", ctypes.c_int), ("lda", ctypes.c_int),
        ("problem", ctypes.c_int), ("structure", ctypes.c_int), ("method", ctypes.c_int),
        ("precision", ctypes.c_int), ("max_batch", ctypes.c_int),
        ("lam", ctypes.c_double), ("beta", ctypes.c_double), ("xi", ctypes.c_double),
        ("xi_growth", ctypes.c_double), ("max_inner", ctypes.c_int),
        ("tol_inner", ctypes.c_double), ("refine_switch", ctypes.c_double),
        ("record_tape", ctypes.c_int), ("checkpoint_every", ctypes.c_int),
        ("time_kernels", ctypes.c_int), ("div_factor", ctypes.c_double),
        ("iteration_form", ctypes.c_int),
    ]


class L1Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path=LIB_PATH):
    """Load libl1alm.so and declare its signatures (no GPU work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1007_3753_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i, f, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_double
    lib.l1_alm_plan.argtypes = [ctypes.POINTER(l1_alm_desc), vp, vp, ctypes.POINTER(vp)]
    lib.l1_alm_solve.argtypes = [vp, vp, i, i, vp, vp, f, i, vp, vp, vp, i, vp, i, vp, i, vp, vp, vp]
    lib.l1_alm_backward.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.l1_alm_kkt.argtypes = [vp, vp, i, i, vp, vp, i, vp, i, vp, i, vp, vp]
    lib.l1_alm_kkt_noalloc.argtypes = [vp, i, i, i, i, i, d, vp, i, i, vp, vp, i, vp, i, vp, i, vp, vp]
    lib.l1_alm_classify.argtypes = [vp, i, i, i, vp, i, vp, vp, vp, vp]
    lib.l1_alm_class_residuals.argtypes = [vp, i, i, i, vp, i, vp, i, vp, i, i, vp, i, vp, vp, vp]
    lib.l1_alm_set_ksplit.argtypes = [vp, vp, i]
    lib.l1_alm_tune_ksplit.argtypes = [vp, i, vp, i, vp]
    lib.l1_alm_align.argtypes = [vp, i, i, i, vp, i, f, i, vp, vp, i, vp, vp, vp]
    lib.l1_alm_last_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i]
    lib.l1_alm_destroy.argtypes = [vp]
    lib.l1_alm_last_error.argtypes = []
    lib.l1_alm_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name != "l1_alm_last_error":
            getattr(lib, name).restype = i
    _lib = lib
    return lib


def check(rc):
    if rc != L1_OK:
        msg = _lib.l1_alm_last_error().decode(errors="replace")
        raise L1Error(rc, msg)


# ---- deterministic teardown -------------------------------------------------
_live = weakref.WeakSet()


def register(obj):
    """Track an object with a ``close()`` that releases library resources."""
    _live.add(obj)


def close_all():
    """Close every live plan (also run at interpreter exit)."""
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass
    if _lib is not None:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                torch.cuda.synchronize()
        except Exception:
            pass


atexit.register(close_all)
