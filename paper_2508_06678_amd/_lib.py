"""ctypes binding of libqg.so (include/qg.h).  Argument marshalling only.

The library must have been built (``paper_2508_06678_amd.build``); loading
fails loudly otherwise -- there is no fallback implementation.
"""
import ctypes
import math
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqg.so")

QG_OK, QG_EINVAL, QG_EUNSUPPORTED, QG_EWORKSPACE, QG_EHIP, QG_ESTATE = range(6)
CLOSURES = {"none": 0, "smag": 1, "leith": 2, "dsmag": 3, "dleith": 4}
SCHEMES = {"rk4": 0, "ab2cn": 1}

EXPORTS = ["qg_workspace_bytes", "qg_init", "qg_step", "qg_adjoint_step", "qg_diag",
           "qg_filter_les", "qg_ideal_sgs", "qg_closure_term", "qg_pcc", "qg_set_coef", "qg_autotune", "qg_tuning", "qg_profile_steps", "qg_stamp_steps", "qg_step_noalloc", "qg_info",
           "qg_destroy", "qg_last_error"]


class QGParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("beta", ctypes.c_double), ("re", ctypes.c_double), ("mu", ctypes.c_double),
                ("u_in", ctypes.c_double), ("v_in", ctypes.c_double), ("eta", ctypes.c_double),
                ("sponge_sigma", ctypes.c_double), ("dt", ctypes.c_double), ("c", ctypes.c_double),
                ("closure", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("test_ratio", ctypes.c_double), ("clip_mode", ctypes.c_int32),
                ("fp64_lowk", ctypes.c_int32), ("scheme", ctypes.c_int32)]


class QGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qg error {code}: {msg}")
        self.code = code


_libs = {}
POISON_LIB_PATH = os.path.join(_PKG, "libqg_ldspoison.so")
STAMPS_LIB_PATH = os.path.join(_PKG, "libqg_stamps.so")


def lib(path=None):
    """Load libqg.so (or the library at `path`, e.g. the LDS-poison debug
    build) once; raise if it has not been built."""
    path = LIB_PATH if path is None else path
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2508_06678_amd.build.build()")
    L = ctypes.CDLL(path)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    P = ctypes.POINTER(QGParams)
    L.qg_workspace_bytes.argtypes = [P, i32, i32, ctypes.POINTER(sz)]
    L.qg_init.argtypes = [P, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, sz, i32, vp,
                          ctypes.POINTER(vp)]
    L.qg_step.argtypes = [vp, vp, i64, i32, vp, i32, vp]
    L.qg_adjoint_step.argtypes = [vp, vp, vp, i64, vp, vp]
    L.qg_diag.argtypes = [vp, vp, vp, vp, vp]
    L.qg_filter_les.argtypes = [vp, vp, vp, vp, vp]
    L.qg_ideal_sgs.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.qg_closure_term.argtypes = [vp, vp, vp, vp]
    L.qg_pcc.argtypes = [vp, vp, vp, vp, vp]
    L.qg_autotune.argtypes = [vp, ctypes.c_char_p, vp]
    L.qg_tuning.argtypes = [vp, ctypes.POINTER(i32)]
    L.qg_step_noalloc.argtypes = [P, vp, vp, vp, i64, vp]
    L.qg_profile_steps.argtypes = [vp, vp, i64, i32, ctypes.POINTER(ctypes.c_float), i32,
                                   ctypes.POINTER(i32), vp]
    L.qg_stamp_steps.argtypes = [vp, vp, i64, vp, sz, vp]
    L.qg_set_coef.argtypes = [vp, ctypes.POINTER(ctypes.c_double), vp]
    L.qg_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i32),
                          ctypes.POINTER(i32)]
    L.qg_destroy.argtypes = [vp]
    L.qg_destroy.restype = None
    L.qg_last_error.argtypes = []
    L.qg_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("qg_destroy", "qg_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _libs[path] = L
    return L


def check(rc, L=None):
    """Raise QGError with the library's message (L: the library that
    returned rc; the default one if None)."""
    if rc != QG_OK:
        raise QGError(rc, (L or lib()).qg_last_error().decode())


def make_params(d):
    """qg_params from a dict with the struct's field names (closure may be a name)."""
    p = QGParams()
    p.nx, p.ny = int(d["nx"]), int(d["ny"])
    for k in ("lx", "ly", "beta", "mu", "u_in", "v_in", "sponge_sigma", "dt", "c"):
        setattr(p, k, float(d.get(k, 0.0)))
    p.re = float(d.get("re", math.inf))
    p.eta = float(d.get("eta", math.inf))
    cl = d.get("closure", 0)
    p.closure = CLOSURES[cl] if isinstance(cl, str) else int(cl)
    p.precision = int(d.get("precision", 64))
    p.test_ratio = float(d.get("test_ratio", 2))
    p.clip_mode = int(d.get("clip_mode", 0))
    p.fp64_lowk = int(d.get("fp64_lowk", 8))
    sc = d.get("scheme", 0)
    p.scheme = SCHEMES[sc] if isinstance(sc, str) else int(sc)
    return p
