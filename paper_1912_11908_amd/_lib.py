"""ctypes binding of libibm.so (the C ABI in include/ibm.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibm.so")

IBM_OK = 0
ERRORS = {-1: "IBM_EINVAL", -2: "IBM_EGEOM", -3: "IBM_EDEVICE", -4: "IBM_ENONFINITE",
          -5: "IBM_ENOSPACE", -6: "IBM_ECAPACITY"}
BC = {"farfield": 0, "extrap": 1, "periodic": 2}
FLUID, FORCING, G1, G2, G3, SOLID = range(6)
REC_INT, REC_DBL = 24, 32
EXPORTS = ["ibm_workspace_bytes", "ibm_create", "ibm_destroy", "ibm_set_time", "ibm_classify",
           "ibm_fill", "ibm_residual", "ibm_forces", "ibm_body_state", "ibm_advance", "ibm_init_state", "ibm_state_to_prim",
           "ibm_status", "ibm_read_counts", "ibm_info_get", "ibm_last_error",
           "ibm_time_update_kernel", "ibm_set_option", "ibm_batch_advance", "ibm_stage_timing",
           "ibm_forces_static"]

BATCH_MAX = 64
FORCES_STATIC_MAX_FACETS = 262144


class IbmCase(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("ni", ctypes.c_int), ("nj", ctypes.c_int), ("nk", ctypes.c_int),
        ("xf", ctypes.c_void_p), ("yf", ctypes.c_void_p), ("zf", ctypes.c_void_p),
        ("bc", ctypes.c_int * 6),
        ("nvert", ctypes.c_int), ("nfacet", ctypes.c_int),
        ("vert", ctypes.c_void_p), ("facet", ctypes.c_void_p),
        ("motion", ctypes.c_int), ("motion_par", ctypes.c_double * 4),
        ("mach", ctypes.c_double), ("reynolds", ctypes.c_double),
        ("prandtl", ctypes.c_double), ("gamma", ctypes.c_double),
        ("scheme", ctypes.c_int), ("ib_family", ctypes.c_int), ("precision", ctypes.c_int),
        ("dt", ctypes.c_double), ("cfl_tau", ctypes.c_double), ("n_inner", ctypes.c_int),
        ("u_inf", ctypes.c_double * 3), ("motion_vel", ctypes.c_double), ("wall_pressure", ctypes.c_int),
        ("reconstruction", ctypes.c_int), ("ib_framework", ctypes.c_int),
    ]


class IbmInfo(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("ni", ctypes.c_int), ("nj", ctypes.c_int), ("nk", ctypes.c_int),
        ("nv", ctypes.c_int), ("state_elems", ctypes.c_longlong), ("ncell", ctypes.c_longlong),
        ("cap_nodes", ctypes.c_int), ("region", ctypes.c_int * 6),
        ("cls", ctypes.c_void_p), ("counts", ctypes.c_void_p),
        ("list_forcing", ctypes.c_void_p), ("list_ghost", ctypes.c_void_p),
        ("rec_int", ctypes.c_void_p), ("rec_dbl", ctypes.c_void_p), ("time", ctypes.c_double),
    ]


_lib = None


class IbmError(RuntimeError):
    def __init__(self, code, where, msg=""):
        super().__init__(f"{where}: {ERRORS.get(code, code)} {msg}".strip())
        self.code = code


def load():
    """Load libibm.so; raises if it is missing (build it with
    ``python -m paper_1912_11908_amd.build`` or ``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.ibm_workspace_bytes.argtypes = [ctypes.POINTER(IbmCase), ctypes.POINTER(ctypes.c_size_t)]
    L.ibm_create.argtypes = [ctypes.POINTER(IbmCase), P, ctypes.c_size_t, ctypes.POINTER(P)]
    L.ibm_destroy.argtypes = [P]
    L.ibm_destroy.restype = None
    L.ibm_set_time.argtypes = [P, D]
    L.ibm_classify.argtypes = [P, P]
    L.ibm_fill.argtypes = [P, P, D, P]
    L.ibm_residual.argtypes = [P, P, P, P]
    L.ibm_forces.argtypes = [P, P, P, P, P, P]
    L.ibm_forces_static.argtypes = [P, P, P, P, P, P]
    L.ibm_body_state.argtypes = [P, P]
    L.ibm_advance.argtypes = [P, P, I, P]
    L.ibm_init_state.argtypes = [P, P, P, P]
    L.ibm_state_to_prim.argtypes = [P, P, P, P]
    L.ibm_status.argtypes = [P, P]
    L.ibm_read_counts.argtypes = [P, P, P]
    L.ibm_info_get.argtypes = [P, ctypes.POINTER(IbmInfo)]
    L.ibm_last_error.argtypes = [P]
    L.ibm_last_error.restype = ctypes.c_char_p
    L.ibm_time_update_kernel.argtypes = [P, P, I, I, P, ctypes.POINTER(ctypes.c_float)]
    L.ibm_set_option.argtypes = [P, I, I]
    L.ibm_batch_advance.argtypes = [P, P, I, I, P]
    F = ctypes.POINTER(ctypes.c_float)
    L.ibm_stage_timing.argtypes = [P, F, ctypes.POINTER(I), F, F]
    for name in EXPORTS:
        if name not in ("ibm_destroy", "ibm_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(rc, where, ctx=None):
    if rc != IBM_OK:
        msg = ""
        if ctx:
            m = load().ibm_last_error(ctx)
            msg = m.decode() if m else ""
        raise IbmError(rc, where, msg)
