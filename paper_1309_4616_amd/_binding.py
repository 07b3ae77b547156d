"""ctypes binding of libexpi.so (argument marshalling only).

Every computation runs in the HIP library; this module converts Python and
PyTorch arguments to the C ABI declared in include/expi.h and turns error
codes into exceptions.  PyTorch provides device memory and the stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libexpi.so")

EXPI_OK = 0
ERRORS = {-1: "EINVAL", -2: "EALIAS", -3: "EWORKSPACE", -4: "ENOTCONV",
          -5: "ENONFINITE", -6: "EHIP", -7: "EUNSUPPORTED"}
F64, F32 = 0, 1
BCS = {"dirichlet0": 0, "neumann0": 1, "interior_only": 2}
COEF_CONST, COEF_SEPARABLE, COEF_FIELD, COEF_DLAP = 0, 1, 2, 3
BDATA = {None: 0, "none": 0, "z1mz_xy": 1, "sinpiz_expmxy": 2}
BDATA_MODES = {"in_kernel": 0, "separate": 1}
G_CUBIC, G_COMBUSTION, G_COMBUSTION_FAST = 0, 1, 2
NONLIN = {"cubic": G_CUBIC, "combustion": G_COMBUSTION, "combustion_fast": G_COMBUSTION_FAST}

# every symbol include/expi.h declares
EXPORTS = ("expi_op_create_stencil", "expi_op_create_csr", "expi_op_destroy", "expi_op_size",
           "expi_op_set_tiles", "expi_op_get_tiles", "expi_op_set_pairs", "expi_op_get_pairs", "expi_op_autotune", "expi_workspace_bytes", "expi_op_interval", "apply_op", "phi_action",
           "expeuler_step", "expi_leja_points", "expi_divided_differences", "expi_last_error",
           "expi_batch_create", "expi_batch_destroy", "expi_batch_set_tiles",
           "expi_batch_total_length", "expi_batch_offsets", "expi_batch_workspace_bytes",
           "expi_batch_prepare", "expi_batch_launch", "expi_batch_capture", "expi_batch_replay",
           "expi_batch_results", "expi_batch_max_rounds", "expi_batch_graph_rounds",
           "expi_batch_launch_persistent", "expi_batch_capture_persistent",
           "expi_batch_autotune", "expi_batch_get_tiles", "expi_batch_set_pairs", "expi_batch_get_pairs", "expi_mlp_param_count", "expi_mlp_scratch_floats",
           "expi_mlp_forward", "expi_mlp_backward", "expi_mlp_adam",
           "expi_noalloc_init", "phi_action_noalloc", "exprk2_step",
           "expi_exprk2_workspace_bytes", "expi_nonlinearity", "expi_op_set_boundary_data",
           "expi_op_create_csr_complex", "expi_skew_phi_action", "expi_divided_differences_skew")

# size of the library's scratch array behind phi_action_noalloc
NOALLOC_SCRATCH_BYTES = 64 << 20


class ExpiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class Stats(ctypes.Structure):
    _fields_ = [("substeps", ctypes.c_int32), ("newton_steps", ctypes.c_int32),
                ("matvecs", ctypes.c_int32), ("retries", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("degree_max", ctypes.c_int32),
                ("degree_last", ctypes.c_int32), ("timed_products", ctypes.c_int32),
                ("err_est", ctypes.c_double), ("interval_a", ctypes.c_double),
                ("interval_b", ctypes.c_double), ("newton_ms", ctypes.c_double),
                ("rnorm", ctypes.c_double), ("t_first", ctypes.c_double * 5),
                ("pred_degree", ctypes.c_int32), ("pred_substeps", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("finalized", ctypes.c_int32),
                ("timed_pairs", ctypes.c_int32), ("pair_ms", ctypes.c_double),
                ("pair_launches", ctypes.c_int32), ("single_launches", ctypes.c_int32),
                ("fused_starts", ctypes.c_int32), ("reserved3", ctypes.c_int32)]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["t_first"] = list(self.t_first)
        return d


class BatchStat(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("substeps", ctypes.c_int32),
                ("newton_steps", ctypes.c_int32), ("degree_max", ctypes.c_int32),
                ("degree_last", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("err_est", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class Params(ctypes.Structure):
    _fields_ = [("l_max", ctypes.c_double), ("m_max", ctypes.c_int32),
                ("max_retries", ctypes.c_int32), ("have_interval", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("interval_a", ctypes.c_double),
                ("interval_b", ctypes.c_double), ("selector", ctypes.c_void_p),
                ("selector_hidden", ctypes.c_int32), ("no_pairs", ctypes.c_int32),
                ("fuse_start", ctypes.c_int32), ("selector_l_max", ctypes.c_double),
                ("selector_features", ctypes.c_void_p)]


@dataclass
class LejaParams:
    l_max: float = 100.0
    m_max: int = 100
    max_retries: int = 4
    interval: tuple | None = None
    profile: int = 0                 # 0 off, 1 / True every launch, 2 one launch per loop
    selector: object = None          # device float tensor (see selector.pack)
    selector_hidden: int = 64
    pairs: bool = True               # fuse consecutive Newton products where supported
    fuse_start: int = 0              # Euler steps: 0 by degree parity, 1 never, 2 always
    selector_l_max: float = 0.0      # largest delta (b - a) the selector may choose (0: 500)
    selector_features: object = None  # device float32 tensor of 8: features of the last prediction

    def to_c(self) -> Params:
        p = Params()
        p.l_max = float(self.l_max)
        p.m_max = int(self.m_max)
        p.max_retries = int(self.max_retries)
        p.profile = int(self.profile)
        p.no_pairs = 0 if self.pairs else 1
        p.fuse_start = int(self.fuse_start)
        p.selector_l_max = float(self.selector_l_max)
        if self.selector_features is not None:
            p.selector_features = ctypes.c_void_p(self.selector_features.data_ptr())
        if self.selector is not None:
            p.selector = ctypes.c_void_p(self.selector.data_ptr())
            p.selector_hidden = int(self.selector_hidden)
        if self.interval is not None:
            p.have_interval = 1
            p.interval_a, p.interval_b = (float(v) for v in self.interval)
        return p


_lib = None


def lib() -> ctypes.CDLL:
    """Load libexpi.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_1309_4616_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    c_int, c_double, c_void_p, c_size_t = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
    i64p = ctypes.POINTER(ctypes.c_int64)
    dblp = ctypes.POINTER(ctypes.c_double)
    L.expi_op_create_stencil.argtypes = [ctypes.POINTER(c_void_p), c_int, i64p, dblp, c_int, c_int,
                                         c_double, c_double, c_void_p, c_void_p, c_void_p, c_void_p]
    L.expi_op_create_stencil.restype = c_int
    L.expi_op_create_csr.argtypes = [ctypes.POINTER(c_void_p), ctypes.c_int64, ctypes.c_int64,
                                     c_void_p, c_void_p, c_void_p]
    L.expi_op_create_csr.restype = c_int
    L.expi_op_destroy.argtypes = [c_void_p]
    L.expi_op_destroy.restype = c_int
    L.expi_op_size.argtypes = [c_void_p]
    L.expi_op_size.restype = ctypes.c_int64
    L.expi_op_set_tiles.argtypes = [c_void_p, c_int, c_int, c_int]
    L.expi_op_set_tiles.restype = c_int
    ip = ctypes.POINTER(c_int)
    L.expi_op_get_tiles.argtypes = [c_void_p, ip, ip, ip]
    L.expi_op_get_tiles.restype = c_int
    L.expi_op_set_pairs.argtypes = [c_void_p, c_int]
    L.expi_op_set_pairs.restype = c_int
    L.expi_op_get_pairs.argtypes = [c_void_p, ip]
    L.expi_op_get_pairs.restype = c_int
    L.expi_op_autotune.argtypes = [c_void_p, c_int, c_int, c_void_p, c_size_t, c_void_p,
                                   ip, ctypes.POINTER(ctypes.c_float), c_int, ip]
    L.expi_op_autotune.restype = c_int
    L.expi_workspace_bytes.argtypes = [c_void_p, c_int]
    L.expi_workspace_bytes.restype = c_size_t
    L.expi_op_interval.argtypes = [c_void_p, dblp, dblp, c_void_p, c_size_t, c_void_p]
    L.expi_op_interval.restype = c_int
    L.apply_op.argtypes = [c_void_p, c_double, c_double, c_void_p, c_void_p, c_int, c_void_p]
    L.apply_op.restype = c_int
    L.phi_action.argtypes = [c_void_p, c_int, c_double, c_void_p, c_void_p, c_double, c_int,
                             ctypes.POINTER(Params), c_void_p, c_size_t, ctypes.POINTER(Stats),
                             c_void_p]
    L.phi_action.restype = c_int
    L.expeuler_step.argtypes = [c_void_p, c_int, c_double, c_void_p, c_double, c_int,
                                ctypes.POINTER(Params), c_void_p, c_size_t, ctypes.POINTER(Stats),
                                c_void_p]
    L.expeuler_step.restype = c_int
    L.exprk2_step.argtypes = L.expeuler_step.argtypes
    L.exprk2_step.restype = c_int
    L.expi_exprk2_workspace_bytes.argtypes = [c_void_p, c_int]
    L.expi_exprk2_workspace_bytes.restype = c_size_t
    L.expi_nonlinearity.argtypes = [c_int, ctypes.c_int64, c_void_p, c_void_p, c_int, c_void_p]
    L.expi_nonlinearity.restype = c_int
    L.expi_op_create_csr_complex.argtypes = L.expi_op_create_csr.argtypes
    L.expi_op_create_csr_complex.restype = c_int
    L.expi_skew_phi_action.argtypes = [c_void_p, c_int, c_double, c_void_p, c_void_p, c_double,
                                       ctypes.POINTER(Params), c_void_p, c_size_t,
                                       ctypes.POINTER(Stats), c_void_p]
    L.expi_skew_phi_action.restype = c_int
    L.expi_divided_differences_skew.argtypes = [c_int, c_double, c_double, c_double, c_int, dblp, dblp]
    L.expi_divided_differences_skew.restype = c_int
    L.expi_op_set_boundary_data.argtypes = [c_void_p, c_int, c_int]
    L.expi_op_set_boundary_data.restype = c_int
    L.expi_noalloc_init.argtypes = []
    L.expi_noalloc_init.restype = c_int
    L.phi_action_noalloc.argtypes = [c_void_p, c_int, c_double, c_void_p, c_void_p, c_double, c_int,
                                     ctypes.POINTER(Params), ctypes.POINTER(Stats), c_void_p]
    L.phi_action_noalloc.restype = c_int
    i32p = ctypes.POINTER(ctypes.c_int32)
    L.expi_batch_create.argtypes = [ctypes.POINTER(c_void_p), c_int, i32p, i32p, dblp, dblp, dblp,
                                    c_int, c_double, c_double, c_int, ctypes.POINTER(Params)]
    L.expi_batch_create.restype = c_int
    L.expi_batch_destroy.argtypes = [c_void_p]
    L.expi_batch_destroy.restype = c_int
    L.expi_batch_set_tiles.argtypes = [c_void_p, c_int, c_int]
    L.expi_batch_set_tiles.restype = c_int
    L.expi_batch_total_length.argtypes = [c_void_p]
    L.expi_batch_total_length.restype = ctypes.c_int64
    L.expi_batch_offsets.argtypes = [c_void_p, i64p]
    L.expi_batch_offsets.restype = c_int
    L.expi_batch_workspace_bytes.argtypes = [c_void_p]
    L.expi_batch_workspace_bytes.restype = c_size_t
    L.expi_batch_prepare.argtypes = [c_void_p, c_void_p, c_size_t, c_void_p]
    L.expi_batch_prepare.restype = c_int
    for name in ("expi_batch_launch", "expi_batch_launch_persistent",
                 "expi_batch_capture_persistent"):
        getattr(L, name).argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
        getattr(L, name).restype = c_int
    L.expi_batch_capture.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_int, c_void_p]
    L.expi_batch_capture.restype = c_int
    L.expi_batch_autotune.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_int, c_void_p,
                                      ctypes.POINTER(c_int), ctypes.POINTER(ctypes.c_float), c_int,
                                      ctypes.POINTER(c_int)]
    L.expi_batch_autotune.restype = c_int
    L.expi_batch_get_tiles.argtypes = [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]
    L.expi_batch_get_tiles.restype = c_int
    L.expi_batch_set_pairs.argtypes = [c_void_p, c_int]
    L.expi_batch_set_pairs.restype = c_int
    L.expi_batch_get_pairs.argtypes = [c_void_p, ctypes.POINTER(c_int)]
    L.expi_batch_get_pairs.restype = c_int
    for name in ("expi_batch_max_rounds", "expi_batch_graph_rounds"):
        getattr(L, name).argtypes = [c_void_p]
        getattr(L, name).restype = c_int
    L.expi_batch_replay.argtypes = [c_void_p, c_void_p]
    L.expi_batch_replay.restype = c_int
    L.expi_batch_results.argtypes = [c_void_p, c_void_p, c_void_p, ctypes.POINTER(BatchStat),
                                     ctypes.POINTER(c_int)]
    L.expi_batch_results.restype = c_int
    L.expi_mlp_param_count.argtypes = [c_int]
    L.expi_mlp_param_count.restype = c_size_t
    L.expi_mlp_scratch_floats.argtypes = [c_int, c_int]
    L.expi_mlp_scratch_floats.restype = c_size_t
    L.expi_mlp_forward.argtypes = [c_int, c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p]
    L.expi_mlp_forward.restype = c_int
    L.expi_mlp_backward.argtypes = [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                    ctypes.c_float, c_void_p, c_void_p, c_void_p, c_void_p]
    L.expi_mlp_backward.restype = c_int
    L.expi_mlp_adam.argtypes = [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_int, ctypes.c_float,
                                ctypes.c_float, ctypes.c_float, ctypes.c_float, c_void_p]
    L.expi_mlp_adam.restype = c_int
    L.expi_leja_points.argtypes = [dblp, c_int]
    L.expi_leja_points.restype = c_int
    L.expi_divided_differences.argtypes = [c_int, c_double, c_double, c_double, c_int, dblp]
    L.expi_divided_differences.restype = c_int
    L.expi_last_error.argtypes = []
    L.expi_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != EXPI_OK:
        raise ExpiError(rc, lib().expi_last_error().decode())


def leja_points(count: int):
    import numpy as np
    out = np.empty(count, dtype=np.float64)
    check(lib().expi_leja_points(out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(count)))
    return out


def divided_differences(k: int, delta: float, c: float, gamma: float, count: int):
    import numpy as np
    out = np.empty(count, dtype=np.float64)
    check(lib().expi_divided_differences(int(k), float(delta), float(c), float(gamma), int(count),
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def divided_differences_skew(k: int, delta: float, c: float, gamma: float, count: int):
    """Complex divided differences of x -> phi_k(-i delta (c + gamma x))."""
    import numpy as np
    re = np.empty(count, dtype=np.float64)
    im = np.empty(count, dtype=np.float64)
    P = ctypes.POINTER(ctypes.c_double)
    check(lib().expi_divided_differences_skew(int(k), float(delta), float(c), float(gamma), int(count),
                                              re.ctypes.data_as(P), im.ctypes.data_as(P)))
    return re + 1j * im
