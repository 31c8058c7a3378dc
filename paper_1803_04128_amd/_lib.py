"""ctypes declarations of libbf.so (include/bf.h).  Loading fails loudly when
the library has not been built: there is no fallback path."""

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbf.so")

BF_OK, BF_EINVAL, BF_ENOMEM, BF_EHIP, BF_EUNSUPPORTED, BF_EBUSY = (
    0, -1, -2, -3, -4, -5)
PHASES = {"dft": 0, "fio1d": 1, "radon2d": 2, "separable": 3,
          "fio1d_warp": 4, "lowrank": 5}
PRECISIONS = {"fp32": 0, "bf16x3": 1, "fp16x3": 2}
OPS = {"N": 0, "T": 1, "C": 2, "H": 3}


class BfGrid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int)]


class BfPhase(C.Structure):
    _fields_ = [("kind", C.c_int), ("nparams", C.c_int),
                ("params", C.POINTER(C.c_double)), ("rank", C.c_int),
                ("U", C.POINTER(C.c_double)), ("V", C.POINTER(C.c_double))]


class BfAmplitude(C.Structure):
    _fields_ = [("r", C.c_int), ("a", C.POINTER(C.c_double)),
                ("b", C.POINTER(C.c_double))]


class BfPlanInfo(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int), ("L", C.c_int),
                ("h", C.c_int), ("q", C.c_int), ("r", C.c_int),
                ("precision", C.c_int), ("N", C.c_longlong),
                ("first_xi_level", C.c_int), ("last_x_level", C.c_int),
                ("n_steps", C.c_int), ("n_passes", C.c_int),
                ("max_rank", C.c_int), ("chunk_nvec", C.c_int),
                ("factor_bytes", C.c_size_t),
                ("workspace_bytes", C.c_size_t),
                ("flops_per_column", C.c_double),
                ("factor_stream_bytes", C.c_double), ("op", C.c_int),
                ("method", C.c_int)]


class BfStepInfo(C.Structure):
    _fields_ = [("kind", C.c_int), ("level", C.c_int), ("r_in", C.c_int),
                ("r_out", C.c_int), ("reads_f", C.c_int),
                ("writes_lambda", C.c_int), ("side_in", C.c_int),
                ("side_out", C.c_int), ("units", C.c_longlong),
                ("tw_entries", C.c_longlong), ("S_entries", C.c_longlong)]


class BfKernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int),
                ("total_ms", C.c_double), ("bytes", C.c_double),
                ("flops", C.c_double), ("state_bytes", C.c_double)]


# BF_STATIC_SCRATCH_BYTES of include/bf.h
STATIC_SCRATCH_BYTES = 256 << 20

PATHS = {"fused": 0, "fused_valu": 1, "per_step": 2, "per_step_mfma": 3}


class BfConfig(C.Structure):
    _fields_ = [("path", C.c_int), ("tile_cols", C.c_int),
                ("tile_cols_used", C.c_int), ("switch_otf", C.c_int),
                ("max_pass_levels", C.c_int), ("twiddle_otf", C.c_int)]


class BfTuneEntry(C.Structure):
    _fields_ = [("config", BfConfig), ("ms", C.c_double)]


SAMPLER = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_int,
                      C.POINTER(C.c_longlong), C.POINTER(C.c_double))

EXPORTS = ["bf_plan", "bf_plan_op", "bf_plan_footprint", "bf_step_query",
           "bf_factor_entries", "bf_apply_static", "bf_lift_decide",
           "bf_plan_lifted", "bf_apply_chain",
           "bf_graph_create_chain", "bf_unwrap",
           "bf_recover_phase", "bf_lowrank_samples", "bf_apply", "bf_workspace_bytes", "bf_apply_ws",
           "bf_destroy", "bf_query", "bf_last_error", "bf_points",
           "bf_lagrange", "bf_profile", "bf_profile_read", "bf_get_config",
           "bf_set_config", "bf_autotune", "bf_graph_create",
           "bf_graph_launch", "bf_graph_destroy"]

_lib = None


class BfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def load():
    """Load libbf.so once; raise ImportError if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python -m paper_1803_04128_amd.build` (hipcc, gfx950)")
    # PyTorch ships its own HIP runtime (same soname as the system one).
    # Import it first so libbf.so binds to that runtime: two HIP runtimes in
    # one process do not share devices.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    lib.bf_plan.argtypes = [P(BfGrid), P(BfPhase), P(BfAmplitude), C.c_int,
                            C.c_int, C.c_int, P(C.c_void_p)]
    lib.bf_plan_op.argtypes = [P(BfGrid), P(BfPhase), P(BfAmplitude),
                               C.c_int, C.c_int, C.c_int, C.c_int,
                               P(C.c_void_p)]
    lib.bf_plan_footprint.argtypes = [P(BfGrid), P(BfPhase),
                                      P(BfAmplitude), C.c_int, C.c_int,
                                      C.c_int, C.c_int, P(C.c_size_t)]
    D, L = P(C.c_double), P(C.c_longlong)
    lib.bf_lift_decide.argtypes = [C.c_longlong, C.c_int, D, D, C.c_int, D,
                                   D, C.c_int, C.c_int, C.c_double, D,
                                   C.c_int, L, C.c_int, C.c_int, L, L,
                                   C.c_int, L, L, C.c_int, P(C.c_int),
                                   P(C.c_int), D, D, D, D, P(C.c_int)]
    lib.bf_plan_lifted.argtypes = [C.c_longlong, C.c_int, D, D, C.c_int, D,
                                   D, C.c_int, P(C.c_void_p)]
    lib.bf_step_query.argtypes = [C.c_void_p, C.c_int, P(BfStepInfo)]
    lib.bf_factor_entries.argtypes = [C.c_void_p, C.c_int, C.c_int,
                                      P(C.c_longlong), C.c_int,
                                      P(C.c_longlong), P(C.c_longlong),
                                      P(C.c_float)]
    lib.bf_unwrap.argtypes = [P(C.c_double), C.c_longlong, C.c_double,
                              P(C.c_double), P(C.c_longlong), C.c_int,
                              P(C.c_int)]
    lib.bf_recover_phase.argtypes = [C.c_longlong, P(C.c_longlong), C.c_int,
                                     P(C.c_longlong), C.c_int, C.c_int,
                                     C.c_double, SAMPLER, C.c_void_p,
                                     C.c_int, P(C.c_double), P(C.c_double),
                                     P(C.c_int)]
    lib.bf_lowrank_samples.argtypes = [C.c_longlong, P(C.c_double),
                                       P(C.c_longlong), C.c_int,
                                       P(C.c_double), P(C.c_longlong),
                                       C.c_int, C.c_int, C.c_int,
                                       P(C.c_double), P(C.c_double),
                                       P(C.c_int)]
    lib.bf_graph_create_chain.argtypes = [P(C.c_void_p), C.c_int, C.c_int,
                                          C.c_void_p, C.c_void_p, C.c_void_p,
                                          P(C.c_void_p)]
    lib.bf_apply_chain.argtypes = [P(C.c_void_p), C.c_int, C.c_int,
                                   C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p]
    lib.bf_apply.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                             C.c_void_p]
    lib.bf_apply_static.argtypes = [C.c_void_p, C.c_int, C.c_void_p,
                                    C.c_void_p, C.c_void_p]
    lib.bf_workspace_bytes.argtypes = [C.c_void_p, C.c_int, P(C.c_size_t)]
    lib.bf_apply_ws.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_size_t, C.c_void_p]
    lib.bf_destroy.argtypes = [C.c_void_p]
    lib.bf_query.argtypes = [C.c_void_p, P(BfPlanInfo)]
    lib.bf_last_error.restype = C.c_char_p
    lib.bf_last_error.argtypes = []
    lib.bf_points.argtypes = [C.c_int, C.c_int, P(C.c_int), C.c_int,
                              P(C.c_int)]
    lib.bf_lagrange.argtypes = [P(C.c_int), C.c_int, P(C.c_double), C.c_int,
                                P(C.c_double)]
    lib.bf_profile.argtypes = [C.c_void_p, C.c_int]
    lib.bf_profile_read.argtypes = [C.c_void_p, P(BfKernelStat), C.c_int,
                                    P(C.c_int)]
    lib.bf_get_config.argtypes = [C.c_void_p, P(BfConfig)]
    lib.bf_set_config.argtypes = [C.c_void_p, P(BfConfig)]
    lib.bf_autotune.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                C.c_int, C.c_void_p, P(BfTuneEntry), C.c_int,
                                P(C.c_int)]
    lib.bf_graph_create.argtypes = [C.c_void_p, C.c_int, C.c_void_p,
                                    C.c_void_p, P(C.c_void_p)]
    lib.bf_graph_launch.argtypes = [C.c_void_p, C.c_void_p]
    lib.bf_graph_destroy.argtypes = [C.c_void_p]
    for name in EXPORTS:
        getattr(lib, name).restype = (C.c_char_p if name == "bf_last_error"
                                      else C.c_int)
    _lib = lib
    return lib


def check(rc):
    if rc != BF_OK:
        raise BfError(rc, load().bf_last_error().decode())
    return rc
