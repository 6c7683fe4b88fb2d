"""ctypes declarations mirroring include/cprand.h."""
import ctypes as C
import os

MAX_ORDER = 8
MAX_RANK = 64

OK = 0
W_PINV = 1
W_MAXIT = 2
W_FALLBACK = 4
EINVAL = -1
ENAN = -2
EHIP = -3
ENOMEM = -4
EUNSUPPORTED = -5

F64, F32, BF16, C64, C128 = 0, 1, 2, 3, 4

NOALLOC_SCRATCH_BYTES = 32 << 20

MIX_NONE, MIX_FFT, MIX_DCT = 0, 1, 2
PREC_NATIVE, PREC_BF16_REFINE, PREC_BF16 = 0, 1, 2
PROPOSAL_UNIFORM, PROPOSAL_TABLE, PROPOSAL_LEARNED, PROPOSAL_MARGINAL, PROPOSAL_MIXTURE = 0, 1, 2, 3, 4
PROPOSAL_LEVERAGE = 5


class cprand_tensor(C.Structure):
    _fields_ = [("order", C.c_int32), ("dtype", C.c_int32),
                ("dims", C.c_int64 * MAX_ORDER), ("strides", C.c_int64 * MAX_ORDER),
                ("data", C.c_void_p)]


class cprand_opts(C.Structure):
    _fields_ = [("R", C.c_int32), ("S", C.c_int32), ("P_hat", C.c_int32), ("max_iters", C.c_int32),
                ("seed", C.c_uint64), ("tol", C.c_double), ("fit_target", C.c_double),
                ("patience", C.c_int32), ("mix", C.c_int32), ("precision", C.c_int32),
                ("proposal", C.c_int32), ("layout", C.c_int32), ("use_graph", C.c_int32),
                ("alpha", C.c_double), ("proposal_cdf", C.POINTER(C.c_void_p)),
                ("mlp_params", C.c_void_p), ("refine_every", C.c_int32), ("fit_beta", C.c_double),
                ("fit_alpha", C.c_double)]


class cprand_report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("flags", C.c_int32), ("fit_est", C.c_double),
                ("setup_ms", C.c_double), ("loop_ms", C.c_double),
                ("fit_history", C.POINTER(C.c_double)),
                ("proposal_history", C.POINTER(C.c_int32)),
                ("norm_ms", C.c_double), ("mix_ms", C.c_double * MAX_ORDER),
                ("layout_ms", C.c_double * MAX_ORDER), ("fused", C.c_int32),
                ("refined_from", C.c_int32)]


LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcprand.so")

# (name, restype, argtypes) for every entry point of include/cprand.h
SIGNATURES = [
    ("cprand_version", C.c_char_p, []),
    ("cprand_strerror", C.c_char_p, [C.c_int]),
    ("cprand_last_error", C.c_char_p, []),
    ("cprand_workspace_size", C.c_size_t, [C.POINTER(cprand_tensor), C.c_int32, C.c_int32, C.c_int32]),
    ("cprand_sample", C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.c_int32, C.c_int32, C.c_uint64,
                                C.c_uint64, C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p, C.c_void_p]),
    ("cprand_mttkrp_sampled", C.c_int, [C.POINTER(cprand_tensor), C.c_int32, C.POINTER(C.c_void_p),
                                        C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("cprand_mttkrp_sampled_noalloc", C.c_int, [C.POINTER(cprand_tensor), C.c_int32, C.POINTER(C.c_void_p),
                                                C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                                C.c_void_p, C.c_void_p]),
    ("cprand_solve", C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                               C.c_void_p]),
    ("cprand_fit_est", C.c_int, [C.POINTER(cprand_tensor), C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p,
                                 C.c_int32, C.c_int32, C.c_uint64, C.c_void_p, C.c_void_p, C.c_size_t,
                                 C.c_void_p]),
    ("cprand_fit_weighted_workspace_size", C.c_size_t, [C.c_int32, C.c_int32]),
    ("cprand_energy_proposals", C.c_int, [C.POINTER(cprand_tensor), C.c_void_p, C.c_double, C.POINTER(C.c_void_p),
                                          C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("cprand_fit_set_weighted", C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.c_int32, C.c_uint64,
                                          C.POINTER(C.c_void_p), C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("cprand_fit_est_weighted", C.c_int, [C.POINTER(cprand_tensor), C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p,
                                          C.c_int32, C.c_int32, C.c_uint64, C.POINTER(C.c_void_p), C.c_double,
                                          C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("cprand_norm", C.c_int, [C.POINTER(cprand_tensor), C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("cprand_mix", C.c_int, [C.POINTER(cprand_tensor), C.c_uint64, C.POINTER(cprand_tensor), C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("cprand_mix_dct", C.c_int, [C.POINTER(cprand_tensor), C.c_uint64, C.POINTER(cprand_tensor), C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("cprand_mix_factor_dct", C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                        C.c_int32, C.c_void_p]),
    ("cprand_mix_factor", C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_int32, C.c_void_p]),
    ("cprand_mode_major_strides", C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.c_int32, C.c_int64,
                                            C.POINTER(C.c_int64)]),
    ("cprand_layout_copy", C.c_int, [C.POINTER(cprand_tensor), C.c_int32, C.POINTER(cprand_tensor),
                                     C.c_void_p]),
    ("cprand_full_workspace_size", C.c_size_t, [C.POINTER(cprand_tensor), C.c_int32]),
    ("cprand_mttkrp_full", C.c_int, [C.POINTER(cprand_tensor), C.c_int32, C.POINTER(C.c_void_p), C.c_int32,
                                     C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("cprand_fit_exact", C.c_int, [C.POINTER(cprand_tensor), C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p,
                                   C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("cprand_cpals", C.c_int, [C.POINTER(cprand_tensor), C.c_int32, C.c_int32, C.c_double, C.POINTER(C.c_void_p),
                               C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_void_p]),
    ("cprand_mlp_param_count", C.c_int32, []),
    ("cprand_proposal_workspace_size", C.c_size_t, [C.c_int32, C.POINTER(C.c_int64), C.c_int32]),
    ("cprand_proposal", C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.c_int32, C.c_int32, C.POINTER(C.c_void_p),
                                  C.c_int32, C.c_void_p, C.c_double, C.POINTER(C.c_void_p), C.c_void_p, C.c_size_t,
                                  C.c_void_p]),
    ("cprand_mlp_features", C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.c_int32, C.c_int32, C.POINTER(C.c_void_p),
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("cprand_mlp_forward", C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    ("cprand_mlp_workspace_size", C.c_size_t, [C.c_int64, C.c_int32]),
    ("cprand_mlp_grad", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("cprand_mlp_adam", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.c_void_p]),
    ("cprand_mlp_train", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_int32,
                                   C.c_float, C.POINTER(C.c_double), C.c_void_p]),
    ("cprand_plan_create", C.c_int, [C.POINTER(cprand_tensor), C.POINTER(cprand_opts), C.POINTER(C.c_void_p)]),
    ("cprand_plan_run", C.c_int, [C.c_void_p, C.POINTER(cprand_tensor), C.POINTER(C.c_void_p), C.c_void_p,
                                  C.POINTER(cprand_report), C.c_void_p]),
    ("cprand_plan_destroy", None, [C.c_void_p]),
    ("cprand_als", C.c_int, [C.POINTER(cprand_tensor), C.POINTER(cprand_opts), C.POINTER(C.c_void_p),
                             C.c_void_p, C.POINTER(cprand_report), C.c_void_p]),
]


def load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError("libcprand.so is not built (%s); run __graft_entry__.build() or "
                          "python paper_1701_06600_amd/build.py" % path)
    lib = C.CDLL(path)
    for name, res, args in SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib
