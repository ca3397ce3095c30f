"""ctypes declarations of the C ABI in include/mm.h (libmm.so, built in-tree).

Importing this module loads libmm.so and raises ImportError if it has not
been built; there is no fallback implementation.
"""

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmm.so")

MM_OK, MM_ENOCONV, MM_EINVAL, MM_ENOMEM, MM_EDEVICE, MM_ENOTBUILT, MM_EBREAKDOWN = 0, 1, -1, -2, -3, -4, -5
MM_F32, MM_BF16, MM_F64 = 0, 1, 2
MM_ACC_F64, MM_ACC_F32X2 = 0, 1
MM_POINT_STORED, MM_POINT_BORESIGHT = 0, 1
MM_M_NONE, MM_M_JACOBI, MM_M_BINNED, MM_M_CIRCULANT, MM_M_LEARNED, MM_M_TILED = 0, 1, 2, 3, 4, 5

STATUS_NAMES = {0: "MM_OK", 1: "MM_ENOCONV", -1: "MM_EINVAL", -2: "MM_ENOMEM",
                -3: "MM_EDEVICE", -4: "MM_ENOTBUILT", -5: "MM_EBREAKDOWN"}


class mm_scan_desc(C.Structure):
    _fields_ = [
        ("ncomp", C.c_int32), ("ny", C.c_int32), ("nx", C.c_int32), ("ndet", C.c_int32),
        ("tod_dtype", C.c_int32), ("nsamp", C.c_int64), ("fsample", C.c_double),
        ("pix", C.c_void_p), ("cos2psi", C.c_void_p), ("sin2psi", C.c_void_p),
        ("inv_noise", C.c_void_p), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
        ("det_group", C.c_int32), ("fft_m1", C.c_int32), ("mask_rcond", C.c_double),
        ("fft_cols", C.c_int32), ("scatter", C.c_int32), ("acc", C.c_int32),
        ("corr_rank", C.c_int32), ("corr_nbins", C.c_int32), ("corr_edges", C.c_void_p),
        ("corr_V", C.c_void_p), ("pointing", C.c_int32), ("bore", C.c_void_p),
        ("det_off", C.c_void_p), ("pointing_code", C.c_int32),
    ]


class mm_precon_opts(C.Structure):
    _fields_ = [("ref_y", C.c_int32), ("ref_x", C.c_int32), ("gauss_sigma_px", C.c_double),
                ("symmetrize", C.c_int32), ("eig_floor_rel", C.c_double),
                ("tile", C.c_int32), ("tiled_workspace", C.c_void_p),
                ("tiled_workspace_bytes", C.c_size_t), ("probe_sets", C.c_int32)]


class mm_pcg_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int32), ("check_every", C.c_int32),
                ("use_x0", C.c_int32), ("snap_every", C.c_int32), ("max_snaps", C.c_int32),
                ("snapshots", C.c_void_p), ("graph", C.c_int32), ("flexible", C.c_int32),
                ("refine", C.c_int32), ("true_residual", C.c_int32)]


class mm_train_opts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("seed", C.c_uint64), ("shuffle", C.c_int32), ("drop_last", C.c_int32)]


class mm_pcg_result(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("rel_resid", C.c_double),
                ("t_solve_s", C.c_double), ("history", C.POINTER(C.c_double)),
                ("alpha", C.POINTER(C.c_double)), ("rho", C.POINTER(C.c_double)),
                ("t_setup_s", C.c_double), ("true_rel_resid", C.c_double),
                ("restarts", C.c_int32)]


class mm_scan_info(C.Structure):
    _fields_ = [("n_active", C.c_int32), ("ref_pixel", C.c_int32), ("n_floored", C.c_int32),
                ("det_group", C.c_int32), ("fft_m1", C.c_int32), ("fft_m2", C.c_int32),
                ("fft_cols", C.c_int32), ("single_pass", C.c_int32), ("csr", C.c_int32), ("workspace_bytes", C.c_size_t),
                ("gather_weights", C.c_int32), ("pass1_pointing", C.c_int32),
                ("t_build_s", C.c_double)]


class mm_profile(C.Structure):
    _fields_ = [("n_stages", C.c_int32), ("ms", C.c_double * 8), ("launches", C.c_int64 * 8),
                ("samples", C.c_int64 * 8)]


PROFILE_STAGES = ["single", "pass1", "pass2", "pass3", "apply_A", "precon", "reduce", "corr"]
MM_SCATTER_AUTO, MM_SCATTER_ATOMIC, MM_SCATTER_SAMPLES = 0, 1, 2
MM_PTC_AUTO, MM_PTC_OFF = 0, 1


# name -> (restype, argtypes)
SIGNATURES = {
    "mm_scan_workspace_bytes": (C.c_size_t, [C.POINTER(mm_scan_desc)]),
    "mm_create_scan": (C.c_int, [C.POINTER(mm_scan_desc), C.c_void_p, C.POINTER(C.c_void_p)]),
    "mm_destroy_scan": (None, [C.c_void_p]),
    "mm_rhs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_apply_A": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_build_precon": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(mm_precon_opts), C.c_void_p]),
    "mm_apply_precon_binned": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_apply_precon_circulant": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_tiled_workspace_bytes": (C.c_size_t, [C.c_void_p, C.c_int32]),
    "mm_apply_precon_tiled": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_pcg_solve": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                               C.POINTER(mm_pcg_opts), C.POINTER(mm_pcg_result), C.c_void_p]),
    "mm_precon_judge": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                  C.POINTER(mm_pcg_opts), C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_pcg_solve_batch": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_int32,
                                     C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                     C.POINTER(mm_pcg_opts), C.POINTER(mm_pcg_result),
                                     C.POINTER(C.c_int32), C.c_void_p]),
    "mm_map_spectra": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_int32,
                                 C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_map_spectra_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_int32,
                                 C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_anorm_error_estimate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                          C.c_void_p]),
    "mm_spectrum_cv_error": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                       C.c_void_p]),
    "mm_cv_crossing_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_int32,
                                      C.c_void_p, C.c_void_p]),
    "mm_get_info": (C.c_int, [C.c_void_p, C.POINTER(mm_scan_info)]),
    "mm_get_mask": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_learned_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "mm_learned_create": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                    C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "mm_learned_destroy": (None, [C.c_void_p]),
    "mm_learned_get": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_learned_attach": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mm_learned_make_pair": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_learned_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                   C.POINTER(mm_train_opts), C.c_void_p, C.c_void_p]),
    "mm_learned_loss": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                  C.POINTER(C.c_double), C.c_void_p]),
    "mm_learned_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_learned_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                  C.POINTER(C.c_double), C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_apply_precon_learned": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "mm_profile_read": (C.c_int, [C.c_void_p, C.POINTER(mm_profile)]),
    "mm_profile_stages": (C.c_int, [C.c_void_p, C.c_uint32]),
    "mm_last_error": (C.c_char_p, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1309_7473_amd.build")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class MMError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib.mm_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


def check(status, where):
    if status not in (MM_OK,):
        raise MMError(status, where)
    return status
