"""ctypes view of libpm.so (declarations mirror include/pm.h).

Argument marshalling only: structures, prototypes and status checking.  The
library must have been built (python -m paper_2211_09815_amd.build); there is
no fallback implementation, so a missing library is an ImportError.
"""
import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpm.so")

PM_OK = 0
PM_EINVAL = -1
PM_ESHAPE = -2
PM_ENOMEM = -3
PM_EDEVICE = -4
PM_EUNSUPPORTED = -5
PM_ENONFINITE = -6

PM_F32 = 0
PM_F64 = 1

PM_K_BIN = 1
PM_K_FFT_R2C_Z = 2
PM_K_FFT_C2R_Z = 3
PM_K_FFT_LINES = 4
PM_K_FFT_POISSON = 5
PM_K_GATHER = 6
PM_K_SCATTER = 7
PM_K_PAINT_TILES = 8
PM_K_HALO = 9
PM_K_LIGHTCONE = 10

PM_STREAM_READ = 0
PM_STREAM_COPY = 1
PM_STREAM_WRITE = 2
KERNEL_FAMILIES = {
    "bin": PM_K_BIN, "scatter": PM_K_SCATTER, "paint_tiles": PM_K_PAINT_TILES, "halo_add": PM_K_HALO,
    "fft_r2c_z": PM_K_FFT_R2C_Z, "fft_lines": PM_K_FFT_LINES, "fft_poisson": PM_K_FFT_POISSON,
    "fft_c2r_z": PM_K_FFT_C2R_Z, "gather": PM_K_GATHER, "lightcone": PM_K_LIGHTCONE,
}
# device kernel symbol of each family (for matching profiler output)
KERNEL_SYMBOLS = {
    "bin": "k_bin", "scatter": "k_scatter", "paint_tiles": "k_paint_tiles", "halo_add": "k_halo_add",
    "fft_r2c_z": "k_fft_r2c_z", "fft_lines": "k_fft_lines", "fft_poisson": "k_fft_x_fused",
    "fft_c2r_z": "k_fft_c2r_z", "gather": "k_gather_tiles", "lightcone": "k_lightcone",
}

c_int = ctypes.c_int
c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_dbl = ctypes.c_double
c_vp = ctypes.c_void_p
c_sz = ctypes.c_size_t


class PmConfig(ctypes.Structure):
    _fields_ = [("mesh", c_i32 * 3), ("ptcl", c_i32 * 3), ("box", c_dbl * 3),
                ("lattice_offset", c_dbl), ("mesh_dtype", c_i32), ("state_dtype", c_i32),
                ("deterministic", c_i32), ("lpt_scratch", c_i32), ("lpt_keep", c_i32)]


class PmStepCoef(ctypes.Structure):
    _fields_ = [("Ka", c_dbl), ("D", c_dbl), ("Kb", c_dbl), ("dKa", c_dbl), ("dD", c_dbl), ("dKb", c_dbl)]


class PmState(ctypes.Structure):
    _fields_ = [("s", c_vp), ("p", c_vp), ("acc", c_vp)]


class PmAdj(ctypes.Structure):
    _fields_ = [("xi", c_vp), ("pi", c_vp)]


class PmCheckpoints(ctypes.Structure):
    _fields_ = [("count", c_int), ("step", ctypes.POINTER(c_int)), ("s", ctypes.POINTER(c_vp)),
                ("p", ctypes.POINTER(c_vp))]


class PmCosmo(ctypes.Structure):
    _fields_ = [("omega_m", c_dbl), ("omega_b", c_dbl), ("h", c_dbl), ("n_s", c_dbl),
                ("sigma8", c_dbl), ("t_cmb", c_dbl)]


class PmIcCoef(ctypes.Structure):
    _fields_ = [("D1", c_dbl), ("D2", c_dbl), ("P1", c_dbl), ("P2", c_dbl), ("A", c_dbl),
                ("dD1", c_dbl), ("dD2", c_dbl), ("dP1", c_dbl), ("dP2", c_dbl), ("dA", c_dbl)]


class PmLcCoef(ctypes.Structure):
    _fields_ = [("a", c_dbl), ("chi", c_dbl), ("dchi", c_dbl), ("w", c_dbl),
                ("chi_om", c_dbl), ("dchi_om", c_dbl), ("w_om", c_dbl)]


class PmLcStep(ctypes.Structure):
    _fields_ = [("c0", PmLcCoef), ("c1", PmLcCoef), ("omega_m", c_dbl), ("observer", c_dbl * 3),
                ("step", c_i32)]


P = ctypes.POINTER
_PROTOS = {
    "pm_plan_create": (c_int, [P(PmConfig), P(c_vp)]),
    "pm_plan_destroy": (c_int, [c_vp]),
    "pm_workspace_bytes": (c_sz, [P(PmConfig)]),
    "pm_last_error": (ctypes.c_char_p, [c_vp]),
    "pm_strerror": (ctypes.c_char_p, [c_int]),
    "pm_paint": (c_int, [c_vp, c_vp, c_vp, c_int, c_vp, c_vp]),
    "pm_fft": (c_int, [c_vp, c_int, c_vp, c_vp, c_int, c_vp]),
    "pm_poisson_grad": (c_int, [c_vp, c_vp, c_vp, c_dbl, c_vp]),
    "pm_readout": (c_int, [c_vp, c_vp, c_vp, c_int, c_vp, c_vp]),
    "pm_force": (c_int, [c_vp, c_vp, c_dbl, c_vp, c_vp]),
    "pm_force_vjp": (c_int, [c_vp, c_vp, c_vp, c_dbl, c_vp, c_vp, c_vp, c_vp]),
    "pm_fwd_init": (c_int, [c_vp, P(PmState), P(PmStepCoef), c_dbl, c_vp]),
    "pm_step_fwd": (c_int, [c_vp, P(PmState), P(PmStepCoef), P(PmStepCoef), c_dbl, c_vp]),
    "pm_adj_init": (c_int, [c_vp, P(PmState), P(PmAdj), P(PmStepCoef), c_dbl, c_vp, c_vp]),
    "pm_step_adj": (c_int, [c_vp, P(PmState), P(PmAdj), P(PmStepCoef), P(PmStepCoef), c_dbl, c_vp, c_vp]),
    "pm_run_fwd": (c_int, [c_vp, P(PmState), P(PmStepCoef), c_int, c_dbl, c_vp]),
    "pm_run_adj": (c_int, [c_vp, P(PmState), P(PmAdj), P(PmStepCoef), c_int, c_dbl, c_vp, c_vp]),
    "pm_run_adj_from": (c_int, [c_vp, P(PmState), P(PmAdj), P(PmStepCoef), c_int, c_dbl, c_vp, c_vp]),
    "pm_run_fwd_ckpt": (c_int, [c_vp, P(PmState), P(PmStepCoef), c_int, c_dbl, P(PmCheckpoints), c_vp]),
    "pm_run_adj_ckpt": (c_int, [c_vp, P(PmState), P(PmAdj), P(PmStepCoef), c_int, c_dbl, P(PmCheckpoints), c_vp,
                                c_vp]),
    "pm_density_mse": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "pm_density": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "pm_tables": (c_int, [P(PmCosmo), P(c_dbl), c_int, P(PmStepCoef), P(PmIcCoef)]),
    "pm_lpt": (c_int, [c_vp, c_vp, P(PmCosmo), P(PmIcCoef), P(PmState), c_vp]),
    "pm_lpt_vjp": (c_int, [c_vp, c_vp, P(PmCosmo), P(PmIcCoef), P(PmAdj), c_vp, c_vp, c_vp]),
    "pm_lightcone_tables": (c_int, [P(PmCosmo), P(c_dbl), c_int, c_dbl, P(PmLcCoef)]),
    "pm_lightcone_reach": (c_int, [c_vp, c_vp, P(c_dbl), c_vp, c_vp]),
    "pm_lightcone_truncate": (c_int, [c_vp, c_vp, c_vp, c_i32, c_vp]),
    "pm_lightcone": (c_int, [c_vp, P(PmLcStep), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "pm_lightcone_vjp": (c_int, [c_vp, P(PmLcStep), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                                 c_vp, c_vp]),
    "pm_adj_bump": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_dbl, c_dbl, c_vp, c_vp, c_vp, c_vp]),
    "pm_kick": (c_int, [c_vp, c_vp, c_vp, c_dbl, c_vp, c_vp]),
    "pm_drift": (c_int, [c_vp, c_vp, c_vp, c_dbl, c_vp, c_vp]),
    "pm_power_spectrum": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "pm_power_spectrum_noalloc": (c_int, [c_int, c_dbl, c_int, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "pm_stream": (c_int, [c_vp, c_int, c_vp, c_vp, c_i64, c_vp]),
    "pm_check_finite": (c_int, [c_vp, c_vp, c_i64, c_int, c_vp, c_vp]),
    "pm_timing_enable": (c_int, [c_vp, ctypes.c_uint]),
    "pm_timing_read": (c_int, [c_vp, c_int, P(c_dbl), P(c_i64), P(c_dbl), P(c_dbl)]),
}

EXPORTED = tuple(_PROTOS.keys())


class PmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libpm error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    """The loaded library (loaded once); ImportError if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpm.so is not built at %s; run `python -m paper_2211_09815_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc, plan=None):
    if rc != PM_OK:
        msg = lib().pm_last_error(plan)
        raise PmError(rc, (msg or b"").decode() or lib().pm_strerror(rc).decode())
    return rc
