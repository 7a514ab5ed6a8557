"""ctypes view of libpimc's C ABI (include/pimc.h).  Argument marshalling only."""

from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpimc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pimc.h")

PIMC_OK = 0
PIMC_ERR_ARG = -1
PIMC_ERR_HIP = -2
PIMC_ERR_NONFINITE = -3
PIMC_ERR_UNSUPPORTED = -4
PIMC_ERR_NOMEM = -5
PIMC_ERR_BOX = -6
PIMC_ERR_TIMEOUT = -7
PIMC_FP64 = 0
PIMC_FP32 = 1
PIMC_PROP_GAUSS = 0
PIMC_PROP_UNIFORM = 1
PIMC_STATES = 1
PIMC_PARAMS = 2
PIMC_GIBBS = 4
PIMC_KINETIC = 8
PIMC_NACC = 10
PIMC_NOALLOC_MAX_SITES = 4096 * 256


class Model(C.Structure):
    _fields_ = [("dt", C.c_double), ("Ro", C.c_double), ("Rd", C.c_double * 4), ("beta", C.c_double),
                ("Va", C.c_double * 3), ("dVa", C.c_double * 3), ("tau0", C.c_double * 3),
                ("tau1", C.c_double * 3), ("x_lo", C.c_double * 4), ("x_hi", C.c_double * 4),
                ("p_lo", C.c_double * 7), ("p_hi", C.c_double * 7), ("p_mask", C.c_uint32),
                ("proposal", C.c_int32), ("k_lo", C.c_double * 12), ("k_hi", C.c_double * 12),
                ("k_mask", C.c_uint32)]


class Path(C.Structure):
    _fields_ = [("M", C.c_int64), ("prec", C.c_int32), ("X", C.c_void_p), ("p", C.c_void_p),
                ("y", C.c_void_p), ("I", C.c_void_p), ("kin", C.c_void_p)]


class Rng(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("chain", C.c_uint32), ("sweep0", C.c_uint64)]


class Stats(C.Structure):
    _fields_ = [("sum", C.c_void_p), ("sumsq", C.c_void_p), ("xref", C.c_void_p),
                ("ptrace", C.c_void_p), ("acc", C.c_void_p), ("burn", C.c_int64), ("stride", C.c_int64),
                ("batch", C.c_void_p), ("nbatch", C.c_int64), ("kacc", C.c_void_p)]


class Debug(C.Structure):
    _fields_ = [("xprop", C.c_void_p), ("dA", C.c_void_p), ("accept", C.c_void_p),
                ("pprop", C.c_void_p), ("pdA", C.c_void_p), ("paccept", C.c_void_p),
                ("kprop", C.c_void_p), ("kdA", C.c_void_p), ("kaccept", C.c_void_p)]


class Batch(C.Structure):
    _fields_ = [("B", C.c_int32), ("prec", C.c_int32), ("offsets", C.POINTER(C.c_int64)),
                ("X", C.c_void_p), ("p", C.c_void_p), ("y", C.c_void_p), ("I", C.c_void_p),
                ("chain", C.c_void_p)]


class BatchStats(C.Structure):
    _fields_ = [("sum", C.c_void_p), ("sumsq", C.c_void_p), ("xref", C.c_void_p),
                ("ptrace", C.c_void_p), ("acc", C.c_void_p), ("burn", C.c_int64), ("stride", C.c_int64),
                ("batch", C.c_void_p), ("nbatch", C.c_int64)]


class InitPhase(C.Structure):
    _fields_ = [("beta0", C.c_double), ("n_cool", C.c_int64), ("n_init", C.c_int64), ("n_skip", C.c_int64),
                ("f_acc", C.c_double), ("alpha", C.c_double), ("beta", C.c_void_p), ("site_scale", C.c_void_p),
                ("w_param", C.c_void_p), ("cnt_site", C.c_void_p), ("cnt_param", C.c_void_p)]


class HmcStats(C.Structure):
    _fields_ = [("acc", C.c_void_p), ("ptrace", C.c_void_p), ("dH", C.c_void_p), ("traj_q", C.c_void_p),
                ("traj_r", C.c_void_p), ("traj_p", C.c_void_p), ("traj_rp", C.c_void_p)]


_SIGS = {
    "pimc_ctx_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    "pimc_ctx_destroy": (None, [C.c_void_p]),
    "pimc_set_sweep_tile": (C.c_int, [C.c_void_p, C.c_int]),
    "pimc_set_sweep_tiles": (C.c_int, [C.c_void_p, C.c_int]),
    "pimc_sync": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pimc_strerror": (C.c_char_p, [C.c_int]),
    "pimc_action": (C.c_int, [C.c_void_p, C.POINTER(Model), C.POINTER(Path), C.c_void_p, C.c_void_p]),
    "pimc_sweep": (C.c_int, [C.c_void_p, C.POINTER(Model), C.POINTER(Path), Rng, C.c_void_p, C.c_int64,
                             C.c_int32, C.POINTER(Stats), C.POINTER(Debug), C.c_void_p]),
    "pimc_sweep_init": (C.c_int, [C.c_void_p, C.POINTER(Model), C.POINTER(Path), Rng, C.c_void_p, C.c_int64,
                                  C.c_int32, C.POINTER(InitPhase), C.POINTER(Stats), C.c_void_p]),
    "pimc_param_update": (C.c_int, [C.c_void_p, C.POINTER(Model), C.POINTER(Path), Rng, C.c_void_p,
                                    C.POINTER(Debug), C.c_void_p]),
    "pimc_model_errors": (C.c_int, [C.c_void_p, C.POINTER(Model), C.POINTER(Path), C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    "pimc_forecast": (C.c_int, [C.c_void_p, C.POINTER(Model), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_int64, C.c_double, C.c_uint64, C.c_int64, C.c_void_p, C.c_void_p]),
    "pimc_action_noalloc": (C.c_int, [C.POINTER(Model), C.POINTER(Path), C.c_void_p, C.c_void_p]),
    "pimc_grad": (C.c_int, [C.c_void_p, C.POINTER(Model), C.POINTER(Path), C.c_void_p, C.c_void_p,
                            C.c_void_p]),
    "pimc_run_batch": (C.c_int, [C.c_void_p, C.POINTER(Model), C.POINTER(Batch), C.c_uint64, C.c_uint64,
                                 C.c_void_p, C.c_int64, C.c_int32, C.POINTER(BatchStats), C.c_void_p]),
    "pimc_hmc": (C.c_int, [C.c_void_p, C.POINTER(Model), C.POINTER(Batch), C.c_uint64, C.c_uint64, C.c_double,
                           C.c_int32, C.POINTER(C.c_double), C.c_int64, C.POINTER(HmcStats), C.c_void_p]),
}

_lib = None


def header_functions(path: str = HEADER):
    """Names of the functions declared in include/pimc.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(pimc_\w+)\s*\(", text, flags=re.M)))


def load():
    """Load libpimc.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class PimcError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        msg = load().pimc_strerror(status).decode()
        super().__init__(f"{what}: {msg} (status {status})" if what else f"{msg} (status {status})")
        self.status = status


def check(status: int, what: str = ""):
    if status != PIMC_OK:
        raise PimcError(status, what)
