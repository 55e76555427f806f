"""ctypes view of libri.so (the C ABI declared in include/ri.h).

torch is imported first so the library binds to the HIP runtime torch already loaded
(both carry the soname libamdhip64.so.7).  Loading fails loudly when the library has
not been built: there is no fallback path.
"""
import ctypes
import os

import torch  # noqa: F401  (must precede the library load, see above)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libri.so")

RI_OK, RI_EINVAL, RI_ENOMEM, RI_EHIP, RI_ESTATE = 0, -1, -2, -3, -4
RI_PD_X, RI_PD_XTILDE, RI_PD_S, RI_PD_V, RI_PD_ITER, RI_PD_E, RI_PD_W = range(7)
STAGES = ("fft_rows", "fft_cols", "degrid", "block_norms", "grid", "grid_halo", "ifft_cols", "ifft_rows",
          "psi_adj", "psi_synth", "update")

c_void_p, c_int, c_int64, c_double, c_size_t, c_uint32 = (
    ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t, ctypes.c_uint32)
P = ctypes.POINTER


class Tuning(ctypes.Structure):
    _fields_ = [("tile", c_int), ("bin", c_int), ("fft_panel", c_int), ("persistent_wgs", c_int),
                ("slice_vis", c_int)]


class PDParams(ctypes.Structure):
    _fields_ = [("tau", c_double), ("sigma", c_double), ("varsigma", c_double), ("kappa", c_double),
                ("psi_norm", c_double), ("phi_norm", c_double)]


class Sched(ctypes.Structure):
    _fields_ = [("d", c_int), ("T", c_int64), ("u", c_void_p), ("masks", c_void_p), ("p_fixed", c_void_p),
                ("c", c_void_p), ("stats_step", c_void_p), ("stats_x", c_void_p), ("eps", c_void_p),
                ("n_nodes", c_double), ("p_min", c_double), ("p_max", c_double), ("counter", c_void_p),
                ("mask", c_void_p), ("p_log", c_void_p), ("mask_log", c_void_p)]


SCHED_UPDATE, SCHED_REFRESH, SCHED_ADAPTIVE, SCHED_DRAW = 1, 2, 4, 8

# name -> (restype, argtypes)
SIGNATURES = {
    "ri_last_error": (ctypes.c_char_p, []),
    "ri_version": (c_int, []),
    "ri_hip_runtime_version": (c_int, [P(c_int)]),
    "ri_plan_create": (c_int, [P(c_void_p), c_int, c_int64, c_void_p, c_int, c_void_p, c_int, c_double,
                               P(Tuning), c_void_p]),
    "ri_plan_destroy": (None, [c_void_p]),
    "ri_plan_info": (c_int, [c_void_p, P(c_int), P(c_int64), P(c_int), P(c_int), P(c_int), P(c_int)]),
    "ri_plan_order": (c_int, [c_void_p, c_void_p]),
    "ri_plan_permute": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    "ri_phi": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ri_phi_adj": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ri_block_sumsq": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "ri_phi_norm": (c_int, [c_void_p, c_void_p, c_int, c_double, P(c_double), P(c_int), c_void_p]),
    "ri_sara_create": (c_int, [P(c_void_p), c_int, c_int, c_uint32, c_void_p]),
    "ri_sara_destroy": (None, [c_void_p]),
    "ri_sara_bases": (c_int, [c_void_p, P(c_int)]),
    "ri_psi": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "ri_psi_adj": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "ri_psi_norm": (c_int, [c_void_p, c_void_p, c_int, c_double, P(c_double), P(c_int), c_void_p]),
    "ri_pd_create": (c_int, [P(c_void_p), c_void_p, c_void_p, c_void_p, c_void_p, P(PDParams), c_void_p]),
    "ri_pd_destroy": (None, [c_void_p]),
    "ri_pd_step": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "ri_pd_step_plain": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "ri_pd_refresh": (c_int, [c_void_p, c_void_p]),
    "ri_pd_residual": (c_int, [c_void_p, c_void_p, c_void_p]),
    "ri_pd_timing": (c_int, [c_void_p, c_int]),
    "ri_pd_stage_times": (c_int, [c_void_p, c_void_p, c_void_p, c_int]),
    "ri_pd_get": (c_int, [c_void_p, c_int, c_void_p, c_size_t, c_void_p]),
    "ri_pd_set": (c_int, [c_void_p, c_int, c_void_p, c_size_t, c_void_p]),
    "ri_pd_step_vjp": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ri_residual_energy": (c_int, [c_void_p, c_void_p, c_int, c_void_p]),
    "ri_probs": (c_int, [c_void_p, c_int, c_double, c_double, c_double, c_void_p, P(c_double)]),
    "ri_sched_step": (c_int, [P(Sched), c_int, c_void_p]),
    "ri_pd_reweight": (c_int, [c_void_p, c_double, c_void_p]),
    "ri_plan_dde": (c_int, [c_void_p, c_int, c_void_p, c_void_p]),
    "ri_pd_residual_noalloc": (c_int, [c_void_p, c_void_p, c_void_p]),
    "ri_pd_weighted": (c_int, [c_void_p, P(c_int)]),
}

_lib = None


class RIError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ri error {code}: {msg}")
        self.code = code


def load():
    """Load libri.so once and declare every signature."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1610_08895_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(code):
    if code != RI_OK:
        raise RIError(code, load().ri_last_error().decode(errors="replace"))
    return code
