"""ctypes binding of libglens.so (the C ABI declared in include/gl.h).

Argument marshalling only: every step of the lens model runs in the library's HIP kernels.
The library is loaded after torch so that both share one HIP runtime; if it is missing the
import fails loudly (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libglens.so")

GL_OK, GL_PENDING = 0, 1
ERRORS = {-1: "GL_E_INVALID", -2: "GL_E_NOMEM", -3: "GL_E_DEVICE", -4: "GL_E_BUDGET",
          -5: "GL_E_NOTFOUND", -6: "GL_E_NUMERIC", -7: "GL_E_UNIMPLEMENTED", -8: "GL_E_CLOSED"}
GL_MASS_SIE, GL_MASS_EPL = 0, 1
GL_PRIOR_NORMAL, GL_PRIOR_LOGNORMAL, GL_PRIOR_TRUNCNORMAL, GL_PRIOR_UNIFORM = 0, 1, 2, 3
GL_MAX_PARAMS = 68

_fp = ctypes.POINTER(ctypes.c_float)


class ModelDesc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int), ("W", ctypes.c_int), ("pixel_scale", ctypes.c_float),
                ("k_super", ctypes.c_int), ("mass", ctypes.c_int), ("shear", ctypes.c_int),
                ("lens_light", ctypes.c_int), ("shapelet_nmax", ctypes.c_int),
                ("psf_size", ctypes.c_int), ("psf", _fp), ("obs", _fp),
                ("sigma_bkg", ctypes.c_float), ("t_exp", ctypes.c_float), ("gain", ctypes.c_float)]


class Prior(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int), ("mu", ctypes.c_float), ("sigma", ctypes.c_float),
                ("lo", ctypes.c_float), ("hi", ctypes.c_float)]


class FitOpts(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int), ("K", ctypes.c_int), ("lr0", ctypes.c_float),
                ("lr1", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("priors", ctypes.POINTER(Prior))]


class FitResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("d", ctypes.c_int), ("best", ctypes.c_int),
                ("theta_best", ctypes.c_float * GL_MAX_PARAMS),
                ("z_best", ctypes.c_float * GL_MAX_PARAMS), ("logl_best", ctypes.c_double),
                ("logpost_best", ctypes.c_double), ("chi2nu", ctypes.c_double),
                ("t_submit", ctypes.c_uint64), ("t_admit", ctypes.c_uint64),
                ("t_done", ctypes.c_uint64)]


class HmcOpts(ctypes.Structure):
    _fields_ = [("chains", ctypes.c_int), ("n_leapfrog", ctypes.c_int), ("n_burn", ctypes.c_int),
                ("n_samples", ctypes.c_int), ("step_size", ctypes.c_float),
                ("target_accept", ctypes.c_float), ("adapt_frac", ctypes.c_float),
                ("seed", ctypes.c_uint64), ("inv_mass", ctypes.POINTER(ctypes.c_float)),
                ("adapt_length", ctypes.c_int), ("max_leapfrog", ctypes.c_int),
                ("inv_mass_form", ctypes.c_int), ("priors", ctypes.POINTER(Prior)),
                ("adapt_mass", ctypes.c_int)]


class HmcInfo(ctypes.Structure):
    _fields_ = [("step_size", ctypes.c_float), ("accept_mean", ctypes.c_double),
                ("trajectories", ctypes.c_int), ("trajectory_length", ctypes.c_float),
                ("mean_leapfrog", ctypes.c_double), ("mass_updates", ctypes.c_int)]


class ViOpts(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int), ("K", ctypes.c_int), ("lr_max", ctypes.c_float),
                ("lr_warmup", ctypes.c_int), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("init_sd", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("priors", ctypes.POINTER(Prior)), ("lr_final", ctypes.c_float),
                ("estimator", ctypes.c_int)]

GL_VI_PATHWISE, GL_VI_SCORE = 0, 1


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_systems", ctypes.c_int),
                ("steps_per_tick", ctypes.c_int), ("fill_subpixels", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("ticks", ctypes.c_uint64),
                ("hbm_in_use", ctypes.c_size_t), ("hbm_peak", ctypes.c_size_t),
                ("active", ctypes.c_int), ("queued", ctypes.c_int),
                ("failed", ctypes.c_uint64), ("last_error", ctypes.c_int)]


GL_PSF_MFMA, GL_PSF_VALU, GL_PSF_BANDED = 0, 1, 2


class Plan(ctypes.Structure):
    _fields_ = [("psf_path", ctypes.c_int), ("tiles", ctypes.c_int), ("fwd_tiles", ctypes.c_int),
                ("bands", ctypes.c_int), ("workspace_bytes", ctypes.c_size_t),
                ("workspace_reserved", ctypes.c_size_t), ("noalloc_max_P", ctypes.c_int),
                ("band_split", ctypes.c_int)]


_vp = ctypes.c_void_p
_i = ctypes.c_int
_SIGNATURES = {
    "gl_model_create": [ctypes.POINTER(ModelDesc), ctypes.POINTER(_vp)],
    "gl_model_destroy": [_vp],
    "gl_model_nparams": [_vp, ctypes.POINTER(_i)],
    "gl_model_reserve": [_vp, _i, _i],
    "gl_model_plan": [_vp, _i, ctypes.POINTER(Plan)],
    "gl_simulate": [_vp, _vp, _i, _vp, _vp],
    "gl_loglik": [_vp, _vp, _i, _vp, _vp],
    "gl_loglik_grad": [_vp, _vp, _i, _vp, _vp, _vp],
    "gl_loglik_grad_noalloc": [_vp, _vp, _i, _vp, _vp, _vp],
    "gl_model_stage_times": [_vp, _vp, _i, _i, _vp, _vp, ctypes.POINTER(ctypes.c_float), _vp],
    "gl_model_stage_times_n": [_vp, _vp, _i, _i, _i, _vp, _vp, ctypes.POINTER(ctypes.c_float),
                               _vp],
    "gl_fit": [_vp, ctypes.POINTER(FitOpts), ctypes.POINTER(FitResult), _vp],
    "gl_fit_state_create": [_vp, ctypes.POINTER(FitOpts), ctypes.POINTER(_vp), _vp],
    "gl_fit_state_destroy": [_vp],
    "gl_fit_state_step": [_vp, _i, _vp],
    "gl_fit_state_load": [_vp, _vp, _vp, _vp, _i, _vp],
    "gl_fit_state_store": [_vp, _vp, _vp, _vp, ctypes.POINTER(_i), _vp],
    "gl_fit_state_result": [_vp, ctypes.POINTER(FitResult), _vp],
    "gl_hmc_create": [_vp, ctypes.POINTER(HmcOpts), _vp, ctypes.POINTER(_vp), _vp],
    "gl_hmc_destroy": [_vp],
    "gl_hmc_run": [_vp, _i, _vp],
    "gl_hmc_samples": [_vp, _vp, _vp],
    "gl_hmc_get_info": [_vp, ctypes.POINTER(HmcInfo), _vp],
    "gl_hmc_get_mass": [_vp, _vp, _vp],
    "gl_hmc_leapfrog": [_vp, _vp, _vp, _i, ctypes.c_float, _vp, _vp, _vp, _vp],
    "gl_vi_create": [_vp, ctypes.POINTER(ViOpts), _vp, ctypes.POINTER(_vp), _vp],
    "gl_vi_destroy": [_vp],
    "gl_vi_step": [_vp, _i, _vp],
    "gl_vi_get": [_vp, _vp, _vp, _vp, _vp],
    "gl_vi_sample": [_vp, _i, ctypes.c_uint64, _vp, _vp],
    "gl_vi_get_state": [_vp, _vp, _vp, _vp, ctypes.POINTER(_i), _vp, _vp],
    "gl_vi_set_state": [_vp, _vp, _vp, _vp, _i, _vp],
    "gl_server_create": [ctypes.POINTER(ServerOpts), ctypes.POINTER(_vp)],
    "gl_server_destroy": [_vp],
    "gl_submit": [_vp, ctypes.POINTER(ModelDesc), ctypes.POINTER(FitOpts),
                  ctypes.POINTER(ctypes.c_uint64)],
    "gl_poll": [_vp, ctypes.c_uint64, ctypes.POINTER(FitResult)],
    "gl_server_get_stats": [_vp, ctypes.POINTER(ServerStats)],
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2202_07663_amd.build` (no CPU fallback exists)")
        _lib = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            f = getattr(_lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        _lib.gl_last_error.argtypes = []
        _lib.gl_last_error.restype = ctypes.c_char_p
    return _lib


class GlError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def check(rc: int) -> int:
    if rc < 0:
        raise GlError(rc, lib().gl_last_error().decode())
    return rc
