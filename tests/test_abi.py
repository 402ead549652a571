"""The C-ABI library loads on a machine without a GPU, exports every function that
include/gl.h declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gl.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(gl_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2202_07663_amd import _lib
    return _lib.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["gl_model_create", "gl_model_destroy", "gl_model_nparams", "gl_simulate",
              "gl_loglik", "gl_loglik_grad", "gl_fit", "gl_server_create", "gl_server_destroy",
              "gl_submit", "gl_poll", "gl_last_error"]:
        assert n in names, n


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def _desc(**kw):
    from paper_2202_07663_amd import _lib
    import numpy as np
    psf = np.ones((3, 3), np.float32) / 9
    obs = np.zeros((8, 8), np.float32)
    d = dict(H=8, W=8, pixel_scale=0.065, k_super=1, mass=1, shear=1, lens_light=0,
             shapelet_nmax=-1, psf_size=3, psf=psf.ctypes.data_as(_lib._fp),
             obs=obs.ctypes.data_as(_lib._fp), sigma_bkg=0.1, t_exp=100.0, gain=1.0)
    d.update(kw)
    return _lib.ModelDesc(**d), (psf, obs)


@pytest.mark.parametrize("field,value,code", [
    ("H", 0, -1), ("W", -3, -1), ("H", 4096, -7), ("pixel_scale", 0.0, -1),
    ("k_super", 0, -1), ("k_super", 9, -7), ("mass", 2, -1), ("shear", 2, -1),
    ("lens_light", -1, -1), ("shapelet_nmax", -2, -1), ("shapelet_nmax", 9, -7),
    ("psf_size", 4, -1), ("psf_size", 33, -7), ("t_exp", 0.0, -1), ("gain", -1.0, -1),
    ("sigma_bkg", -0.1, -1)])
def test_model_create_validates(lib, field, value, code):
    d, keep = _desc(**{field: value})
    h = ctypes.c_void_p()
    assert lib.gl_model_create(ctypes.byref(d), ctypes.byref(h)) == code
    assert h.value is None
    assert lib.gl_last_error() != b""


def test_null_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.gl_model_create(None, ctypes.byref(h)) == -1
    assert lib.gl_model_nparams(None, None) == -1
    assert lib.gl_loglik(None, None, 4, None, None) == -1
    assert lib.gl_loglik_grad(None, None, 4, None, None, None) == -1
    assert lib.gl_simulate(None, None, 4, None, None) == -1
    assert lib.gl_model_reserve(None, 4, 0) == -1
    assert lib.gl_model_plan(None, 4, None) == -1
    assert lib.gl_model_destroy(None) == 0
    assert b"NULL" in lib.gl_last_error() or lib.gl_last_error() == b""


def test_nonfinite_psf_rejected(lib):
    import numpy as np
    from paper_2202_07663_amd import _lib
    psf = np.full((3, 3), np.nan, np.float32)
    d, keep = _desc(psf=psf.ctypes.data_as(_lib._fp))
    h = ctypes.c_void_p()
    assert lib.gl_model_create(ctypes.byref(d), ctypes.byref(h)) == -1
    assert b"psf" in lib.gl_last_error()


def test_hmc_entry_points_reject_null_handles(lib):
    from paper_2202_07663_amd import _lib
    h = ctypes.c_void_p()
    o = _lib.HmcOpts(chains=4, n_leapfrog=2, n_burn=1, n_samples=1, step_size=0.1,
                     target_accept=0.75, adapt_frac=0.8)
    assert lib.gl_hmc_create(None, ctypes.byref(o), None, ctypes.byref(h), None) == -1
    assert lib.gl_last_error()
    assert lib.gl_hmc_create(None, ctypes.byref(o), None, None, None) == -1
    assert lib.gl_hmc_run(None, 1, None) == -1
    assert lib.gl_hmc_samples(None, None, None) == -1
    assert lib.gl_hmc_get_info(None, None, None) == -1
    assert lib.gl_hmc_leapfrog(None, None, None, 1, 0.1, None, None, None, None) == -1
    assert lib.gl_hmc_destroy(None) == 0
