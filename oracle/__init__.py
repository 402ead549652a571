"""FP64 CPU oracle for the GIGA-Lens lens model (arXiv:2202.07663, Sec. 2.1-2.2).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of the
benchmark use it; the product package never imports it. It shares no code with the HIP
path. The arithmetic lives in ``oracle.cpp`` (plain FP64 C++, dual numbers for the exact
gradient) and ``fit.py`` (priors, bijectors and the Adam step, in numpy FP64); this module
is the ctypes marshalling for the C part.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


class _Desc(ctypes.Structure):
    _fields_ = [
        ("H", ctypes.c_int), ("W", ctypes.c_int), ("k", ctypes.c_int),
        ("pix", ctypes.c_double),
        ("epl", ctypes.c_int), ("shear", ctypes.c_int), ("lens_light", ctypes.c_int),
        ("nmax", ctypes.c_int),
        ("K", ctypes.c_int), ("psf", _dp),
        ("sigma_bkg", ctypes.c_double), ("t_exp", ctypes.c_double), ("gain", ctypes.c_double),
    ]


def lib():
    """Load (building first if needed) the oracle shared library."""
    global _lib
    if _lib is None:
        src = os.path.join(_HERE, "oracle.cpp")
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
            from . import build as _build
            _build.build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _lib.or_nparams.restype = ctypes.c_int
        _lib.or_num_threads.restype = ctypes.c_int
        _lib.or_set_num_threads.argtypes = [ctypes.c_int]
        _lib.or_set_num_threads.restype = None
        _lib.or_loglik_grad.restype = ctypes.c_int
        _lib.or_log_likelihood_image.restype = ctypes.c_double
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


@dataclass
class Model:
    """Lens model description (mirrors the fields of the product's model descriptor)."""
    H: int
    W: int
    k: int
    pix: float
    epl: bool
    shear: bool
    lens_light: bool
    nmax: int
    psf: np.ndarray
    sigma_bkg: float
    t_exp: float
    gain: float = 1.0

    def desc(self) -> _Desc:
        self._psf64 = _f64(self.psf)
        K = self._psf64.shape[0]
        assert self._psf64.shape == (K, K) and K % 2 == 1
        return _Desc(self.H, self.W, self.k, self.pix, int(self.epl), int(self.shear),
                     int(self.lens_light), self.nmax, K, _ptr(self._psf64),
                     self.sigma_bkg, self.t_exp, self.gain)

    @property
    def nparams(self) -> int:
        return lib().or_nparams(ctypes.byref(self.desc()))


def num_threads() -> int:
    """Threads the oracle's parallel loops use (OpenMP)."""
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    """Threads for the oracle's later parallel loops (the CPU baseline times 1 and all)."""
    lib().or_set_num_threads(int(n))


def simulate(m: Model, theta) -> np.ndarray:
    theta = _f64(np.atleast_2d(theta))
    P = theta.shape[0]
    assert theta.shape[1] == m.nparams
    out = np.zeros((P, m.H, m.W))
    d = m.desc()
    lib().or_simulate(ctypes.byref(d), _ptr(theta), P, _ptr(out))
    return out


def loglik(m: Model, theta, obs) -> np.ndarray:
    theta = _f64(np.atleast_2d(theta))
    obs = _f64(obs)
    assert obs.shape == (m.H, m.W) and theta.shape[1] == m.nparams
    out = np.zeros(theta.shape[0])
    d = m.desc()
    lib().or_loglik(ctypes.byref(d), _ptr(theta), theta.shape[0], _ptr(obs), _ptr(out))
    return out


def loglik_grad(m: Model, theta, obs):
    theta = _f64(np.atleast_2d(theta))
    obs = _f64(obs)
    assert obs.shape == (m.H, m.W) and theta.shape[1] == m.nparams
    P, d = theta.shape
    ll = np.zeros(P)
    g = np.zeros((P, d))
    desc = m.desc()
    rc = lib().or_loglik_grad(ctypes.byref(desc), _ptr(theta), P, _ptr(obs), _ptr(ll), _ptr(g))
    if rc != 0:
        raise ValueError("oracle gradient supports at most 72 parameters")
    return ll, g


def log_likelihood_image(m: Model, img, obs) -> float:
    img, obs = _f64(img), _f64(obs)
    d = m.desc()
    return lib().or_log_likelihood_image(ctypes.byref(d), _ptr(img), _ptr(obs))


def surface_brightness(m: Model, theta, x, y) -> np.ndarray:
    theta, x, y = _f64(theta), _f64(x), _f64(y)
    out = np.zeros_like(x)
    d = m.desc()
    lib().or_surface_brightness(ctypes.byref(d), _ptr(theta), x.size, _ptr(x), _ptr(y), _ptr(out))
    return out


# ---- component evaluators (for the closed-form pins) ----

def _xy(x, y):
    x, y = np.broadcast_arrays(_f64(x), _f64(y))
    return _f64(x), _f64(y)


def epl_deflection(x, y, theta_e, gamma, e1, e2, xc=0.0, yc=0.0):
    x, y = _xy(x, y)
    ax, ay = np.zeros_like(x), np.zeros_like(x)
    lib().or_epl_deflection(x.size, _ptr(x), _ptr(y), *map(ctypes.c_double,
                            (theta_e, gamma, e1, e2, xc, yc)), _ptr(ax), _ptr(ay))
    return ax, ay


def sie_deflection(x, y, theta_e, e1, e2, xc=0.0, yc=0.0):
    x, y = _xy(x, y)
    ax, ay = np.zeros_like(x), np.zeros_like(x)
    lib().or_sie_deflection(x.size, _ptr(x), _ptr(y), *map(ctypes.c_double,
                            (theta_e, e1, e2, xc, yc)), _ptr(ax), _ptr(ay))
    return ax, ay


def epl_kappa(x, y, theta_e, gamma, e1, e2, xc=0.0, yc=0.0):
    x, y = _xy(x, y)
    out = np.zeros_like(x)
    lib().or_epl_kappa(x.size, _ptr(x), _ptr(y), *map(ctypes.c_double,
                       (theta_e, gamma, e1, e2, xc, yc)), _ptr(out))
    return out


def hyp2f1(t, z):
    z = np.asarray(z, dtype=np.complex128)
    zr, zi = _f64(z.real), _f64(z.imag)
    fr, fi = np.zeros_like(zr), np.zeros_like(zr)
    lib().or_hyp2f1(zr.size, ctypes.c_double(t), _ptr(zr), _ptr(zi), _ptr(fr), _ptr(fi))
    return fr + 1j * fi


def shear_deflection(x, y, g1, g2):
    x, y = _xy(x, y)
    ax, ay = np.zeros_like(x), np.zeros_like(x)
    lib().or_shear_deflection(x.size, _ptr(x), _ptr(y), ctypes.c_double(g1), ctypes.c_double(g2),
                              _ptr(ax), _ptr(ay))
    return ax, ay


def sersic(x, y, r_eff, n, e1, e2, xc, yc, i0):
    x, y = _xy(x, y)
    out = np.zeros_like(x)
    lib().or_sersic(x.size, _ptr(x), _ptr(y), *map(ctypes.c_double,
                    (r_eff, n, e1, e2, xc, yc, i0)), _ptr(out))
    return out


def hermite_functions(u, nmax):
    u = _f64(u).ravel()
    out = np.zeros((u.size, nmax + 1))
    lib().or_hermite_functions(u.size, _ptr(u), nmax, _ptr(out))
    return out


def shapelets(x, y, xc, yc, beta, coeffs, nmax):
    x, y = _xy(x, y)
    coeffs = _f64(coeffs)
    assert coeffs.size == (nmax + 1) * (nmax + 2) // 2
    out = np.zeros_like(x)
    lib().or_shapelets(x.size, _ptr(x), _ptr(y), ctypes.c_double(xc), ctypes.c_double(yc),
                       ctypes.c_double(beta), _ptr(coeffs), nmax, _ptr(out))
    return out
