"""Shared test helpers: oracle model from a workload spec, and the parity tolerances.

Tolerances (FP32 GPU vs FP64 oracle):
  log L:     |dlogL| <= 1e-4 |logL_ref|
  gradient:  per particle ||g - g_ref||_2 <= 1e-3 ||g_ref||_2, and per component
             |dg_i| <= 1e-3 (|g_ref,i| + rms over particles of g_ref,i)
"""
import os

import numpy as np

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
LOGL_RTOL = 1e-4
GRAD_RTOL = 1e-3


def oracle_model(spec: synth.Spec, psf=None) -> oracle.Model:
    psf = spec.psf if psf is None else psf
    return oracle.Model(H=spec.H, W=spec.W, k=spec.k, pix=float(np.float32(spec.pix)), epl=spec.epl,
                        shear=spec.shear, lens_light=spec.lens_light, nmax=spec.nmax,
                        psf=np.asarray(psf, np.float32).astype(np.float64),
                        sigma_bkg=float(np.float32(spec.sigma_bkg)),
                        t_exp=float(np.float32(spec.t_exp)), gain=float(np.float32(spec.gain)))


def load_workload(name: str, seed: int = 0):
    obs = np.load(os.path.join(GOLDEN, f"obs_{name}_s{seed}.npy"))
    truth = np.load(os.path.join(GOLDEN, f"truth_{name}_s{seed}.npy"))
    return obs, truth


def logl_errors(gpu, ref):
    gpu, ref = np.asarray(gpu, np.float64), np.asarray(ref, np.float64)
    return np.abs(gpu - ref) / np.abs(ref)


def assert_logl_close(gpu, ref, rtol=LOGL_RTOL):
    err = logl_errors(gpu, ref)
    assert np.all(np.isfinite(gpu)), "non-finite GPU log L"
    assert err.max() <= rtol, f"log L rel err max {err.max():.3e} at {int(err.argmax())}"
    return err.max()


def grad_errors(gpu, ref):
    gpu, ref = np.asarray(gpu, np.float64), np.asarray(ref, np.float64)
    norm_err = np.linalg.norm(gpu - ref, axis=1) / np.linalg.norm(ref, axis=1)
    rms = np.sqrt(np.mean(ref ** 2, axis=0))
    comp_err = np.abs(gpu - ref) / (np.abs(ref) + rms[None, :])
    return norm_err, comp_err


def assert_grad_close(gpu, ref, rtol=GRAD_RTOL, names=None):
    assert np.all(np.isfinite(gpu)), "non-finite GPU gradient"
    norm_err, comp_err = grad_errors(gpu, ref)
    i, j = np.unravel_index(int(comp_err.argmax()), comp_err.shape)
    label = names[j] if names is not None else j
    assert norm_err.max() <= rtol, f"grad norm rel err {norm_err.max():.3e} at particle {int(norm_err.argmax())}"
    assert comp_err.max() <= rtol, (f"grad component err {comp_err.max():.3e} at particle {i}, "
                                    f"param {label}: gpu {gpu[i, j]:.6e} ref {ref[i, j]:.6e}")
    return norm_err.max(), comp_err.max()
