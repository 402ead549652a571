"""MI355X-native batched lens likelihood and adjoint (GIGA-Lens, arXiv:2202.07663).

Thin Python layer over libglens.so (C ABI in include/gl.h). PyTorch supplies device memory
and streams; every step of the lens model runs in the library's HIP kernels.

    m = Model(H=60, W=60, pixel_scale=0.065, k_super=2, mass="epl", lens_light=True,
              shapelet_nmax=6, psf=psf, obs=obs, sigma_bkg=0.1, t_exp=1000.0)
    logl = m.loglik(theta)                 # theta: cuda float32 [P, d] -> float64 [P]
    logl, grad = m.loglik_grad(theta)      # grad: float32 [P, d]
    logl = LogLik.apply(theta, m)          # differentiable (backward uses the adjoint)
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import GlError, check, lib

__all__ = ["Model", "LogLik", "FitState", "fit", "VI", "HMC", "Server", "GlError", "param_names", "nparams",
           "make_priors", "make_fit_opts", "result_dict"]


def nparams(mass: str, shear: bool, lens_light: bool, shapelet_nmax: int) -> int:
    return ((6 if mass == "epl" else 5) + (2 if shear else 0) + (7 if lens_light else 0) + 7
            + (0 if shapelet_nmax < 0 else 1 + (shapelet_nmax + 1) * (shapelet_nmax + 2) // 2))


def param_names(mass: str, shear: bool, lens_light: bool, shapelet_nmax: int) -> list:
    n = ["theta_E"] + (["gamma"] if mass == "epl" else []) + ["e1", "e2", "x", "y"]
    n += ["gamma1", "gamma2"] if shear else []
    n += ["l_R", "l_n", "l_e1", "l_e2", "l_x", "l_y", "l_I"] if lens_light else []
    n += ["s_R", "s_n", "s_e1", "s_e2", "s_x", "s_y", "s_I"]
    if shapelet_nmax >= 0:
        n += ["beta"] + [f"c{i}" for i in range(nparams("sie", False, False, shapelet_nmax) - 13)]
    return n


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def make_desc(H, W, pixel_scale, k_super, mass, shear, lens_light, shapelet_nmax, psf, obs,
              sigma_bkg, t_exp, gain):
    """Build a gl_model_desc; returns (desc, keepalive arrays)."""
    psf = _f32(psf)
    keep = [psf]
    obs_p = None
    if obs is not None:
        obs = _f32(obs)
        assert obs.shape == (H, W), "obs must be H x W"
        keep.append(obs)
        obs_p = obs.ctypes.data_as(_lib._fp)
    assert psf.ndim == 2 and psf.shape[0] == psf.shape[1], "psf must be K x K"
    d = _lib.ModelDesc(H, W, pixel_scale, k_super,
                       _lib.GL_MASS_EPL if mass == "epl" else _lib.GL_MASS_SIE,
                       int(shear), int(lens_light), shapelet_nmax, psf.shape[0],
                       psf.ctypes.data_as(_lib._fp), obs_p, sigma_bkg, t_exp, gain)
    return d, keep


class Model:
    """One lens system (image grid, components, PSF, observed image, noise model) on the
    current GPU. Calls are ordered on the current torch stream."""

    def __init__(self, H: int, W: int, pixel_scale: float, k_super: int, mass: str = "epl",
                 shear: bool = True, lens_light: bool = True, shapelet_nmax: int = -1,
                 psf=None, obs=None, sigma_bkg: float = 0.1, t_exp: float = 1000.0,
                 gain: float = 1.0):
        assert mass in ("sie", "epl")
        self.H, self.W, self.k_super = H, W, k_super
        self.mass, self.shear, self.lens_light, self.nmax = mass, shear, lens_light, shapelet_nmax
        self.has_obs = obs is not None
        desc, keep = make_desc(H, W, pixel_scale, k_super, mass, shear, lens_light,
                               shapelet_nmax, psf, obs, sigma_bkg, t_exp, gain)
        self._desc, self._keep = desc, keep
        h = ctypes.c_void_p()
        check(lib().gl_model_create(ctypes.byref(desc), ctypes.byref(h)))
        self._h = h
        d = ctypes.c_int()
        check(lib().gl_model_nparams(self._h, ctypes.byref(d)))
        self.d = d.value
        self.names = param_names(mass, shear, lens_light, shapelet_nmax)
        assert len(self.names) == self.d

    @classmethod
    def from_spec(cls, spec, obs=None):
        """Build from a ``synth.Spec``-like object."""
        return cls(spec.H, spec.W, spec.pix, spec.k, "epl" if spec.epl else "sie", spec.shear,
                   spec.lens_light, spec.nmax, spec.psf, obs, spec.sigma_bkg, spec.t_exp,
                   spec.gain)

    def close(self):
        if getattr(self, "_h", None):
            lib().gl_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _theta(self, theta: torch.Tensor) -> torch.Tensor:
        if not (isinstance(theta, torch.Tensor) and theta.is_cuda):
            raise TypeError("theta must be a CUDA tensor")
        if theta.dtype != torch.float32 or theta.dim() != 2 or theta.shape[1] != self.d:
            raise ValueError(f"theta must be float32 [P, {self.d}]")
        return theta.contiguous()

    PSF_PATHS = {_lib.GL_PSF_MFMA: "mfma", _lib.GL_PSF_VALU: "valu", _lib.GL_PSF_BANDED: "banded"}

    def reserve(self, P: int, with_fit: bool = False):
        """Size the device work space for calls of up to P vectors (later calls then only
        enqueue work)."""
        check(lib().gl_model_reserve(self._h, int(P), int(with_fit)))

    def plan(self, P: int) -> dict:
        """How a call with P vectors is split: PSF path, tiles, bands (and the lanes sharing a
        strip's PSF columns in the banded pass), work-space bytes."""
        r = _lib.Plan()
        check(lib().gl_model_plan(self._h, int(P), ctypes.byref(r)))
        return {"psf_path": self.PSF_PATHS[r.psf_path], "tiles": r.tiles,
                "fwd_tiles": r.fwd_tiles, "bands": r.bands,
                "workspace_bytes": r.workspace_bytes, "workspace_reserved": r.workspace_reserved,
                "noalloc_max_P": r.noalloc_max_P, "band_split": r.band_split}

    def simulate(self, theta: torch.Tensor, stream=None) -> torch.Tensor:
        theta = self._theta(theta)
        P = theta.shape[0]
        img = torch.empty((P, self.H, self.W), dtype=torch.float32, device=theta.device)
        check(lib().gl_simulate(self._h, theta.data_ptr(), P, img.data_ptr(), _stream_ptr(stream)))
        return img

    def loglik(self, theta: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        theta = self._theta(theta)
        P = theta.shape[0]
        ll = out if out is not None else torch.empty(P, dtype=torch.float64, device=theta.device)
        check(lib().gl_loglik(self._h, theta.data_ptr(), P, ll.data_ptr(), _stream_ptr(stream)))
        return ll

    def loglik_grad(self, theta: torch.Tensor, out=None, stream=None):
        theta = self._theta(theta)
        P = theta.shape[0]
        if out is None:
            ll = torch.empty(P, dtype=torch.float64, device=theta.device)
            g = torch.empty((P, self.d), dtype=torch.float32, device=theta.device)
        else:
            ll, g = out
        check(lib().gl_loglik_grad(self._h, theta.data_ptr(), P, ll.data_ptr(), g.data_ptr(),
                                   _stream_ptr(stream)))
        return ll, g

    STAGES = ("prologue", "subpix_fwd", "conv_lik", "subpix_adj", "finalize")

    def stage_times(self, theta: torch.Tensor, with_grad: bool = True, stream=None,
                    n_calls: int = 1) -> dict:
        """Run the pipeline n_calls times back to back with HIP events between its kernels
        (blocking); returns the mean milliseconds of each stage."""
        theta = self._theta(theta)
        P = theta.shape[0]
        ll = torch.empty(P, dtype=torch.float64, device=theta.device)
        g = torch.empty((P, self.d), dtype=torch.float32, device=theta.device)
        ms = (ctypes.c_float * 5)()
        check(lib().gl_model_stage_times_n(self._h, theta.data_ptr(), P, int(with_grad),
                                           int(n_calls), ll.data_ptr(), g.data_ptr(), ms,
                                           _stream_ptr(stream)))
        return dict(zip(self.STAGES, list(ms)))


class LogLik(torch.autograd.Function):
    """log L(theta) as a differentiable function of theta [P, d] (float32, CUDA).

    forward runs gl_loglik_grad once and saves the gradient; backward returns
    grad_out[:, None] * grad (log L is one scalar per parameter vector, so this is the exact
    vector-Jacobian product)."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, model: Model):
        ll, g = model.loglik_grad(theta.detach())
        ctx.save_for_backward(g)
        return ll

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return (grad_out.to(g.dtype)[:, None] * g), None


# ------------------------------------------------------------------------------------------
# Multi-start fit
# ------------------------------------------------------------------------------------------

def make_priors(priors) -> "ctypes.Array":
    """gl_prior array from a list of dicts {family, mu, sigma, lo, hi}."""
    arr = (_lib.Prior * len(priors))()
    for i, p in enumerate(priors):
        arr[i] = _lib.Prior(int(p["family"]), float(p.get("mu", 0.0)), float(p.get("sigma", 1.0)),
                            float(p.get("lo", 0.0)), float(p.get("hi", 0.0)))
    return arr


def make_fit_opts(P, K, priors, lr0=1e-2, lr1=1e-3, seed=0, beta1=0.9, beta2=0.999, eps=1e-8):
    pa = make_priors(priors)
    o = _lib.FitOpts(P, K, lr0, lr1, beta1, beta2, eps, seed,
                     ctypes.cast(pa, ctypes.POINTER(_lib.Prior)))
    return o, pa


def result_dict(r) -> dict:
    return {"status": r.status, "d": r.d, "best": r.best,
            "theta_best": np.array(r.theta_best[:r.d], np.float32),
            "z_best": np.array(r.z_best[:r.d], np.float32), "logl_best": r.logl_best,
            "logpost_best": r.logpost_best, "chi2nu": r.chi2nu, "t_submit": r.t_submit,
            "t_admit": r.t_admit, "t_done": r.t_done}


class FitState:
    """Device state of one multi-start fit (z, Adam moments, step) on a Model.
    Starts are drawn from the prior on creation."""

    def __init__(self, model: Model, P: int, K: int, priors, lr0=1e-2, lr1=1e-3, seed=0,
                 stream=None):
        assert len(priors) == model.d
        self.model, self.P, self.K = model, P, K
        opts, self._pa = make_fit_opts(P, K, priors, lr0, lr1, seed)
        h = ctypes.c_void_p()
        check(lib().gl_fit_state_create(model._h, ctypes.byref(opts), ctypes.byref(h),
                                        _stream_ptr(stream)))
        self._h = h

    def step(self, n: int = 1, stream=None):
        check(lib().gl_fit_state_step(self._h, n, _stream_ptr(stream)))

    def load(self, z: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, stream=None):
        z, m, v = (t.contiguous() for t in (z, m, v))
        for t in (z, m, v):
            assert t.is_cuda and t.dtype == torch.float32 and t.shape == (self.P, self.model.d)
        check(lib().gl_fit_state_load(self._h, z.data_ptr(), m.data_ptr(), v.data_ptr(), step,
                                      _stream_ptr(stream)))
        self._keep = (z, m, v)

    def store(self, stream=None):
        shape = (self.P, self.model.d)
        z, m, v = (torch.empty(shape, dtype=torch.float32, device="cuda") for _ in range(3))
        step = ctypes.c_int()
        check(lib().gl_fit_state_store(self._h, z.data_ptr(), m.data_ptr(), v.data_ptr(),
                                       ctypes.byref(step), _stream_ptr(stream)))
        return z, m, v, step.value

    def result(self, stream=None) -> dict:
        r = _lib.FitResult()
        check(lib().gl_fit_state_result(self._h, ctypes.byref(r), _stream_ptr(stream)))
        return result_dict(r)

    def close(self):
        if getattr(self, "_h", None):
            lib().gl_fit_state_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fit(model: Model, P: int, K: int, priors, lr0=1e-2, lr1=1e-3, seed=0, stream=None) -> dict:
    """One fixed-budget multi-start fit of one system (blocking); returns the best particle."""
    opts, _keep = make_fit_opts(P, K, priors, lr0, lr1, seed)
    r = _lib.FitResult()
    check(lib().gl_fit(model._h, ctypes.byref(opts), ctypes.byref(r), _stream_ptr(stream)))
    return result_dict(r)


# ------------------------------------------------------------------------------------------
# Variational inference (Sec. 2.4)
# ------------------------------------------------------------------------------------------
class VI:
    """Multivariate normal surrogate of one system's posterior in unconstrained space, fitted
    by the library's kernels (one batched likelihood-gradient launch per iteration).
    mu0: [d] start of the mean (the paper: the MAP point, e.g. fit(...)["z_best"]).
    lr_final: 0 keeps lr_max after the warm-up (the paper); > 0 decays the rate geometrically
    to lr_final on the last iteration. estimator: "pathwise" (default) or "score" (the
    score-function form the paper prints, eq. elbo-grad)."""

    ESTIMATORS = {"pathwise": _lib.GL_VI_PATHWISE, "score": _lib.GL_VI_SCORE}

    def __init__(self, model: Model, n_samples: int, K: int, priors, mu0, lr_max: float = 1e-3,
                 lr_warmup: int = 500, init_sd: float = 1e-3, seed: int = 0, beta1=0.9,
                 beta2=0.999, eps=1e-8, lr_final: float = 0.0, estimator: str = "pathwise",
                 stream=None):
        assert len(priors) == model.d
        self.model, self.n, self.K, self.d = model, n_samples, K, model.d
        self._pa = make_priors(priors)
        o = _lib.ViOpts(n_samples=n_samples, K=K, lr_max=lr_max, lr_warmup=lr_warmup,
                        beta1=beta1, beta2=beta2, eps=eps, init_sd=init_sd, seed=seed,
                        priors=self._pa, lr_final=lr_final,
                        estimator=self.ESTIMATORS[estimator])
        mu = torch.as_tensor(np.asarray(mu0, np.float64)).reshape(model.d).cuda()
        h = ctypes.c_void_p()
        check(lib().gl_vi_create(model._h, ctypes.byref(o), mu.data_ptr(), ctypes.byref(h),
                                 _stream_ptr(stream)))
        self._h = h
        torch.cuda.synchronize()

    @property
    def nx(self) -> int:
        return self.d + self.d * (self.d + 1) // 2

    def step(self, n: int | None = None, stream=None):
        """Run the next n iterations (all that are left by default)."""
        if n is None:
            n = self.K - self.get_state(stream)["k"]
        check(lib().gl_vi_step(self._h, n, _stream_ptr(stream)))

    def get(self, stream=None) -> dict:
        """mean [d], Cholesky factor [d, d] and covariance [d, d] (cuda float64)."""
        d = self.d
        mu = torch.empty(d, dtype=torch.float64, device="cuda")
        chol = torch.empty((d, d), dtype=torch.float64, device="cuda")
        cov = torch.empty((d, d), dtype=torch.float64, device="cuda")
        check(lib().gl_vi_get(self._h, mu.data_ptr(), chol.data_ptr(), cov.data_ptr(),
                              _stream_ptr(stream)))
        return {"mu": mu, "chol": chol, "cov": cov}

    def sample(self, n: int, seed: int = 0, stream=None) -> torch.Tensor:
        z = torch.empty((n, self.d), dtype=torch.float64, device="cuda")
        check(lib().gl_vi_sample(self._h, n, seed, z.data_ptr(), _stream_ptr(stream)))
        return z

    def get_state(self, stream=None) -> dict:
        x, m, s = (torch.empty(self.nx, dtype=torch.float64, device="cuda") for _ in range(3))
        loss = torch.empty(self.K, dtype=torch.float64, device="cuda")
        k = ctypes.c_int()
        check(lib().gl_vi_get_state(self._h, x.data_ptr(), m.data_ptr(), s.data_ptr(),
                                    ctypes.byref(k), loss.data_ptr(), _stream_ptr(stream)))
        return {"x": x, "m": m, "s": s, "k": k.value, "loss": loss}

    def set_state(self, x, m, s, k: int, stream=None):
        x, m, s = (torch.as_tensor(t, dtype=torch.float64).reshape(self.nx).cuda().contiguous()
                   for t in (x, m, s))
        check(lib().gl_vi_set_state(self._h, x.data_ptr(), m.data_ptr(), s.data_ptr(), k,
                                    _stream_ptr(stream)))
        self._keep = (x, m, s)

    def close(self):
        if getattr(self, "_h", None):
            lib().gl_vi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------
# Preconditioned Hamiltonian Monte Carlo (Sec. 2.5)
# ------------------------------------------------------------------------------------------
class HMC:
    """`chains` HMC chains on the posterior of one system in unconstrained space, run by the
    library's kernels (one batched likelihood-gradient launch per leapfrog step).
    z0: optional [chains, d] unconstrained starts (e.g. the fit's best particle plus
    jitter; kept in FP64); inv_mass: optional inverse mass matrix M^-1, the diagonal [d] or the full
    [d, d] (the paper uses the variational posterior covariance of z); mass_chol: instead, the
    lower Cholesky factor of M^-1 (e.g. VI.get()["chol"]). adapt_mass: re-estimate M^-1 from
    the chains in three windows of the adaptation period (not in the paper)."""

    def __init__(self, model: Model, chains: int, n_leapfrog: int, n_burn: int, n_samples: int,
                 priors, step_size: float = 1e-2, target_accept: float = 0.75,
                 adapt_frac: float = 0.8, seed: int = 0, z0: torch.Tensor | None = None,
                 inv_mass=None, mass_chol=None, adapt_length: bool = False,
                 max_leapfrog: int = 1000, adapt_mass: bool = False, stream=None):
        assert len(priors) == model.d
        self.model, self.C = model, chains
        self.n_burn, self.n_samples = n_burn, n_samples
        self._pa = make_priors(priors)
        o = _lib.HmcOpts(chains=chains, n_leapfrog=n_leapfrog, n_burn=n_burn,
                         n_samples=n_samples, step_size=step_size, target_accept=target_accept,
                         adapt_frac=adapt_frac, seed=seed, priors=self._pa,
                         adapt_length=int(adapt_length), max_leapfrog=max_leapfrog,
                         adapt_mass=int(adapt_mass))
        if inv_mass is not None or mass_chol is not None:
            assert inv_mass is None or mass_chol is None
            im = np.ascontiguousarray(np.asarray(inv_mass if mass_chol is None else mass_chol,
                                                 np.float32))
            assert im.shape in ((model.d,), (model.d, model.d))
            self._im = (ctypes.c_float * im.size)(*im.ravel().tolist())
            o.inv_mass = self._im
            o.inv_mass_form = 2 if mass_chol is not None else int(im.ndim == 2)
        zp = None
        if z0 is not None:
            z0 = z0.to(torch.float64).contiguous()
            assert z0.is_cuda and z0.shape == (chains, model.d)
            zp = z0.data_ptr()
        h = ctypes.c_void_p()
        check(lib().gl_hmc_create(model._h, ctypes.byref(o), zp, ctypes.byref(h),
                                  _stream_ptr(stream)))
        self._h = h

    def run(self, n: int | None = None, stream=None):
        """Run the next n trajectories (all that are left by default)."""
        if n is None:
            n = self.n_burn + self.n_samples - self.info(stream)["trajectories"]
        check(lib().gl_hmc_run(self._h, n, _stream_ptr(stream)))

    def samples(self, stream=None) -> torch.Tensor:
        """[n_samples, chains, d] physical parameters of the recorded trajectories."""
        out = torch.empty((self.n_samples, self.C, self.model.d), dtype=torch.float32,
                          device="cuda")
        check(lib().gl_hmc_samples(self._h, out.data_ptr(), _stream_ptr(stream)))
        return out

    def info(self, stream=None) -> dict:
        r = _lib.HmcInfo()
        check(lib().gl_hmc_get_info(self._h, ctypes.byref(r), _stream_ptr(stream)))
        return {"step_size": r.step_size, "accept_mean": r.accept_mean,
                "trajectories": r.trajectories, "trajectory_length": r.trajectory_length,
                "mean_leapfrog": r.mean_leapfrog, "mass_updates": r.mass_updates}

    def mass_chol(self, stream=None) -> torch.Tensor:
        """[d, d] current lower Cholesky factor of M^-1 (FP32, cuda)."""
        out = torch.empty((self.model.d, self.model.d), dtype=torch.float32, device="cuda")
        check(lib().gl_hmc_get_mass(self._h, out.data_ptr(), _stream_ptr(stream)))
        return out

    def leapfrog(self, z: torch.Tensor, p: torch.Tensor, L: int, eps: float, stream=None):
        """L leapfrog steps from (z, p) (no accept): returns z_L (FP64), p_L (FP32) and
        log p~(z_L | I)."""
        z, p = z.to(torch.float64).contiguous(), p.to(torch.float32).contiguous()
        for t in (z, p):
            assert t.is_cuda and t.shape == (self.C, self.model.d)
        zo, po = torch.empty_like(z), torch.empty_like(p)
        lp = torch.empty(self.C, dtype=torch.float64, device="cuda")
        check(lib().gl_hmc_leapfrog(self._h, z.data_ptr(), p.data_ptr(), L, eps, zo.data_ptr(),
                                    po.data_ptr(), lp.data_ptr(), _stream_ptr(stream)))
        return zo, po, lp

    def close(self):
        if getattr(self, "_h", None):
            lib().gl_hmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------
# Continuous-batching server
# ------------------------------------------------------------------------------------------

class Server:
    """Fit server on the current GPU: gl_submit queues a system, gl_poll collects results."""

    def __init__(self, hbm_budget_bytes: int = 16 << 30, max_systems: int = 16,
                 steps_per_tick: int = 10, fill_subpixels: float = 0.0):
        o = _lib.ServerOpts(hbm_budget_bytes, max_systems, steps_per_tick, fill_subpixels)
        h = ctypes.c_void_p()
        check(lib().gl_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    def submit(self, spec, obs, P: int, K: int, priors, lr0=1e-2, lr1=1e-3, seed=0) -> int:
        """Queue one fit of the system `spec` (a synth.Spec-like object) with image `obs`."""
        desc, _keep = make_desc(spec.H, spec.W, spec.pix, spec.k, "epl" if spec.epl else "sie",
                                spec.shear, spec.lens_light, spec.nmax, spec.psf, obs,
                                spec.sigma_bkg, spec.t_exp, spec.gain)
        opts, _pa = make_fit_opts(P, K, priors, lr0, lr1, seed)
        t = ctypes.c_uint64()
        check(lib().gl_submit(self._h, ctypes.byref(desc), ctypes.byref(opts), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """None while pending, else the result dict (the ticket is then released)."""
        r = _lib.FitResult()
        rc = check(lib().gl_poll(self._h, ticket, ctypes.byref(r)))
        return None if rc == _lib.GL_PENDING else result_dict(r)

    def wait(self, ticket: int, timeout: float = 600.0, interval: float = 0.002) -> dict:
        import time
        t0 = time.monotonic()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.monotonic() - t0 > timeout:
                raise TimeoutError(f"ticket {ticket} not done after {timeout} s")
            time.sleep(interval)

    def stats(self) -> dict:
        s = _lib.ServerStats()
        check(lib().gl_server_get_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _lib.ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().gl_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
