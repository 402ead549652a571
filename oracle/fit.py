"""FP64 oracle of the multi-start fit step (TEST INFRASTRUCTURE ONLY).

Follows Sec. 2.2 (bijectors, Jacobian-corrected prior) and Sec. 2.3 (objective and Adam):
  * bijector per parameter, chosen by its prior family: normal -> identity, log-normal ->
    exp (eq. exp), truncated normal and uniform on (lo, hi) -> the sigmoid map
    lo + (hi - lo) / (1 + e^-z) (eq. sigmoid);
  * log p~(z) = log p(g(z)) + log |J| (Jacobian-corrected prior), likelihood unchanged;
  * objective f(z) = -(log L(g(z)) + log p~(z)) (eq. obj-fun);
  * Adam (Kingma & Ba) with learning rate lr0 -> lr1 linear over K steps (Table 1).
Arrays are [P, d] in z (unconstrained) space; priors are a list of dicts
{"family": 0..3, "mu", "sigma", "lo", "hi"} with the gl.h family codes.
"""
from __future__ import annotations

import math

import numpy as np

from . import loglik_grad

NORMAL, LOGNORMAL, TRUNCNORMAL, UNIFORM = 0, 1, 2, 3
_LOG_SQRT_2PI = 0.5 * math.log(2 * math.pi)


def _std_normal_cdf(x):
    return 0.5 * math.erfc(-x / math.sqrt(2.0))


def bijector(z, priors):
    """theta = g(z), component-wise."""
    z = np.asarray(z, np.float64)
    th = np.empty_like(z)
    for j, pr in enumerate(priors):
        f = pr["family"]
        if f == LOGNORMAL:
            th[..., j] = np.exp(z[..., j])
        elif f in (TRUNCNORMAL, UNIFORM):
            th[..., j] = pr["lo"] + (pr["hi"] - pr["lo"]) / (1.0 + np.exp(-z[..., j]))
        else:
            th[..., j] = z[..., j]
    return th


def bijector_inverse(theta, priors):
    theta = np.asarray(theta, np.float64)
    z = np.empty_like(theta)
    for j, pr in enumerate(priors):
        f = pr["family"]
        if f == LOGNORMAL:
            z[..., j] = np.log(theta[..., j])
        elif f in (TRUNCNORMAL, UNIFORM):
            u = (theta[..., j] - pr["lo"]) / (pr["hi"] - pr["lo"])
            z[..., j] = np.log(u) - np.log1p(-u)
        else:
            z[..., j] = theta[..., j]
    return z


def log_det_jacobian(z, priors):
    """log |d g / d z| summed over components."""
    z = np.asarray(z, np.float64)
    out = np.zeros(z.shape[:-1])
    for j, pr in enumerate(priors):
        f = pr["family"]
        if f == LOGNORMAL:
            out += z[..., j]
        elif f in (TRUNCNORMAL, UNIFORM):
            # log s = -softplus(-z), log(1 - s) = -softplus(z), s = 1 / (1 + e^-z)
            out += (math.log(pr["hi"] - pr["lo"]) - np.logaddexp(0.0, -z[..., j])
                    - np.logaddexp(0.0, z[..., j]))
    return out


def log_prior(theta, priors):
    """log p(theta) = sum of the independent 1-D log densities (Sec. 2.1.2)."""
    theta = np.asarray(theta, np.float64)
    out = np.zeros(theta.shape[:-1])
    for j, pr in enumerate(priors):
        x, f = theta[..., j], pr["family"]
        mu, sg = pr.get("mu", 0.0), pr.get("sigma", 1.0)
        if f == NORMAL:
            out += -0.5 * ((x - mu) / sg) ** 2 - math.log(sg) - _LOG_SQRT_2PI
        elif f == LOGNORMAL:
            out += -0.5 * ((np.log(x) - mu) / sg) ** 2 - math.log(sg) - _LOG_SQRT_2PI - np.log(x)
        elif f == TRUNCNORMAL:
            Z = _std_normal_cdf((pr["hi"] - mu) / sg) - _std_normal_cdf((pr["lo"] - mu) / sg)
            out += -0.5 * ((x - mu) / sg) ** 2 - math.log(sg) - _LOG_SQRT_2PI - math.log(Z)
        else:
            out += -math.log(pr["hi"] - pr["lo"])
    return out


def log_prior_z(z, priors):
    """log p~(z) = log p(g(z)) + log|J(z)|."""
    return log_prior(bijector(z, priors), priors) + log_det_jacobian(z, priors)


def _dtheta_dz(z, priors):
    z = np.asarray(z, np.float64)
    out = np.ones_like(z)
    for j, pr in enumerate(priors):
        f = pr["family"]
        if f == LOGNORMAL:
            out[..., j] = np.exp(z[..., j])
        elif f in (TRUNCNORMAL, UNIFORM):
            s = 1.0 / (1.0 + np.exp(-z[..., j]))
            out[..., j] = (pr["hi"] - pr["lo"]) * s * (1.0 - s)
    return out


def grad_log_prior_z(z, priors):
    """d log p~ / d z, written out per family."""
    z = np.asarray(z, np.float64)
    g = np.zeros_like(z)
    th = bijector(z, priors)
    for j, pr in enumerate(priors):
        f = pr["family"]
        mu, sg = pr.get("mu", 0.0), pr.get("sigma", 1.0)
        if f in (NORMAL, LOGNORMAL):
            # log-normal with the exp bijector is a normal density in z
            g[..., j] = -(z[..., j] - mu) / sg ** 2
        elif f == TRUNCNORMAL:
            s = 1.0 / (1.0 + np.exp(-z[..., j]))
            g[..., j] = (-(th[..., j] - mu) / sg ** 2 * (pr["hi"] - pr["lo"]) * s * (1 - s)
                         + 1.0 - 2.0 * s)
        else:
            s = 1.0 / (1.0 + np.exp(-z[..., j]))
            g[..., j] = 1.0 - 2.0 * s
    return g


def objective_and_grad(model, z, obs, priors):
    """f(z) and d f / d z for rows of z (eq. obj-fun), with the oracle's exact log L gradient."""
    th = bijector(z, priors)
    ll, gth = loglik_grad(model, th, obs)
    lp = log_prior_z(z, priors)
    gz = -(gth * _dtheta_dz(z, priors) + grad_log_prior_z(z, priors))
    return -(ll + lp), gz, ll


def learning_rate(step, K, lr0, lr1):
    """Linear decay from lr0 to lr1 over K steps; `step` counts from 0 (Table 1)."""
    return lr0 + (lr1 - lr0) * min(step, K) / K


def adam_step(z, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) at 0-based step `step`."""
    t = step + 1
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return z - lr * mhat / (np.sqrt(vhat) + eps), m, v


def draw_starts(priors, seed, P):
    """The P multi-start points in unconstrained space (Sec. 2.3: starts drawn from the
    prior), from the counter-based generator of oracle.rng with counter
    (particle, parameter, 0x6c656e73, 0): u1, u2 from the two word pairs; normal and
    log-normal priors take the Box-Muller normal, truncated normals the inverse CDF at
    Phi(a) + u1 (Phi(b) - Phi(a)), uniforms u1; bounded families map through the logit of
    the position within (lo, hi) clipped to [1e-7, 1 - 1e-7]. Prior parameters are used at
    float32, the precision the library stores them in; the result is rounded to float32."""
    from scipy.special import erfinv
    from . import rng
    d = len(priors)
    p_idx = np.arange(P, dtype=np.uint64)[:, None]
    j_idx = np.arange(d, dtype=np.uint64)[None, :]
    ctr = np.stack(np.broadcast_arrays(p_idx, j_idx, np.uint64(0x6C656E73), np.uint64(0)), axis=-1)
    w = rng.philox4x32_10(ctr, rng.split_seed(seed))
    u1, u2 = rng.u01(w[..., 0], w[..., 1]), rng.u01(w[..., 2], w[..., 3])
    out = np.empty((P, d))
    f32 = lambda x: float(np.float32(x))
    for j, pr in enumerate(priors):
        fam = pr["family"]
        mu, sg = f32(pr.get("mu", 0.0)), f32(pr.get("sigma", 1.0))
        lo, hi = f32(pr.get("lo", 0.0)), f32(pr.get("hi", 0.0))
        if fam in (NORMAL, LOGNORMAL):
            n = np.sqrt(-2.0 * np.log(u1[:, j])) * np.cos(2.0 * np.pi * u2[:, j])
            out[:, j] = mu + sg * n
            continue
        if fam == TRUNCNORMAL:
            # the standardised bounds in float32 arithmetic, as the library forms them
            za = float((np.float32(lo) - np.float32(mu)) / np.float32(sg))
            zb = float((np.float32(hi) - np.float32(mu)) / np.float32(sg))
            a, b = _std_normal_cdf(za), _std_normal_cdf(zb)
            x = mu + sg * math.sqrt(2.0) * erfinv(2.0 * (a + u1[:, j] * (b - a)) - 1.0)
            u = (x - lo) / (hi - lo)
        else:
            u = u1[:, j]
        u = np.clip(u, 1e-7, 1.0 - 1e-7)
        out[:, j] = np.log(u) - np.log1p(-u)
    return out.astype(np.float32)
