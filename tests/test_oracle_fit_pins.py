"""Pins of the oracle's fit step (priors, bijectors, objective, Adam) to scipy and to finite
differences; Sec. 2.2 and Sec. 2.3 of arXiv:2202.07663. CPU only."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import fit
import synth
from tests.helpers import oracle_model

PRIORS = [
    {"family": fit.NORMAL, "mu": 0.1, "sigma": 0.2},
    {"family": fit.LOGNORMAL, "mu": math.log(1.25), "sigma": 0.4},
    {"family": fit.TRUNCNORMAL, "mu": 2.0, "sigma": 0.5, "lo": 1.0, "hi": 3.0},
    {"family": fit.UNIFORM, "lo": 0.5, "hi": 8.0},
]


def _theta_in_support(n, seed=0):
    rng = np.random.default_rng(seed)
    return np.stack([rng.normal(0.1, 0.3, n), np.exp(rng.normal(0.2, 0.5, n)),
                     rng.uniform(1.01, 2.99, n), rng.uniform(0.6, 7.9, n)], axis=1)


def test_log_prior_matches_scipy():
    th = _theta_in_support(50)
    got = fit.log_prior(th, PRIORS)
    ref = (stats.norm(0.1, 0.2).logpdf(th[:, 0])
           + stats.lognorm(s=0.4, scale=1.25).logpdf(th[:, 1])
           + stats.truncnorm((1 - 2) / 0.5, (3 - 2) / 0.5, loc=2, scale=0.5).logpdf(th[:, 2])
           + stats.uniform(0.5, 7.5).logpdf(th[:, 3]))
    np.testing.assert_allclose(got, ref, rtol=1e-12)


def test_bijector_round_trip_and_support():
    th = _theta_in_support(40, 1)
    z = fit.bijector_inverse(th, PRIORS)
    np.testing.assert_allclose(fit.bijector(z, PRIORS), th, rtol=1e-12)
    big = fit.bijector(np.array([[50.0, 5.0, 30.0, -30.0]]), PRIORS)[0]
    assert 1.0 < big[2] <= 3.0 and 0.5 <= big[3] < 8.0 and big[1] > 0


def test_log_det_jacobian_by_finite_differences():
    """Sec. 2.2: log|J| of the component-wise bijector, against central differences of g."""
    z = fit.bijector_inverse(_theta_in_support(30, 2), PRIORS)
    h = 1e-6
    fd = np.zeros(z.shape[0])
    for j in range(z.shape[1]):
        zp, zm = z.copy(), z.copy()
        zp[:, j] += h
        zm[:, j] -= h
        fd += np.log(np.abs((fit.bijector(zp, PRIORS)[:, j] - fit.bijector(zm, PRIORS)[:, j]) / (2 * h)))
    np.testing.assert_allclose(fit.log_det_jacobian(z, PRIORS), fd, rtol=1e-8, atol=1e-8)


def test_reparameterised_prior_is_a_density_in_z():
    """p~(z) = p(g(z)) |J| integrates to one over z (change of variables, Sec. 2.2)."""
    zs = np.linspace(-40, 40, 400001)
    for pr in PRIORS:
        z = np.zeros((zs.size, 1))
        z[:, 0] = zs
        dens = np.exp(fit.log_prior_z(z, [pr]))
        np.testing.assert_allclose(np.trapezoid(dens, zs), 1.0, rtol=1e-6)


def test_grad_log_prior_z_by_finite_differences():
    z = fit.bijector_inverse(_theta_in_support(20, 3), PRIORS)
    g = fit.grad_log_prior_z(z, PRIORS)
    h = 1e-6
    for j in range(z.shape[1]):
        zp, zm = z.copy(), z.copy()
        zp[:, j] += h
        zm[:, j] -= h
        fd = (fit.log_prior_z(zp, PRIORS) - fit.log_prior_z(zm, PRIORS)) / (2 * h)
        np.testing.assert_allclose(g[:, j], fd, rtol=1e-6, atol=1e-7)


def test_objective_gradient_by_finite_differences():
    spec = synth.Spec("f", 10, 12, 1, epl=True, lens_light=False, nmax=1,
                      psf=synth.moffat_psf(5, 0.15, 2.5), sigma_bkg=0.2, t_exp=100.0)
    m = oracle_model(spec)
    priors = prior_list_for(spec)
    truth = synth.draw_truth(spec, 4).astype(np.float64)
    obs = oracle.simulate(m, truth)[0] + np.random.default_rng(0).normal(0, 0.2, (10, 12))
    th = truth * (1 + 0.02 * np.random.default_rng(1).normal(size=truth.size))
    z = fit.bijector_inverse(th[None, :], priors)
    f0, gz, _ = fit.objective_and_grad(m, z, obs, priors)
    for j in range(z.shape[1]):
        h = 1e-6 * max(1.0, abs(z[0, j]))
        zp, zm = z.copy(), z.copy()
        zp[0, j] += h
        zm[0, j] -= h
        fd = (fit.objective_and_grad(m, zp, obs, priors)[0] -
              fit.objective_and_grad(m, zm, obs, priors)[0]) / (2 * h)
        assert abs(gz[0, j] - fd[0]) <= 1e-5 * (abs(fd[0]) + 1e-3 * np.abs(gz).max()), j


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g, bias correction makes m_hat = g and v_hat = g^2 at every
    step, so each update is exactly lr g / (|g| + eps)."""
    z = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    g = np.array([2.0, -0.5, 1e-3])
    total = np.zeros(3)
    for k in range(7):
        lr = fit.learning_rate(k, 300, 1e-2, 1e-3)
        total += lr * g / (np.abs(g) + 1e-8)
        z, m, v = fit.adam_step(z, m, v, g, k, lr)
    np.testing.assert_allclose(z, -total, rtol=1e-12)


def test_learning_rate_schedule_endpoints():
    """Table 1: 1e-2 -> 1e-3, linear over 300 iterations."""
    assert fit.learning_rate(0, 300, 1e-2, 1e-3) == 1e-2
    assert abs(fit.learning_rate(300, 300, 1e-2, 1e-3) - 1e-3) < 1e-18
    assert abs(fit.learning_rate(150, 300, 1e-2, 1e-3) - 5.5e-3) < 1e-15


def prior_list_for(spec):
    """Broadened prior of the parameter layout (the paper's blue distributions of eq.
    sim-dist where it lists them)."""
    from synth import fit_priors
    return fit_priors(spec)


def test_draw_starts_follow_the_prior():
    """Sec. 2.3: starts are draws from the prior. The oracle's draws (its own Philox and
    transforms) pass Kolmogorov-Smirnov tests against scipy's distributions for every
    family, and depend only on (seed, particle, parameter)."""
    z = fit.draw_starts(PRIORS, 99, 20000).astype(np.float64)
    th = fit.bijector(z, PRIORS)
    cdfs = [stats.norm(0.1, 0.2).cdf, stats.lognorm(s=0.4, scale=1.25).cdf,
            stats.truncnorm((1 - 2) / 0.5, (3 - 2) / 0.5, loc=2, scale=0.5).cdf,
            stats.uniform(0.5, 7.5).cdf]
    for j, cdf in enumerate(cdfs):
        assert stats.kstest(th[:, j], cdf).pvalue > 1e-3, j
    np.testing.assert_array_equal(fit.draw_starts(PRIORS, 99, 50), z[:50].astype(np.float32))
    assert not np.array_equal(fit.draw_starts(PRIORS, 98, 50), z[:50].astype(np.float32))
