"""Pins of the oracle's VI step (Sec. 2.4 of arXiv:2202.07663) and of its counter-based
generator: published known-answer vectors, closed forms on Gaussian targets, finite
differences on the lens posterior. CPU only."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import fit as ofit
from oracle import hmc as ohmc
from oracle import rng
from oracle import vi
import synth
from tests.helpers import load_workload, oracle_model


@pytest.mark.parametrize("ctr,key,want", [
    # known-answer vectors of Philox4x32-10 (Salmon et al. 2011, distributed with Random123)
    ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
    ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
    ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
])
def test_philox_known_answers(ctr, key, want):
    got = rng.philox4x32_10(np.array(ctr, np.uint64), np.array(key, np.uint64))
    assert [int(x) for x in got] == want


def test_uniforms_stay_inside_the_open_interval():
    assert rng.u01(0, 0) == 0.5 / 2.0 ** 52
    top = rng.u01(0xFFFFFFFF, 0xFFFFFFFF)
    assert top < 1.0 and top == (2.0 ** 52 - 0.5) / 2.0 ** 52
    assert rng.u01(0x40, 0) == 2.0 ** 26 * 0 + (1 * 2.0 ** 26 + 0.5) / 2.0 ** 52


def test_normals_are_standard_normal():
    x = rng.normals(7, np.arange(20000), 3, 5, 0x1234)
    assert stats.kstest(x, "norm").pvalue > 1e-3
    y = rng.normals(7, np.arange(20000), 4, 5, 0x1234)  # another counter word: independent
    assert abs(np.corrcoef(x, y)[0, 1]) < 0.03
    np.testing.assert_array_equal(x, rng.normals(7, np.arange(20000), 3, 5, 0x1234))


def test_cholesky_bijector():
    rng_ = np.random.default_rng(0)
    d = 5
    v = rng_.normal(size=vi.n_chol(d))
    L = vi.cholesky_factor(v, d)
    assert np.allclose(L, np.tril(L)) and np.all(np.diag(L) > 0)
    np.testing.assert_allclose(vi.cholesky_inverse(L), v, rtol=1e-14, atol=1e-14)
    np.testing.assert_array_equal(vi.cholesky_factor(np.zeros(vi.n_chol(d)), d), np.eye(d))
    # row-major fill of the lower triangle: entry 1 is L[1, 0], entry 2 is L[1, 1]
    e = np.zeros(vi.n_chol(d))
    e[1] = 0.7
    assert vi.cholesky_factor(e, d)[1, 0] == 0.7
    # the covariance it implies equals numpy's Cholesky round trip
    S = L @ L.T
    np.testing.assert_allclose(np.linalg.cholesky(S), L, rtol=1e-12, atol=1e-12)


def test_learning_rate_schedule():
    """Table 1: 0 -> 1e-3 over 500 iterations, quadratic."""
    assert vi.learning_rate(0, 1e-3, 500) == 0.0
    assert math.isclose(vi.learning_rate(250, 1e-3, 500), 0.75e-3)
    assert math.isclose(vi.learning_rate(500, 1e-3, 500), 1e-3)
    assert math.isclose(vi.learning_rate(900, 1e-3, 500), 1e-3)
    lr = [vi.learning_rate(k, 1.0, 10) for k in range(11)]
    assert all(b > a for a, b in zip(lr, lr[1:]))


def test_learning_rate_geometric_decay():
    """The optional decay after the warm-up: lr_max at the end of the warm-up, lr_final on
    the last iteration, their geometric mean half-way (a constant ratio per iteration), and
    the paper's constant rate when lr_final is 0."""
    K, w = 1001, 200
    assert math.isclose(vi.learning_rate(w, 3e-3, w, 1e-5, K), 3e-3)
    assert math.isclose(vi.learning_rate(K - 1, 3e-3, w, 1e-5, K), 1e-5)
    assert math.isclose(vi.learning_rate(w + 400, 3e-3, w, 1e-5, K), math.sqrt(3e-3 * 1e-5))
    r = [vi.learning_rate(k + 1, 3e-3, w, 1e-5, K) / vi.learning_rate(k, 3e-3, w, 1e-5, K)
         for k in range(w, K - 1)]
    assert max(r) - min(r) < 1e-12 and math.isclose(r[0], (1e-5 / 3e-3) ** (1 / 800))
    assert math.isclose(vi.learning_rate(199, 3e-3, w, 1e-5, K),
                        vi.learning_rate(199, 3e-3, w))
    assert vi.learning_rate(900, 3e-3, w, 0.0, K) == 3e-3
    assert vi.learning_rate(0, 3e-3, 0, 1e-5, K) == 3e-3


def _quadratic(A, c):
    def fg(z):
        u = z - c
        return 0.5 * np.einsum("ni,ij,nj->n", u, A, u), u @ A
    return fg


def _exact_moment_draws(d):
    """+- sqrt(d) e_i: zero mean and identity second moment exactly."""
    return np.concatenate([np.eye(d), -np.eye(d)]) * math.sqrt(d)


def test_gradient_and_loss_on_a_gaussian_target_with_exact_moment_draws():
    """f = (z - c)^T A (z - c) / 2: with draws of exactly zero mean and identity covariance
    the estimator is exact: grad_mu = A (mu - c), grad L_ij = (A L)_ij (i > j),
    grad log L_ii = L_ii (A L)_ii - 1, and the loss equals KL(q || N(c, A^-1)) up to the
    target's log normaliser."""
    rng_ = np.random.default_rng(1)
    d = 4
    B = rng_.normal(size=(d, d))
    A = B @ B.T / d + 0.5 * np.eye(d)
    c = rng_.normal(size=d)
    eps = _exact_moment_draws(d)
    logZ = 0.5 * d * math.log(2 * math.pi) - 0.5 * np.linalg.slogdet(A)[1]
    for trial in range(3):
        mu = rng_.normal(size=d)
        v = 0.3 * rng_.normal(size=vi.n_chol(d))
        L = vi.cholesky_factor(v, d)
        loss, g_mu, g_v, n = vi.loss_and_grad_fn(_quadratic(A, c), mu, v, eps)
        assert n == 2 * d
        np.testing.assert_allclose(g_mu, A @ (mu - c), rtol=1e-12, atol=1e-12)
        AL = A @ L
        want = AL.copy()
        want[np.diag_indices(d)] = np.diag(L) * np.diag(AL) - 1.0
        np.testing.assert_allclose(g_v, want[np.tril_indices(d)], rtol=1e-12, atol=1e-12)
        S = L @ L.T
        kl = 0.5 * (np.trace(A @ S) + (mu - c) @ A @ (mu - c) - d
                    - np.linalg.slogdet(A @ S)[1])
        assert math.isclose(loss, kl - logZ, rel_tol=1e-12, abs_tol=1e-12)


def test_log_q_is_the_normal_density():
    rng_ = np.random.default_rng(11)
    d = 5
    mu = rng_.normal(size=d)
    v = 0.4 * rng_.normal(size=vi.n_chol(d))
    L = vi.cholesky_factor(v, d)
    z = rng_.normal(size=(7, d)) + mu
    want = stats.multivariate_normal(mean=mu, cov=L @ L.T).logpdf(z)
    np.testing.assert_allclose(vi.log_q(z, mu, v), want, rtol=1e-12, atol=1e-12)


def test_score_matches_finite_differences_of_log_q():
    """The score of eq. elbo-grad (gradient of log q at fixed z) against central differences
    of log q in every entry of (mu, v)."""
    rng_ = np.random.default_rng(12)
    d = 4
    mu = rng_.normal(size=d)
    v = 0.4 * rng_.normal(size=vi.n_chol(d))
    z = rng_.normal(size=(3, d)) * 1.5 + mu
    s_mu, s_v = vi.score(z, mu, v)
    h = 1e-6
    for q in range(d + vi.n_chol(d)):
        x = np.concatenate([mu, v])
        xp, xm = x.copy(), x.copy()
        xp[q] += h
        xm[q] -= h
        fd = (vi.log_q(z, xp[:d], xp[d:]) - vi.log_q(z, xm[:d], xm[d:])) / (2 * h)
        got = s_mu[:, q] if q < d else s_v[:, q - d]
        np.testing.assert_allclose(got, fd, rtol=1e-6, atol=1e-7)


def test_score_has_zero_mean_under_exact_moment_draws():
    """E_q[grad log q] = 0: with draws of exactly zero mean and identity second moment the
    mean score vanishes in every entry."""
    rng_ = np.random.default_rng(13)
    d = 4
    mu = rng_.normal(size=d)
    v = 0.4 * rng_.normal(size=vi.n_chol(d))
    L = vi.cholesky_factor(v, d)
    z = mu[None, :] + _exact_moment_draws(d) @ L.T
    s_mu, s_v = vi.score(z, mu, v)
    np.testing.assert_allclose(s_mu.mean(axis=0), 0.0, atol=1e-12)
    np.testing.assert_allclose(s_v.mean(axis=0), 0.0, atol=1e-12)


def test_score_estimator_has_the_pathwise_expectation_on_a_gaussian_target():
    """Both estimators are unbiased for the same ELBO gradient: on f = (z - c)^T A (z - c)/2
    the score-function form over many draws lands on the closed form A (mu - c), (A L)_ij,
    L_ii (A L)_ii - 1 within a few of its standard errors."""
    rng_ = np.random.default_rng(14)
    d = 3
    B = rng_.normal(size=(d, d))
    A = B @ B.T / d + 0.5 * np.eye(d)
    c = rng_.normal(size=d)
    mu = rng_.normal(size=d)
    v = 0.3 * rng_.normal(size=vi.n_chol(d))
    L = vi.cholesky_factor(v, d)
    AL = A @ L
    want_v = AL.copy()
    want_v[np.diag_indices(d)] = np.diag(L) * np.diag(AL) - 1.0
    want = np.concatenate([A @ (mu - c), want_v[np.tril_indices(d)]])
    eps = rng_.normal(size=(400_000, d))
    _, g_mu, g_v, n = vi.loss_and_grad_score_fn(_quadratic(A, c), mu, v, eps)
    assert n == eps.shape[0]
    got = np.concatenate([g_mu, g_v])
    # per-draw terms give the standard error of the mean
    z = mu[None, :] + eps @ L.T
    f, _ = _quadratic(A, c)(z)
    w = vi.log_q(z, mu, v) + f
    s_mu, s_v = vi.score(z, mu, v)
    terms = w[:, None] * np.concatenate([s_mu, s_v], axis=1)
    se = terms.std(axis=0) / math.sqrt(n)
    assert np.all(np.abs(got - want) < 5 * se), (got - want) / se


def test_vi_converges_to_a_gaussian_target():
    """On a Gaussian target the optimum of the ELBO is the target itself: mu -> c and
    L L^T -> A^-1 (Adam on random draws: the iterates of the last 1000 steps are averaged
    to take out the optimiser's noise)."""
    rng_ = np.random.default_rng(2)
    d = 3
    B = rng_.normal(size=(d, d))
    A = B @ B.T + np.eye(d)
    c = rng_.normal(size=d)
    fg = _quadratic(A, c)
    mu = np.zeros(d)
    v = vi.cholesky_inverse(1e-3 * np.eye(d))
    m = np.zeros(d + vi.n_chol(d))
    s = np.zeros_like(m)
    mu_avg, cov_avg = np.zeros(d), np.zeros((d, d))
    for k in range(3000):
        eps = vi.draws(11, d, 200, k)
        mu, v, m, s, _ = vi.vi_step(fg, mu, v, m, s, k, eps, vi.learning_rate(k, 1e-2, 300))
        if k >= 2000:
            L = vi.cholesky_factor(v, d)
            mu_avg += mu / 1000
            cov_avg += L @ L.T / 1000
    cov = np.linalg.inv(A)
    sd = np.sqrt(np.diag(cov))
    assert np.abs((mu_avg - c) / sd).max() < 0.05
    np.testing.assert_allclose(cov_avg, cov, atol=0.03 * sd.max() ** 2)


@pytest.fixture(scope="module")
def lens():
    spec = synth.spec_c1()
    obs, truth = load_workload(spec.name)
    priors = synth.fit_priors(spec)
    fg = ohmc.lens_objective(oracle_model(spec), obs, priors)
    z_true = ofit.bijector_inverse(truth[None, :].astype(np.float64), priors)[0]
    z_mode, hess = ohmc.newton_mode(fg, z_true)
    return fg, z_mode, hess


def test_vi_gradient_matches_finite_differences_on_the_lens_posterior(lens):
    """With the draws held fixed the loss is a smooth function of (mu, v): its pathwise
    gradient equals central differences (catches transposed or misplaced L entries)."""
    fg, z_mode, hess = lens
    d = z_mode.size
    L0 = np.linalg.cholesky(np.linalg.inv(hess))
    rng_ = np.random.default_rng(3)
    mu = z_mode + 0.3 * L0 @ rng_.normal(size=d)
    v = vi.cholesky_inverse(L0 * np.exp(0.2 * rng_.normal(size=(d, 1))))
    eps = vi.draws(5, d, 64, 0)
    loss, g_mu, g_v, n = vi.loss_and_grad_fn(fg, mu, v, eps)
    assert n == 64
    x0 = np.concatenate([mu, v])
    g = np.concatenate([g_mu, g_v])
    scale = np.concatenate([np.sqrt(np.diag(np.linalg.inv(hess))), 0.02 * np.abs(v) + 1e-7])
    idx = list(range(d)) + list(d + np.flatnonzero(np.tril_indices(d)[0] == np.tril_indices(d)[1])) \
        + list(d + rng_.choice(vi.n_chol(d), 12, replace=False))
    for i in idx:
        h = 1e-3 * scale[i]
        xp, xm = x0.copy(), x0.copy()
        xp[i] += h
        xm[i] -= h
        fp = vi.loss_and_grad_fn(fg, xp[:d], xp[d:], eps)[0]
        fm = vi.loss_and_grad_fn(fg, xm[:d], xm[d:], eps)[0]
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-4 * (abs(g[i]) + np.abs(g[:d] * scale[:d]).max() / scale[i]), \
            (i, fd, g[i])
