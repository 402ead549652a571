"""Pins of the oracle's HMC pieces (Sec. 2.5 of arXiv:2202.07663) to closed forms and to
properties of the leapfrog integrator and of dual averaging. CPU only."""
import math

import numpy as np
import pytest

from oracle import fit as ofit
from oracle import hmc
import synth
from tests.helpers import load_workload, oracle_model


def _quadratic(a, c):
    a, c = np.asarray(a, np.float64), np.asarray(c, np.float64)

    def fg(z):
        u = z - c
        return 0.5 * np.sum(a * u * u, axis=-1), a * u
    return fg


def test_leapfrog_matches_the_linear_map_on_a_quadratic():
    """For f = sum a_j (z_j - c_j)^2 / 2 and inverse mass m_j, one leapfrog step is the linear
    map (u, p) -> (u (1 - e^2 a m / 2) + e m p, p (1 - e^2 a m / 2) - e a u (1 - e^2 a m / 4))
    per coordinate (u = z - c); L steps are its L-th matrix power."""
    rng = np.random.default_rng(0)
    d, C, L, eps = 5, 3, 7, 0.23
    a = rng.uniform(0.5, 3.0, d)
    c = rng.normal(size=d)
    m = rng.uniform(0.3, 2.0, d)
    z0 = rng.normal(size=(C, d))
    p0 = rng.normal(size=(C, d))
    zL, pL, f0, fL = hmc.leapfrog_fn(_quadratic(a, c), z0, p0, eps, L, m)
    for j in range(d):
        w = eps * eps * a[j] * m[j]
        step = np.array([[1 - w / 2, eps * m[j]], [-eps * a[j] * (1 - w / 4), 1 - w / 2]])
        ML = np.linalg.matrix_power(step, L)
        u_ref = ML[0, 0] * (z0[:, j] - c[j]) + ML[0, 1] * p0[:, j]
        p_ref = ML[1, 0] * (z0[:, j] - c[j]) + ML[1, 1] * p0[:, j]
        np.testing.assert_allclose(zL[:, j] - c[j], u_ref, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(pL[:, j], p_ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(f0, _quadratic(a, c)(z0)[0], rtol=1e-14)
    np.testing.assert_allclose(fL, _quadratic(a, c)(zL)[0], rtol=1e-14)


def test_leapfrog_matches_the_linear_map_with_a_dense_mass_matrix():
    """f = u^T A u / 2, M^-1 = S: one step maps (u, p) to
    ((I - e^2 S A / 2) u + e S p, (I - e^2 A S / 2) p - e A (I - e^2 S A / 4) u)."""
    rng = np.random.default_rng(5)
    d, L, eps = 4, 6, 0.3
    B = rng.normal(size=(d, d))
    A = B @ B.T / d + 0.5 * np.eye(d)
    B = rng.normal(size=(d, d))
    S = B @ B.T / d + 0.3 * np.eye(d)
    c = rng.normal(size=d)

    def fg(z):
        u = z - c
        return 0.5 * np.einsum("ci,ij,cj->c", u, A, u), u @ A
    z0, p0 = rng.normal(size=(3, d)), rng.normal(size=(3, d))
    zL, pL, _, _ = hmc.leapfrog_fn(fg, z0, p0, eps, L, S)
    I = np.eye(d)
    step = np.block([[I - eps ** 2 * S @ A / 2, eps * S],
                     [-eps * A @ (I - eps ** 2 * S @ A / 4), I - eps ** 2 * A @ S / 2]])
    x = np.concatenate([z0 - c, p0], axis=1) @ np.linalg.matrix_power(step, L).T
    np.testing.assert_allclose(zL - c, x[:, :d], rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(pL, x[:, d:], rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(hmc.kinetic(p0, S), 0.5 * np.einsum("ci,ij,cj->c", p0, S, p0))


def test_leapfrog_approaches_the_harmonic_oscillator():
    """As eps -> 0 at fixed time T = eps L the integrator follows Hamilton's equations:
    u(T) = u0 cos(w T) + p0 m sin(w T) / w with w^2 = a m (error O(eps^2))."""
    a, m, c = np.array([2.0]), np.array([0.5]), np.array([0.3])
    z0, p0 = np.array([[1.1]]), np.array([[-0.4]])
    T, w = 2.0, 1.0
    exact = (z0 - c) * math.cos(w * T) + p0 * m * math.sin(w * T) / w
    errs = []
    for L in (20, 40, 80):
        zL, _, _, _ = hmc.leapfrog_fn(_quadratic(a, c), z0, p0, T / L, L, m)
        errs.append(abs((zL - c - exact).item()))
    assert errs[-1] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


@pytest.fixture(scope="module")
def lens():
    spec = synth.spec_c1()
    obs, truth = load_workload(spec.name)
    priors = synth.fit_priors(spec)
    fg = hmc.lens_objective(oracle_model(spec), obs, priors)
    z_true = ofit.bijector_inverse(truth[None, :].astype(np.float64), priors)[0]
    z_mode, hess = hmc.newton_mode(fg, z_true)
    return fg, z_mode, hess


def test_laplace_mode_is_a_stationary_point_with_a_positive_definite_hessian(lens):
    fg, z_mode, hess = lens
    _, g = fg(z_mode[None, :])
    scale = np.sqrt(np.diag(hess))  # gradient in units of the posterior width
    assert np.abs(g[0] / scale).max() < 1e-6
    assert np.linalg.eigvalsh(hess).min() > 0
    # the FD Hessian agrees with finite differences of f itself along a random direction
    rng = np.random.default_rng(1)
    v = rng.normal(size=z_mode.size) / scale
    h = 0.3
    f = fg(np.stack([z_mode + h * v, z_mode, z_mode - h * v]))[0]
    np.testing.assert_allclose((f[0] - 2 * f[1] + f[2]) / h ** 2, v @ hess @ v, rtol=2e-2)


def _chains(lens, C, seed, spread=1.0):
    """Chains around the mode with the Laplace covariance as M^-1 (the paper's choice, with
    the variational covariance in its place), momenta drawn from N(0, M)."""
    fg, z_mode, hess = lens
    cov = np.linalg.inv(hess)
    rng = np.random.default_rng(seed)
    z = z_mode + spread * rng.normal(size=(C, z_mode.size)) @ np.linalg.cholesky(cov).T
    p = rng.normal(size=z.shape) @ np.linalg.cholesky(hess).T
    return fg, z, p, cov


def test_leapfrog_is_reversible_on_the_lens_posterior(lens):
    """Negating the momentum at the end and integrating again returns to the start."""
    fg, z, p, im = _chains(lens, 6, 2)
    z1, p1, _, _ = hmc.leapfrog_fn(fg, z, p, 0.3, 8, im)
    z2, p2, _, _ = hmc.leapfrog_fn(fg, z1, -p1, 0.3, 8, im)
    width = np.sqrt(np.diag(im))
    assert np.abs((z2 - z) / width).max() < 1e-6
    assert np.abs((p2 + p) * width).max() < 1e-6
    assert np.abs((z1 - z) / width).max() > 0.1  # it did move


def test_energy_error_is_second_order_on_the_lens_posterior(lens):
    """|H(z_L, p_L) - H(z_0, p_0)| over a fixed time eps L falls as eps^2."""
    fg, z, p, im = _chains(lens, 8, 3)
    errs = []
    for eps, L in ((0.2, 5), (0.1, 10), (0.05, 20)):
        zL, pL, f0, fL = hmc.leapfrog_fn(fg, z, p, eps, L, im)
        errs.append(np.abs(hmc.hamiltonian(fL, pL, im) - hmc.hamiltonian(f0, p, im)))
    r1, r2 = np.median(errs[0] / errs[1]), np.median(errs[1] / errs[2])
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, (r1, r2)
    assert np.median(errs[0]) < 0.5


def test_volume_is_preserved_on_the_lens_posterior(lens):
    """The leapfrog map is symplectic: the Jacobian of (z, p) -> (z_L, p_L) has determinant 1
    (by central differences, in coordinates scaled by the posterior width)."""
    fg, z, p, im = _chains(lens, 1, 4)
    s = np.sqrt(np.diag(im))
    d = z.shape[1]
    x0 = np.concatenate([z[0] / s, p[0] * s])
    h = 1e-4
    pts = np.repeat(x0[None, :], 4 * d, axis=0)
    for i in range(2 * d):
        pts[2 * i, i] += h
        pts[2 * i + 1, i] -= h
    zL, pL, _, _ = hmc.leapfrog_fn(fg, pts[:, :d] * s, pts[:, d:] / s, 0.2, 4, im)
    y = np.concatenate([zL / s, pL * s], axis=1)
    J = (y[0::2] - y[1::2]).T / (2 * h)
    sign, logdet = np.linalg.slogdet(J)
    assert sign > 0 and abs(logdet) < 1e-4


def test_accept_probability():
    h0 = np.array([1.0, 1.0, 1.0, 0.0, 0.0])
    h1 = np.array([0.5, 1.0, 3.0, np.inf, np.nan])
    np.testing.assert_allclose(hmc.accept_probability(h0, h1), [1.0, 1.0, math.exp(-2.0), 0, 0])


@pytest.mark.parametrize("target", [0.6, 0.75, 0.9])
def test_dual_averaging_reaches_the_target_acceptance(target):
    """Driven by a deterministic acceptance curve a(eps) = 1 / (1 + (eps / e*)^4), the averaged
    step size converges to the eps with a(eps) = target."""
    e_star = 0.37
    da = hmc.DualAveraging(1.0, target=target)
    for _ in range(3000):
        da.update(1.0 / (1.0 + (da.eps / e_star) ** 4))
    want = e_star * ((1.0 - target) / target) ** 0.25
    assert abs(da.final() / want - 1.0) < 0.02


def test_dual_averaging_first_steps():
    """m = 1: H_1 = (delta - a_1) / (1 + t0); log eps_1 = mu - H_1 / gamma; eps_bar_1 = eps_1.
    With the acceptance at the target the step size jumps to 10 eps_0 (mu = log 10 eps_0)."""
    da = hmc.DualAveraging(0.1, target=0.75)
    assert math.isclose(da.update(0.75), 1.0, rel_tol=1e-12)
    assert math.isclose(da.final(), 1.0, rel_tol=1e-12)
    da = hmc.DualAveraging(0.1, target=0.75)
    e1 = da.update(0.0)  # too large a step: shrink
    assert math.isclose(math.log(e1), math.log(1.0) - 0.75 / 11 / 0.05, rel_tol=1e-12)


def test_van_der_corput_sequence():
    assert [hmc.halton(k) for k in range(1, 9)] == [0.5, 0.25, 0.75, 0.125, 0.625, 0.375,
                                                     0.875, 0.0625]


# On a standard normal target with identity mass the flow is a rotation: with t = u T,
# |z'|^2 - |z|^2 = sin^2 t (|p|^2 - |z|^2) + sin 2t z.p, so ChEES(t) = d sin^2 t, and the
# jittered criterion E_u[d sin^2(u T)] = d (1/2 - sin 2T / (4T)) peaks where tan 2T = 2T.
T_STAR = 4.493409457909064 / 2.0  # first positive root of tan x = x, halved


@pytest.mark.parametrize("scale,inv_mass,want", [
    (1.0, 1.0, T_STAR),          # standard normal, identity mass
    (3.0, 1.0, 3.0 * T_STAR),    # the optimum scales with the target's width
    (3.0, 9.0, T_STAR),          # ... and is T* again once M^-1 whitens the target
])
def test_chees_adaptation_finds_the_optimal_length(scale, inv_mass, want):
    d = 4
    fg = lambda z: (0.5 * np.sum(z * z, axis=1) / scale ** 2, z / scale ** 2)
    rng = np.random.default_rng(1)
    eps = 0.05 * scale / math.sqrt(inv_mass)
    ad, z = hmc.chees_run(fg, scale * rng.standard_normal((512, d)), np.full(d, inv_mass),
                          eps, 0.5 * want, 600, rng)
    assert abs(ad.final() / want - 1.0) < 0.08, (ad.final(), want)
    assert abs(np.std(z) / scale - 1.0) < 0.05  # still samples the target


def test_mass_windows_schedule():
    """Initial buffer 15%, windows 1 : 2 : 4, terminal buffer 10%, none below 7 trajectories
    of windows (values worked by hand)."""
    assert hmc.mass_windows(200) == [30, 51, 94, 180]  # 30 + 150: 21, 43, 86
    assert hmc.mass_windows(800) == [120, 205, 377, 720]  # 120 + 600: 85, 172, 343
    assert hmc.mass_windows(20) == [3, 5, 9, 18]
    assert hmc.mass_windows(9) == [1, 2, 4, 9]  # span 8 (the buffers floor to 1 and 0)
    assert hmc.mass_windows(7) == []  # span 7 - 1 - 0 = 6
    assert hmc.mass_windows(8) == [1, 2, 4, 8]  # span 7
    assert hmc.mass_windows(0) == [] and hmc.mass_windows(4) == []
    for n in range(8, 2000, 37):
        b = hmc.mass_windows(n)
        lengths = np.diff(b)
        assert b[0] == int(0.15 * n) and b[-1] == n - int(0.10 * n)
        assert np.all(lengths >= 0) and lengths[2] >= lengths[1] >= lengths[0]


def test_window_inv_mass():
    """The sample covariance (numpy's, divisor n - 1) on the diagonal, its off-diagonal
    scaled by n / (n + 5); positive definite even from fewer samples than dimensions; close
    to the generating covariance for a large Gaussian sample."""
    rng = np.random.default_rng(3)
    d = 6
    A = rng.normal(size=(d, d))
    cov = A @ A.T + 0.1 * np.eye(d)
    Z = rng.multivariate_normal(np.arange(d), cov, size=40)
    S = np.cov(Z.T)
    M = hmc.window_inv_mass(Z)
    np.testing.assert_allclose(np.diag(M), np.diag(S), rtol=1e-12)
    off = ~np.eye(d, dtype=bool)
    np.testing.assert_allclose(M[off], S[off] * 40 / 45, rtol=1e-12)
    assert np.all(np.linalg.eigvalsh(hmc.window_inv_mass(Z[:4])) > 0)
    big = rng.multivariate_normal(np.zeros(d), cov, size=200000)
    np.testing.assert_allclose(hmc.window_inv_mass(big), cov, atol=0.02 * np.abs(cov).max())
