"""FP64 oracle of the preconditioned Hamiltonian Monte Carlo step (TEST INFRASTRUCTURE ONLY).

Sec. 2.5: sampling in unconstrained space with target log p~(z | I_obs) = log L(g(z)) +
log p~(z); momenta p ~ N(0, M), where the paper takes M as the inverse of the variational
posterior covariance (here inv_mass = M^-1, diagonal or dense);
Hamiltonian H = -log p~(z | I) + p^T M^-1 p / 2; leapfrog integration with step eps and
L steps; Metropolis acceptance min(1, exp(H0 - H1)). The step size is tuned by the dual
averaging of Hoffman & Gelman (2014, Sec. 3.2) towards a target acceptance probability
(0.75 in the paper) during the first part of burn-in. The optional windowed re-estimation of
M^-1 (not in the paper) is given by its window schedule and estimator (mass_windows,
window_inv_mass).
"""
from __future__ import annotations

import math

import numpy as np

from .fit import objective_and_grad


def _apply_inv_mass(inv_mass, p):
    """M^-1 p for rows p: inv_mass is the diagonal [d] or the full symmetric matrix [d, d]."""
    inv_mass = np.asarray(inv_mass, np.float64)
    if inv_mass.ndim == 2:
        return p @ inv_mass.T
    return inv_mass * p


def kinetic(p, inv_mass):
    """p^T M^-1 p / 2 per row."""
    p = np.asarray(p, np.float64)
    return 0.5 * np.sum(p * _apply_inv_mass(inv_mass, p), axis=-1)


def leapfrog_fn(fg, z, p, eps, L, inv_mass):
    """L leapfrog steps of size eps for H = f(z) + p^T M^-1 p / 2, where fg(z) returns f and
    its gradient (rows are independent chains) and M^-1 is diagonal ([d]) or dense ([d, d]):
    a half kick, then L drifts separated by full kicks, and a final half kick.
    Returns z_L, p_L, f(z_0), f(z_L)."""
    z = np.array(z, np.float64)
    p = np.array(p, np.float64)
    f0, gf = fg(z)
    f = f0
    p = p - 0.5 * eps * gf
    for step in range(L):
        z = z + eps * _apply_inv_mass(inv_mass, p)
        f, gf = fg(z)
        p = p - (eps if step < L - 1 else 0.5 * eps) * gf
    return z, p, f0, f


def leapfrog(model, z, p, eps, L, obs, priors, inv_mass):
    """Leapfrog on the lens posterior in unconstrained space: f = -log p~(z | I)."""
    return leapfrog_fn(lens_objective(model, obs, priors), z, p, eps, L, inv_mass)


def hamiltonian(f, p, inv_mass):
    return f + kinetic(p, inv_mass)


def accept_probability(h0, h1):
    dh = np.asarray(h0) - np.asarray(h1)
    with np.errstate(over="ignore", invalid="ignore"):
        a = np.minimum(1.0, np.exp(dh))
    return np.where(np.isfinite(a), a, 0.0)


class DualAveraging:
    """Hoffman & Gelman (2014), Sec. 3.2: H_m = (1 - 1/(m + t0)) H_{m-1} + (delta - a_m)/(m + t0);
    log eps_m = mu - sqrt(m)/gamma H_m; log eps_bar_m = m^-kappa log eps_m
    + (1 - m^-kappa) log eps_bar_{m-1}; mu = log(10 eps_0)."""

    def __init__(self, eps0, target=0.75, gamma=0.05, t0=10.0, kappa=0.75):
        self.mu = math.log(10.0 * eps0)
        self.target, self.gamma, self.t0, self.kappa = target, gamma, t0, kappa
        self.h = 0.0
        self.log_eps_bar = 0.0
        self.m = 0
        self.eps = eps0

    def update(self, accept):
        self.m += 1
        m = self.m
        w = 1.0 / (m + self.t0)
        self.h = (1.0 - w) * self.h + w * (self.target - accept)
        log_eps = self.mu - math.sqrt(m) / self.gamma * self.h
        log_eps = min(max(log_eps, self.mu - 40.0), self.mu + 40.0)  # no underflow to 0
        eta = m ** (-self.kappa)
        self.log_eps_bar = eta * log_eps + (1.0 - eta) * self.log_eps_bar
        self.eps = math.exp(log_eps)
        return self.eps

    def final(self):
        return math.exp(self.log_eps_bar)


def hessian_fd(fg, z, h=1e-4):
    """Hessian of f at one point z [d] by central differences of the exact gradient,
    symmetrised. All 2 d perturbed points go through fg as one batch."""
    z = np.asarray(z, np.float64)
    d = z.size
    pts = np.repeat(z[None, :], 2 * d, axis=0)
    pts[np.arange(d), np.arange(d)] += h
    pts[d + np.arange(d), np.arange(d)] -= h
    _, g = fg(pts)
    hess = (g[:d] - g[d:]) / (2 * h)
    return 0.5 * (hess + hess.T)


def newton_mode(fg, z0, iters=6, h=1e-4):
    """Posterior mode by Newton's method on f from a start in its basin; returns the mode
    and the Hessian there (the Laplace approximation's precision matrix)."""
    z = np.asarray(z0, np.float64).copy()
    for _ in range(iters):
        _, g = fg(z[None, :])
        hess = hessian_fd(fg, z, h)
        z = z - np.linalg.solve(hess, g[0])
    return z, hessian_fd(fg, z, h)


def lens_objective(model, obs, priors):
    """fg(z) -> (f, d f / d z) for the lens posterior in unconstrained space."""
    def fg(zz):
        f, g, _ = objective_and_grad(model, zz, obs, priors)
        return f, g
    return fg


# ------------------------------------------------------------------------------------------
# Trajectory-length adaptation (Hoffman, Radul & Sountsov 2021, "An adaptive MCMC scheme
# for setting trajectory lengths in Hamiltonian Monte Carlo"): the length T of every
# trajectory is jittered, t = u T with u from a low-discrepancy sequence shared by all chains,
# and log T follows stochastic gradient ascent on the ChEES criterion
#   ChEES(T) = E[(|z' - E z'|^2 - |z - E z|^2)^2] / 4
# (change in the expected squared jump distance), whose gradient estimate per chain i is
#   g_i = (|z'_i - zbar'|^2 - |z_i - zbar|^2) ((z'_i - zbar') . M^-1 p'_i) u,
# averaged over chains with the acceptance probabilities as weights; means are over chains.
# ------------------------------------------------------------------------------------------

def halton(k, base=2):
    """The k-th (k >= 1) element of the van der Corput sequence in the given base."""
    f, r = 1.0, 0.0
    while k > 0:
        f /= base
        r += f * (k % base)
        k //= base
    return r


def chees_gradient(z0, z1, p1, inv_mass, accept, u):
    """Acceptance-weighted ChEES gradient estimate w.r.t. T from the chains' starts z0,
    proposals z1 and end momenta p1 (rows are chains)."""
    z0, z1 = np.asarray(z0, np.float64), np.asarray(z1, np.float64)
    c0, c1 = z0 - z0.mean(axis=0), z1 - z1.mean(axis=0)
    v1 = _apply_inv_mass(inv_mass, np.asarray(p1, np.float64))
    diff = np.sum(c1 * c1, axis=1) - np.sum(c0 * c0, axis=1)
    g = diff * np.sum(c1 * v1, axis=1) * u
    a = np.asarray(accept, np.float64)
    return float(np.sum(a * g) / max(np.sum(a), 1e-300))


class LengthAdaptation:
    """Adam (beta1 = 0, beta2 = 0.95, as in the reference implementation the paper uses)
    ascending the ChEES gradient in log T, with rate 0.025 and the gradient taken w.r.t.
    log T (g T); the averaged length follows the dual-averaging weights m^-kappa."""

    def __init__(self, T0, rate=0.025, beta2=0.95, eps=1e-8, kappa=0.75):
        self.logT = math.log(T0)
        self.rate, self.beta2, self.eps, self.kappa = rate, beta2, eps, kappa
        self.v = 0.0
        self.m = 0
        self.log_bar = self.logT

    def update(self, grad_T):
        self.m += 1
        g = grad_T * math.exp(self.logT)  # d / d log T
        self.v = self.beta2 * self.v + (1.0 - self.beta2) * g * g
        vhat = self.v / (1.0 - self.beta2 ** self.m)
        self.logT += self.rate * g / (math.sqrt(vhat) + self.eps)
        eta = self.m ** (-self.kappa)
        self.log_bar = eta * self.logT + (1.0 - eta) * self.log_bar
        return math.exp(self.logT)

    def final(self):
        return math.exp(self.log_bar)


def chees_run(fg, z, inv_mass, eps, T0, n_iter, rng, target=None):
    """A plain HMC run with ChEES length adaptation at a fixed step size (for pins): every
    iteration draws momenta, integrates for ceil(u T / eps) leapfrog steps, accepts, and
    updates T. Returns the adaptation state and the final positions."""
    z = np.array(z, np.float64)
    inv_mass = np.asarray(inv_mass, np.float64)
    chol_m = np.linalg.cholesky(np.linalg.inv(inv_mass)) if inv_mass.ndim == 2 else None
    ad = LengthAdaptation(T0)
    T = T0
    for k in range(1, n_iter + 1):
        n = rng.standard_normal(z.shape)
        p = n @ chol_m.T if chol_m is not None else n / np.sqrt(inv_mass)
        u = halton(k)
        L = max(1, int(math.ceil(u * T / eps)))
        z1, p1, f0, f1 = leapfrog_fn(fg, z, p, eps, L, inv_mass)
        acc = accept_probability(hamiltonian(f0, p, inv_mass), hamiltonian(f1, p1, inv_mass))
        T = ad.update(chees_gradient(z, z1, p1, inv_mass, acc, u))
        keep = rng.uniform(size=len(z)) < acc
        z = np.where(keep[:, None], z1, z)
    return ad, z


def mass_windows(n_adapt):
    """Window boundaries of the optional mass adaptation (not in the paper; Stan's windowed
    scheme): an initial buffer of floor(0.15 n_adapt) trajectories, three windows of lengths in
    the ratio 1 : 2 : 4 (cut at floor(span / 7) and floor(3 span / 7)), a terminal buffer of
    floor(0.10 n_adapt); window k holds the positions after trajectories [b[k], b[k + 1]).
    No windows when they would span fewer than 7 trajectories."""
    b0, b1 = int(0.15 * n_adapt), int(0.10 * n_adapt)
    span = n_adapt - b0 - b1
    if span < 7:
        return []
    return [b0, b0 + span // 7, b0 + (3 * span) // 7, b0 + span]


def window_inv_mass(Z):
    """M^-1 estimated from a window's positions Z [n, d]: the sample covariance (divisor
    n - 1) with its off-diagonal entries scaled by n / (n + 5), i.e. shrunk towards its
    diagonal."""
    Z = np.asarray(Z, np.float64)
    n = Z.shape[0]
    dev = Z - Z.mean(axis=0)
    S = dev.T @ dev / (n - 1)
    w = n / (n + 5.0)
    return w * S + (1.0 - w) * np.diag(np.diag(S))
