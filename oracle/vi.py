"""FP64 oracle of the variational-inference step (TEST INFRASTRUCTURE ONLY).

Sec. 2.4: a multivariate normal surrogate q = N(mu, Sigma) in unconstrained space is fitted
to the posterior p~(z | I_obs) by minimising the ELBO loss E_q[log q(z) - log p~(I_obs, z)]
with Adam; Sigma = L L^T through a Cholesky bijector: the d(d+1)/2 unconstrained values fill
the lower triangle of L row by row and the diagonal entries are exponentiated. Initial state
mu = the MAP point, Sigma = 1e-6 I; the learning rate rises from 0 to its maximum with a
quadratic polynomial schedule over the first iterations (Table 1: 0 -> 1e-3 over 500).

Gradient estimators. The default reads the gradient as the pathwise (reparameterisation)
form, an unbiased estimator of the same ELBO gradient. With z = mu + L eps, eps ~ N(0, I),
the loss is E[f(z)] - sum_i log L_ii - (d/2)(1 + log 2 pi), f = -log p~(z | I), so its
gradients are E[grad f] for mu, E[(grad f)_i eps_j] for the off-diagonal L_ij (i > j), and
L_ii E[(grad f)_i eps_i] - 1 for the log-diagonal entries. The score-function form the paper
prints (eq. elbo-grad), E[(log q(z) - log p~(I, z)) grad log q(z)], is the option
estimator="score". Either expectation is the mean over the n_VI draws of one iteration
(draws with a non-finite objective are left out of the mean).
"""
from __future__ import annotations

import math

import numpy as np

from . import rng
from .fit import adam_step, objective_and_grad


def n_chol(d: int) -> int:
    return d * (d + 1) // 2


def tril_index(d: int):
    """Row-major positions (i, j), i >= j, of the unconstrained vector's entries."""
    return np.tril_indices(d)


def cholesky_factor(v, d):
    """Cholesky bijector: vector [d(d+1)/2] -> lower-triangular L with exp on the diagonal."""
    L = np.zeros((d, d))
    L[tril_index(d)] = np.asarray(v, np.float64)
    L[np.diag_indices(d)] = np.exp(np.diag(L))
    return L


def cholesky_inverse(L):
    """Inverse of the bijector: lower-triangular L with a positive diagonal -> vector."""
    L = np.array(L, np.float64)
    L[np.diag_indices(L.shape[0])] = np.log(np.diag(L))
    return L[tril_index(L.shape[0])]


def learning_rate(k, lr_max, warmup, lr_final=0.0, K=0):
    """Polynomial schedule of power 2 from 0 to lr_max over `warmup` iterations (the form
    of a polynomial decay from init 0 to end lr_max): lr_max (1 - (1 - k/warmup)^2), then
    constant (Sec. 2.4's schedule). With lr_final > 0 (an option of this implementation, not
    the paper's), the rate after the warm-up falls geometrically from lr_max at k = warmup to
    lr_final at the last of K iterations, k = K - 1."""
    if k < warmup:
        frac = 1.0 - k / warmup
        return lr_max * (1.0 - frac * frac)
    span = K - 1 - warmup
    if lr_final <= 0 or span <= 0:
        return lr_max
    t = min(1.0, (k - warmup) / span)
    return lr_max * (lr_final / lr_max) ** t


def draws(seed, d, n, k):
    """The n x d standard normals of iteration k: counter (sample, parameter, k, tag)."""
    s = np.arange(n)[:, None]
    j = np.arange(d)[None, :]
    return rng.normals(seed, s, j, np.full((1, 1), k), 0x76690000)


def loss_and_grad_fn(fg, mu, v, eps):
    """ELBO loss and its gradient w.r.t. (mu, v) for a target given by fg(z) -> (f, grad f)
    rows, with the standard-normal draws eps [n, d]."""
    mu = np.asarray(mu, np.float64)
    d = mu.size
    L = cholesky_factor(v, d)
    z = mu[None, :] + eps @ L.T
    f, g = fg(z)
    ok = np.isfinite(f) & np.all(np.isfinite(g), axis=1)
    n = int(ok.sum())
    f, g, e = f[ok], g[ok], eps[ok]
    loss = f.sum() / n - np.log(np.diag(L)).sum() - 0.5 * d * (1.0 + math.log(2.0 * math.pi))
    g_mu = g.sum(axis=0) / n
    gL = g.T @ e / n  # [i, j] = mean of g_i eps_j
    gv = gL.copy()
    gv[np.diag_indices(d)] = np.diag(L) * np.diag(gL) - 1.0
    return loss, g_mu, gv[tril_index(d)], n


def log_q(z, mu, v):
    """log N(z; mu, L L^T) of rows z [n, d] under the surrogate (mu, v)."""
    mu = np.asarray(mu, np.float64)
    d = mu.size
    L = cholesky_factor(v, d)
    r = np.linalg.solve(L, (np.atleast_2d(z) - mu[None, :]).T).T  # L^-1 (z - mu)
    return (-0.5 * np.sum(r * r, axis=1) - np.log(np.diag(L)).sum()
            - 0.5 * d * math.log(2.0 * math.pi))


def score(z, mu, v):
    """Gradient of log q(z; mu, v) with respect to (mu, v) at fixed rows z [n, d] (the score
    of Sec. 2.4's eq. elbo-grad). With r = L^-1 (z - mu): d/d mu = L^-T r; d/d L_ij
    (i > j) = (L^-T r r^T)_ij; d/d log L_ii = L_ii (L^-T r r^T)_ii - 1. Returns [n, d] and
    [n, d(d+1)/2]."""
    mu = np.asarray(mu, np.float64)
    d = mu.size
    L = cholesky_factor(v, d)
    r = np.linalg.solve(L, (np.atleast_2d(z) - mu[None, :]).T).T
    u = np.linalg.solve(L.T, r.T).T  # rows L^-T r
    g_mu = u
    G = u[:, :, None] * r[:, None, :]  # [n, i, j] = (L^-T r)_i r_j
    ii = np.arange(d)
    G[:, ii, ii] = np.diag(L)[None, :] * G[:, ii, ii] - 1.0
    ti, tj = tril_index(d)
    return g_mu, G[:, ti, tj]


def loss_and_grad_score_fn(fg, mu, v, eps):
    """The ELBO gradient in the score-function form the paper prints (eq. elbo-grad):
    E_q[(log q(z) - log p~(I, z)) grad log q(z)], the expectation the mean over the draws
    z = mu + L eps whose objective is finite; log p~(I, z) = -f(z). Only f enters (no
    gradient of the target). Returns the loss (as loss_and_grad_fn), the gradient for mu and
    for v, and the number of draws used."""
    mu = np.asarray(mu, np.float64)
    d = mu.size
    L = cholesky_factor(v, d)
    z = mu[None, :] + eps @ L.T
    f, g = fg(z)
    ok = np.isfinite(f) & np.all(np.isfinite(g), axis=1)
    n = int(ok.sum())
    f, z = f[ok], z[ok]
    w = log_q(z, mu, v) + f
    s_mu, s_v = score(z, mu, v)
    loss = f.sum() / n - np.log(np.diag(L)).sum() - 0.5 * d * (1.0 + math.log(2.0 * math.pi))
    return loss, (w[:, None] * s_mu).sum(axis=0) / n, (w[:, None] * s_v).sum(axis=0) / n, n


def loss_and_grad(model, mu, v, eps, obs, priors):
    """loss_and_grad_fn on the lens posterior in unconstrained space."""
    def fg(z):
        f, g, _ = objective_and_grad(model, z, obs, priors)
        return f, g
    return loss_and_grad_fn(fg, mu, v, eps)


def vi_step(fg, mu, v, m, s, k, eps, lr, beta1=0.9, beta2=0.999, adam_eps=1e-8,
            estimator="pathwise"):
    """One VI iteration: the loss gradient at (mu, v) with draws eps (the pathwise or the
    score-function estimator), then Adam (moments m, s over the concatenated (mu, v)) at
    0-based step k with learning rate lr."""
    est = loss_and_grad_fn if estimator == "pathwise" else loss_and_grad_score_fn
    loss, g_mu, g_v, _ = est(fg, mu, v, eps)
    x = np.concatenate([mu, v])
    x, m, s = adam_step(x, m, s, np.concatenate([g_mu, g_v]), k, lr, beta1, beta2, adam_eps)
    d = len(mu)
    return x[:d], x[d:], m, s, loss
