"""Convergence diagnostics of MCMC output (Sec. 2.5 judges the HMC chains by the split
Gelman-Rubin statistic and the effective sample size).

Both follow Gelman et al., Bayesian Data Analysis (3rd ed.), Sec. 11.4-11.5: every chain is
split in half, so that m = 2 C sequences of n = N // 2 draws are compared.

    split R-hat: W = mean within-sequence variance, B / n = variance of the sequence means,
                 var+ = (n - 1) / n W + B / n, R-hat = sqrt(var+ / W)
    ESS:         m n / (1 + 2 sum_t rho_t), rho_t = 1 - (W - mean_j acov_j(t)) / var+,
                 summed over Geyer's initial positive sequence (pairs rho_{2k} + rho_{2k+1}
                 while positive, made monotone).

Inputs are host arrays [N, C] or [N, C, d] (draws, chains, parameters).
"""
from __future__ import annotations

import numpy as np


def _split(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, np.float64)
    if x.ndim == 2:
        x = x[:, :, None]
    n = x.shape[0] // 2
    if n < 2:
        raise ValueError("need at least 4 draws per chain")
    return np.concatenate([x[:n], x[x.shape[0] - n:]], axis=1)  # [n, 2C, d]


def _w_var(s: np.ndarray):
    n = s.shape[0]
    w = s.var(axis=0, ddof=1).mean(axis=0)
    b_n = s.mean(axis=0).var(axis=0, ddof=1)
    return w, (n - 1) / n * w + b_n


def split_rhat(x: np.ndarray) -> np.ndarray:
    """Split R-hat per parameter (shape [d], or a scalar for [N, C] input)."""
    s = _split(x)
    w, var = _w_var(s)
    r = np.sqrt(var / w)
    return r[0] if np.ndim(x) == 2 else r


def _autocov(s: np.ndarray) -> np.ndarray:
    """Autocovariance (biased, 1/n) of each sequence at lags 0..n-1: [n, m, d]."""
    n = s.shape[0]
    c = s - s.mean(axis=0)
    f = np.fft.rfft(c, n=2 * n, axis=0)
    return np.fft.irfft(f * np.conj(f), n=2 * n, axis=0)[:n] / n


def ess(x: np.ndarray) -> np.ndarray:
    """Effective sample size per parameter (shape [d], or a scalar for [N, C] input)."""
    s = _split(x)
    n, m, d = s.shape
    w, var = _w_var(s)
    acov = _autocov(s).mean(axis=1)  # [n, d]
    out = np.empty(d)
    for j in range(d):
        rho = 1.0 - (w[j] - acov[:, j]) / var[j]
        rho[0] = 1.0
        total, prev = 0.0, np.inf
        for t in range(0, n - 1, 2):
            pair = rho[t] + rho[t + 1]
            if pair <= 0:
                break
            pair = min(pair, prev)  # initial monotone sequence
            total += pair
            prev = pair
        tau = -1.0 + 2.0 * total  # = 1 + 2 sum_{t >= 1} rho_t
        out[j] = m * n / max(tau, 1.0 / np.log10(max(m * n, 10)))
    return out[0] if np.ndim(x) == 2 else out
