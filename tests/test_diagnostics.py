"""Pins of the MCMC diagnostics (split R-hat, ESS; Sec. 2.5 reports both for the HMC chains)
to closed forms and to brute-force sums. CPU only."""
import numpy as np
import pytest

from paper_2202_07663_amd import diagnostics as dg


def _ar1(rho, N, C, seed):
    rng = np.random.default_rng(seed)
    x = np.empty((N, C))
    x[0] = rng.normal(size=C)
    e = rng.normal(size=(N, C)) * np.sqrt(1 - rho ** 2)
    for t in range(1, N):
        x[t] = rho * x[t - 1] + e[t]
    return x


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9])
def test_ess_of_an_ar1_process(rho):
    """Stationary AR(1) with coefficient rho: integrated autocorrelation time
    tau = (1 + rho) / (1 - rho), so ESS = N C / tau."""
    N, C = 20000, 8
    x = _ar1(rho, N, C, 1)
    want = N * C * (1 - rho) / (1 + rho)
    assert abs(dg.ess(x) / want - 1) < 0.1


def test_ess_and_rhat_are_per_parameter():
    x = np.stack([_ar1(0.0, 4000, 4, 2), _ar1(0.8, 4000, 4, 3)], axis=-1)
    e = dg.ess(x)
    assert e.shape == (2,) and e[0] > 3 * e[1]
    assert dg.split_rhat(x).shape == (2,)


def test_rhat_brute_force_on_a_tiny_input():
    """Split R-hat written out with loops for 2 chains of 6 draws (4 half-chains of 3)."""
    x = np.array([[0.1, 1.0], [0.4, 1.3], [-0.2, 0.7], [0.3, 1.1], [0.0, 0.9], [0.5, 1.6]])
    seqs = [x[:3, 0], x[3:, 0], x[:3, 1], x[3:, 1]]
    n, m = 3, 4
    means = [sum(s) / n for s in seqs]
    grand = sum(means) / m
    B = n / (m - 1) * sum((mu - grand) ** 2 for mu in means)
    W = sum(sum((v - mu) ** 2 for v in s) / (n - 1) for s, mu in zip(seqs, means)) / m
    var = (n - 1) / n * W + B / n
    assert abs(dg.split_rhat(x) - (var / W) ** 0.5) < 1e-12


def test_ess_brute_force_autocorrelation():
    """ESS from rho_t computed by a direct double loop over lags (small input)."""
    x = _ar1(0.6, 200, 3, 4)
    s = np.concatenate([x[:100], x[100:]], axis=1)  # split: 6 sequences of 100
    n, m = s.shape
    W = np.mean([np.var(s[:, j], ddof=1) for j in range(m)])
    B_n = np.var(s.mean(axis=0), ddof=1)
    var = (n - 1) / n * W + B_n
    rho = np.empty(n)
    for t in range(n):
        ac = 0.0
        for j in range(m):
            c = s[:, j] - s[:, j].mean()
            ac += sum(c[i] * c[i + t] for i in range(n - t)) / n
        rho[t] = 1 - (W - ac / m) / var
    rho[0] = 1.0
    total, prev = 0.0, np.inf
    for t in range(0, n - 1, 2):
        pair = rho[t] + rho[t + 1]
        if pair <= 0:
            break
        pair = min(pair, prev)
        total += pair
        prev = pair
    want = m * n / (2 * total - 1)
    assert abs(dg.ess(x) / want - 1) < 1e-9


def test_rhat_flags_chains_that_disagree():
    rng = np.random.default_rng(5)
    x = rng.normal(size=(1000, 4))
    assert abs(dg.split_rhat(x) - 1) < 0.01
    x[:, 0] += 3.0  # one chain in another mode
    assert dg.split_rhat(x) > 1.5
    y = rng.normal(size=(1000, 4)) + np.linspace(0, 3, 1000)[:, None]  # drifting chains
    assert dg.split_rhat(y) > 1.1  # the split catches within-chain trends
