"""Seeded input generators: the noise models' first two moments and the matched prior of the
paper's simulated systems (eq. sim-dist) against the simulation draws themselves."""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("gen", ["poisson", "gauss"])
def test_noise_moments(gen):
    # both noise models have mean I and variance sigma_bkg^2 + I / (G t_exp) (Sec. 2.1.2)
    sigma, t = 0.2, 100.0
    clean = np.repeat(np.array([0.0, 0.5, 2.0, 20.0], np.float32), 50_000).reshape(4, -1)
    add = synth.add_noise if gen == "poisson" else synth.add_gaussian_noise
    obs = add(clean, 3, sigma, t).astype(np.float64)
    for row, c in zip(obs, clean[:, 0]):
        var = sigma ** 2 + c / t
        assert abs(row.mean() - c) < 5 * np.sqrt(var / row.size)
        assert abs(row.var() / var - 1) < 0.03


def test_gaussian_noise_has_no_skew():
    # the Gaussian stand-in keeps the shot noise's variance but not its third moment
    clean = np.full((1, 400_000), 0.05, np.float32)
    for add, want_skew in ((synth.add_noise, True), (synth.add_gaussian_noise, False)):
        r = add(clean, 5, 0.0, 100.0).astype(np.float64)[0] - 0.05
        skew = np.mean(r ** 3) / np.mean(r ** 2) ** 1.5
        # Poisson(5) has skewness 1/sqrt(5) = 0.447
        assert (abs(skew - 0.447) < 0.03) if want_skew else (abs(skew) < 0.02)


def test_matched_prior_is_the_simulation_distribution():
    sp = synth.spec_paper80()
    broad, matched = synth.fit_priors(sp), synth.fit_priors(sp, matched=True)
    draws = synth.paper_sim_params(np.random.default_rng(7), 200_000, sp.pix).astype(np.float64)
    for j, (b, m) in enumerate(zip(broad, matched)):
        x = draws[:, j]
        if m["family"] == synth.LOGNORMAL:
            assert abs(np.log(x).mean() - m["mu"]) < 0.01 and abs(np.log(x).std() - m["sigma"]) < 0.01
            assert b["mu"] == m["mu"] and b["sigma"] > m["sigma"]
        elif m["family"] == synth.NORMAL:
            assert abs(x.mean() - m["mu"]) < 0.02 * m["sigma"]
            assert abs(x.std() / m["sigma"] - 1) < 0.01
            assert b["sigma"] == 2 * m["sigma"]
        elif m["family"] == synth.UNIFORM:
            assert m["lo"] <= x.min() and x.max() <= m["hi"]
            assert abs(x.min() - m["lo"]) < 1e-3 and abs(x.max() - m["hi"]) < 1e-3
        else:  # truncated normal: inside its bounds, centred, narrower than the broad prior
            assert m["lo"] <= x.min() and x.max() <= m["hi"]
            assert abs(x.mean() - m["mu"]) < 0.01 and b["sigma"] == 2 * m["sigma"]
