"""GPU tests of the HMC sampler (Sec. 2.5) through the C ABI: leapfrog parity with the FP64
oracle (oracle/hmc.py), reversibility, step-size adaptation, and the sampled distribution
against the Laplace approximation of a high signal-to-noise posterior."""
import numpy as np
import pytest

import oracle
from oracle import fit as ofit
from oracle import hmc as ohmc
import synth
from paper_2202_07663_amd import diagnostics as dg
from tests.helpers import load_workload, oracle_model

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    import paper_2202_07663_amd as g
    return g


def _say(*a):
    print(*a, flush=True)


def _laplace_sie40():
    spec = synth.spec_c1()
    obs, truth = load_workload(spec.name)
    priors = synth.fit_priors(spec)
    fg = ohmc.lens_objective(oracle_model(spec), obs, priors)
    z_true = ofit.bijector_inverse(truth[None, :].astype(np.float64), priors)[0]
    z_mode, hess = ohmc.newton_mode(fg, z_true)
    return spec, obs, priors, fg, z_mode, np.linalg.inv(hess)


def _near_truth_epl36():
    """A small EPL + lens light + shapelet system; M^-1 = 1 / diag(Hessian) at the truth."""
    spec = synth.Spec("hmcepl", 36, 36, 2, epl=True, lens_light=True, nmax=3,
                      psf=synth.moffat_psf(9, 0.15, 2.5), sigma_bkg=0.1, t_exp=1000.0)
    truth = synth.draw_truth(spec, 31)
    om = oracle_model(spec)
    obs = synth.add_noise(oracle.simulate(om, truth.astype(np.float64))[0], 31, 0.1, 1000.0)
    priors = synth.fit_priors(spec)
    fg = ohmc.lens_objective(om, obs, priors)
    z = ofit.bijector_inverse(truth[None, :].astype(np.float64), priors)[0]
    return spec, obs, priors, fg, z, 1.0 / np.abs(np.diag(ohmc.hessian_fd(fg, z)))


@pytest.fixture(scope="module")
def sie40():
    return _laplace_sie40()


def _whiten(inv_mass):
    im = np.asarray(inv_mass, np.float64)
    return np.sqrt(np.diag(im) if im.ndim == 2 else im)


def _white(inv_mass):
    """Maps taking position and momentum differences to units where M^-1 = I:
    dz -> C^-1 dz, dp -> C^T dp for M^-1 = C C^T."""
    im = np.asarray(inv_mass, np.float64)
    C = np.linalg.cholesky(im) if im.ndim == 2 else np.diag(np.sqrt(im))
    Ci = np.linalg.inv(C)
    return (lambda dz: dz @ Ci.T), (lambda dp: dp @ C)


@pytest.mark.parametrize("case", ["sie40_dense", "epl36_diag"])
def test_leapfrog_parity(G, sie40, case):
    """L leapfrog steps on the GPU (FP32 positions and momenta, the library's gradient) from
    the same (z, p) as the oracle's FP64 integration. Compared in units of the posterior
    width: |dz| / w and |dp| w within 2e-3 (1 + the distance travelled), the end log
    posterior within the log-likelihood bar (relative 1e-4)."""
    if case == "sie40_dense":
        spec, obs, priors, fg, z_c, im = sie40
        eps, L = 0.3, 5
    else:
        spec, obs, priors, fg, z_c, im = _near_truth_epl36()
        eps, L = 0.05, 6
    w = _whiten(im)
    C = 16
    rng = np.random.default_rng(7)
    z0 = z_c + 0.7 * rng.normal(size=(C, z_c.size)) * w
    p0 = (rng.normal(size=z0.shape) / w).astype(np.float32)
    model = G.Model.from_spec(spec, obs)
    h = G.HMC(model, C, L, 0, 0, priors, inv_mass=im, z0=torch.from_numpy(z0).cuda())
    zg, pg, lpg = (t.cpu().numpy().astype(np.float64)
                   for t in h.leapfrog(torch.from_numpy(z0).cuda(), torch.from_numpy(p0).cuda(),
                                       L, eps))
    zr, pr, _, fr = ohmc.leapfrog_fn(fg, z0, p0.astype(np.float64), eps, L,
                                     np.asarray(im, np.float64))
    assert np.all(np.isfinite(zr)) and np.all(np.isfinite(fr))
    wz, wp = _white(im)
    travel = max(np.abs(wz(zr - z0)).max(), np.abs(wp(pr - p0)).max())
    ez, ep = np.abs(wz(zg - zr)).max(), np.abs(wp(pg - pr)).max()
    elp = np.abs(lpg + fr).max() / np.abs(fr).max()
    _say(case, "travel", travel, "max |dz|", ez, "max |dp|", ep, "lp rel", elp)
    # per-parameter detail, and the gradient of log p~ at the start against the oracle
    _say("dz/w by param", np.round(np.abs((zg - zr) / w).max(axis=0), 4))
    _say("dp w by param", np.round(np.abs((pg - pr) * w).max(axis=0), 4))
    th0 = torch.from_numpy(ofit.bijector(z0.astype(np.float64), priors).astype(np.float32)).cuda()
    _, gth = model.loglik_grad(th0)
    _, gth_ref = oracle.loglik_grad(oracle_model(spec), th0.cpu().numpy().astype(np.float64), obs)
    gw = np.abs((gth.cpu().numpy() - gth_ref)).max(axis=0) / (np.abs(gth_ref).max(axis=0) + 1e-30)
    _say("grad rel err by param", np.round(gw, 6))
    assert ez <= 2e-3 * (1 + travel) and ep <= 2e-3 * (1 + travel)
    assert elp <= 1e-4


def test_leapfrog_is_reversible_on_the_gpu(G, sie40):
    """Integrating back with the momentum negated returns to the start (in units where
    M^-1 = I), up to the FP32 rounding of momenta and of the likelihood's parameters."""
    spec, obs, priors, fg, z_c, im = sie40
    w = _whiten(im)
    C = 32
    rng = np.random.default_rng(8)
    z0 = torch.from_numpy(z_c + rng.normal(size=(C, z_c.size)) * w).cuda()
    p0 = torch.from_numpy((rng.normal(size=(C, z_c.size)) / w).astype(np.float32)).cuda()
    model = G.Model.from_spec(spec, obs)
    h = G.HMC(model, C, 5, 0, 0, priors, inv_mass=im, z0=z0)
    z1, p1, _ = h.leapfrog(z0, p0, 8, 0.3)
    z2, p2, _ = h.leapfrog(z1, -p1, 8, 0.3)
    wz, wp = _white(im)
    d = lambda t: t.cpu().numpy().astype(np.float64)
    moved = np.abs(wz(d(z1) - d(z0))).max()
    ez = np.abs(wz(d(z2) - d(z0))).max()
    ep = np.abs(wp(d(p2) + d(p0))).max()
    _say("moved", moved, "return error z", ez, "p", ep)
    assert moved > 0.1 and ez < 2e-3 and ep < 2e-3


def test_sampler_matches_the_laplace_posterior(G, sie40):
    """At this signal-to-noise the posterior is close to Gaussian: 64 chains (the paper's
    L = 5, M^-1 = the posterior covariance, target acceptance 0.75 adapted over 80% of
    burn-in) reproduce the Laplace mean and widths, with R-hat < 1.05 and the acceptance
    near its target. The initial step (1.0) is far from the adapted one."""
    spec, obs, priors, fg, z_c, cov = sie40
    C, nb, ns = 64, 150, 250
    rng = np.random.default_rng(9)
    z0 = z_c + rng.normal(size=(C, z_c.size)) @ np.linalg.cholesky(cov).T
    model = G.Model.from_spec(spec, obs)
    h = G.HMC(model, C, 5, nb, ns, priors, step_size=1.0, seed=11, inv_mass=cov,
              z0=torch.from_numpy(z0).cuda())
    h.run()
    info = h.info()
    th = h.samples().cpu().numpy().astype(np.float64)  # [ns, C, d]
    z = ofit.bijector_inverse(th.reshape(-1, th.shape[-1]), priors).reshape(th.shape)
    sd = np.sqrt(np.diag(cov))
    mean_err = np.abs(z.mean(axis=(0, 1)) - z_c) / sd
    sd_ratio = z.std(axis=(0, 1)) / sd
    rhat, ess = dg.split_rhat(z), dg.ess(z)
    _say("eps", info["step_size"], "accept", info["accept_mean"], "mean err/sd", mean_err.max(),
         "sd ratio", sd_ratio.min(), sd_ratio.max(), "rhat", rhat.max(), "ess", ess.min())
    assert info["trajectories"] == nb + ns
    assert abs(info["accept_mean"] - 0.75) < 0.1
    assert 0.1 < info["step_size"] < 1.0
    assert rhat.max() < 1.05 and ess.min() > 500
    assert mean_err.max() < 0.15
    assert np.all(np.abs(sd_ratio - 1) < 0.12)


def test_sampler_is_deterministic_and_seeded(G, sie40):
    spec, obs, priors, fg, z_c, cov = sie40
    z0 = torch.from_numpy(np.tile(z_c, (8, 1))).cuda()
    model = G.Model.from_spec(spec, obs)
    runs = []
    for seed in (3, 3, 4):
        h = G.HMC(model, 8, 5, 10, 10, priors, step_size=0.3, seed=seed, inv_mass=cov, z0=z0)
        h.run(12)
        h.run(8)
        runs.append(h.samples().cpu().numpy())
        h.close()
    np.testing.assert_array_equal(runs[0], runs[1])
    assert not np.array_equal(runs[0], runs[2])


def test_sampler_from_prior_starts_and_bad_options(G, sie40):
    """Chains drawn from the prior (far from the posterior, where log L may overflow) run
    without failing and report finite samples; invalid options are refused."""
    spec, obs, priors, _, _, cov = sie40
    model = G.Model.from_spec(spec, obs)
    h = G.HMC(model, 16, 3, 2, 2, priors, step_size=1e-3, seed=1)
    h.run()
    assert np.all(np.isfinite(h.samples().cpu().numpy()))
    with pytest.raises(G.GlError):
        h.run(1)  # nothing left
    bad = -np.eye(spec.d)
    with pytest.raises(G.GlError):
        G.HMC(model, 4, 3, 1, 1, priors, inv_mass=bad)
    with pytest.raises(G.GlError):
        G.HMC(model, 4, 3, 1, 1, priors, target_accept=1.5)


def test_trajectory_length_adaptation(G, sie40):
    """With M^-1 = the posterior covariance the target is close to a standard normal in
    whitened units, where the jittered ChEES criterion peaks at T* = 2.247 (tan 2T = 2T;
    pinned on the oracle). Adapting eps and T over 80% of 300 burn-in trajectories lands near
    T*, the jittered lengths average about T / (2 eps) steps, and the samples still match the
    Laplace posterior."""
    spec, obs, priors, fg, z_c, cov = sie40
    C, nb, ns = 64, 300, 200  # 500 trajectories, run 50 at a time
    rng = np.random.default_rng(12)
    z0 = z_c + rng.normal(size=(C, z_c.size)) @ np.linalg.cholesky(cov).T
    model = G.Model.from_spec(spec, obs)
    # a high acceptance target keeps eps small enough that L = ceil(u T / eps) resolves T
    h = G.HMC(model, C, 5, nb, ns, priors, step_size=0.3, seed=13, inv_mass=cov,
              z0=torch.from_numpy(z0).cuda(), adapt_length=True, target_accept=0.95)
    Ts = []
    for _ in range(10):
        h.run(50)
        Ts.append(round(h.info()["trajectory_length"], 3))
    _say("T along the run", Ts)
    info = h.info()
    th = h.samples().cpu().numpy().astype(np.float64)
    z = ofit.bijector_inverse(th.reshape(-1, th.shape[-1]), priors).reshape(th.shape)
    sd = np.sqrt(np.diag(cov))
    mean_err = np.abs(z.mean(axis=(0, 1)) - z_c) / sd
    sd_ratio = z.std(axis=(0, 1)) / sd
    _say("T", info["trajectory_length"], "eps", info["step_size"], "mean L",
         info["mean_leapfrog"], "accept", info["accept_mean"], "mean err", mean_err.max(),
         "sd ratio", sd_ratio.min(), sd_ratio.max(), "rhat", dg.split_rhat(z).max())
    assert 1.6 < info["trajectory_length"] < 3.0
    assert info["mean_leapfrog"] > 1.0
    assert abs(info["accept_mean"] - 0.95) < 0.05
    assert mean_err.max() < 0.15 and np.all(np.abs(sd_ratio - 1) < 0.12)
    assert dg.split_rhat(z).max() < 1.05


def test_length_adaptation_survives_a_far_rejected_chain(G, sie40):
    """The length gradient is an acceptance-weighted mean over chains. A chain started far
    from the posterior makes proposals with a huge ChEES term and acceptance probability 0;
    with weight 0 it must leave the adapted length and step size finite (in FP32 such a term
    can overflow, and 0 x inf is NaN)."""
    spec, obs, priors, fg, z_c, cov = sie40
    C = 32
    rng = np.random.default_rng(5)
    z0 = z_c + rng.normal(size=(C, z_c.size)) @ np.linalg.cholesky(cov).T
    z0[3] = z_c + 1e6 * np.sqrt(np.diag(cov))  # a start 1e6 posterior widths away
    model = G.Model.from_spec(spec, obs)
    h = G.HMC(model, C, 5, 60, 10, priors, step_size=0.3, seed=17, inv_mass=cov,
              z0=torch.from_numpy(z0).cuda(), adapt_length=True)
    h.run()
    info = h.info()
    _say("far chain: T", info["trajectory_length"], "eps", info["step_size"], "accept",
         info["accept_mean"])
    assert np.isfinite(info["trajectory_length"]) and info["trajectory_length"] > 0
    assert np.isfinite(info["step_size"]) and info["step_size"] > 0
    assert np.all(np.isfinite(h.samples().cpu().numpy()[:, np.arange(C) != 3]))


def test_mass_adaptation(G, sie40):
    """Windowed re-estimation of M^-1 (adapt_mass). From a mass matrix with the wrong widths
    (the posterior's diagonal scaled by factors of 1/8 .. 8) and no correlations, the three
    window estimates replace it; the last one matches the posterior covariance (the Laplace
    approximation from the oracle) in whitened units to within sampling error, and the
    samples match the Laplace posterior. Without windows (a burn-in too short for them) the
    factor stays the one given."""
    spec, obs, priors, fg, z_c, cov = sie40
    d = z_c.size
    C, nb, ns = 64, 400, 300
    rng = np.random.default_rng(21)
    z0 = z_c + rng.normal(size=(C, d)) @ np.linalg.cholesky(cov).T
    bad = np.diag(cov) * np.exp(rng.uniform(-np.log(64), np.log(64), d))
    model = G.Model.from_spec(spec, obs)
    h = G.HMC(model, C, 5, nb, ns, priors, step_size=0.3, seed=23, inv_mass=bad,
              z0=torch.from_numpy(z0).cuda(), adapt_mass=True)
    h.run()
    info = h.info()
    F = h.mass_chol().cpu().numpy().astype(np.float64)
    Lc = np.linalg.cholesky(cov)
    W = np.linalg.solve(Lc, np.linalg.solve(Lc, F @ F.T).T)  # Lc^-1 (F F^T) Lc^-T
    ev = np.linalg.eigvalsh((W + W.T) / 2)
    th = h.samples().cpu().numpy().astype(np.float64)
    z = ofit.bijector_inverse(th.reshape(-1, d), priors).reshape(th.shape)
    sd = np.sqrt(np.diag(cov))
    mean_err = np.abs(z.mean(axis=(0, 1)) - z_c) / sd
    sd_ratio = z.std(axis=(0, 1)) / sd
    rhat, ess = dg.split_rhat(z), dg.ess(z)
    _say("mass updates", info["mass_updates"], "whitened eigenvalues", ev.min(), ev.max(),
         "eps", info["step_size"], "accept", info["accept_mean"], "rhat", rhat.max(), "ess",
         ess.min(), "mean err", mean_err.max(), "sd ratio", sd_ratio.min(), sd_ratio.max())
    assert info["mass_updates"] == 3
    assert np.allclose(F, np.tril(F))
    assert ev.min() > 0.6 and ev.max() < 1.5
    assert rhat.max() < 1.05 and ess.min() > 500
    assert mean_err.max() < 0.15 and np.all(np.abs(sd_ratio - 1) < 0.12)
    # n_adapt = floor(0.8 x 5) = 4 trajectories: too few for windows
    h2 = G.HMC(model, 8, 3, 5, 2, priors, step_size=0.3, seed=1, inv_mass=bad,
               z0=torch.from_numpy(z0[:8]).cuda(), adapt_mass=True)
    h2.run()
    assert h2.info()["mass_updates"] == 0
    np.testing.assert_allclose(h2.mass_chol().cpu().numpy(), np.diag(np.sqrt(bad)), rtol=1e-6)
    with pytest.raises(G.GlError):
        G.HMC(model, 4, 3, 1, 1, priors, adapt_mass=2)


def test_mass_estimate_matches_the_oracle(G, sie40):
    """The window estimate itself against the oracle's estimator, on positions known
    exactly: with a step size of 30 posterior widths every proposal is rejected, and a
    target acceptance of 1e-6 keeps the adapted step there, so each chain stays at its start
    and a window of w trajectories holds each start w times. After the last window M^-1 is the
    oracle's window_inv_mass of those positions (window lengths from its mass_windows), to
    the FP32 rounding of the factor."""
    spec, obs, priors, fg, z_c, cov = sie40
    d = z_c.size
    C, nb = 32, 20
    rng = np.random.default_rng(8)
    z0 = z_c + rng.normal(size=(C, d)) @ np.linalg.cholesky(cov).T
    model = G.Model.from_spec(spec, obs)
    h = G.HMC(model, C, 3, nb, 1, priors, step_size=30.0, target_accept=1e-6, adapt_frac=1.0,
              seed=29, inv_mass=cov, z0=torch.from_numpy(z0).cuda(), adapt_mass=True)
    h.run()
    info = h.info()
    b = ohmc.mass_windows(nb)
    ref = np.linalg.cholesky(ohmc.window_inv_mass(np.tile(z0, (b[3] - b[2], 1))))
    F = h.mass_chol().cpu().numpy().astype(np.float64)
    th = h.samples().cpu().numpy()[0]
    _say("windows", b, "accept", info["accept_mean"], "eps", info["step_size"],
         "max |F - ref| / max |ref|", np.abs(F - ref).max() / np.abs(ref).max())
    assert info["mass_updates"] == 3 and info["accept_mean"] == 0.0
    np.testing.assert_allclose(th, ofit.bijector(z0, priors), rtol=2e-6, atol=1e-7)
    np.testing.assert_allclose(F, ref, rtol=2e-5, atol=2e-6 * np.abs(ref).max())


def test_mass_and_length_adaptation_together(G, sie40):
    """Mass adaptation with the trajectory length adapted too (ChEES): from the same mass
    matrix with the wrong widths, the length settles on a finite value, the three window
    estimates are taken, and the samples match the Laplace posterior."""
    spec, obs, priors, fg, z_c, cov = sie40
    d = z_c.size
    C, nb, ns = 64, 300, 200
    rng = np.random.default_rng(31)
    z0 = z_c + rng.normal(size=(C, d)) @ np.linalg.cholesky(cov).T
    bad = np.diag(cov) * np.exp(rng.uniform(-np.log(64), np.log(64), d))
    model = G.Model.from_spec(spec, obs)
    h = G.HMC(model, C, 5, nb, ns, priors, step_size=0.3, seed=37, inv_mass=bad,
              z0=torch.from_numpy(z0).cuda(), adapt_mass=True, adapt_length=True,
              max_leapfrog=50)
    h.run()
    info = h.info()
    th = h.samples().cpu().numpy().astype(np.float64)
    z = ofit.bijector_inverse(th.reshape(-1, d), priors).reshape(th.shape)
    sd = np.sqrt(np.diag(cov))
    mean_err = np.abs(z.mean(axis=(0, 1)) - z_c) / sd
    sd_ratio = z.std(axis=(0, 1)) / sd
    rhat = dg.split_rhat(z)
    _say("T", info["trajectory_length"], "eps", info["step_size"], "mean L",
         info["mean_leapfrog"], "updates", info["mass_updates"], "rhat", rhat.max(),
         "mean err", mean_err.max(), "sd ratio", sd_ratio.min(), sd_ratio.max())
    assert info["mass_updates"] == 3
    assert np.isfinite(info["trajectory_length"]) and info["trajectory_length"] > 0
    assert rhat.max() < 1.05
    assert mean_err.max() < 0.15 and np.all(np.abs(sd_ratio - 1) < 0.12)
