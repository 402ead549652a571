"""GPU <-> oracle parity of the C-ABI library (gl_simulate, gl_loglik, gl_loglik_grad).

Inputs are seeded and synthetic (synth), with the observed images stored by
tests/golden/make_workloads.py from the oracle. Both sides consume the same float32 values.
Tolerances: see tests/helpers.py.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import (assert_grad_close, assert_logl_close, load_workload,
                           oracle_model)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def glens():
    import paper_2202_07663_amd as g
    return g


def _run(model, theta_np, grad=True):
    th = torch.from_numpy(np.ascontiguousarray(theta_np, np.float32)).cuda()
    if grad:
        ll, g = model.loglik_grad(th)
        torch.cuda.synchronize()
        return ll.cpu().numpy(), g.cpu().numpy()
    ll = model.loglik(th)
    torch.cuda.synchronize()
    return ll.cpu().numpy()


def _say(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------------------------------
# Workload 1: SIE + shear, Sersic source, 40x40, k = 1, Gaussian 11x11, 64 vectors
# ------------------------------------------------------------------------------------------

def test_sie40_loglik_and_grad_64(glens):
    spec = synth.spec_c1()
    obs, truth = load_workload(spec.name)
    theta = synth.draw_particles(spec, truth, 64, seed=0)
    _say("case sie40 P=64")
    m = glens.Model.from_spec(spec, obs)
    ll, g = _run(m, theta)
    ll_ref, g_ref = oracle.loglik_grad(oracle_model(spec), theta.astype(np.float64), obs)
    e1 = assert_logl_close(ll, ll_ref)
    e2 = assert_grad_close(g, g_ref, names=spec.names)
    _say("sie40 logl err", e1, "grad err", e2)
    ll2 = _run(m, theta, grad=False)
    np.testing.assert_array_equal(ll, ll2)  # log L identical with and without the adjoint


# ------------------------------------------------------------------------------------------
# Workload 2: EPL + shear, Sersic lens light, Sersic + shapelets (n_max 6), 60x60, k = 2,
# Moffat 21x21, 4096 vectors
# ------------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def epl60_case():
    spec = synth.spec_c2()
    obs, truth = load_workload(spec.name)
    theta = synth.draw_particles(spec, truth, 4096, seed=0)
    return spec, obs, theta


def test_epl60_loglik_4096(glens, epl60_case):
    spec, obs, theta = epl60_case
    _say("case epl60 loglik P=4096")
    m = glens.Model.from_spec(spec, obs)
    ll = _run(m, theta, grad=False)
    ll_ref = oracle.loglik(oracle_model(spec), theta.astype(np.float64), obs)
    _say("epl60 logl err", assert_logl_close(ll, ll_ref))


def test_epl60_grad_4096_sampled(glens, epl60_case):
    """Gradient at the full launch (4096 vectors, the benchmark's configuration), checked on a
    sample of 192 vectors against the oracle's dual-number gradient."""
    spec, obs, theta = epl60_case
    _say("case epl60 grad P=4096")
    m = glens.Model.from_spec(spec, obs)
    ll, g = _run(m, theta)
    idx = np.r_[np.arange(0, 2048, 32), np.arange(2048, 4096, 16)]
    ll_ref, g_ref = oracle.loglik_grad(oracle_model(spec), theta[idx].astype(np.float64), obs)
    e1 = assert_logl_close(ll[idx], ll_ref)
    e2 = assert_grad_close(g[idx], g_ref, names=spec.names)
    _say("epl60 grad logl err", e1, "grad err", e2)


def test_largest_system_4096_sampled(glens):
    """The largest system of the serving stream (100 x 100 px, k = 2, EPL + shear, Sersic lens
    light, Sersic + shapelets n_max 8: d = 68, 160 000 sub-pixels per vector) in a 4096-vector
    launch, the largest per-vector work the library takes at the benchmark's batch size: log L
    and gradient of a sample of the vectors against the oracle."""
    spec = synth.spec_custom(100, 2, True, True, 8, K=21)
    truth = synth.draw_truth(spec, 11)
    om = oracle_model(spec)
    obs = synth.add_noise(oracle.simulate(om, truth[None, :].astype(np.float64))[0], 11,
                          spec.sigma_bkg, spec.t_exp)
    theta = synth.draw_particles(spec, truth, 4096, seed=5)
    _say("case n100 d68 grad P=4096")
    m = glens.Model.from_spec(spec, obs)
    assert m.d == 68
    ll, g = _run(m, theta)
    assert np.all(np.isfinite(ll)) and np.all(np.isfinite(g))
    idx = np.r_[0, 1, 700, 2047, 2048, 3333, 4094, 4095]
    ll_ref, g_ref = oracle.loglik_grad(om, theta[idx].astype(np.float64), obs)
    e1 = assert_logl_close(ll[idx], ll_ref)
    e2 = assert_grad_close(g[idx], g_ref, names=spec.names)
    _say("n100 logl err", e1, "grad err", e2)


def test_epl60_simulate_image(glens, epl60_case):
    spec, obs, theta = epl60_case
    m = glens.Model.from_spec(spec, obs)
    th = torch.from_numpy(theta[:24]).cuda()
    img = m.simulate(th).cpu().numpy()
    ref = oracle.simulate(oracle_model(spec), theta[:24].astype(np.float64))
    scale = np.abs(ref).max(axis=(1, 2), keepdims=True)
    err = np.abs(img - ref) / scale
    assert err.max() < 2e-5, err.max()


# ------------------------------------------------------------------------------------------
# Ragged shapes, tiles, component sets
# ------------------------------------------------------------------------------------------

CASES = [
    # H, W, k, K, epl, lens_light, nmax, shear, P
    (37, 23, 3, 5, True, True, 2, True, 5),
    (17, 29, 1, 1, False, True, -1, False, 7),
    (40, 40, 2, 9, True, False, 0, True, 3),
    (64, 48, 2, 21, True, True, 8, True, 4),
    (31, 31, 4, 3, False, False, 4, True, 6),
    (100, 100, 2, 21, True, True, 6, True, 2),
    (9, 300 // 30, 1, 31, True, True, 1, True, 3),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}k{c[2]}K{c[3]}" for c in CASES])
def test_ragged_configs(glens, case):
    H, W, k, K, epl, ll_on, nmax, shear, P = case
    psf = synth.asymmetric_psf(K, seed=K) if K > 1 else np.ones((1, 1), np.float32)
    spec = synth.Spec("x", H, W, k, epl=epl, lens_light=ll_on, nmax=nmax, psf=psf,
                      sigma_bkg=0.1, t_exp=1000.0, shear=shear)
    truth = synth.draw_truth(spec, 7)
    om = oracle_model(spec)
    clean = oracle.simulate(om, truth.astype(np.float64))[0]
    obs = synth.add_noise(clean, 7, spec.sigma_bkg, spec.t_exp)
    theta = synth.draw_particles(spec, truth, P, seed=3)
    _say("case", case)
    m = glens.Model.from_spec(spec, obs)
    ll, g = _run(m, theta)
    ll_ref, g_ref = oracle.loglik_grad(om, theta.astype(np.float64), obs)
    assert_logl_close(ll, ll_ref)
    assert_grad_close(g, g_ref, names=spec.names)
    img = m.simulate(torch.from_numpy(theta).cuda()).cpu().numpy()
    ref = oracle.simulate(om, theta.astype(np.float64))
    err = np.abs(img - ref) / np.abs(ref).max(axis=(1, 2), keepdims=True)
    assert err.max() < 2e-5, err.max()


@pytest.mark.parametrize("eps", [1e-6, 1e-4, 0.0005, 0.0199, 0.0201, 0.05, 0.0999, 0.1001, 0.3,
                                 0.55, 0.7])
@pytest.mark.parametrize("epl", [False, True])
def test_mass_ellipticity_range(glens, eps, epl):
    """Both SIE branches (series below |eps| = 0.1, closed form above), both ways of getting
    the series derivative dS/dX in the adjoint (its own series below |eps| = 0.02, the
    first-order identity above), the EPL series up to its longest expansion, the |eps|
    clamp at 0.6, and nearly round lenses (|eps| = 1e-6, 1e-4), where the oracle's (q, phi)
    form is still differentiable (at |eps| = 0 exactly its phi is not)."""
    spec = synth.Spec("e", 32, 32, 2, epl=epl, lens_light=False, nmax=2,
                      psf=synth.moffat_psf(7, 0.15, 2.5), sigma_bkg=0.1, t_exp=1000.0)
    truth = synth.draw_truth(spec, 11)
    om = oracle_model(spec)
    obs = synth.add_noise(oracle.simulate(om, truth.astype(np.float64))[0], 11, 0.1, 1000.0)
    theta = synth.draw_particles(spec, truth, 8, seed=5)
    ang = np.linspace(0, 2 * np.pi, 8, endpoint=False) + 0.1
    ie = 2 if epl else 1
    theta[:, ie] = eps * np.cos(ang)
    theta[:, ie + 1] = eps * np.sin(ang)
    m = glens.Model.from_spec(spec, obs)
    ll, g = _run(m, theta)
    ll_ref, g_ref = oracle.loglik_grad(om, theta.astype(np.float64), obs)
    assert_logl_close(ll, ll_ref)
    assert_grad_close(g, g_ref, names=spec.names)


@pytest.mark.parametrize("offset", [(0.0, 0.0), (3e-7, -2e-7), (-6e-7, 1e-7)],
                         ids=["on", "near1", "near2"])
@pytest.mark.parametrize("epl", [False, True])
def test_lens_centre_on_a_sub_pixel(glens, epl, offset):
    """A lens centre on, or within 1e-6 arcsec of, a sub-pixel centre: the elliptical radius
    there sits at its floor (R^2 >= 1e-12) on both sides. Log L and the whole gradient are
    compared with the oracle, whose derivative there is that of the frozen-radius formula
    (the SIE's closed form, the EPL's series; the frozen radius carries the eps-dependence
    of the mass radius). That one sub-pixel's mass Jacobian is ~1e6 times a normal one's, so
    it dominates the centre and eccentricity gradients."""
    spec = synth.Spec("c", 31, 31, 1, epl=epl, lens_light=False, nmax=2,
                      psf=synth.moffat_psf(7, 0.15, 2.5), sigma_bkg=0.1, t_exp=1000.0)
    truth = synth.draw_truth(spec, 12)
    ic = 4 if epl else 3  # lens centre (x, y): pixel (15, 15) is centred on the origin
    truth[ic] = truth[ic + 1] = 0.0
    om = oracle_model(spec)
    obs = synth.add_noise(oracle.simulate(om, truth.astype(np.float64))[0], 12, 0.1, 1000.0)
    theta = synth.draw_particles(spec, truth, 8, seed=3)
    theta[:, ic] = np.float32(offset[0])
    theta[:, ic + 1] = np.float32(offset[1])
    _say("case centre", epl, offset)
    m = glens.Model.from_spec(spec, obs)
    ll, g = _run(m, theta)
    ll_ref, g_ref = oracle.loglik_grad(om, theta.astype(np.float64), obs)
    assert_logl_close(ll, ll_ref)
    e = assert_grad_close(g, g_ref, names=spec.names)
    _say("centre", epl, offset, "grad err", e)
    img = m.simulate(torch.from_numpy(theta).cuda()).cpu().numpy()
    ref = oracle.simulate(om, theta.astype(np.float64))
    assert (np.abs(img - ref) / np.abs(ref).max(axis=(1, 2), keepdims=True)).max() < 2e-5


@pytest.mark.parametrize("eps", [1e-6, 1e-4])
def test_light_ellipticity_near_round(glens, eps):
    """Nearly round lens light and source (|eps| = 1e-6, 1e-4): the kernels' rotation-free
    quadratic form against the oracle's (q, phi) form, which is still differentiable there
    (at |eps| = 0 exactly its phi is not)."""
    spec = synth.Spec("l", 36, 36, 2, epl=True, lens_light=True, nmax=3,
                      psf=synth.moffat_psf(9, 0.15, 2.5), sigma_bkg=0.1, t_exp=1000.0)
    truth = synth.draw_truth(spec, 13)
    om = oracle_model(spec)
    obs = synth.add_noise(oracle.simulate(om, truth.astype(np.float64))[0], 13, 0.1, 1000.0)
    theta = synth.draw_particles(spec, truth, 8, seed=6)
    ang = np.linspace(0, 2 * np.pi, 8, endpoint=False) + 0.3
    il, isrc = 8, 15  # lens light and source (eps1, eps2) follow the 8 mass parameters
    for i0 in (il + 2, isrc + 2):
        theta[:, i0] = eps * np.cos(ang)
        theta[:, i0 + 1] = eps * np.sin(ang)
    assert spec.names[il + 2] == "l_e1" and spec.names[isrc + 2] == "s_e1"
    m = glens.Model.from_spec(spec, obs)
    ll, g = _run(m, theta)
    ll_ref, g_ref = oracle.loglik_grad(om, theta.astype(np.float64), obs)
    assert_logl_close(ll, ll_ref)
    assert_grad_close(g, g_ref, names=spec.names)


# ------------------------------------------------------------------------------------------
# Edge cases and API behaviour
# ------------------------------------------------------------------------------------------

def test_empty_batch_is_noop(glens):
    spec = synth.spec_c1()
    obs, _ = load_workload(spec.name)
    m = glens.Model.from_spec(spec, obs)
    th = torch.zeros((0, m.d), dtype=torch.float32, device="cuda")
    assert m.loglik(th).numel() == 0
    ll, g = m.loglik_grad(th)
    assert ll.numel() == 0 and g.shape == (0, m.d)


def test_nan_particle_is_isolated(glens):
    spec = synth.spec_c1()
    obs, truth = load_workload(spec.name)
    theta = synth.draw_particles(spec, truth, 8, seed=1)
    theta[3, 0] = np.nan
    m = glens.Model.from_spec(spec, obs)
    ll, g = _run(m, theta)
    assert ll[3] == -np.inf and np.all(g[3] == 0)
    ok = np.r_[0:3, 4:8]
    ll_ref, g_ref = oracle.loglik_grad(oracle_model(spec), theta[ok].astype(np.float64), obs)
    assert_logl_close(ll[ok], ll_ref)
    assert_grad_close(g[ok], g_ref)


def test_nan_in_any_parameter_is_isolated(glens):
    """A NaN in any one parameter (mass, shear, lens light, source, shapelet scale or
    coefficient) makes that vector's log L -inf and its gradient zero, whatever clamp or floor
    the parameter meets on the way; the other vectors of the launch are unaffected."""
    spec = synth.Spec("nan36", 36, 36, 2, epl=True, lens_light=True, nmax=2,
                      psf=synth.moffat_psf(9, 0.15, 2.5), sigma_bkg=0.1, t_exp=1000.0)
    truth = synth.draw_truth(spec, 13)
    om = oracle_model(spec)
    obs = synth.add_noise(oracle.simulate(om, truth[None, :].astype(np.float64))[0], 13, 0.1,
                          1000.0)
    d = spec.d
    # 16 clean vectors (near the truth and from the broadened draws, as in the other parity
    # cases: the per-component bound takes its scale from the batch), then d vectors with one
    # NaN each
    n = 16
    theta = np.concatenate([synth.draw_particles(spec, truth, n, seed=2),
                            synth.draw_particles(spec, truth, d, seed=3)])
    for j in range(d):
        theta[n + j, j] = np.nan
    m = glens.Model.from_spec(spec, obs)
    ll, g = _run(m, theta)
    bad = [spec.names[j] for j in range(d)
           if not (ll[n + j] == -np.inf and np.all(g[n + j] == 0))]
    assert not bad, bad
    ll_ref, g_ref = oracle.loglik_grad(om, theta[:n].astype(np.float64), obs)
    assert_logl_close(ll[:n], ll_ref)
    assert_grad_close(g[:n], g_ref, names=spec.names)


def test_host_pointer_rejected(glens):
    spec = synth.spec_c1()
    obs, _ = load_workload(spec.name)
    m = glens.Model.from_spec(spec, obs)
    th = torch.zeros((4, m.d), dtype=torch.float32)
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    from paper_2202_07663_amd import _lib
    rc = _lib.lib().gl_loglik(m._h, th.data_ptr(), 4, out.data_ptr(), None)
    assert rc == -1 and b"theta" in _lib.lib().gl_last_error()


def test_stage_times_loop(glens):
    """The stage-timing entry point: n back-to-back calls give the results of gl_loglik_grad
    (bitwise) and a positive duration for every stage; n out of range is refused."""
    import ctypes
    from paper_2202_07663_amd import _lib
    spec = synth.spec_c1()
    obs, truth = load_workload(spec.name)
    theta = synth.draw_particles(spec, truth, 64, seed=4)
    m = glens.Model.from_spec(spec, obs)
    ll_ref, g_ref = _run(m, theta)
    th = torch.from_numpy(theta).cuda()
    ll = torch.zeros(64, dtype=torch.float64, device="cuda")
    g = torch.zeros((64, m.d), dtype=torch.float32, device="cuda")
    ms = (ctypes.c_float * 5)()
    L = _lib.lib()
    for bad in (0, 10001):
        rc = L.gl_model_stage_times_n(m._h, th.data_ptr(), 64, 1, bad, ll.data_ptr(),
                                      g.data_ptr(), ms, None)
        assert rc == -1 and b"n_calls" in L.gl_last_error()
    _say("case stage_times_n sie40 P=64 n=7")
    check = _lib.check
    check(L.gl_model_stage_times_n(m._h, th.data_ptr(), 64, 1, 7, ll.data_ptr(), g.data_ptr(),
                                   ms, None))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ll.cpu().numpy(), ll_ref)
    np.testing.assert_array_equal(g.cpu().numpy(), g_ref)
    assert all(t > 0 for t in ms), list(ms)
    st = m.stage_times(th, with_grad=False, n_calls=3)
    assert st["subpix_adj"] == 0 and st["finalize"] == 0 and st["subpix_fwd"] > 0


def test_repeat_is_bitwise_identical(glens, epl60_case):
    spec, obs, theta = epl60_case
    m = glens.Model.from_spec(spec, obs)
    a = _run(m, theta[:512])
    b = _run(m, theta[:512])
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_batch_composition_invariance(glens, epl60_case):
    """At a fixed batch size, a vector's result does not depend on which other vectors share
    the launch (bitwise): the work split and every summation order depend only on the
    model and P. Across batch sizes the sub-pixel tiling changes, and so does the PSF pass's
    summation order for very small batches (their strips' PSF columns are split over lanes),
    so log L and the gradient agree to FP32 summation-order rounding only."""
    spec, obs, theta = epl60_case
    m = glens.Model.from_spec(spec, obs)
    a = _run(m, theta[:300])
    mixed = np.concatenate([theta[3000:3290], theta[290:300]])
    b = _run(m, mixed)
    np.testing.assert_array_equal(a[0][290:300], b[0][290:])
    np.testing.assert_array_equal(a[1][290:300], b[1][290:])
    c = _run(m, theta[290:300])
    np.testing.assert_allclose(c[0], a[0][290:300], rtol=1e-5)
    np.testing.assert_allclose(c[1], a[1][290:300], rtol=1e-5,
                               atol=1e-5 * np.abs(a[1][290:300]).max())


def test_autograd_function(glens):
    spec = synth.spec_c1()
    obs, truth = load_workload(spec.name)
    theta = synth.draw_particles(spec, truth, 16, seed=2)
    m = glens.Model.from_spec(spec, obs)
    th = torch.from_numpy(theta).cuda().requires_grad_(True)
    ll = glens.LogLik.apply(th, m)
    w = torch.linspace(0.5, 2.0, 16, device="cuda", dtype=torch.float64)
    (ll * w).sum().backward()
    _, g = m.loglik_grad(th.detach())
    expect = (w.float()[:, None] * g).cpu().numpy()
    np.testing.assert_allclose(th.grad.cpu().numpy(), expect, rtol=1e-6)
