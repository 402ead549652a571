"""Pins of the FP64 oracle to things other than itself: library routines (scipy), closed
forms, invariants of lensing, and brute force on tiny inputs. CPU only.

Each test names the passage of the paper (arXiv:2202.07663) or the mathematics it checks.
"""
import numpy as np
import pytest
from scipy import integrate, signal, special, stats

import oracle
import synth

RNG = np.random.default_rng(1234)


def _fd_jacobian(fun, x, y, h=1e-6):
    """Central-difference Jacobian of a 2-vector field (ax, ay) at points (x, y)."""
    axp, ayp = fun(x + h, y)
    axm, aym = fun(x - h, y)
    bxp, byp = fun(x, y + h)
    bxm, bym = fun(x, y - h)
    return ((axp - axm) / (2 * h), (bxp - bxm) / (2 * h),
            (ayp - aym) / (2 * h), (byp - bym) / (2 * h))


def _points(n=64, rmin=0.3, rmax=2.5, seed=0):
    rng = np.random.default_rng(seed)
    r = rng.uniform(rmin, rmax, n)
    a = rng.uniform(0, 2 * np.pi, n)
    return r * np.cos(a), r * np.sin(a)


# ------------------------------------------------------------------------------------------
# EPL (Sec. 2.1.1; deflection via the Gauss hypergeometric function)
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("t", [0.4, 0.8, 1.0, 1.2, 1.6])
def test_hyp2f1_series_matches_scipy(t):
    """The series equals scipy's 2F1(1, t/2; 2 - t/2; z) for complex |z| < 1."""
    rng = np.random.default_rng(int(t * 10))
    rad = rng.uniform(0, 0.75, 200)
    ang = rng.uniform(0, 2 * np.pi, 200)
    z = rad * np.exp(1j * ang)
    got = oracle.hyp2f1(t, z)
    ref = special.hyp2f1(1.0, t / 2, 2 - t / 2, z)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-14)


def test_hyp2f1_series_truncation_consistent_with_paper():
    """Sec. 2.1.1: < 1e-16 truncation error within 35 terms for q >~ 0.5. For q = 0.5,
    |z| = (1-q)/(1+q) = 1/3 and every coefficient is at most 1, so the tail after 35 terms
    is below (1/3)^35 / (1 - 1/3) ~ 2.3e-17: the series sum agrees with scipy to ~1e-16."""
    z = (1 / 3) * np.exp(1j * np.linspace(0, 2 * np.pi, 50))
    got = oracle.hyp2f1(1.0, z)
    ref = special.hyp2f1(1.0, 0.5, 1.5, z)
    assert np.max(np.abs(got - ref)) < 8 * np.finfo(float).eps  # rounding, not truncation
    assert (1 / 3) ** 35 / (2 / 3) < 1e-16


@pytest.mark.parametrize("gamma,e1,e2", [(2.0, 0.1, -0.05), (1.7, -0.2, 0.15), (2.3, 0.05, 0.3),
                                         (2.0, 0.35, 0.2), (1.5, 0.0, 0.4)])
def test_epl_divergence_is_twice_kappa(gamma, e1, e2):
    """div alpha = 2 kappa (Poisson equation of lensing) with kappa exactly as printed in
    Sec. 2.1.1. Pins the deflection's normalisation and its dependence on q and gamma."""
    x, y = _points()
    f = lambda xx, yy: oracle.epl_deflection(xx, yy, 1.2, gamma, e1, e2, 0.03, -0.02)  # noqa
    dxx, dxy, dyx, dyy = _fd_jacobian(f, x, y)
    kappa = oracle.epl_kappa(x, y, 1.2, gamma, e1, e2, 0.03, -0.02)
    np.testing.assert_allclose(dxx + dyy, 2 * kappa, rtol=2e-7, atol=1e-8)


@pytest.mark.parametrize("gamma,e1,e2", [(2.0, 0.1, -0.05), (1.7, -0.2, 0.15), (2.3, 0.05, 0.3)])
def test_epl_curl_free(gamma, e1, e2):
    """alpha is a gradient field, so its curl vanishes. A conjugated series term or a
    wrongly oriented back-rotation breaks this."""
    x, y = _points(seed=1)
    f = lambda xx, yy: oracle.epl_deflection(xx, yy, 1.1, gamma, e1, e2, -0.04, 0.05)  # noqa
    dxx, dxy, dyx, dyy = _fd_jacobian(f, x, y)
    np.testing.assert_allclose(dxy, dyx, atol=2e-8)


@pytest.mark.parametrize("gamma,e1,e2", [(1.8, 0.12, 0.07), (2.2, -0.25, 0.1)])
def test_epl_is_gradient_of_homogeneous_potential(gamma, e1, e2):
    """kappa is homogeneous of degree 1 - gamma about the lens centre, so the potential is
    psi = (x - x_c) . alpha / (3 - gamma) and grad psi = alpha."""
    xc, yc = 0.02, -0.03
    psi = lambda xx, yy: ((xx - xc) * oracle.epl_deflection(xx, yy, 1.3, gamma, e1, e2, xc, yc)[0]  # noqa
                          + (yy - yc) * oracle.epl_deflection(xx, yy, 1.3, gamma, e1, e2, xc, yc)[1]) / (3 - gamma)
    x, y = _points(seed=2)
    h = 1e-6
    gx = (psi(x + h, y) - psi(x - h, y)) / (2 * h)
    gy = (psi(x, y + h) - psi(x, y - h)) / (2 * h)
    ax, ay = oracle.epl_deflection(x, y, 1.3, gamma, e1, e2, xc, yc)
    np.testing.assert_allclose(gx, ax, rtol=1e-7, atol=1e-8)
    np.testing.assert_allclose(gy, ay, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("gamma", [1.5, 1.9, 2.0, 2.4])
def test_epl_circular_power_law(gamma):
    """q = 1: alpha is radial with |alpha| = theta_E (r / theta_E)^(2 - gamma) (enclosed
    mass of a circular power law)."""
    x, y = _points(seed=3)
    te = 1.25
    ax, ay = oracle.epl_deflection(x, y, te, gamma, 0.0, 0.0)
    r = np.hypot(x, y)
    np.testing.assert_allclose(np.hypot(ax, ay), te * (r / te) ** (2 - gamma), rtol=1e-13)
    np.testing.assert_allclose(ax * y - ay * x, 0.0, atol=1e-13)


@pytest.mark.parametrize("e1,e2", [(0.1, 0.0), (0.2, -0.3), (-0.05, 0.02), (0.4, 0.1)])
def test_epl_slope_two_equals_sie_closed_form(e1, e2):
    """gamma = 2 (t = 1) reduces the series to the SIE closed form (atan / atanh)."""
    x, y = _points(seed=4)
    a1 = oracle.epl_deflection(x, y, 1.2, 2.0, e1, e2, 0.01, 0.02)
    a2 = oracle.sie_deflection(x, y, 1.2, e1, e2, 0.01, 0.02)
    np.testing.assert_allclose(a1[0], a2[0], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(a1[1], a2[1], rtol=1e-12, atol=1e-13)


def test_epl_major_axis_orientation():
    """(eps1, eps2) = (1-q)/(1+q) (cos 2phi, sin 2phi) and the frame rotation of eq.
    coord-trans put the major axis at position angle phi: kappa at distance a along the
    major axis equals kappa at distance a q along the minor axis."""
    for phi in [0.0, 0.3, np.pi / 4, 1.2]:
        q = 0.6
        f = (1 - q) / (1 + q)
        e1, e2 = f * np.cos(2 * phi), f * np.sin(2 * phi)
        a = np.array([0.7, 1.1, 1.9])
        kmaj = oracle.epl_kappa(a * np.cos(phi), a * np.sin(phi), 1.2, 2.1, e1, e2)
        kmin = oracle.epl_kappa(-a * q * np.sin(phi), a * q * np.cos(phi), 1.2, 2.1, e1, e2)
        np.testing.assert_allclose(kmaj, kmin, rtol=1e-12)
        kmin_far = oracle.epl_kappa(-a * np.sin(phi), a * np.cos(phi), 1.2, 2.1, e1, e2)
        assert np.all(kmaj > kmin_far)


def test_sie_pins():
    """SIE: div alpha = 2 kappa with kappa = theta_E / (2 sqrt(q x^2 + y^2/q)); curl-free;
    q -> 1 gives |alpha| = theta_E."""
    x, y = _points(seed=5)
    f = lambda xx, yy: oracle.sie_deflection(xx, yy, 1.3, 0.15, -0.1, 0.02, 0.01)  # noqa
    dxx, dxy, dyx, dyy = _fd_jacobian(f, x, y)
    kappa = oracle.epl_kappa(x, y, 1.3, 2.0, 0.15, -0.1, 0.02, 0.01)
    np.testing.assert_allclose(dxx + dyy, 2 * kappa, rtol=2e-7, atol=1e-8)
    np.testing.assert_allclose(dxy, dyx, atol=2e-8)
    ax, ay = oracle.sie_deflection(x, y, 1.3, 1e-9, 0.0)
    np.testing.assert_allclose(np.hypot(ax, ay), 1.3, rtol=1e-7)
    ax, ay = oracle.sie_deflection(x, y, 1.3, 0.0, 0.0)
    np.testing.assert_allclose(np.hypot(ax, ay), 1.3, rtol=1e-14)


def test_mass_ellipticity_clamp():
    """Reading: |eps| above 0.6 is rescaled onto 0.6 (q stays positive)."""
    x, y = _points(seed=6)
    a = oracle.epl_deflection(x, y, 1.2, 2.0, 0.9, 0.0)
    b = oracle.epl_deflection(x, y, 1.2, 2.0, 0.6, 0.0)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-14)


# ------------------------------------------------------------------------------------------
# External shear (eq. alpha_ext)
# ------------------------------------------------------------------------------------------

def test_shear_hessian():
    """alpha_ext is the gradient of psi = g1 (x^2 - y^2)/2 + g2 x y: Hessian
    [[g1, g2], [g2, -g1]], zero divergence (no mass)."""
    x, y = _points(seed=7)
    g1, g2 = 0.04, -0.07
    f = lambda xx, yy: oracle.shear_deflection(xx, yy, g1, g2)  # noqa
    dxx, dxy, dyx, dyy = _fd_jacobian(f, x, y)
    np.testing.assert_allclose(dxx, g1, atol=1e-9)
    np.testing.assert_allclose(dyy, -g1, atol=1e-9)
    np.testing.assert_allclose(dxy, g2, atol=1e-9)
    np.testing.assert_allclose(dyx, g2, atol=1e-9)
    psi = lambda xx, yy: g1 * (xx ** 2 - yy ** 2) / 2 + g2 * xx * yy  # noqa
    h = 1e-6
    ax, ay = oracle.shear_deflection(x, y, g1, g2)
    np.testing.assert_allclose(ax, (psi(x + h, y) - psi(x - h, y)) / (2 * h), atol=1e-9)


# ------------------------------------------------------------------------------------------
# Sersic (eq. Sersic, b_n = 1.9992 n - 0.3271)
# ------------------------------------------------------------------------------------------

def _sersic_flux_within(R, n, i0, r_eff):
    bn = 1.9992 * n - 0.3271
    x = bn * (R / r_eff) ** (1 / n)
    return 2 * np.pi * n * i0 * r_eff ** 2 * np.exp(bn) * special.gammainc(2 * n, x) * \
        special.gamma(2 * n) / bn ** (2 * n)


@pytest.mark.parametrize("n,e1,e2", [(1.0, 0.0, 0.0), (2.5, 0.2, -0.1), (4.0, -0.3, 0.25)])
def test_sersic_enclosed_flux(n, e1, e2):
    """The flux inside the isophote of elliptical radius R is the circular closed form
    2 pi n I0 R_eff^2 e^b_n gamma(2n, b_n (R/R_eff)^(1/n)) / b_n^(2n), whatever q and phi
    (the map to the light frame is a rotation plus an area-preserving stretch). Integrated
    numerically on the oracle's profile over an ellipse of q = 1 geometry in circular
    coordinates u = (sqrt(q) x_l, y_l / sqrt(q))."""
    r_eff, i0, xc, yc = 0.4, 3.0, 0.05, -0.02
    eps = np.hypot(e1, e2)
    q = (1 - eps) / (1 + eps)
    phi = 0.5 * np.arctan2(e2, e1)
    Rmax = 2.0

    def integrand(theta, R):
        xl = R * np.cos(theta) / np.sqrt(q)
        yl = R * np.sin(theta) * np.sqrt(q)
        x = xc + np.cos(phi) * xl - np.sin(phi) * yl
        y = yc + np.sin(phi) * xl + np.cos(phi) * yl
        return oracle.sersic(np.array([x]), np.array([y]), r_eff, n, e1, e2, xc, yc, i0)[0] * R

    got, _ = integrate.dblquad(integrand, 0, Rmax, 0, 2 * np.pi, epsabs=1e-10, epsrel=1e-9)
    ref = _sersic_flux_within(Rmax, n, i0, r_eff)
    np.testing.assert_allclose(got, ref, rtol=2e-7)


def test_sersic_half_light_and_amplitude():
    """I0 is the intensity at R_eff, and b_n as printed makes R_eff enclose about half of
    the total light (Capaccioli's approximation: within 1% for 0.5 < n < 10)."""
    for n in [0.8, 1.5, 3.0, 6.0]:
        v = oracle.sersic(np.array([0.3]), np.array([0.0]), 0.3, n, 0, 0, 0, 0, 2.0)[0]
        np.testing.assert_allclose(v, 2.0, rtol=1e-14)
        half = _sersic_flux_within(0.3, n, 1.0, 0.3) / _sersic_flux_within(1e6, n, 1.0, 0.3)
        assert abs(half - 0.5) < 0.01


def test_sersic_orientation():
    """Same convention as the mass: equal intensity at a along the major axis and at a q
    along the minor axis."""
    phi, q = 0.7, 0.5
    f = (1 - q) / (1 + q)
    e1, e2 = f * np.cos(2 * phi), f * np.sin(2 * phi)
    a = np.array([0.2, 0.5])
    imaj = oracle.sersic(a * np.cos(phi), a * np.sin(phi), 0.4, 2.0, e1, e2, 0, 0, 1.0)
    imin = oracle.sersic(-a * q * np.sin(phi), a * q * np.cos(phi), 0.4, 2.0, e1, e2, 0, 0, 1.0)
    np.testing.assert_allclose(imaj, imin, rtol=1e-12)


# ------------------------------------------------------------------------------------------
# Shapelets (Refregier 2003; named in Sec. 4, no formula printed)
# ------------------------------------------------------------------------------------------

def test_hermite_functions_match_scipy():
    u = np.linspace(-4, 4, 41)
    nmax = 10
    got = oracle.hermite_functions(u, nmax)
    for n in range(nmax + 1):
        ref = special.eval_hermite(n, u) * np.exp(-u ** 2 / 2) / np.sqrt(
            2.0 ** n * np.sqrt(np.pi) * special.factorial(n))
        np.testing.assert_allclose(got[:, n], ref, rtol=1e-12, atol=1e-15)


def test_shapelet_basis_orthonormal():
    """int B_a B_b dx dy = delta_ab (Gauss-Hermite quadrature, exact for these
    polynomial-times-Gaussian integrands)."""
    nmax, beta, xc, yc = 6, 0.15, 0.03, -0.01
    M = (nmax + 1) * (nmax + 2) // 2
    t, w = special.roots_hermite(20)
    # B_a B_b = poly * exp(-(u^2+v^2)); integrate in u = (x-xc)/beta
    U, V = np.meshgrid(t, t, indexing="ij")
    Wt = np.outer(w, w) * np.exp(U ** 2 + V ** 2)
    x, y = xc + beta * U.ravel(), yc + beta * V.ravel()
    B = np.stack([oracle.shapelets(x, y, xc, yc, beta, np.eye(M)[i], nmax) for i in range(M)])
    G = (B * Wt.ravel()) @ B.T * beta ** 2
    np.testing.assert_allclose(G, np.eye(M), atol=1e-12)


def test_shapelet_b00_is_normalised_gaussian():
    x, y = np.array([0.1, -0.05, 0.0]), np.array([0.02, 0.1, 0.0])
    beta = 0.12
    got = oracle.shapelets(x, y, 0.0, 0.0, beta, np.array([1.0]), 0)
    ref = np.exp(-(x ** 2 + y ** 2) / (2 * beta ** 2)) / (np.sqrt(np.pi) * beta)
    np.testing.assert_allclose(got, ref, rtol=1e-14)


def test_shapelet_ordering():
    """Coefficient k runs over n = 0..n_max, n1 = n..0, n2 = n - n1 (reading): coefficient
    2 is (n1, n2) = (0, 1), i.e. the first Hermite function in y."""
    x, y = np.array([0.07]), np.array([0.04])
    beta = 0.1
    got = oracle.shapelets(x, y, 0, 0, beta, np.array([0, 0, 1.0]), 1)
    phi = oracle.hermite_functions(np.array([0.7, 0.4]), 1)
    np.testing.assert_allclose(got, phi[0, 0] * phi[1, 1] / beta, rtol=1e-14)


# ------------------------------------------------------------------------------------------
# Grid, downsampling, PSF (Sec. 2.1.1)
# ------------------------------------------------------------------------------------------

def _tiny_model(H=7, W=9, k=2, psf=None, epl=True, lens_light=True, nmax=2):
    psf = np.ones((1, 1)) if psf is None else psf
    return oracle.Model(H=H, W=W, k=k, pix=0.13, epl=epl, shear=True, lens_light=lens_light,
                        nmax=nmax, psf=psf, sigma_bkg=0.1, t_exp=500.0)


def _tiny_theta(m):
    spec = synth.Spec("t", m.H, m.W, m.k, m.epl, m.lens_light, m.nmax, psf=np.ones((1, 1)),
                      sigma_bkg=0.1, t_exp=1.0)
    th = synth.draw_truth(spec, 3).astype(np.float64)
    return th


def test_downsample_is_mean_of_subpixels_brute_force():
    """Pixel (i, j) centred at ((j - (W-1)/2) s, (i - (H-1)/2) s), sub-pixel (a, b) offset by
    (((b + 1/2)/k - 1/2) s, ((a + 1/2)/k - 1/2) s); the image pixel is their mean."""
    for k in (1, 2, 3):
        m = _tiny_model(k=k)
        th = _tiny_theta(m)
        img = oracle.simulate(m, th)[0]
        ref = np.zeros((m.H, m.W))
        for i in range(m.H):
            for j in range(m.W):
                xs, ys = [], []
                for a in range(k):
                    for b in range(k):
                        xs.append((j - (m.W - 1) / 2) * m.pix + ((b + 0.5) / k - 0.5) * m.pix)
                        ys.append((i - (m.H - 1) / 2) * m.pix + ((a + 0.5) / k - 0.5) * m.pix)
                ref[i, j] = oracle.surface_brightness(m, th, np.array(xs), np.array(ys)).mean()
        np.testing.assert_allclose(img, ref, rtol=1e-14, atol=1e-14)


def test_constant_surface_brightness_survives_downsampling():
    """With no lens light and a huge, flat source (n = 0.5 Sersic of enormous radius) the
    supersampled image is constant, and the k x k mean keeps it so."""
    m = _tiny_model(k=3, lens_light=False, nmax=-1)
    th = _tiny_theta(m)
    th[7:14] = [1e6, 0.5, 0.0, 0.0, 0.0, 0.0, 2.5]  # R, n, e1, e2, x, y, I
    img = oracle.simulate(m, th)[0]
    np.testing.assert_allclose(img, img[0, 0], rtol=1e-9)


def test_psf_is_scipy_convolve_same():
    """PSF: zero-padded 'same' convolution (not correlation: the kernel is lopsided)."""
    psf = synth.asymmetric_psf(5, seed=1).astype(np.float64)
    m1 = _tiny_model(H=11, W=8, psf=psf)
    m0 = _tiny_model(H=11, W=8)
    th = _tiny_theta(m1)
    low = oracle.simulate(m0, th)[0]
    got = oracle.simulate(m1, th)[0]
    ref = signal.convolve2d(low, psf, mode="same", boundary="fill", fillvalue=0.0)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-14)
    corr = signal.correlate2d(low, psf, mode="same", boundary="fill", fillvalue=0.0)
    assert np.max(np.abs(got - corr)) > 1e-3 * np.max(np.abs(got))


def test_psf_flux_conservation_interior():
    """A unit-sum PSF conserves the flux of a compact source far from the edges."""
    psf = synth.moffat_psf(7, 0.15, 2.5).astype(np.float64)
    m = _tiny_model(H=41, W=41, k=1, psf=psf, lens_light=False, nmax=-1)
    m0 = _tiny_model(H=41, W=41, k=1, lens_light=False, nmax=-1)
    th = _tiny_theta(m)
    th[0] = 1e-6  # negligible lensing: compact unlensed source at the centre
    th[5:7] = 0.0
    th[7:14] = [0.1, 1.0, 0.0, 0.0, 0.0, 0.0, 1.0]
    np.testing.assert_allclose(oracle.simulate(m, th).sum(), oracle.simulate(m0, th).sum(),
                               rtol=1e-9)


# ------------------------------------------------------------------------------------------
# Likelihood (eq. model-def)
# ------------------------------------------------------------------------------------------

def test_loglik_matches_scipy_norm():
    m = _tiny_model()
    rng = np.random.default_rng(0)
    img = rng.normal(2.0, 3.0, size=(m.H, m.W))   # includes negative model pixels
    obs = rng.normal(2.0, 3.0, size=(m.H, m.W))
    var = m.sigma_bkg ** 2 + np.maximum(img, 0) / (m.gain * m.t_exp)
    ref = stats.norm.logpdf(obs, img, np.sqrt(var)).sum()
    np.testing.assert_allclose(oracle.log_likelihood_image(m, img, obs), ref, rtol=1e-13)


def test_loglik_perfect_fit_is_normalisation_only():
    m = _tiny_model()
    img = np.abs(np.random.default_rng(1).normal(size=(m.H, m.W)))
    var = m.sigma_bkg ** 2 + img / (m.gain * m.t_exp)
    np.testing.assert_allclose(oracle.log_likelihood_image(m, img, img),
                               -0.5 * np.sum(np.log(2 * np.pi * var)), rtol=1e-14)


def test_loglik_of_simulate_consistent():
    m = _tiny_model()
    th = _tiny_theta(m)
    obs = np.random.default_rng(2).normal(size=(m.H, m.W))
    img = oracle.simulate(m, th)[0]
    np.testing.assert_allclose(oracle.loglik(m, th, obs)[0],
                               oracle.log_likelihood_image(m, img, obs), rtol=1e-14)


# ------------------------------------------------------------------------------------------
# Whole model: closed-form Einstein ring
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("epl", [False, True])
def test_einstein_ring_closed_form(epl):
    """SIS (eps = 0, slope 2, no shear) at the origin lensing a circular Sersic source at
    the origin, k = 1, delta PSF: beta = x (1 - theta_E/|x|), so the image is
    I_src(| |x| - theta_E |): a ring of the source's central brightness at |x| = theta_E."""
    m = oracle.Model(H=24, W=24, k=1, pix=0.1, epl=epl, shear=False, lens_light=False,
                     nmax=-1, psf=np.ones((1, 1)), sigma_bkg=0.1, t_exp=1.0)
    te = 0.8
    th = ([te, 2.0] if epl else [te]) + [0.0, 0.0, 0.0, 0.0] + [0.2, 1.5, 0.0, 0.0, 0.0, 0.0, 4.0]
    th = np.array(th)
    img = oracle.simulate(m, th)[0]
    jj, ii = np.meshgrid(np.arange(24), np.arange(24))
    r = np.hypot((jj - 11.5) * 0.1, (ii - 11.5) * 0.1)
    ref = oracle.sersic(np.abs(r - te), np.zeros_like(r), 0.2, 1.5, 0, 0, 0, 0, 4.0)
    bn = 1.9992 * 1.5 - 0.3271
    ref2 = 4.0 * np.exp(-bn * ((np.abs(r - te) / 0.2) ** (1 / 1.5) - 1))
    np.testing.assert_allclose(img, ref, rtol=1e-12)
    np.testing.assert_allclose(img, ref2, rtol=1e-12)


# ------------------------------------------------------------------------------------------
# Gradient: dual numbers vs FP64 central differences (h = 1e-5 max(1, |theta_i|))
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("epl,lens_light,nmax,k,K", [(False, False, -1, 1, 5), (True, True, 3, 2, 5),
                                                     (True, False, 1, 1, 3)])
def test_dual_gradient_matches_central_differences(epl, lens_light, nmax, k, K):
    psf = synth.asymmetric_psf(K, seed=2).astype(np.float64)
    m = oracle.Model(H=10, W=12, k=k, pix=0.15, epl=epl, shear=True, lens_light=lens_light,
                     nmax=nmax, psf=psf, sigma_bkg=0.2, t_exp=50.0)
    th = _tiny_theta(m)
    th += 0.02 * np.random.default_rng(5).normal(size=th.shape)  # away from the truth
    obs = oracle.simulate(m, _tiny_theta(m))[0] + np.random.default_rng(6).normal(0, 0.2, (m.H, m.W))
    ll, g = oracle.loglik_grad(m, th, obs)
    np.testing.assert_allclose(ll[0], oracle.loglik(m, th, obs)[0], rtol=1e-14)
    fd = np.zeros_like(th)
    for i in range(th.size):
        h = 1e-5 * max(1.0, abs(th[i]))
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (oracle.loglik(m, tp, obs)[0] - oracle.loglik(m, tm, obs)[0]) / (2 * h)
    scale = np.abs(g[0]) + 1e-6 * np.linalg.norm(g[0])
    assert np.max(np.abs(g[0] - fd) / scale) < 1e-5, (g[0], fd)
