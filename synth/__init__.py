"""Seeded synthetic inputs for the lens-model workloads.

Shared by the tests, the benchmark and the stored-workload script. It draws parameter
vectors, builds PSF kernels and applies the paper's noise model to a clean image; it holds
none of the lens model's arithmetic (deflection, light profiles, downsampling,
convolution, likelihood). Every array it returns is already rounded to float32, the
product's input precision, so that both sides of a parity test consume identical values.

Parameter layout (one row per parameter vector), following the paper's parameter list
(Sec. 2.1.2, eq. sim-dist):
  mass:       theta_E, [gamma_epl], eps1, eps2, x, y, gamma_ext1, gamma_ext2
  lens light: R, n, eps1, eps2, x, y, I                       (optional)
  source:     R, n, eps1, eps2, x, y, I
  shapelets:  beta, c_0 .. c_{M-1}                            (optional)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PIX = 0.065  # arcsec per pixel (Sec. 3: HST WFC3 cut-outs at 0.065")


# ----------------------------------------------------------------------------------------
# PSF kernels (the paper's TinyTim PSF is not available; these stand in for it).
# Point-sampled at pixel centres on a K x K grid and normalised to unit sum.
# ----------------------------------------------------------------------------------------

def _radius2(K: int, pix: float) -> np.ndarray:
    c = (K - 1) / 2
    i = (np.arange(K) - c) * pix
    return i[:, None] ** 2 + i[None, :] ** 2


def gaussian_psf(K: int, fwhm: float, pix: float = PIX) -> np.ndarray:
    sigma = fwhm / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    k = np.exp(-0.5 * _radius2(K, pix) / sigma ** 2)
    return (k / k.sum()).astype(np.float32)


def moffat_psf(K: int, fwhm: float, beta: float, pix: float = PIX) -> np.ndarray:
    a = fwhm / (2.0 * np.sqrt(2.0 ** (1.0 / beta) - 1.0))
    k = (1.0 + _radius2(K, pix) / a ** 2) ** (-beta)
    return (k / k.sum()).astype(np.float32)


def asymmetric_psf(K: int, seed: int = 0) -> np.ndarray:
    """A deliberately lopsided kernel: tells convolution from correlation in tests."""
    rng = np.random.default_rng(seed)
    k = rng.uniform(0.0, 1.0, size=(K, K))
    k[0, :] *= 3.0
    return (k / k.sum()).astype(np.float32)


# ----------------------------------------------------------------------------------------
# Image / model specification
# ----------------------------------------------------------------------------------------

@dataclass
class Spec:
    name: str
    H: int
    W: int
    k: int
    epl: bool
    lens_light: bool
    nmax: int
    psf: np.ndarray
    sigma_bkg: float
    t_exp: float
    gain: float = 1.0
    shear: bool = True
    pix: float = PIX
    dist: str = "workload"  # "paper": the paper's simulation distribution and prior
    names: list = field(default_factory=list)

    def __post_init__(self):
        self.names = param_names(self.epl, self.shear, self.lens_light, self.nmax)

    @property
    def d(self) -> int:
        return len(self.names)


def n_shapelet_coeffs(nmax: int) -> int:
    return 0 if nmax < 0 else (nmax + 1) * (nmax + 2) // 2


def param_names(epl: bool, shear: bool, lens_light: bool, nmax: int) -> list:
    names = ["theta_E"] + (["gamma"] if epl else []) + ["e1", "e2", "x", "y"]
    if shear:
        names += ["gamma1", "gamma2"]
    if lens_light:
        names += ["l_R", "l_n", "l_e1", "l_e2", "l_x", "l_y", "l_I"]
    names += ["s_R", "s_n", "s_e1", "s_e2", "s_x", "s_y", "s_I"]
    if nmax >= 0:
        names += ["beta"] + [f"c{i}" for i in range(n_shapelet_coeffs(nmax))]
    return names


def spec_c1() -> Spec:
    """SIE + shear, Sersic source, 40x40 at 0.065", k = 1, Gaussian FWHM 0.08" (11x11)."""
    return Spec("sie40", 40, 40, 1, epl=False, lens_light=False, nmax=-1,
                psf=gaussian_psf(11, 0.08), sigma_bkg=0.1, t_exp=1000.0)


def spec_c2() -> Spec:
    """EPL + shear, Sersic lens light, Sersic + shapelets (n_max = 6) source, 60x60 at
    0.065", k = 2, Moffat 21x21 (FWHM 0.15", beta 2.5)."""
    return Spec("epl60", 60, 60, 2, epl=True, lens_light=True, nmax=6,
                psf=moffat_psf(21, 0.15, 2.5), sigma_bkg=0.1, t_exp=1000.0)


def spec_paper80() -> Spec:
    """The configuration of the paper's simulated systems (Sec. 3): EPL + shear, Sersic lens
    light, Sersic source (22 parameters), 80x80 at 0.065", k = 2, sigma_bkg = 0.2, t_exp =
    100 s, gain 1. The paper's HST PSF model is not available: a Moffat 21x21 (FWHM 0.15",
    beta 2.5) stands in for it."""
    return Spec("paper80", 80, 80, 2, epl=True, lens_light=True, nmax=-1,
                psf=moffat_psf(21, 0.15, 2.5), sigma_bkg=0.2, t_exp=100.0, dist="paper")


# The paper's simulation distribution and (broadened) prior of eq. sim-dist, per parameter
# in the gl.h order (EPL + shear, Sersic lens light, Sersic source): (family, simulation
# arguments, prior arguments). ln = log-normal (median, sigma of the log), tn = truncated
# normal (mean, sigma, low, high), n = normal (mean, sigma), u = uniform (low, high).
# Reading: the paper's half-light intensities I_l, I_s are surface brightnesses per square
# arcsecond (with them its arcs have the quoted signal-to-noise of about 100), while the
# amplitude of this library's Sersic profile is the value of a pixel; PAPER_AMP_INDEX marks
# the two amplitudes, whose medians are multiplied by the pixel area.
PAPER_DIST = [
    ("ln", (1.25, 0.25), (1.25, 0.4)),             # theta_E
    ("tn", (2.0, 0.25, 1.0, 3.0), (2.0, 0.5, 1.0, 3.0)),  # gamma_epl
    ("n", (0.0, 0.1), (0.0, 0.2)), ("n", (0.0, 0.1), (0.0, 0.2)),      # eps_epl
    ("n", (0.0, 0.03), (0.0, 0.06)), ("n", (0.0, 0.03), (0.0, 0.06)),  # lens centre
    ("n", (0.0, 0.05), (0.0, 0.1)), ("n", (0.0, 0.05), (0.0, 0.1)),    # external shear
    ("ln", (1.6, 0.15), (1.6, 0.25)),              # R_l
    ("u", (2.0, 6.0), (0.5, 8.0)),                 # n_l
    ("tn", (0.0, 0.05, -0.15, 0.15), (0.0, 0.1, -0.15, 0.15)),
    ("tn", (0.0, 0.05, -0.15, 0.15), (0.0, 0.1, -0.15, 0.15)),         # eps_l
    ("n", (0.0, 0.01), (0.0, 0.02)), ("n", (0.0, 0.01), (0.0, 0.02)),  # lens light centre
    ("ln", (300.0, 0.3), (300.0, 0.5)),            # I_l
    ("ln", (0.25, 0.15), (0.25, 0.25)),            # R_s
    ("u", (0.5, 4.0), (0.5, 8.0)),                 # n_s
    ("tn", (0.0, 0.15, -0.5, 0.5), (0.0, 0.3, -0.5, 0.5)),
    ("tn", (0.0, 0.15, -0.5, 0.5), (0.0, 0.3, -0.5, 0.5)),             # eps_s
    ("n", (0.0, 0.25), (0.0, 0.5)), ("n", (0.0, 0.25), (0.0, 0.5)),    # source centre
    ("ln", (150.0, 0.5), (150.0, 0.9)),            # I_s
]


PAPER_AMP_INDEX = (14, 21)


def _paper_median(i, median, pix):
    return median * pix * pix if i in PAPER_AMP_INDEX else median


def paper_sim_params(rng: np.random.Generator, size: int, pix: float = PIX) -> np.ndarray:
    """Draws from the paper's simulation distribution (eq. sim-dist), [size, 22]."""
    cols = []
    for i, (fam, a, _) in enumerate(PAPER_DIST):
        if fam == "ln":
            cols.append(np.exp(rng.normal(np.log(_paper_median(i, a[0], pix)), a[1], size)))
        elif fam == "tn":
            cols.append(_trunc_normal(rng, a[0], a[1], a[2], a[3], size))
        elif fam == "n":
            cols.append(rng.normal(a[0], a[1], size))
        else:
            cols.append(rng.uniform(a[0], a[1], size))
    return np.stack(cols, axis=1).astype(np.float32)


def spec_custom(N: int, k: int, epl: bool, lens_light: bool, nmax: int, K: int = 21,
                sigma_bkg: float = 0.1, t_exp: float = 1000.0, shear: bool = True) -> Spec:
    psf = moffat_psf(K, 0.15, 2.5) if K > 1 else np.ones((1, 1), np.float32)
    return Spec(f"n{N}k{k}{'epl' if epl else 'sie'}{'L' if lens_light else ''}s{nmax}",
                N, N, k, epl=epl, lens_light=lens_light, nmax=nmax, psf=psf,
                sigma_bkg=sigma_bkg, t_exp=t_exp, shear=shear)


# ----------------------------------------------------------------------------------------
# Parameter draws
# ----------------------------------------------------------------------------------------

def _trunc_normal(rng, mu, sigma, lo, hi, size=None):
    out = rng.normal(mu, sigma, size=size)
    bad = (out < lo) | (out > hi)
    while np.any(bad):
        out = np.where(bad, rng.normal(mu, sigma, size=np.shape(out)), out)
        bad = (out < lo) | (out > hi)
    return out


def _ellipticity(rng, sigma, max_abs, size):
    e = rng.normal(0.0, sigma, size=(size, 2))
    bad = np.hypot(e[:, 0], e[:, 1]) >= max_abs
    while np.any(bad):
        e[bad] = rng.normal(0.0, sigma, size=(int(bad.sum()), 2))
        bad = np.hypot(e[:, 0], e[:, 1]) >= max_abs
    return e


def draw_params(spec: Spec, rng: np.random.Generator, size: int, broad: float = 1.0) -> np.ndarray:
    """Parameter vectors from the workload distribution (``broad`` = 1) or a broadened
    version of it (``broad`` = 2, the prior the particles start from).

    Mass: theta_E ~ U[1, 1.5], gamma ~ U[1.8, 2.2], eps ~ N(0, 0.1) with |eps| < 0.4,
    centre ~ N(0, 0.05), shear ~ N(0, 0.05). Lens light: R ~ U[0.5, 1.5], n ~ U[2, 6],
    eps ~ TN(0, 0.05; +-0.15), centre ~ N(0, 0.01), I ~ lognormal(ln 300, 0.3) (eq.
    sim-dist). Source: R ~ U[0.1, 0.4], n ~ U[1, 4], eps ~ TN(0, 0.15; +-0.5) (eq.
    sim-dist), centre ~ N(0, 0.1), I ~ U[5, 20]. Shapelets: beta ~ U[0.05, 0.2], c ~ N(0, 1).
    """
    b = broad
    n = size

    def uni(lo, hi):
        # broadened about the centre; positive quantities never drop below half their
        # original lower bound
        c, h = 0.5 * (lo + hi), 0.5 * (hi - lo) * b
        return rng.uniform(max(c - h, 0.5 * lo) if b != 1.0 else lo, c + h, size=n)

    cols = [uni(1.0, 1.5)]
    if spec.epl:
        cols.append(uni(1.8, 2.2))
    e = _ellipticity(rng, 0.1 * b, 0.4 if b == 1.0 else 0.5, n)
    cols += [e[:, 0], e[:, 1], rng.normal(0, 0.05 * b, n), rng.normal(0, 0.05 * b, n)]
    if spec.shear:
        cols += [rng.normal(0, 0.05 * b, n), rng.normal(0, 0.05 * b, n)]
    if spec.lens_light:
        cols += [uni(0.5, 1.5), uni(2.0, 6.0),
                 _trunc_normal(rng, 0, 0.05 * b, -0.15, 0.15, n),
                 _trunc_normal(rng, 0, 0.05 * b, -0.15, 0.15, n),
                 rng.normal(0, 0.01 * b, n), rng.normal(0, 0.01 * b, n),
                 np.exp(rng.normal(np.log(300.0), 0.3 * b, n))]
    cols += [uni(0.1, 0.4), uni(1.0, 4.0),
             _trunc_normal(rng, 0, 0.15 * b, -0.5, 0.5, n),
             _trunc_normal(rng, 0, 0.15 * b, -0.5, 0.5, n),
             rng.normal(0, 0.1 * b, n), rng.normal(0, 0.1 * b, n), uni(5.0, 20.0)]
    if spec.nmax >= 0:
        cols.append(uni(0.05, 0.2))
        for _ in range(n_shapelet_coeffs(spec.nmax)):
            cols.append(rng.normal(0, 1.0 * b, n))
    out = np.stack(cols, axis=1)
    assert out.shape == (n, spec.d)
    return out.astype(np.float32)


def param_spread(spec: Spec) -> np.ndarray:
    """Standard deviation of each parameter's workload distribution (used to size the
    perturbations of the particles drawn around the truth)."""
    u = lambda lo, hi: (hi - lo) / np.sqrt(12.0)  # noqa: E731
    s = [u(1.0, 1.5)] + ([u(1.8, 2.2)] if spec.epl else []) + [0.1, 0.1, 0.05, 0.05]
    if spec.shear:
        s += [0.05, 0.05]
    if spec.lens_light:
        s += [u(0.5, 1.5), u(2, 6), 0.05, 0.05, 0.01, 0.01, 300 * 0.3]
    s += [u(0.1, 0.4), u(1, 4), 0.15, 0.15, 0.1, 0.1, u(5, 20)]
    if spec.nmax >= 0:
        s += [u(0.05, 0.2)] + [1.0] * n_shapelet_coeffs(spec.nmax)
    return np.asarray(s)


def draw_truth(spec: Spec, seed: int) -> np.ndarray:
    if spec.dist == "paper":
        return paper_sim_params(np.random.default_rng(seed), 1, spec.pix)[0]
    return draw_params(spec, np.random.default_rng(seed), 1)[0]


def draw_particles(spec: Spec, truth: np.ndarray, P: int, seed: int,
                   near_frac: float = 0.5, near_scale: float = 0.01) -> np.ndarray:
    """P parameter vectors: the first round(near_frac * P) are the truth plus a Gaussian
    perturbation of near_scale * max(|truth|, spread) per parameter; the rest come from the
    broadened (x2) workload distribution."""
    rng = np.random.default_rng(10_000 + seed)
    n_near = int(round(near_frac * P))
    scale = near_scale * np.maximum(np.abs(truth.astype(np.float64)), param_spread(spec))
    near = truth[None, :].astype(np.float64) + rng.normal(size=(n_near, spec.d)) * scale
    far = draw_params(spec, rng, P - n_near, broad=2.0).astype(np.float64)
    return np.concatenate([near, far], axis=0).astype(np.float32)


def add_noise(clean: np.ndarray, seed: int, sigma_bkg: float, t_exp: float,
              gain: float = 1.0) -> np.ndarray:
    """Observed image from a clean model image: Poisson shot noise on the expected counts
    max(I, 0) G t_exp, converted back to counts/s, plus Gaussian background noise
    (the noise model of Sec. 2.1.2)."""
    rng = np.random.default_rng(20_000 + seed)
    lam = np.maximum(np.asarray(clean, np.float64), 0.0) * gain * t_exp
    shot = rng.poisson(lam) / (gain * t_exp)
    return (shot + rng.normal(0.0, sigma_bkg, size=np.shape(clean))).astype(np.float32)


def add_gaussian_noise(clean: np.ndarray, seed: int, sigma_bkg: float, t_exp: float,
                       gain: float = 1.0) -> np.ndarray:
    """Observed image whose noise is Gaussian with the variance the likelihood assumes,
    sigma_bkg^2 + max(I, 0) / (G t_exp): the Poisson shot noise's first two moments
    without its skewness."""
    rng = np.random.default_rng(20_000 + seed)
    c = np.asarray(clean, np.float64)
    sd = np.sqrt(sigma_bkg ** 2 + np.maximum(c, 0.0) / (gain * t_exp))
    return (c + rng.normal(size=np.shape(clean)) * sd).astype(np.float32)


# ----------------------------------------------------------------------------------------
# Fit priors (passed to the fit as gl_prior entries). Families and widths follow the
# paper's broadened prior (blue entries of eq. sim-dist) where its parameter and scale
# match these workloads; lens-light radius, source radius and source intensity are centred
# on these workloads' draws instead. Shapelets (no prior in the paper): beta uniform on
# (0.02, 0.4), coefficients N(0, 2) (the draws' N(0, 1) broadened by the paper's factor 2).
# ----------------------------------------------------------------------------------------
NORMAL, LOGNORMAL, TRUNCNORMAL, UNIFORM = 0, 1, 2, 3


def fit_priors(spec: Spec, matched: bool = False) -> list:
    """Per-parameter priors of the fit. matched (only for the paper's distribution): the
    simulation distribution itself instead of the paper's broadened prior."""
    def N(mu, s):
        return {"family": NORMAL, "mu": mu, "sigma": s, "lo": 0.0, "hi": 0.0}

    def LN(m, s):
        return {"family": LOGNORMAL, "mu": float(np.log(m)), "sigma": s, "lo": 0.0, "hi": 0.0}

    def TN(mu, s, lo, hi):
        return {"family": TRUNCNORMAL, "mu": mu, "sigma": s, "lo": lo, "hi": hi}

    def U(lo, hi):
        return {"family": UNIFORM, "mu": 0.0, "sigma": 1.0, "lo": lo, "hi": hi}

    if spec.dist == "paper":  # the prior of eq. sim-dist
        out = []
        for i, (f, a, b) in enumerate(PAPER_DIST):
            if matched:
                b = a
            if f == "ln":
                out.append(LN(_paper_median(i, b[0], spec.pix), b[1]))
            else:
                out.append({"tn": TN, "n": N, "u": U}[f](*b))
        return [dict(p) for p in out]
    pr = [LN(1.25, 0.4)] + ([TN(2.0, 0.5, 1.0, 3.0)] if spec.epl else [])
    pr += [N(0, 0.2), N(0, 0.2), N(0, 0.1), N(0, 0.1)]
    if spec.shear:
        pr += [N(0, 0.1), N(0, 0.1)]
    if spec.lens_light:
        pr += [LN(1.0, 0.5), U(0.5, 8.0), TN(0, 0.1, -0.15, 0.15), TN(0, 0.1, -0.15, 0.15),
               N(0, 0.02), N(0, 0.02), LN(300.0, 0.5)]
    pr += [LN(0.25, 0.5), U(0.5, 8.0), TN(0, 0.3, -0.5, 0.5), TN(0, 0.3, -0.5, 0.5),
           N(0, 0.5), N(0, 0.5), LN(12.0, 0.9)]
    if spec.nmax >= 0:
        # shapelets: beta over (0.02, 0.4) (draws U[0.05, 0.2]); coefficients N(0, 2), the
        # draws' N(0, 1) broadened x2 as every normal prior of eq. sim-dist is
        pr += [U(0.02, 0.4)] + [N(0, 2.0)] * n_shapelet_coeffs(spec.nmax)
    assert len(pr) == spec.d
    return [dict(p) for p in pr]
