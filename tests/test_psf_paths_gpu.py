"""GPU parity of every PSF-pass code path (Sec. 2.1.1: the image is finally convolved with the
PSF) at launch sizes that select it, against the FP64 oracle.

The library picks, per system and batch size (gl_model_plan):
  * the matrix-core pass for P >= 512 when K <= 21 and the image fits 64 tiles of 16 rows
    (and at any P for images of at most 8 rows, which make one band);
  * the whole-image VALU pass for P >= 512 otherwise (K = 23..31, or more than 64 tiles);
  * the banded VALU pass for P < 512 (one band: the whole-image kernel), with each strip's
    PSF columns split over 2 or 4 lanes when the batch is very small.
Each case asserts on the host which path the plan takes, runs the full launch, and compares a
sample of its vectors (log L, gradient, model image) with the oracle. The PSFs are asymmetric,
so a correlation in place of the convolution would fail.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import assert_grad_close, assert_logl_close, oracle_model

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    import paper_2202_07663_amd as g
    return g


def _say(*a):
    print(*a, flush=True)


# name, H, W, k, K, epl, lens_light, nmax, P, expected path, expected band split
CASES = [
    ("K25", 40, 36, 1, 25, False, False, 2, 512, "valu", 1),
    ("K31", 33, 41, 2, 31, True, True, 2, 512, "valu", 1),
    ("128x128K21", 128, 128, 1, 21, True, True, 4, 512, "valu", 1),    # 8 x 11 = 88 tiles
    ("128x100K21", 128, 100, 1, 21, False, True, -1, 512, "valu", 1),  # 8 x 9 = 72 tiles
    ("101x101K21", 101, 101, 1, 21, True, False, 2, 512, "mfma", 1),   # 7 x 9 = 63 tiles
    ("7x40K5", 7, 40, 2, 5, True, True, 3, 512, "mfma", 1),            # H < 8: one tile row
    ("5x9K9", 5, 9, 1, 9, False, False, 0, 600, "mfma", 1),            # image smaller than K
    ("24x44K19", 24, 44, 2, 19, True, False, 4, 512, "mfma", 1),       # 4 tile columns of 12
    ("24x44K19small", 24, 44, 2, 19, True, False, 4, 96, "banded", 4),
    ("K27small", 30, 30, 1, 27, False, True, 1, 64, "banded", 4),
    ("40x40K21P256", 40, 40, 1, 21, True, True, 6, 256, "banded", 2),  # 2 lanes per strip
    ("60x60K21P300", 60, 60, 2, 21, True, True, 6, 300, "banded", 1),  # 2 bands, unsplit
    ("7x40K5small", 7, 40, 1, 5, False, False, 2, 8, "mfma", 1),       # H <= 8: one band
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_psf_path_parity(G, case):
    name, H, W, k, K, epl, ll_on, nmax, P, path, split = case
    psf = synth.asymmetric_psf(K, seed=K + H)
    spec = synth.Spec(name, H, W, k, epl=epl, lens_light=ll_on, nmax=nmax, psf=psf,
                      sigma_bkg=0.1, t_exp=1000.0)
    truth = synth.draw_truth(spec, 40 + K)
    om = oracle_model(spec)
    obs = synth.add_noise(oracle.simulate(om, truth.astype(np.float64))[0], 40 + K,
                          spec.sigma_bkg, spec.t_exp)
    theta = synth.draw_particles(spec, truth, P, seed=K)
    m = G.Model.from_spec(spec, obs)
    plan = m.plan(P)
    _say("case", name, "P", P, "plan", plan)
    assert plan["psf_path"] == path
    assert plan["band_split"] == split
    th = torch.from_numpy(theta).cuda()
    ll, g = m.loglik_grad(th)
    ll_only = m.loglik(th)
    img = m.simulate(th)
    torch.cuda.synchronize()
    ll, g, ll_only, img = (t.cpu().numpy() for t in (ll, g, ll_only, img))
    idx = np.unique(np.r_[0, 1, P // 3, P // 2 + 1, P - 2, P - 1])
    ll_ref, g_ref = oracle.loglik_grad(om, theta[idx].astype(np.float64), obs)
    e1 = assert_logl_close(ll[idx], ll_ref)
    e2 = assert_grad_close(g[idx], g_ref, names=spec.names)
    np.testing.assert_array_equal(ll, ll_only)  # the same PSF pass with and without the adjoint
    ref = oracle.simulate(om, theta[idx].astype(np.float64))
    err = np.abs(img[idx] - ref) / np.abs(ref).max(axis=(1, 2), keepdims=True)
    _say(name, "logl err", e1, "grad err", e2, "image err", err.max())
    assert err.max() < 2e-5
