"""GPU parity of the matrix-core PSF pass.

A whole-image launch (here P = 512 vectors, one row band each) with a PSF of at most 21 x 21
takes the matrix-core PSF pass; small launches take the banded VALU kernels. These cases use
asymmetric PSFs (a wrong flip or transposition shows) and ragged image shapes (partial tiles in
both directions, images smaller than the PSF, the largest tile count one workgroup takes).
Sampled vectors of the large launch are compared with the oracle, and with the same vectors
run through a small launch.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import assert_grad_close, assert_logl_close, oracle_model

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

P = 512
SAMPLE = [0, 1, 97, 255, 256, 400, 510, 511]

CASES = [
    # H, W, k, K, epl, lens_light, nmax, shear
    (37, 23, 2, 5, True, True, 2, True),      # partial tiles, 16 output columns per tile
    (64, 48, 2, 21, True, True, 6, True),     # 12 output columns per tile
    (31, 31, 1, 17, False, False, 4, True),   # K = 17: 16 columns per tile
    (100, 100, 1, 21, True, True, 0, True),   # 7 x 9 = 63 tiles (16 per wave)
    (17, 29, 1, 1, False, True, -1, False),   # no PSF
    (9, 10, 2, 19, True, True, 1, True),      # image smaller than the PSF
]


@pytest.fixture(scope="module")
def glens():
    import paper_2202_07663_amd as g
    return g


def _run(model, theta):
    th = torch.from_numpy(np.ascontiguousarray(theta, np.float32)).cuda()
    ll, g = model.loglik_grad(th)
    torch.cuda.synchronize()
    return ll.cpu().numpy(), g.cpu().numpy()


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}k{c[2]}K{c[3]}" for c in CASES])
def test_matrix_core_psf_pass(glens, case):
    H, W, k, K, epl, ll_on, nmax, shear = case
    print("case", case, flush=True)
    psf = synth.asymmetric_psf(K, seed=K) if K > 1 else np.ones((1, 1), np.float32)
    spec = synth.Spec("x", H, W, k, epl=epl, lens_light=ll_on, nmax=nmax, psf=psf,
                      sigma_bkg=0.1, t_exp=1000.0, shear=shear)
    truth = synth.draw_truth(spec, 11)
    om = oracle_model(spec)
    obs = synth.add_noise(oracle.simulate(om, truth.astype(np.float64))[0], 11, spec.sigma_bkg,
                          spec.t_exp)
    theta = synth.draw_particles(spec, truth, P, seed=5)
    m = glens.Model.from_spec(spec, obs)
    ll, g = _run(m, theta)
    idx = np.array(SAMPLE)
    ll_ref, g_ref = oracle.loglik_grad(om, theta[idx].astype(np.float64), obs)
    e1 = assert_logl_close(ll[idx], ll_ref)
    e2 = assert_grad_close(g[idx], g_ref, names=spec.names)
    # the same vectors in a small launch (banded VALU PSF kernels): both paths are FP32
    # computations of the same sums, so their distances to the oracle are of one size
    ll_s, g_s = _run(m, theta[idx])
    f1 = assert_logl_close(ll_s, ll_ref)
    f2 = assert_grad_close(g_s, g_ref, names=spec.names)
    print("matrix cores: logl err", e1, "grad err", e2, "| VALU: logl err", f1, "grad err", f2,
          flush=True)
    assert e1 <= 3 * f1 + 1e-6 and e2[0] <= 3 * f2[0] + 1e-6
    # model images of the large launch (the image-only mode of the pass)
    img = m.simulate(torch.from_numpy(theta).cuda()).cpu().numpy()
    ref = oracle.simulate(om, theta[idx].astype(np.float64))
    err = np.abs(img[idx] - ref) / np.abs(ref).max(axis=(1, 2), keepdims=True)
    assert err.max() < 2e-5, err.max()
    m.close()


def test_non_finite_vector_is_isolated_in_matrix_core_pass(glens):
    """A NaN parameter vector in a 512-vector launch gets log L = -inf; the other vectors'
    results are bitwise those of the same launch with a finite vector in its place (each
    particle's image scale and sums are its own)."""
    spec = synth.spec_c2()
    from tests.helpers import load_workload
    obs, truth = load_workload(spec.name)
    theta = synth.draw_particles(spec, truth, P, seed=9)
    m = glens.Model.from_spec(spec, obs)
    ll_a, g_a = _run(m, theta)
    bad = theta.copy()
    bad[7, 0] = np.nan
    ll_b, g_b = _run(m, bad)
    keep = np.arange(P) != 7
    assert ll_b[7] == -np.inf
    np.testing.assert_array_equal(ll_a[keep], ll_b[keep])
    np.testing.assert_array_equal(g_a[keep], g_b[keep])
    m.close()
