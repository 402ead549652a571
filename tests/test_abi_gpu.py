"""C-ABI behaviour on the GPU: compute calls write their outputs only within [P] / [P][d] /
[P][H][W] and leave their inputs as they were, for batch sizes on each PSF path (banded,
matrix cores, whole-image VALU) and ragged tile counts; and they are ordered on the stream
they are given."""
import numpy as np
import pytest

import synth
from tests.helpers import load_workload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SENTINEL = 12345.678


@pytest.fixture(scope="module")
def G():
    import paper_2202_07663_amd as g
    return g


def _say(*a):
    print(*a, flush=True)


def _k25_system():
    """A 40x40 system with a 25x25 PSF (the whole-image VALU PSF kernel at P >= 512); its
    observed image is a flat 0.1 counts/s (any finite image serves here)."""
    spec = synth.spec_custom(40, 1, epl=True, lens_light=True, nmax=2, K=25)
    return spec, np.full((spec.H, spec.W), 0.1, np.float32), synth.draw_truth(spec, 0)


@pytest.mark.parametrize("spec_fn,P", [(synth.spec_c1, 1), (synth.spec_c1, 65),
                                       (synth.spec_c2, 63), (synth.spec_c2, 513),
                                       ("k25", 512)])
def test_outputs_stay_within_their_extent(G, spec_fn, P):
    from paper_2202_07663_amd import _lib
    if spec_fn == "k25":
        spec, obs, truth = _k25_system()
    else:
        spec = spec_fn()
        obs, truth = load_workload(spec.name)
    m = G.Model.from_spec(spec, obs)
    d, H, W = m.d, spec.H, spec.W
    path = m.plan(P)["psf_path"]
    _say("case extent", spec.name, "P", P, "psf path", path)
    assert path == {1: "banded", 63: "banded", 65: "banded", 513: "mfma", 512: "valu"}[P]
    theta = torch.from_numpy(synth.draw_particles(spec, truth, P, seed=3)).cuda()
    theta_before = theta.clone()
    pad = 3
    ll = torch.full((P + pad,), SENTINEL, dtype=torch.float64, device="cuda")
    g = torch.full((P + pad, d), SENTINEL, dtype=torch.float32, device="cuda")
    img = torch.full((P + pad, H, W), SENTINEL, dtype=torch.float32, device="cuda")
    L = _lib.lib()
    _lib.check(L.gl_loglik_grad(m._h, theta.data_ptr(), P, ll.data_ptr(), g.data_ptr(), None))
    torch.cuda.synchronize()
    assert torch.isfinite(ll[:P]).all() and torch.isfinite(g[:P]).all()
    assert (ll[P:] == SENTINEL).all() and (g[P:] == SENTINEL).all()
    ll.fill_(SENTINEL)
    _lib.check(L.gl_loglik(m._h, theta.data_ptr(), P, ll.data_ptr(), None))
    _lib.check(L.gl_simulate(m._h, theta.data_ptr(), P, img.data_ptr(), None))
    torch.cuda.synchronize()
    assert torch.isfinite(ll[:P]).all() and (ll[P:] == SENTINEL).all()
    assert torch.isfinite(img[:P]).all() and (img[P:] == SENTINEL).all()
    assert torch.equal(theta, theta_before)


def test_calls_are_ordered_on_their_stream(G):
    """On a side stream: a long matrix product, then the parameter rows copied in, then
    gl_loglik_grad and gl_simulate on that stream. The results equal those of the same rows
    computed beforehand, so the library read theta after the copy and wrote before the
    stream's next work."""
    spec = synth.spec_c1()
    obs, truth = load_workload(spec.name)
    m = G.Model.from_spec(spec, obs)
    P = 64
    good = torch.from_numpy(synth.draw_particles(spec, truth, P, seed=5)).cuda()
    ll_ref, g_ref = m.loglik_grad(good)
    img_ref = m.simulate(good)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    buf = torch.zeros_like(good)
    a = torch.randn(4096, 4096, device="cuda")
    torch.cuda.synchronize()
    _say("case stream order")
    with torch.cuda.stream(s):
        for _ in range(8):
            a = (a @ a) * (1.0 / 64.0)  # keeps the side stream busy for a while
        buf.copy_(good)
        ll, g = m.loglik_grad(buf, stream=s)
        img = m.simulate(buf, stream=s)
        ll2 = ll.clone()  # stream work that reads the outputs
    s.synchronize()
    assert torch.equal(ll, ll_ref) and torch.equal(g, g_ref) and torch.equal(img, img_ref)
    assert torch.equal(ll2, ll_ref)
