"""The allocation-free variant of gl_loglik_grad (gl_loglik_grad_noalloc), through the C ABI:
its work space is the library's fixed per-device array, and its results equal
gl_loglik_grad's bitwise (same kernels, same work split for the same P). Two calls in a
row, the second on a smaller batch, then a batch above the array's limit, which is refused
before any work is enqueued."""
import ctypes

import numpy as np
import pytest

import synth
from tests.helpers import load_workload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)


def _noalloc(lib, m, th, ll, g):
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return lib.gl_loglik_grad_noalloc(m._h, th.data_ptr(), th.shape[0], ll.data_ptr(),
                                      g.data_ptr(), stream)


@pytest.mark.parametrize("case", ["epl60", "sie40"])
def test_noalloc_matches_loglik_grad(case):
    import paper_2202_07663_amd as G
    from paper_2202_07663_amd import _lib
    lib = _lib.lib()
    spec = synth.spec_c2() if case == "epl60" else synth.spec_c1()
    obs, truth = load_workload(spec.name)
    m = G.Model.from_spec(spec, obs)
    cap = m.plan(1)["noalloc_max_P"]
    _say("case", case, "noalloc_max_P", cap)
    assert cap >= 256
    theta = synth.draw_particles(spec, truth, cap, seed=11)
    for P in (cap, 37):  # two calls in a row, the second smaller
        th = torch.from_numpy(theta[:P]).cuda()
        ll = torch.full((P,), np.nan, dtype=torch.float64, device="cuda")
        g = torch.full((P, m.d), np.nan, dtype=torch.float32, device="cuda")
        rc = _noalloc(lib, m, th, ll, g)
        assert rc == 0, lib.gl_last_error()
        ll_ref, g_ref = m.loglik_grad(th)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ll.cpu().numpy(), ll_ref.cpu().numpy())
        np.testing.assert_array_equal(g.cpu().numpy(), g_ref.cpu().numpy())
        _say(case, "P", P, "bitwise equal to gl_loglik_grad")
    # above the limit: refused with GL_E_BUDGET, nothing written
    P = cap + 1
    th = torch.from_numpy(synth.draw_particles(spec, truth, P, seed=12)).cuda()
    ll = torch.zeros(P, dtype=torch.float64, device="cuda")
    g = torch.zeros((P, m.d), dtype=torch.float32, device="cuda")
    assert _noalloc(lib, m, th, ll, g) == -4
    assert b"allocation-free" in lib.gl_last_error()
    torch.cuda.synchronize()
    assert float(ll.abs().max()) == 0.0
