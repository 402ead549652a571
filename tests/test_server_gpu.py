"""GPU tests of the continuous-batching fit server (gl_submit / gl_poll)."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import load_workload, oracle_model

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    import paper_2202_07663_amd as g
    return g


def _system(N, k, epl, lens_light, nmax, seed):
    spec = synth.spec_custom(N, k, epl, lens_light, nmax, K=21)
    truth = synth.draw_truth(spec, seed)
    obs = synth.add_noise(oracle.simulate(oracle_model(spec), truth.astype(np.float64))[0],
                          seed, spec.sigma_bkg, spec.t_exp)
    return spec, obs


MIX = [(40, 2, False, False, -1, 1, 256), (60, 2, True, True, 6, 2, 512),
       (32, 2, True, False, 4, 3, 384), (48, 1, False, True, 0, 4, 256),
       (60, 2, True, True, 6, 5, 256), (36, 2, False, True, 8, 6, 512)]


def _submit(srv, case, K=20, seed=7):
    N, k, epl, ll, nmax, s, P = case
    spec, obs = _system(N, k, epl, ll, nmax, s)
    return srv.submit(spec, obs, P, K, synth.fit_priors(spec), seed=seed)


def test_result_same_alone_and_in_the_mix(G):
    """Each system's result is bitwise identical whether it is served alone or together with
    systems of other sizes and component sets (shared grouped launches, staggered
    admission)."""
    alone = []
    for case in MIX:
        srv = G.Server(hbm_budget_bytes=4 << 30, max_systems=1, steps_per_tick=5)
        alone.append(srv.wait(_submit(srv, case)))
        srv.close()
    srv = G.Server(hbm_budget_bytes=4 << 30, max_systems=4, steps_per_tick=3,
                   fill_subpixels=1e12)
    tickets = [_submit(srv, c) for c in MIX]
    mixed = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(MIX) and st["hbm_in_use"] == 0
    for a, b in zip(alone, mixed):
        assert a["status"] == 0 and b["status"] == 0
        assert a["best"] == b["best"]
        assert a["logpost_best"] == b["logpost_best"]
        np.testing.assert_array_equal(a["theta_best"], b["theta_best"])
        assert b["t_submit"] <= b["t_admit"] <= b["t_done"]


def test_server_matches_gl_fit(G):
    case = MIX[1]
    N, k, epl, ll, nmax, s, P = case
    spec, obs = _system(N, k, epl, ll, nmax, s)
    model = G.Model.from_spec(spec, obs)
    ref = G.fit(model, P, 20, synth.fit_priors(spec), seed=7)
    srv = G.Server()
    got = srv.wait(_submit(srv, case))
    srv.close()
    assert got["logpost_best"] == ref["logpost_best"]
    np.testing.assert_array_equal(got["theta_best"], ref["theta_best"])


def test_small_budget_forces_queueing(G):
    """A budget that holds one of these systems at a time (a request here is ~20 MB, most of it
    the sub-pixel source offsets the adjoint reuses): everything still completes, in order,
    and device memory in use never exceeds the budget."""
    case = MIX[0]
    srv = G.Server(hbm_budget_bytes=32 << 20, max_systems=8, steps_per_tick=4,
                   fill_subpixels=1e12)
    tickets = [_submit(srv, case, K=8, seed=i) for i in range(4)]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert all(r["status"] == 0 for r in res)
    assert st["hbm_peak"] <= 32 << 20
    admits = [r["t_admit"] for r in res]
    dones = [r["t_done"] for r in res]
    assert admits == sorted(admits)
    assert all(admits[i + 1] >= dones[i] for i in range(3))  # one system at a time


def test_over_budget_request_rejected(G):
    srv = G.Server(hbm_budget_bytes=1 << 20)
    with pytest.raises(G.GlError) as e:
        _submit(srv, MIX[1])
    assert "GL_E_BUDGET" in str(e.value)
    srv.close()


def test_failing_request_is_isolated(G):
    """A request whose likelihood is non-finite for every particle (an observed image of
    1e30 counts/s) ends with GL_E_NUMERIC; the requests around it are unaffected."""
    srv = G.Server(max_systems=4, steps_per_tick=5)
    spec, obs = _system(40, 2, False, False, -1, 1)
    good1 = _submit(srv, MIX[0])
    bad = srv.submit(spec, np.full_like(obs, 1e30), 256, 20, synth.fit_priors(spec), seed=7)
    good2 = _submit(srv, MIX[2])
    r1, rb, r2 = srv.wait(good1), srv.wait(bad), srv.wait(good2)
    srv.close()
    assert rb["status"] == -6
    assert r1["status"] == 0 and r2["status"] == 0


def test_unknown_ticket(G):
    srv = G.Server()
    with pytest.raises(G.GlError) as e:
        srv.poll(12345)
    assert "GL_E_NOTFOUND" in str(e.value)
    srv.close()


def test_admission_failure_is_reported(G):
    """A request the device cannot hold (budget larger than the device, so admission's
    allocation fails) retires with GL_E_NOMEM; the server counts it and serves the next
    request normally."""
    srv = G.Server(hbm_budget_bytes=1 << 50, max_systems=4, steps_per_tick=5)
    spec, obs = _system(40, 4, True, True, 8, 9)
    big = srv.submit(spec, obs, 1 << 21, 5, synth.fit_priors(spec), seed=1)  # ~1.6 TB
    r = srv.wait(big)
    assert r["status"] == -2, r["status"]
    ok = srv.wait(_submit(srv, MIX[0], K=5))
    st = srv.stats()
    srv.close()
    assert ok["status"] == 0
    assert st["failed"] == 1 and st["last_error"] == -2 and st["completed"] == 2
    assert st["hbm_in_use"] == 0
