"""The step's non-finite check and the serving loop's failure isolation.

* rk_step flags a NaN or an infinity anywhere in the state (velocity or
  temperature) through the device reduction of every stage: FCNS_ENONFINITE
  in the synchronous mode, from fcns_check_finite in the deferred mode; a new
  set_state clears it.
* In the server, a request started from a state holding a NaN fails alone
  (FCNS_ENONFINITE) and every other request's result is bitwise its
  single-problem solve; cancelling a queued or running request ends it with
  FCNS_ECANCELED without touching the others.
The NaN is planted in the host input only; every kernel runs to its normal
end.
"""
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fcns():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2002_01392_amd as P
    P.load_library()
    return P


def _solver(fcns, w, v0, th0):
    s = fcns.Solver.from_workload(w)
    s.set_state(torch.from_numpy(v0), torch.from_numpy(th0) if th0 is not None else None)
    return s


@pytest.mark.parametrize("where", ["velocity", "theta", "inf"])
def test_rk_step_reports_a_non_finite_state(fcns, where):
    w = W.rayleigh_benard(32, 24, 33, 1e5, C=31, dt=1e-3, steps=2, seed=700, noise_rms=1e-2)
    v0, th0 = w.initial_state()
    bad_v, bad_t = v0.copy(), th0.copy()
    if where == "velocity":
        bad_v[1, 7, 3, 5] = np.nan
    elif where == "theta":
        bad_t[9, 2, 11] = np.nan
    else:
        bad_v[0, 4, 4, 4] = np.inf
    s = _solver(fcns, w, bad_v, bad_t)
    with pytest.raises(fcns.FcnsError) as e:
        s.rk_step(w.dt, 1)
    assert e.value.code == fcns.FCNS_ENONFINITE
    # deferred mode: the call returns, the check reports
    s.set_state(torch.from_numpy(bad_v), torch.from_numpy(bad_t))
    s.set_finite_check("deferred")
    s.rk_step(w.dt, 2)
    with pytest.raises(fcns.FcnsError) as e:
        s.check_finite()
    assert e.value.code == fcns.FCNS_ENONFINITE
    # a finite state clears the flag
    s.set_finite_check("sync")
    s.set_state(torch.from_numpy(v0), torch.from_numpy(th0))
    s.rk_step(w.dt, 2)
    s.check_finite()
    v, th, _ = s.get_state()
    torch.cuda.synchronize()
    assert bool(torch.isfinite(v).all()) and bool(torch.isfinite(th).all())


def _requests():
    return [
        W.channel(32, 32, 33, 1000.0, C=31, dt=1e-3, steps=8, seed=711, perturbation="curl_eigen"),
        W.rayleigh_benard(32, 32, 33, 1e5, C=31, dt=1e-3, steps=8, seed=712,
                          perturbation="curl_eigen"),
        W.channel(64, 64, 65, 2000.0, C=31, dt=5e-4, steps=6, seed=713),
        W.rayleigh_benard(64, 64, 65, 1e6, C=31, dt=5e-4, steps=6, seed=714),
        W.channel(32, 32, 33, 3000.0, C=31, dt=1e-3, steps=8, seed=715),
    ]


def _alone(fcns, w, v0, th0):
    s = _solver(fcns, w, v0, th0)
    s.rk_step(w.dt, w.steps)
    v, th, _ = s.get_state()
    torch.cuda.synchronize()
    return v.cpu().numpy(), (th.cpu().numpy() if th is not None else None)


def _drain(srv, n, timeout=120):
    deadline = time.monotonic() + timeout
    while True:
        _, _, d = srv.poll()
        if d == n:
            return
        assert time.monotonic() < deadline, "server did not finish"
        time.sleep(1e-4)


def test_server_isolates_a_request_that_blows_up(fcns):
    ws = _requests()
    states = [w.initial_state() for w in ws]
    bad = 1
    v_bad = states[bad][0].copy()
    v_bad[2, 10, 5, 5] = np.nan
    states[bad] = (v_bad, states[bad][1])
    srv = fcns.Server(max_active=4, max_bytes=8 << 30)
    ids = []
    for w, (v0, th0) in zip(ws, states):
        prob, _tab = fcns.workload_problem(w)
        ids.append(srv.submit(prob, v0, th0, w.dt, w.steps))
    _drain(srv, len(ids))
    for i, (w, (v0, th0), rid) in enumerate(zip(ws, states, ids)):
        v, th, info = srv.result(rid)
        if i == bad:
            assert info["status"] == fcns.FCNS_ENONFINITE
            assert len(srv.step_times(rid)) <= 4     # stopped within the lookahead
            continue
        assert info["status"] == fcns.FCNS_OK, w.name
        rv, rth = _alone(fcns, w, v0, th0)
        assert np.array_equal(v, rv), w.name
        if th is not None:
            assert np.array_equal(th, rth), w.name
    srv.close()


def test_server_cancel_queued_and_running(fcns):
    ws = _requests()
    ws[0] = W.channel(64, 64, 65, 2000.0, C=31, dt=5e-4, steps=200, seed=721)   # long
    states = [w.initial_state() for w in ws]
    srv = fcns.Server(max_active=2, max_bytes=8 << 30)
    ids = []
    for w, (v0, th0) in zip(ws, states):
        prob, _tab = fcns.workload_problem(w)
        ids.append(srv.submit(prob, v0, th0, w.dt, w.steps))
    srv.poll()                  # admits the first two
    srv.cancel(ids[0])          # running
    srv.cancel(ids[4])          # still queued
    _drain(srv, len(ids))
    for i, (w, (v0, th0), rid) in enumerate(zip(ws, states, ids)):
        v, th, info = srv.result(rid)
        if i in (0, 4):
            assert info["status"] == fcns.FCNS_ECANCELED
            continue
        assert info["status"] == fcns.FCNS_OK, w.name
        rv, rth = _alone(fcns, w, v0, th0)
        assert np.array_equal(v, rv), w.name
        if th is not None:
            assert np.array_equal(th, rth), w.name
    assert len(srv.step_times(ids[0])) < 200     # the long request stopped early
    srv.close()
