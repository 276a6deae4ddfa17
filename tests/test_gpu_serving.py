"""The serving engine (fcns_server_*): admitted requests of different shapes
overlap on the device, and each result is bitwise the one a single-problem
solve of the same request gives (alone and in the mix), including requests
served by a reused resident context (new physical parameters) and under a
memory budget that admits one context at a time."""
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


def _requests():
    return [
        W.channel(32, 32, 33, 1000.0, C=31, dt=1e-3, steps=6, seed=601),
        W.channel(32, 32, 33, 3000.0, C=31, dt=1e-3, steps=6, seed=602),   # same shape
        W.rayleigh_benard(32, 32, 33, 1e5, C=31, dt=1e-3, steps=6, seed=603),
        W.channel(64, 64, 65, 2000.0, C=31, dt=5e-4, steps=4, seed=604),
        W.rayleigh_benard(64, 64, 65, 1e6, C=31, dt=5e-4, steps=4, seed=605),
        W.rayleigh_benard(32, 32, 33, 1e6, C=31, dt=1e-3, steps=6, seed=606),  # same shape
    ]


def _serve(fcns, ws, states, max_active, max_bytes):
    srv = fcns.Server(max_active=max_active, max_bytes=max_bytes)
    ids = []
    for w, (v0, th0) in zip(ws, states):
        prob, _tab = fcns.workload_problem(w)
        ids.append(srv.submit(prob, v0, th0, w.dt, w.steps))
    most = 0
    deadline = time.monotonic() + 120
    while True:
        q, a, d = srv.poll()
        most = max(most, a)
        if d == len(ids):
            break
        assert time.monotonic() < deadline, "server did not finish"
        time.sleep(1e-4)
    return srv, ids, most


def _alone(fcns, w, v0, th0):
    s = fcns.Solver.from_workload(w)
    s.set_state(torch.from_numpy(v0), torch.from_numpy(th0) if th0 is not None else None)
    s.rk_step(w.dt, w.steps)
    v, th, _ = s.get_state()
    torch.cuda.synchronize()
    return v.cpu().numpy(), (th.cpu().numpy() if th is not None else None)


@pytest.mark.parametrize("max_active,budget_contexts", [(4, None), (3, 1)])
def test_server_results_match_single_problem_solves(fcns, max_active, budget_contexts):
    ws = _requests()
    states = [w.initial_state() for w in ws]
    if budget_contexts is None:
        budget = 8 << 30
    else:
        # room for the largest context (plus staging) only: one at a time for
        # the large shapes, evicting idle contexts of other shapes
        big = max(fcns.footprint(fcns.workload_problem(w)[0]) + 4 * 8 * w.nx * w.ny * w.nz
                  for w in ws)
        budget = big + 1024
    srv, ids, most = _serve(fcns, ws, states, max_active, budget)
    assert most <= max_active
    if budget_contexts is None:
        assert most >= 2          # requests did overlap
    for w, (v0, th0), rid in zip(ws, states, ids):
        v, th, info = srv.result(rid)
        rv, rth = _alone(fcns, w, v0, th0)
        assert info["finite"]
        assert np.array_equal(v, rv), w.name
        if th is not None:
            assert np.array_equal(th, rth), w.name
        assert info["t_submit"] <= info["t_admit"] <= info["t_done"]
        steps = srv.step_times(rid)
        assert len(steps) == w.steps and (steps > 0).all()
        srv.release(rid)
    srv.close()


def test_server_rejects_a_request_larger_than_the_budget(fcns):
    w = W.channel(32, 32, 33, 1000.0, C=31, dt=1e-3, steps=2, seed=607)
    v0, _ = w.initial_state()
    srv = fcns.Server(max_active=2, max_bytes=1 << 20)
    prob, _tab = fcns.workload_problem(w)
    rid = srv.submit(prob, v0, None, w.dt, w.steps)
    q, a, d = srv.poll()
    assert d == 1 and a == 0 and q == 0
    with pytest.raises(fcns.FcnsError) as e:
        srv.result(rid)
    assert e.value.code == -2
    srv.close()


def test_batch_step_matches_single_solves(fcns):
    # several shapes stepped together on their own streams: each result is
    # bitwise its own rk_step
    ws = _requests()[:5]
    states = [w.initial_state() for w in ws]
    streams = [torch.cuda.Stream() for _ in ws]
    solvers = []
    for w, (v0, th0), st in zip(ws, states, streams):
        s = fcns.Solver.from_workload(w, stream=st)
        s.set_state(torch.from_numpy(v0), torch.from_numpy(th0) if th0 is not None else None)
        solvers.append(s)
    torch.cuda.synchronize()
    fcns.batch_step(solvers, [w.dt for w in ws], [w.steps for w in ws])
    torch.cuda.synchronize()
    for s, w, (v0, th0) in zip(solvers, ws, states):
        v, th, _ = s.get_state()
        torch.cuda.synchronize()
        rv, rth = _alone(fcns, w, v0, th0)
        assert np.array_equal(v.cpu().numpy(), rv), w.name
        if th is not None:
            assert np.array_equal(th.cpu().numpy(), rth), w.name


def test_server_applies_tuned_choices_per_shape(fcns):
    ws = _requests()
    states = [w.initial_state() for w in ws]
    # a tuning table for the 64^3 Rayleigh-Benard shape, and choices the
    # 32^3 channel shape cannot take (8-line y tiles need ny = 512)
    rb64 = ws[4]
    t = fcns.Solver.from_workload(rb64)
    t.set_state(torch.from_numpy(states[4][0]), torch.from_numpy(states[4][1]))
    t.autotune()
    text = t.choices()
    t.close()
    srv = fcns.Server(max_active=4, max_bytes=8 << 30)
    # (each problem's table must stay alive while the call reads it)
    p_rb, tab_rb = fcns.workload_problem(rb64)
    p_ch, tab_ch = fcns.workload_problem(ws[0])
    srv.set_choices(p_rb, text)
    srv.set_choices(p_ch, "ylines=8")
    ids = []
    for w, (v0, th0) in zip(ws, states):
        prob, _tab = fcns.workload_problem(w)
        ids.append(srv.submit(prob, v0, th0, w.dt, w.steps))
    deadline = time.monotonic() + 120
    while srv.poll()[2] < len(ids):
        assert time.monotonic() < deadline, "server did not finish"
        time.sleep(1e-4)
    for i, (w, (v0, th0), rid) in enumerate(zip(ws, states, ids)):
        if i in (0, 1):   # the shape whose choices its contexts cannot take
            with pytest.raises(fcns.FcnsError) as e:
                srv.result(rid)
            assert e.value.code == fcns.FCNS_EINVAL
            continue
        v, th, info = srv.result(rid)
        s = fcns.Solver.from_workload(w)
        if i == 4:
            s.set_choices(text)
        s.set_state(torch.from_numpy(v0), torch.from_numpy(th0) if th0 is not None else None)
        s.rk_step(w.dt, w.steps)
        rv, rth, _ = s.get_state()
        torch.cuda.synchronize()
        assert np.array_equal(v, rv.cpu().numpy()), w.name
        if th is not None:
            assert np.array_equal(th, rth.cpu().numpy()), w.name
    srv.close()


def test_server_mix_limit_keeps_large_requests_apart(fcns):
    ws = _requests() + [W.rayleigh_benard(64, 64, 65, 1e5, C=31, dt=5e-4, steps=4, seed=607)]
    states = [w.initial_state() for w in ws]
    srv = fcns.Server(max_active=4, max_bytes=8 << 30)
    srv.set_mix(1, 64 * 64 * 65)      # the three 64^3 requests are large
    ids = []
    for w, (v0, th0) in zip(ws, states):
        prob, _tab = fcns.workload_problem(w)
        ids.append(srv.submit(prob, v0, th0, w.dt, w.steps))
    deadline = time.monotonic() + 120
    while srv.poll()[2] < len(ids):
        assert time.monotonic() < deadline, "server did not finish"
        time.sleep(1e-4)
    spans = []
    for w, (v0, th0), rid in zip(ws, states, ids):
        v, th, info = srv.result(rid)
        if w.nx == 64:
            spans.append((info["t_admit"], info["t_done"]))
        rv, rth = _alone(fcns, w, v0, th0)
        assert np.array_equal(v, rv), w.name
        if th is not None:
            assert np.array_equal(th, rth), w.name
    spans.sort()
    assert len(spans) == 3
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert a1 <= b0, "two large requests ran together"
    with pytest.raises(fcns.FcnsError):
        srv.set_mix(-1, 10)
    srv.close()
