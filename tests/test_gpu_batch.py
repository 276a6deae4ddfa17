"""Several problems of different shapes in one launch (fcns_batch_*): the
fused z pass of every member runs in one kernel per RK stage.  Each member's
result matches its own step with the fused z pass (the same per-workgroup
code) to rounding, and the FP64 oracle to the 1e-11 bar; members fail
alone; the batch refuses contexts it cannot take."""
import numpy as np
import pytest

import workloads as W
from oracle.ns import Oracle, Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fcns():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2002_01392_amd as P
    P.load_library()
    return P


def rel_l2(a, b):
    a = a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)
    b = b.detach().cpu().numpy() if hasattr(b, "detach") else np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def _members():
    # N' = 64, 80, 96, 128 (radices up to 5) and 58 = 2 * 29 (a prime stage)
    return [
        W.rayleigh_benard(32, 32, 33, 1e5, C=31, dt=1e-3, steps=3, seed=801,
                          perturbation="curl_eigen", noise_rms=1e-2),
        W.channel(48, 32, 49, 2000.0, C=31, dt=5e-4, steps=3, seed=802, noise_rms=0.05),
        W.rayleigh_benard(64, 48, 65, 1e6, C=31, dt=5e-4, steps=3, seed=803, noise_rms=1e-2),
        W.channel(16, 8, 33, 1500.0, C=25, dt=5e-4, steps=3, seed=804, noise_rms=0.05),
        W.rayleigh_benard(24, 40, 97, 1e5, C=31, dt=5e-4, steps=3, seed=805, noise_rms=1e-2),
    ]


def _solvers(fcns, ws, states, order=2, fused=False):
    out = []
    for w, (v0, th0) in zip(ws, states):
        s = fcns.Solver.from_workload(w, rk_order=order, keep_pressure=True,
                                      stream=torch.cuda.Stream())
        s.set_state(torch.from_numpy(v0), torch.from_numpy(th0) if th0 is not None else None)
        if fused:
            s.set_z_fused(True)
        out.append(s)
    torch.cuda.synchronize()
    return out


def _results(solvers):
    res = []
    for s in solvers:
        v, th, p = s.get_state(pressure=True)
        s.synchronize()
        res.append((v.cpu().numpy(), th.cpu().numpy() if th is not None else None,
                    p.cpu().numpy()))
    return res


@pytest.mark.parametrize("order", [2, 3])
def test_batch_matches_each_member_alone_and_the_oracle(fcns, order):
    ws = _members()
    states = [w.initial_state() for w in ws]
    members = _solvers(fcns, ws, states, order)
    b = fcns.Batch(members, [w.dt for w in ws])
    b.run(3)
    got = _results(members)
    b.close()
    alone = _solvers(fcns, ws, states, order, fused=True)
    for s, w in zip(alone, ws):
        s.rk_step(w.dt, 3)
    ref = _results(alone)
    for w, g, r in zip(ws, got, ref):
        assert rel_l2(g[0], r[0]) < 1e-13, w.name
        if g[1] is not None:
            assert rel_l2(g[1], r[1]) < 1e-13, w.name
        assert rel_l2(g[2], r[2]) < 1e-12, w.name
    for w, (v0, th0), g in list(zip(ws, states, got))[:3]:
        o = Oracle(Problem(**w.problem_kwargs(), rk_order=order))
        o.set_state(v0, th0)
        o.rk_step(w.dt, 3)
        rv, rth, rp = o.get_state()
        assert rel_l2(g[0], rv) < 1e-11, w.name
        if rth is not None:
            assert rel_l2(g[1], rth) < 1e-11, w.name
        assert rel_l2(g[2], rp) < 1e-10, w.name


def test_batch_member_with_a_nan_fails_alone(fcns):
    ws = _members()[:3]
    states = [w.initial_state() for w in ws]
    v_bad = states[1][0].copy()
    v_bad[0, 7, 3, 3] = np.nan
    bad_states = [states[0], (v_bad, states[1][1]), states[2]]
    members = _solvers(fcns, ws, bad_states)
    for s in members:
        s.set_finite_check("deferred")
    b = fcns.Batch(members, [w.dt for w in ws])
    b.run(2)
    with pytest.raises(fcns.FcnsError) as e:
        members[1].check_finite()
    assert e.value.code == fcns.FCNS_ENONFINITE
    members[0].check_finite()
    members[2].check_finite()
    got = _results(members)
    b.close()
    alone = _solvers(fcns, [ws[0], ws[2]], [states[0], states[2]], fused=True)
    for s, w in zip(alone, [ws[0], ws[2]]):
        s.rk_step(w.dt, 2)
    ref = _results(alone)
    assert rel_l2(got[0][0], ref[0][0]) < 1e-13
    assert rel_l2(got[2][0], ref[1][0]) < 1e-13


def test_batch_refuses_what_it_cannot_take(fcns):
    w = W.rayleigh_benard(32, 32, 33, 1e5, C=31, dt=1e-3, steps=1, seed=806)
    big = W.rayleigh_benard(16, 8, 257, 1e5, d=7, C=33, dt=1e-3, steps=1, seed=807)  # N' = 290
    a = fcns.Solver.from_workload(w)
    m = fcns.Solver.from_workload(w, precision="mixed")
    c = fcns.Solver.from_workload(big)
    o3 = fcns.Solver.from_workload(w, rk_order=3)
    for pair in ([a, m], [a, c], [a, o3]):
        with pytest.raises(fcns.FcnsError) as e:
            fcns.Batch(pair, [1e-3, 1e-3])
        assert e.value.code == fcns.FCNS_EINVAL
