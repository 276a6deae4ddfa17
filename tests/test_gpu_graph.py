"""HIP-graph replay of the RK step (fcns_rk_graph) against the eager step:
every replay, with eager work and synchronisations between the replays, is
bitwise the eager result; a new dt recaptures."""
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


@pytest.mark.parametrize("kind,precision", [("channel", "fp64"), ("rb", "fp64"), ("rb", "mixed")])
def test_graph_replays_match_eager_steps(fcns, kind, precision):
    if kind == "channel":
        w = W.get("channel_32x32x33")
    else:
        w = W.rayleigh_benard(32, 24, 33, 1e5, C=31, dt=2e-3, steps=4, kmax=3, mmax=3,
                              noise_rms=1e-2)
    v0, th0 = w.initial_state()
    tv = torch.from_numpy(v0)
    tt = torch.from_numpy(th0) if th0 is not None else None
    eager = fcns.Solver.from_workload(w, keep_pressure=True, precision=precision)
    graph = fcns.Solver.from_workload(w, keep_pressure=True, precision=precision)
    eager.set_state(tv, tt)
    graph.set_state(tv, tt)
    for k in range(4):
        dt = w.dt if k < 3 else 0.5 * w.dt       # the last replay recaptures
        eager.rk_step(dt, 1)
        graph.rk_graph(dt, 1)
        ve, te, pe = eager.get_state(pressure=True)
        vg, tg, pg = graph.get_state(pressure=True)   # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(ve, vg), k
        assert torch.equal(pe, pg), k
        if te is not None:
            assert torch.equal(te, tg), k
    # several steps per call
    eager.rk_step(w.dt, 3)
    graph.rk_graph(w.dt, 3)
    ve, _, _ = eager.get_state()
    vg, _, _ = graph.get_state()
    torch.cuda.synchronize()
    assert torch.equal(ve, vg)


def test_a_change_of_launch_choices_recaptures(fcns):
    # the fused and the split z pass agree to rounding only, so a replay of
    # the step captured before the change would not match the eager steps
    w = W.rayleigh_benard(32, 24, 33, 1e5, C=31, dt=2e-3, steps=4, kmax=3, mmax=3,
                          noise_rms=1e-2)
    v0, th0 = w.initial_state()
    eager = fcns.Solver.from_workload(w)
    graph = fcns.Solver.from_workload(w)
    for s in (eager, graph):
        s.set_state(torch.from_numpy(v0), torch.from_numpy(th0))
    eager.rk_step(w.dt, 2)
    graph.rk_graph(w.dt, 2)
    for s in (eager, graph):
        s.set_z_fused(True)
        s.set_slab(8)
    eager.rk_step(w.dt, 2)
    graph.rk_graph(w.dt, 2)
    ve, te, _ = eager.get_state()
    vg, tg, _ = graph.get_state()
    torch.cuda.synchronize()
    assert torch.equal(ve, vg) and torch.equal(te, tg)
