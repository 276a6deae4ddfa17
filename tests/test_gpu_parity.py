"""GPU (HIP, through the C ABI) versus the FP64 oracle, element by element.

Tolerance: 1e-11 relative L2 for FP64 results (the bar the solver is built
to), tighter where no FC continuation is involved.  The continuation tables
have entries up to ~1e4 (App. B: the ill-conditioning sits in the tables),
so one continuation already carries ~1e-12 relative rounding noise.
Sizes span several workgroup tiles with ragged tails, both FFT code paths
(N' with only small radices, and N' = 58 = 2 * 29 and 282 = 2 * 3 * 47), and
the edge cases of the interface.
"""
import numpy as np
import pytest

import workloads as W
from oracle.fcgram import fc_derivative_lines, fc_extend_lines
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
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def solver(P, nx, ny, nz, C=25, lx=2 * np.pi, ly=2 * np.pi, lz=1.0, nu=0.0, **kw):
    return P.Solver(nx, ny, nz, lx, ly, lz, nu, d=5, C=C, **kw)


# ------------------------------------------------------------------ fc_extend / fc_derivative
@pytest.mark.parametrize("nz,C,nlines", [(33, 25, 7), (65, 31, 300), (257, 31, 1031),
                                         (257, 25, 129)])
def test_fc_extend_parity(fcns, nz, C, nlines):
    s = solver(fcns, 8, 8, nz, C=C)
    f = W.rng(100 + nz).standard_normal((nlines, nz))
    got = s.fc_extend(torch.from_numpy(f))
    torch.cuda.synchronize()
    ref = fc_extend_lines(f, 5, C)
    assert np.array_equal(got[:, :nz].cpu().numpy(), f)
    assert rel_l2(got, ref) < 1e-14


@pytest.mark.parametrize("nz,C,nlines", [(33, 25, 5), (65, 31, 77), (257, 31, 513),
                                         (257, 25, 40), (129, 31, 16)])
@pytest.mark.parametrize("order", [1, 2])
def test_fc_derivative_parity(fcns, nz, C, nlines, order):
    s = solver(fcns, 8, 8, nz, C=C, lz=1.7)
    z = np.linspace(0, 1.7, nz)
    r = W.rng(7 * nz + order)
    f = np.stack([np.sin(r.uniform(1, 9) * z + r.uniform()) * np.exp(r.uniform(-1, 1) * z)
                  for _ in range(nlines)])
    got = s.fc_derivative(torch.from_numpy(f), order)
    torch.cuda.synchronize()
    ref = fc_derivative_lines(f, 5, C, 1.7, order)
    assert rel_l2(got, ref) < 1e-11


def test_empty_and_invalid_inputs(fcns):
    s = solver(fcns, 8, 8, 33)
    out = s.fc_extend(torch.zeros((0, 33), dtype=torch.float64))
    assert out.shape == (0, 58)
    with pytest.raises(fcns.FcnsError) as e:
        s.rk_step(1e-3, 1)
    assert e.value.code == -5
    with pytest.raises(fcns.FcnsError):
        solver(fcns, 9, 8, 33)            # odd nx
    with pytest.raises(fcns.FcnsError):
        solver(fcns, 8, 8, 34)            # odd N' = 59
    with pytest.raises(fcns.FcnsError):
        s.fc_derivative(torch.zeros((2, 33), dtype=torch.float64), order=3)


# ------------------------------------------------------------------ transforms and state
@pytest.mark.parametrize("nx,ny,nz,C", [(16, 12, 33, 25), (24, 20, 65, 31), (64, 40, 97, 31)])
def test_state_round_trip_and_spectrum(fcns, nx, ny, nz, C):
    lx, ly, lz = 2.0, 3.0, 1.3
    s = fcns.Solver(nx, ny, nz, lx, ly, lz, 0.01, d=5, C=C)
    v = np.stack([W.smooth_field(nx, ny, nz, lx, ly, lz, 10 + i) for i in range(3)])
    s.set_state(torch.from_numpy(v))
    got, _, _ = s.get_state()
    spec = s.get_spectral(0)
    torch.cuda.synchronize()
    assert rel_l2(got, v) < 1e-12
    o = Oracle(Problem(nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz, nu=0.01, C=C))
    o.set_state(v)
    assert rel_l2(spec, o.Vt[0]) < 1e-11


# ------------------------------------------------------------------ nonlinear term
@pytest.mark.parametrize("filtered", [False, True])
@pytest.mark.parametrize("nx,ny,nz,C", [(16, 16, 33, 25), (32, 24, 65, 31), (16, 288, 17, 25)])
def test_rhs_nonlinear_parity(fcns, filtered, nx, ny, nz, C):
    # ny = 288: the length of the compiled z plan, here run by the run-time
    # y engine (radices 8 4 3 3)
    lx, ly, lz = 2.0, 2.0, 1.0
    s = fcns.Solver(nx, ny, nz, lx, ly, lz, 0.01, d=5, C=C, boussinesq=True, kappa=0.01,
                    gamma=1.0)
    v = np.stack([W.smooth_field(nx, ny, nz, lx, ly, lz, 20 + i) for i in range(3)])
    th = W.smooth_field(nx, ny, nz, lx, ly, lz, 30)
    nlv, nlt = s.rhs_nonlinear(torch.from_numpy(v), torch.from_numpy(th), filtered)
    torch.cuda.synchronize()
    o = Oracle(Problem(nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz, nu=0.01, C=C,
                       boussinesq=True, kappa=0.01, gamma=1.0))
    rv, rt = o.rhs_nonlinear(v, th, filtered)
    assert rel_l2(nlv, rv) < 1e-11
    assert rel_l2(nlt, rt) < 1e-11


@pytest.mark.parametrize("nx,ny,nz,C,filtered", [(512, 512, 11, 25, True), (256, 256, 11, 25, False)])
def test_rhs_nonlinear_compile_time_plans(fcns, nx, ny, nz, C, filtered):
    # nx = ny = 512 and 256 take the x and y kernels built for those lengths
    lx, ly, lz = 2.0, 2.0, 1.0
    s = fcns.Solver(nx, ny, nz, lx, ly, lz, 0.01, d=5, C=C, boussinesq=True, kappa=0.01,
                    gamma=1.0)
    v = np.stack([W.smooth_field(nx, ny, nz, lx, ly, lz, 20 + i) for i in range(3)])
    th = W.smooth_field(nx, ny, nz, lx, ly, lz, 30)
    nlv, nlt = s.rhs_nonlinear(torch.from_numpy(v), torch.from_numpy(th), filtered)
    torch.cuda.synchronize()
    o = Oracle(Problem(nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz, nu=0.01, C=C,
                       boussinesq=True, kappa=0.01, gamma=1.0))
    rv, rt = o.rhs_nonlinear(v, th, filtered)
    assert rel_l2(nlv, rv) < 1e-11
    assert rel_l2(nlt, rt) < 1e-11


def test_rhs_nonlinear_velocity_only_512(fcns):
    # three transported fields on 512-point rows
    nx, ny, nz, C, lx, ly, lz = 512, 24, 17, 25, 2.0, 1.0, 1.0
    s = fcns.Solver(nx, ny, nz, lx, ly, lz, 0.01, d=5, C=C)
    v = np.stack([W.smooth_field(nx, ny, nz, lx, ly, lz, 50 + i, kmax=6) for i in range(3)])
    nlv, _ = s.rhs_nonlinear(torch.from_numpy(v), None, False)
    torch.cuda.synchronize()
    o = Oracle(Problem(nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz, nu=0.01, C=C))
    rv, _ = o.rhs_nonlinear(v, None, False)
    assert rel_l2(nlv, rv) < 1e-11


@pytest.mark.parametrize("boussinesq", [False, True])
def test_rhs_nonlinear_wave_rows_256_partial(fcns, boussinesq):
    # 256-point rows, two per wavefront and eight per workgroup: 17 x 10 rows
    # leave the last workgroup one wavefront with rows and three without
    nx, ny, nz, C, lx, ly, lz = 256, 10, 17, 25, 2.0, 1.0, 1.0
    kw = dict(boussinesq=True, kappa=0.01, gamma=1.0) if boussinesq else {}
    s = fcns.Solver(nx, ny, nz, lx, ly, lz, 0.01, d=5, C=C, **kw)
    v = np.stack([W.smooth_field(nx, ny, nz, lx, ly, lz, 60 + i, kmax=6) for i in range(3)])
    th = W.smooth_field(nx, ny, nz, lx, ly, lz, 64, kmax=6) if boussinesq else None
    nlv, nlt = s.rhs_nonlinear(torch.from_numpy(v),
                               torch.from_numpy(th) if boussinesq else None, False)
    torch.cuda.synchronize()
    o = Oracle(Problem(nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz, nu=0.01, C=C, **kw))
    rv, rt = o.rhs_nonlinear(v, th, False)
    assert rel_l2(nlv, rv) < 1e-11
    if boussinesq:
        assert rel_l2(nlt, rt) < 1e-11


# ------------------------------------------------------------------ projection
@pytest.mark.parametrize("nx,ny,nz,C,c", [(16, 16, 33, 25, 0.5), (32, 24, 65, 31, 1e-3),
                                          (20, 36, 129, 31, 2.0)])
def test_pressure_project_parity(fcns, nx, ny, nz, C, c):
    lx, ly, lz = 2 * np.pi, 3.0, 1.0
    s = fcns.Solver(nx, ny, nz, lx, ly, lz, 0.0, d=5, C=C)
    vs = np.stack([W.smooth_field(nx, ny, nz, lx, ly, lz, 40 + i) for i in range(3)])
    v, gp = s.pressure_project(torch.from_numpy(vs), c)
    torch.cuda.synchronize()
    o = Oracle(Problem(nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz, nu=0.0, C=C))
    rv, rg = o.pressure_project(vs, c)
    assert rel_l2(v, rv) < 1e-11
    assert rel_l2(gp, rg) < 1e-11
    # v_z vanishes at the walls to rounding (Sec. 6: <w^2_wall> ~ 1e-35)
    vz = v[2].cpu().numpy()
    assert np.abs(vz[0]).max() < 1e-12 * np.abs(vs).max()
    assert np.abs(vz[-1]).max() < 1e-12 * np.abs(vs).max()


# ------------------------------------------------------------------ time stepping
def _run_pair(fcns, w, steps, keep_pressure=True, rk_order=2):
    v0, th0 = w.initial_state()
    s = fcns.Solver.from_workload(w, keep_pressure=keep_pressure, rk_order=rk_order)
    s.set_state(torch.from_numpy(v0), torch.from_numpy(th0) if th0 is not None else None)
    s.rk_step(w.dt, steps)
    v, th, p = s.get_state(pressure=keep_pressure)
    gw = s.get_wall_grad()
    torch.cuda.synchronize()
    o = Oracle(Problem(**w.problem_kwargs(), rk_order=rk_order))
    o.set_state(v0, th0)
    o.rk_step(w.dt, steps)
    rv, rth, rp = o.get_state()
    return (v, th, p, gw), (rv, rth, rp, o.G)


def test_rk_channel_small_workload(fcns):
    # the 32x32x33 channel workload (d = 5, C = 25, N' = 58), its 10 steps
    w = W.get("channel_32x32x33")
    (v, _, p, gw), (rv, _, rp, rg) = _run_pair(fcns, w, w.steps)
    assert rel_l2(v, rv) < 1e-11
    assert rel_l2(p, rp) < 1e-10
    assert rel_l2(gw, rg) < 1e-10


def test_rk_rayleigh_benard_small(fcns):
    w = W.rayleigh_benard(32, 24, 33, 1e5, C=31, dt=2e-3, steps=8, kmax=3, mmax=3,
                          noise_rms=1e-2)
    (v, th, p, _), (rv, rth, rp, _) = _run_pair(fcns, w, w.steps)
    print(f"[rb small] rel L2: v {rel_l2(v, rv):.2e} theta {rel_l2(th, rth):.2e} "
          f"p {rel_l2(p, rp):.2e}", flush=True)
    assert rel_l2(th, rth) < 1e-11
    assert rel_l2(v, rv) < 1e-11
    assert rel_l2(p, rp) < 1e-10


def test_rk_rayleigh_benard_compile_time_z_plan(fcns):
    # nz = 257 with C = 31: N' = 288, the z kernels built for that length
    w = W.rayleigh_benard(16, 8, 257, 1e6, C=31, dt=1e-3, steps=3, kmax=2, mmax=3,
                          noise_rms=1e-2)
    (v, th, p, gw), (rv, rth, rp, rg) = _run_pair(fcns, w, w.steps)
    assert rel_l2(th, rth) < 1e-11
    assert rel_l2(v, rv) < 1e-11
    assert rel_l2(p, rp) < 1e-10
    assert rel_l2(gw, rg) < 1e-10


def test_rk_channel_big_prime_length(fcns):
    # N' = 282 = 2 * 3 * 47 (the C = 25 table on nz = 257) on a narrow grid
    w = W.channel(16, 8, 257, 2000.0, d=5, C=25, dt=5e-4, steps=3, seed=9, noise_rms=0.05)
    (v, _, _, _), (rv, _, _, _) = _run_pair(fcns, w, w.steps, keep_pressure=False)
    assert rel_l2(v, rv) < 1e-11


@pytest.mark.parametrize("order", [1, 3, 4])
def test_rk_orders_channel(fcns, order):
    # o = 1 (the Euler splitting of Sec. 4.1) and the o = 3, 4 stages of Sec. 4.4
    w = W.get("channel_32x32x33")
    (v, _, p, gw), (rv, _, rp, rg) = _run_pair(fcns, w, 5, rk_order=order)
    assert rel_l2(v, rv) < 1e-11
    assert rel_l2(p, rp) < 1e-10
    assert rel_l2(gw, rg) < 1e-10


def test_rk_order3_rayleigh_benard(fcns):
    w = W.rayleigh_benard(32, 24, 33, 1e5, C=31, dt=2e-3, steps=4, kmax=3, mmax=3,
                          noise_rms=1e-2)
    (v, th, _, _), (rv, rth, _, _) = _run_pair(fcns, w, w.steps, rk_order=3)
    print(f"[rb order 3] rel L2: v {rel_l2(v, rv):.2e} theta {rel_l2(th, rth):.2e}", flush=True)
    assert rel_l2(th, rth) < 1e-11
    assert rel_l2(v, rv) < 1e-11


def test_rk_is_deterministic_and_restartable(fcns):
    w = W.get("channel_32x32x33")
    v0, _ = w.initial_state()
    a = fcns.Solver.from_workload(w)
    a.set_state(torch.from_numpy(v0))
    a.rk_step(w.dt, 4)
    snap = [a.get_spectral(f).clone() for f in range(3)]
    gw = a.get_wall_grad().clone()
    a.rk_step(w.dt, 3)
    va, _, _ = a.get_state()
    b = fcns.Solver.from_workload(w)
    b.set_spectral(snap, gw)
    b.rk_step(w.dt, 3)
    vb, _, _ = b.get_state()
    c = fcns.Solver.from_workload(w)
    c.set_state(torch.from_numpy(v0))
    c.rk_step(w.dt, 7)
    vc, _, _ = c.get_state()
    torch.cuda.synchronize()
    assert torch.equal(va, vb)     # resume is bitwise identical
    assert torch.equal(va, vc)     # and so is a repeated run


def test_kernel_timing_classes_and_mask(fcns):
    # every class, then one class only; the step's results do not depend on it
    w = W.get("channel_32x32x33")
    v0, _ = w.initial_state()
    a = fcns.Solver.from_workload(w)
    a.set_state(torch.from_numpy(v0))
    a.set_timing(True)
    a.timing_reset()
    a.rk_step(w.dt, 2)
    rep = a.timing_report()
    assert set(rep) == set(a.TIMING_CLASSES)
    used = {k: (n, ms) for k, (n, ms) in rep.items() if n > 0}
    # one launch per substep of each class the step uses: the x and y passes
    # and either the fused z pass or its three separate kernels
    assert {"y_back_dy", "y_back_dz", "x_nl", "y_fwd"} <= set(used), rep
    assert "z_pass" in used or {"z_stageA", "z_stageB", "z_back"} <= set(used), rep
    assert all(n == 4 for n, _ in used.values()), rep
    assert all(ms > 0 for _, ms in used.values()), rep
    a.set_timing(True, classes=["x_nl"])
    a.timing_reset()
    a.rk_step(w.dt, 3)
    rep = a.timing_report()
    assert rep["x_nl"][0] == 6
    assert all(n == 0 for k, (n, _) in rep.items() if k != "x_nl"), rep
    with pytest.raises(fcns.FcnsError):
        a._check(a.lib.fcns_set_timing_mask(a.ctx, 1 << len(a.TIMING_CLASSES)))
    a.set_timing(False)
    va, _, _ = a.get_state()
    b = fcns.Solver.from_workload(w)
    b.set_state(torch.from_numpy(v0))
    b.rk_step(w.dt, 5)
    vb, _, _ = b.get_state()
    torch.cuda.synchronize()
    assert torch.equal(va, vb)


# ------------------------------------------------------------------ diagnostics
def _diag_pair(fcns, w, steps):
    from oracle.diagnostics import diagnostics, spectra
    v0, th0 = w.initial_state()
    s = fcns.Solver.from_workload(w)
    s.set_state(torch.from_numpy(v0), torch.from_numpy(th0) if th0 is not None else None)
    s.rk_step(w.dt, steps)
    o = Oracle(Problem(**w.problem_kwargs()))
    o.set_state(v0, th0)
    o.rk_step(w.dt, steps)
    return s, o, diagnostics, spectra


@pytest.mark.parametrize("kind", ["channel", "rb"])
def test_diagnostics_match_oracle(fcns, kind):
    if kind == "channel":
        w = W.channel(32, 24, 33, 2000.0, C=25, dt=1e-3, steps=4, seed=21, noise_rms=0.05)
    else:
        w = W.rayleigh_benard(32, 24, 33, 1e5, C=31, dt=2e-3, steps=4, kmax=3, mmax=3,
                              noise_rms=1e-2)
    s, o, diagnostics, spectra = _diag_pair(fcns, w, w.steps)
    got = s.diagnostics()
    ref = diagnostics(o)
    # residues of cancellation (the FC divergence, the wall values) are
    # compared as rms values against the velocity scale, the others relatively
    vscale = np.sqrt(2 * ref["energy"])
    kmax = np.pi * max(w.nx / w.lx, w.ny / w.ly, (w.nz - 1) / w.lz)
    residue = {"div2": vscale * kmax, "slip_bottom": vscale, "slip_top": vscale,
               "w2_bottom": vscale, "w2_top": vscale}
    delta = w.lz / 2
    for k, r in ref.items():
        g = got[k]
        if np.isnan(r):
            assert np.isnan(g), k
        elif k in residue:
            assert abs(np.sqrt(g) - np.sqrt(r)) <= 1e-11 * residue[k], (k, g, r)
        elif k.startswith("dudz"):
            assert abs(g - r) <= 1e-11 * vscale * kmax, (k, g, r)
        elif k.startswith("re_tau"):
            # u_tau^2 = nu |dU/dz|
            ut2 = lambda x: (x * w.nu / delta) ** 2
            assert abs(ut2(g) - ut2(r)) <= 1e-11 * w.nu * vscale * kmax, (k, g, r)
        elif k.startswith("nu_"):
            assert abs(g - r) <= 1e-11 * max(1.0, abs(r)), (k, g, r)
        else:
            assert abs(g - r) <= 1e-11 * abs(r), (k, g, r)
    for f in range(w.nfields):
        ex, ey = s.spectra(f, 7)
        rx, ry = spectra(o, f, 7)
        assert rel_l2(ex, rx) < 1e-11 and rel_l2(ey, ry) < 1e-11


# ------------------------------------------------------------------ autotuner
@pytest.mark.parametrize("name", ["channel_32x32x33", "prime"])
def test_autotuned_steps_keep_parity(fcns, name):
    if name == "prime":   # run-time z plan 2 * 3 * 47: its radix orders are tried
        w = W.channel(16, 8, 257, 2000.0, d=5, C=25, dt=5e-4, steps=3, seed=9, noise_rms=0.05)
    else:
        w = W.get(name)
    v0, _ = w.initial_state()
    s = fcns.Solver.from_workload(w)
    s.set_state(torch.from_numpy(v0))
    rep = s.autotune()
    assert rep.startswith("y: grid") and "x: variant" in rep and "z: radices" in rep
    s.rk_step(w.dt, w.steps)
    v, _, _ = s.get_state()
    torch.cuda.synchronize()
    o = Oracle(Problem(**w.problem_kwargs()))
    o.set_state(v0)
    o.rk_step(w.dt, w.steps)
    rv, _, _ = o.get_state()
    assert rel_l2(v, rv) < 1e-11
