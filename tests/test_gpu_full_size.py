"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (the compile-time 512- and 256-point plans in x and y, the
288-point plan in z for the Rayleigh-Benard grid, the run-time plan with the
radix-47 stage for the channel grid).

The oracle cannot run a whole 512 x 512 x 257 step in test time, so these
tests use what holds at any size:
* a single horizontal Fourier mode of tiny amplitude evolves linearly (the
  advective term is quadratic, 1e-13 relative), and the linear step of one
  (kx, ky) mode depends only on the wavenumbers, so the oracle on an 8 x 8
  grid with the same box gives the exact expected coefficients of the mode;
* the step commutes with a shift by one grid cell in x and in y.
"""
import math

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
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _mode_state(xp, w, nx, ny, p, q, eps, device=None):
    """psi = cos(ph) sin(pi z / Lz), ph = 2 pi (p x / Lx + q y / Ly) + 0.3:
    v = curl(psi z^) (divergence-free, zero at the walls) and, for the
    Boussinesq system, theta = psi, both times eps.  [nz][ny][nx] arrays."""
    kw = {} if device is None else {"device": device}
    f64 = np.float64 if xp is np else torch.float64
    x = xp.arange(nx, dtype=f64, **kw) * (w.lx / nx)
    y = xp.arange(ny, dtype=f64, **kw) * (w.ly / ny)
    z = xp.arange(w.nz, dtype=f64, **kw) * (w.lz / (w.nz - 1))
    kx, ky = 2 * math.pi * p / w.lx, 2 * math.pi * q / w.ly
    ph = kx * x[None, :] + ky * y[:, None] + 0.3
    sz = xp.sin(math.pi * z / w.lz)[:, None, None]
    c, s = xp.cos(ph)[None], xp.sin(ph)[None]
    u = eps * (-ky) * s * sz                  # d psi / dy
    v = eps * kx * s * sz                     # -d psi / dx
    wv = 0.0 * u
    vel = xp.stack([u, v, wv])
    th = eps * c * sz if w.boussinesq else None
    return vel, th


@pytest.mark.parametrize("name,p,q", [("rb_512x512x257", 1, 2), ("channel_256x256x257", 2, 1)])
def test_single_mode_step_matches_oracle_at_full_size(fcns, name, p, q):
    w = W.get(name)
    if w.kind == "channel":
        w = W.get(name, forcing_x=0.0)      # the mean flow would couple modes
    eps = 1e-13
    s = fcns.Solver.from_workload(w)
    v0, th0 = _mode_state(torch, w, w.nx, w.ny, p, q, eps, device="cuda")
    s.set_state(v0, th0)
    s.rk_step(w.dt, 1)
    gpu = [s.get_spectral(f)[:, q, p].cpu().numpy() / (w.nx * w.ny) for f in range(w.nfields)]
    torch.cuda.synchronize()
    n = 8
    ws = W.get(name, nx=n, ny=n, forcing_x=0.0)
    vs, ths = _mode_state(np, ws, n, n, p, q, eps)
    o = Oracle(Problem(**ws.problem_kwargs()))
    o.set_state(vs, ths)
    o.rk_step(w.dt, 1)
    ref = [o.Vt[i][:, q, p] / (n * n) for i in range(3)]
    if w.boussinesq:
        ref.append(o.Tt[:, q, p] / (n * n))
    assert rel_l2(np.concatenate(gpu), np.concatenate(ref)) < 1e-11


@pytest.mark.parametrize("name", ["rb_512x512x257", "channel_256x256x257"])
def test_step_commutes_with_grid_shifts_at_full_size(fcns, name):
    w = W.get(name)
    r = W.rng(77)
    dev = "cuda"
    x = torch.arange(w.nx, dtype=torch.float64, device=dev) * (2 * math.pi / w.nx)
    y = torch.arange(w.ny, dtype=torch.float64, device=dev) * (2 * math.pi / w.ny)
    z = torch.arange(w.nz, dtype=torch.float64, device=dev) * (1.0 / (w.nz - 1))
    env = (torch.sin(math.pi * z) ** 2)[:, None, None]

    def field(scale):
        acc = torch.zeros((w.nz, w.ny, w.nx), dtype=torch.float64, device=dev)
        for _ in range(6):
            a, b, c = r.standard_normal(3)
            pk, qk, mk = r.integers(0, 6, 3)
            acc += (scale * a) * torch.cos(pk * x[None, None, :] + b) \
                * torch.cos(qk * y[None, :, None] + c) * (env * torch.cos(mk * math.pi * z)[:, None, None])
        return acc

    v0 = torch.stack([field(0.5) for _ in range(3)])
    th0 = field(1e-2) if w.boussinesq else None
    outs = []
    for sx, sy in ((0, 0), (1, 3)):
        s = fcns.Solver.from_workload(w)
        vin = torch.roll(v0, shifts=(sy, sx), dims=(-2, -1)).contiguous()
        tin = torch.roll(th0, shifts=(sy, sx), dims=(-2, -1)).contiguous() if th0 is not None else None
        s.set_state(vin, tin)
        s.rk_step(w.dt, 1)
        v, th, _ = s.get_state()
        outs.append((v, th))
        torch.cuda.synchronize()
        s.close()
    (va, ta), (vb, tb) = outs
    va = torch.roll(va, shifts=(3, 1), dims=(-2, -1))
    assert (torch.linalg.vector_norm(va - vb) / torch.linalg.vector_norm(vb)).item() < 1e-11
    if ta is not None:
        ta = torch.roll(ta, shifts=(3, 1), dims=(-2, -1))
        assert (torch.linalg.vector_norm(ta - tb) / torch.linalg.vector_norm(tb)).item() < 1e-11
    assert bool(torch.isfinite(vb).all())
