"""Pins of the oracle's own discrete Fourier transforms, of its exponential
filter (Sec. 4.3) and of its pressure output (Sec. 4.2).

The transforms are checked against the definition of the DFT evaluated term
by term; the filter against the two facts Sec. 4.3 states (the largest
wavenumber of each direction is attenuated by exp(-beta), well-resolved modes
are left alone) and against a nonlinear term whose filtered value is known in
closed form; the pressure against potentials whose gradient the projection
must remove (Sec. 4.2: the inhomogeneous part, the closed-form homogeneous
part, and the hydrostatic balance of a horizontally uniform temperature).
"""
import math
import os

import numpy as np
import pytest

from oracle import fft as dft
from oracle.ns import BETA_DEFAULT, Oracle, Problem
import workloads as W

# every transform length the oracle meets: N' = nz + C of the workloads and
# tests (C = 25: 42, 58, 66, 90, 122, 154, 218, 282, 538; C = 31: 64, 96, 128,
# 160, 224, 288) and the periodic lengths
N_CONTINUED = [42, 58, 64, 66, 90, 96, 122, 128, 154, 160, 218, 224, 282, 288, 538]
N_PERIODIC = [2, 4, 6, 8, 12, 16, 32, 64, 96, 128, 192, 256, 512]


def _dft_by_definition(x, sign=-1):
    """X_k = sum_j x_j exp(sign 2 pi i j k / N), one k at a time."""
    n = x.shape[0]
    j = np.arange(n)
    out = np.empty_like(x, dtype=np.complex128)
    for k in range(n):
        w = np.exp(sign * 2j * np.pi * ((j * k) % n) / n)
        out[k] = (w[:, None] * x).sum(axis=0)
    return out


@pytest.mark.parametrize("n", N_CONTINUED + N_PERIODIC)
def test_fft_matches_the_dft_definition(n):
    r = W.rng(1000 + n)
    x = r.standard_normal((n, 3)) + 1j * r.standard_normal((n, 3))
    ref = _dft_by_definition(x)
    got = dft.fft(x, 0)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()
    inv = _dft_by_definition(x, +1) / n
    assert np.abs(dft.ifft(x, 0) - inv).max() < 1e-13 * np.abs(inv).max()
    # the O(N^2) matrix form of the oracle agrees with both
    assert np.abs(dft.dft(x, 0) - ref).max() < 1e-13 * np.abs(ref).max()


def test_fft_closed_forms_and_axes():
    n = 90
    e0 = np.zeros(n)
    e0[0] = 1.0
    assert np.abs(dft.fft(e0) - 1.0).max() < 1e-15          # delta -> all ones
    m = 7
    wave = np.exp(2j * np.pi * m * np.arange(n) / n)
    spec = dft.fft(wave)
    expect = np.zeros(n, dtype=complex)
    expect[m] = n
    assert np.abs(spec - expect).max() < 1e-12              # one mode -> N delta_m
    r = W.rng(7)
    a = r.standard_normal((6, 10, 16))
    # along the last and middle axes, real forms, Parseval
    full = dft.fft(dft.fft(a, -1), -2)
    half = dft.fft(dft.rfft(a, -1), -2)
    assert np.abs(full[..., :9] - half).max() < 1e-12
    back = dft.irfft(dft.ifft(half, -2), 16, -1)
    assert np.abs(back - a).max() < 1e-14
    assert abs(np.sum(np.abs(full) ** 2) / (10 * 16) - np.sum(a ** 2)) < 1e-10 * np.sum(a ** 2)
    assert np.array_equal(dft.signed_index(6), np.array([0, 1, 2, -3, -2, -1], dtype=float))
    assert np.array_equal(dft.signed_index(5), np.array([0, 1, 2, -2, -1], dtype=float))


def test_oracle_uses_no_fft_library():
    here = os.path.join(os.path.dirname(__file__), "..", "oracle")
    for name in os.listdir(here):
        if name.endswith(".py"):
            src = open(os.path.join(here, name)).read()
            for lib in ("np.fft", "numpy.fft", "scipy.fft", "scipy.fftpack", "pocketfft"):
                assert lib not in src, (name, lib)


# ---------------------------------------------------------------- filter (Sec. 4.3)
def _oracle(nx=16, ny=12, nz=33, lx=2 * np.pi, ly=3.0, lz=1.0, **kw):
    return Oracle(Problem(nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz, nu=kw.pop("nu", 0.0),
                          C=kw.pop("C", 25), **kw))


@pytest.mark.parametrize("nx,ny,nz", [(16, 12, 33), (32, 64, 41)])
def test_filter_attenuates_each_nyquist_by_exp_minus_beta(nx, ny, nz):
    o = _oracle(nx=nx, ny=ny, nz=nz)
    s = o.sigma
    npr = o.np_
    eb = math.exp(-BETA_DEFAULT)
    assert abs(BETA_DEFAULT - 16 * math.log(10)) < 1e-15
    # Sec. 4.3: the largest wavenumber of a direction is attenuated by e^-beta
    assert abs(s[0, 0, nx // 2] / eb - 1) < 1e-12
    assert abs(s[0, ny // 2, 0] / eb - 1) < 1e-12
    assert abs(s[npr // 2, 0, 0] / eb - 1) < 1e-12
    assert abs(s[npr // 2, ny // 2, nx // 2] / eb ** 3 - 1) < 1e-12
    # and the well-resolved modes (|m| <= N/4) are left alone
    assert s[0, 0, : nx // 4 + 1].min() >= 1 - 1e-15
    my = dft.signed_index(ny)
    assert s[0, np.abs(my) <= ny // 4, 0].min() >= 1 - 1e-15
    mz = dft.signed_index(npr)
    assert s[np.abs(mz) <= npr // 4, 0, 0].min() >= 1 - 1e-15
    # symmetric in +-m and non-increasing in |m| in every direction
    assert np.all(np.diff(s[0, 0, :]) <= 0)
    for axis_vals, m in ((s[0, :, 0], my), (s[:, 0, 0], mz)):
        for k in range(1, len(m) // 2):
            assert axis_vals[k] == axis_vals[len(m) - k]
        order = np.argsort(np.abs(m), kind="stable")
        assert np.all(np.diff(axis_vals[order]) <= 0)


def test_filtered_nonlinear_term_closed_form():
    # u = cos(3 x') + sin(4 y'), v = cos(4 y'), w = 0 (x' = 2 pi x / Lx, y' =
    # 2 pi y / Ly) on a 16 x 16 grid: -(v.grad)u = 1.5 k1 sin(6 x') +
    # 3 k1 sin(4 y') sin(3 x') - 2 k2 (1 + cos(8 y')), -(v.grad)v = 2 k2 sin(8 y')
    # (zero on the grid).  cos(8 y') is the y Nyquist mode: the filter removes
    # it to e^-beta; the modes at |m| <= 3N/8 keep their amplitude to 1e-10.
    nx = ny = 16
    nz, lx, ly, lz = 33, 2.0, 3.0, 1.0
    o = _oracle(nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz)
    x, y, z = W.grid(nx, ny, nz, lx, ly, lz)
    X, Y = np.meshgrid(x, y, indexing="xy")
    k1, k2 = 2 * np.pi / lx, 2 * np.pi / ly
    xs, ys = k1 * X, k2 * Y
    one = np.ones((nz, 1, 1))
    v = np.stack([one * (np.cos(3 * xs) + np.sin(4 * ys))[None], one * np.cos(4 * ys)[None],
                  np.zeros((nz, ny, nx))])
    smooth = 1.5 * k1 * np.sin(6 * xs) + 3 * k1 * np.sin(4 * ys) * np.sin(3 * xs) - 2 * k2
    nyq = -2 * k2 * np.cos(8 * ys)
    raw, _ = o.rhs_nonlinear(v)
    filt, _ = o.rhs_nonlinear(v, filtered=True)
    scale = np.abs(smooth).max()
    assert np.abs(raw[0] - (smooth + nyq)[None]).max() < 1e-9 * scale
    assert np.abs(filt[0] - smooth[None]).max() < 1e-9 * scale
    assert np.abs(filt[1:]).max() < 1e-9 * scale


# ---------------------------------------------------------------- pressure (Sec. 4.2)
def _manufactured(nz, seed=3):
    nx, ny, lx, ly, lz = 16, 16, 2 * np.pi, 2 * np.pi, 1.0
    x, y, z = W.grid(nx, ny, nz, lx, ly, lz)
    vs = W.solenoidal_noise(nx, ny, nz, lx, ly, lz, 2, 2, 1.0, seed)
    X, Y = np.meshgrid(x, y, indexing="xy")
    Z = z[:, None, None]
    P = np.exp(0.7 * Z) + Z ** 3
    dP = 0.7 * np.exp(0.7 * Z) + 3 * Z ** 2
    T = (np.cos(X + 2 * Y) + 0.5)[None]
    phi = T * P
    gphi = np.stack([(-np.sin(X + 2 * Y))[None] * P, (-2 * np.sin(X + 2 * Y))[None] * P,
                     T * dP])
    return vs, phi, gphi, (nx, ny, lx, ly, lz)


def test_projection_pressure_is_the_potential():
    # v* = v_s + grad(phi), v_s solenoidal and zero at the walls: the
    # projection returns p = phi / c up to a constant (the inhomogeneous part
    # carries the z-dependence, D z the mean pencil's linear part)
    c = 0.25
    errs = []
    for nz in (33, 65, 129):
        vs, phi, gphi, (nx, ny, lx, ly, lz) = _manufactured(nz)
        o = _oracle(nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz)
        _, _, p = o.pressure_project(vs + gphi, c, pressure=True)
        ref = phi / c
        ref = ref - ref.mean()
        errs.append(np.abs(p - ref).max() / np.abs(ref).max())
    assert errs[-1] < 1e-6 and errs[0] / errs[-1] > 30, errs


def test_projection_pressure_of_a_harmonic_potential():
    # phi = cos x cos y (a e^{g(z-Lz)} + b e^{-gz}) is the closed-form
    # homogeneous solution of Sec. 4.2 (A = a, B = b): p = phi / c
    nz, c = 65, 0.5
    o = _oracle(nx=8, ny=8, nz=nz, lx=2 * np.pi, ly=2 * np.pi, lz=1.0)
    x, y, z = W.grid(8, 8, nz, 2 * np.pi, 2 * np.pi, 1.0)
    X, Y = np.meshgrid(x, y, indexing="xy")
    g = math.sqrt(2.0)
    a, b = 0.7, -0.4
    Z = z[:, None, None]
    prof = a * np.exp(g * (Z - 1)) + b * np.exp(-g * Z)
    dprof = g * (a * np.exp(g * (Z - 1)) - b * np.exp(-g * Z))
    cc = (np.cos(X) * np.cos(Y))[None]
    phi = cc * prof
    gphi = np.stack([(-np.sin(X) * np.cos(Y))[None] * prof,
                     (-np.cos(X) * np.sin(Y))[None] * prof, cc * dprof])
    _, _, p = o.pressure_project(gphi, c, pressure=True)
    ref = phi / c
    assert np.abs(p - (ref - ref.mean())).max() < 1e-6 * np.abs(ref).max()


@pytest.mark.parametrize("order", [1, 2])
def test_hydrostatic_pressure_of_the_step(order):
    # Sec. 7 Boussinesq step with v = 0 and theta = sin(pi z) (uniform in x, y),
    # kappa = 0: the buoyancy gamma theta z is a gradient, so the step keeps
    # v = 0 and theta, and get_state's pressure is its potential,
    # p = gamma int theta dz = -(gamma / pi) cos(pi z) up to a constant
    nx, ny, nz, gam = 8, 8, 65, 1.3
    o = _oracle(nx=nx, ny=ny, nz=nz, lx=2.0, ly=2.0, lz=1.0, nu=1e-3, boussinesq=True,
                kappa=0.0, gamma=gam, rk_order=order)
    z = np.linspace(0.0, 1.0, nz)
    th0 = np.sin(np.pi * z)[:, None, None] * np.ones((1, ny, nx))
    o.set_state(np.zeros((3, nz, ny, nx)), th0)
    o.rk_step(0.01, 3)
    v, th, p = o.get_state()
    ref = -(gam / np.pi) * np.cos(np.pi * z)[:, None, None] * np.ones((1, ny, nx))
    ref -= ref.mean()
    assert np.abs(p - ref).max() < 1e-6 * np.abs(ref).max()
    assert np.abs(v).max() < 1e-8
    assert np.abs(th - th0).max() < 1e-12
