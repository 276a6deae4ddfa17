"""Pins of the oracle's flow diagnostics (Sec. 6 and 7 definitions) and of
the App. A solenoidal noise generator, against closed forms and textbook
values."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.diagnostics import diagnostics, spectra
from oracle.ns import Oracle, Problem


def test_chandrasekhar_reid_lambdas_are_the_clamped_beam_roots():
    # App. A: g_m'(+-1/2) = 0; the roots are the clamped-clamped beam
    # eigenvalues (Chandrasekhar 1961, App. V): 4.7300, 7.8532, 10.9956, 14.1372
    lam = W.clamped_beam_lambdas(4)
    ref = [4.730040744862704, 7.853204624095838, 10.995607838001671, 14.137165491257464]
    assert np.allclose(lam, ref, rtol=0, atol=1e-12)
    # and they make g_m and g_m' vanish at both walls
    for m, l in enumerate(lam, start=1):
        g, dg, _ = W._g_cr(m, l, np.array([-0.5, 0.5]))
        assert np.abs(g).max() < 1e-12 and np.abs(dg).max() < 1e-9 * l


def test_curl_eigen_noise_is_no_slip_and_solenoidal():
    # App. A: no-slip (v = 0 and dw/dz = 0 at the walls) and divergence-free;
    # the FC divergence converges at high order as nz doubles
    divs = []
    for nz in (33, 65):
        v = W.curl_eigen_noise(32, 32, nz, 2 * np.pi, 2 * np.pi, 1.0, 1.0, 3)
        assert np.abs(v[:, 0]).max() < 1e-13 and np.abs(v[:, -1]).max() < 1e-13
        o = Oracle(Problem(nx=32, ny=32, nz=nz, lx=2 * np.pi, ly=2 * np.pi, lz=1.0, nu=0.01))
        o.set_state(v)
        divs.append(math.sqrt(np.mean(o.divergence(o.Vt) ** 2)))
    assert divs[1] < divs[0] / 8 and divs[1] < 1e-3


def test_poiseuille_diagnostics_closed_form():
    # Sec. 6: laminar u = G z (Lz - z) / (2 nu): dU/dz(0) = G Lz / (2 nu),
    # u_tau = sqrt(G Lz / 2), Re_tau = u_tau (Lz/2) / nu; slip and w vanish
    nx, ny, nz, lz, nu, G = 8, 8, 33, 2.0, 0.01, 3e-3
    o = Oracle(Problem(nx=nx, ny=ny, nz=nz, lx=2.0, ly=2.0, lz=lz, nu=nu, forcing_x=G))
    z = np.linspace(0, lz, nz)
    u = G * z * (lz - z) / (2 * nu)
    v = np.zeros((3, nz, ny, nx))
    v[0] = u[:, None, None]
    o.set_state(v)
    d = diagnostics(o)
    assert abs(d["dudz_bottom"] - G * lz / (2 * nu)) < 1e-8 * G * lz / nu
    assert abs(d["dudz_top"] + G * lz / (2 * nu)) < 1e-8 * G * lz / nu
    re_tau = math.sqrt(G * lz / 2) * (lz / 2) / nu
    assert abs(d["re_tau_bottom"] - re_tau) < 1e-8 * re_tau
    assert abs(d["re_tau_top"] - re_tau) < 1e-8 * re_tau
    assert abs(d["energy"] - 0.5 * np.mean(u ** 2)) < 1e-14
    assert d["slip_bottom"] < 1e-28 and d["w2_top"] == 0.0
    assert d["div2"] < 1e-28


def test_nusselt_closed_form():
    # Sec. 7: Nu = 1 - (1/gamma) d theta/dz at the wall (conduction: Nu = 1);
    # theta = a sin(pi z) gives 1 - a pi / gamma below and 1 + a pi / gamma above
    # (to the FC accuracy of a wall derivative at nz = 65)
    nx, ny, nz, a, gam = 8, 8, 65, 0.3, 2.0
    o = Oracle(Problem(nx=nx, ny=ny, nz=nz, lx=2.0, ly=2.0, lz=1.0, nu=0.01, boussinesq=True,
                       kappa=0.01, gamma=gam))
    z = np.linspace(0, 1, nz)
    th = np.broadcast_to((a * np.sin(np.pi * z))[:, None, None], (nz, ny, nx)).copy()
    o.set_state(np.zeros((3, nz, ny, nx)), th)
    d = diagnostics(o)
    assert abs(d["nu_bottom"] - (1 - a * np.pi / gam)) < 1e-6
    assert abs(d["nu_top"] - (1 + a * np.pi / gam)) < 1e-6
    o.set_state(np.zeros((3, nz, ny, nx)), 0 * th)
    d = diagnostics(o)
    assert d["nu_bottom"] == 1.0 and d["nu_top"] == 1.0


def test_spectra_and_divergence_closed_form():
    # Sec. 6 spectra: a single mode cos(3 kx0 x) f(z) puts f(z)^2 / 2 at kx = 3
    # and sums to the x-y mean of u^2; the divergence of (sin(kx x) g, 0, 0)
    # is kx cos(kx x) g, so <div^2> = kx^2 <g^2> / 2
    nx, ny, nz, lx = 32, 16, 33, 2.0
    o = Oracle(Problem(nx=nx, ny=ny, nz=nz, lx=lx, ly=2.0, lz=1.0, nu=0.01))
    x, y, z = W.grid(nx, ny, nz, lx, 2.0, 1.0)
    kx = 2 * np.pi * 3 / lx
    g = np.sin(np.pi * z) * (1 + z)
    v = np.zeros((3, nz, ny, nx))
    v[0] = np.sin(kx * x)[None, None, :] * g[:, None, None]
    o.set_state(v)
    ex, ey = spectra(o, 0, 10)
    assert abs(ex[3] - g[10] ** 2 / 2) < 1e-14
    assert abs(ex.sum() - ex[3]) < 1e-14 and abs(ey.sum() - np.mean(v[0][10] ** 2)) < 1e-14
    d = diagnostics(o)
    assert abs(d["div2"] - kx ** 2 * np.mean(g ** 2) / 2) < 1e-12 * kx ** 2
