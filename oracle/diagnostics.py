"""Flow diagnostics of an oracle state (TEST INFRASTRUCTURE ONLY, see
``oracle/__init__``), computed on the physical grid from their definitions.

* kinetic energy: one half of the mean of |v|^2 over the Nx*Ny*Nz grid points;
* FC divergence: the mean of (div v)^2 over the grid (the quantity whose
  smallness Sec. 6 reports);
* wall values: the means over the wall planes of u^2 + v^2 (slip) and w^2
  (Sec. 6 reports both);
* friction Reynolds number (Sec. 6): u_tau = sqrt(nu |dU/dz|) at a wall, with
  U the x-y mean of u, and Re_tau = u_tau delta / nu, delta = Lz / 2;
* Nusselt number at each wall (Sec. 7) in the sign that makes the conductive
  state Nu = 1: Nu = 1 - (1/gamma) <d theta / dz>_xy;
* 1D spectra at one height (Sec. 6, the two spectra equations): E(kx) sums
  |v^(kx, ky)|^2 over ky and E(ky) sums over kx, with the +-kx halves folded
  onto kx >= 0 and the transform normalised so that each spectrum sums to the
  x-y mean of v^2 at that height.

z derivatives are B_z(i k~z V^) of the continued state, as in the step.
"""
from __future__ import annotations

import math

import numpy as np

from . import fft as dft
from .ns import Oracle

NAMES = ("energy", "div2", "slip_bottom", "slip_top", "w2_bottom", "w2_top",
         "dudz_bottom", "dudz_top", "re_tau_bottom", "re_tau_top", "nu_bottom", "nu_top",
         "theta2")


def _dz_phys(o: Oracle, W):
    return o.Bxy(o.Bz(1j * o.KZ * W))


def diagnostics(o: Oracle):
    """The NAMES values of the oracle's current state (dict)."""
    p = o.p
    v, th, _ = o.get_state()
    out = {}
    out["energy"] = 0.5 * float(np.mean(v[0] ** 2 + v[1] ** 2 + v[2] ** 2))
    out["div2"] = float(np.mean(o.divergence(o.Vt) ** 2))
    out["slip_bottom"] = float(np.mean(v[0][0] ** 2 + v[1][0] ** 2))
    out["slip_top"] = float(np.mean(v[0][-1] ** 2 + v[1][-1] ** 2))
    out["w2_bottom"] = float(np.mean(v[2][0] ** 2))
    out["w2_top"] = float(np.mean(v[2][-1] ** 2))
    dudz = _dz_phys(o, o.Vt[0])
    out["dudz_bottom"] = float(np.mean(dudz[0]))
    out["dudz_top"] = float(np.mean(dudz[-1]))
    delta = p.lz / 2.0
    for wall, g in (("bottom", out["dudz_bottom"]), ("top", -out["dudz_top"])):
        out[f"re_tau_{wall}"] = (math.sqrt(p.nu * abs(g)) * delta / p.nu) if p.nu > 0 else 0.0
    if p.boussinesq:
        dtdz = _dz_phys(o, o.Tt)
        out["nu_bottom"] = 1.0 - float(np.mean(dtdz[0])) / p.gamma
        out["nu_top"] = 1.0 - float(np.mean(dtdz[-1])) / p.gamma
        out["theta2"] = float(np.mean(th ** 2))
    else:
        out["nu_bottom"] = out["nu_top"] = float("nan")
        out["theta2"] = 0.0
    return out


def spectra(o: Oracle, field, z):
    """(E(kx) for kx = 0..Nx/2, E(ky) for ky in FFT order) of physical field
    `field` (0..2 velocity, 3 theta) at grid height index z."""
    v, th, _ = o.get_state()
    a = th if field == 3 else v[field]
    nx, ny = o.p.nx, o.p.ny
    f = dft.fft(dft.fft(a[z], -1), -2) / (nx * ny)   # [ky][kx], all kx
    e = np.abs(f) ** 2
    ex = np.zeros(nx // 2 + 1)
    for m in range(nx):
        ex[min(m, nx - m)] += e[:, m].sum()
    ey = e.sum(axis=1)
    return ex, ey
