"""Time-splitting Runge-Kutta FC-Gram step for incompressible flow (Sec. 4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Domain (Sec. 2): (0,Lx) x (0,Ly) x (0,Lz), periodic in x and y, no-slip walls at
z = 0 and z = Lz.  Physical arrays are float64 [Nz][Ny][Nx] (x fastest),
x_q = q Lx/Nx, y_r = r Ly/Ny, z_s = s Lz/(Nz-1).

Spaces
------
physical   [Nz][Ny][Nx] real
mixed      (kx, ky, z): [Nz][Ny][Nx/2+1] complex, F_xy = r2c FFT in x then
           c2c FFT in y, both unnormalized; B_xy is the inverse
continued  (kx, ky, kz): [N'][Ny][Nx/2+1] complex, F_z / B_z of ``FCGram``
           (Sec. 3: the FC-Gram transform commutes with the FFTs in x, y)

State: the continued spectral velocity (and temperature) coefficients
V^t, re-extended only where the paper performs an FC-Gram transform (the
pressureless field v* in step 3 and the homogeneous pressure gradient in step
5 of Sec. 4.4, and every forward transform of a physical product).

Readings where the paper is silent, garbled or self-inconsistent (each also
listed in the design notes of the repository):
* advection enters the pressureless update as -(v.grad)v (Sec. 2 governing
  equations; the printed '+' in Sec. 4.1 and 4.4 contradicts them);
* pressure in increment units phi = c_j p: grad(phi^I) = k(k.V*)/k^2 as printed
  in Sec. 4.4 step 3, b and t are the wall values of z.(v* - grad(phi^I)), the
  homogeneous solution uses A, B of Sec. 4.2, and the (0,0) mode carries
  phi^H = D z with D = (b+t)/2 (A = B = 0 there);
* stage coefficients c_j = dt/(o-j+1) (equal to j dt/o for the paper's o=2);
* filter argument eta = 2|m|/N per direction (largest wavenumber attenuated
  by exp(-beta) as Sec. 4.3 states), applied to the nonlinear term only;
* Nyquist modes: odd derivatives, the projection and the homogeneous rate
  gamma = |k~_h| use k~ (Nyquist zeroed); the Laplacian uses the true k.  With
  the true k in gamma the homogeneous gradient of a Nyquist pencil is not
  solenoidal for the discrete divergence and the step is unstable; every
  pencil with gamma = 0 (the mean and the Nyquist pencils) takes the (0,0)
  form phi^H = D z;
* first-stage wall pressure gradient G = 0 after ``set_state``;
* channel forcing +G x (G > 0; Sec. 6 laminar profile G z (Lz - z) / (2 nu));
* buoyancy +gamma theta z with source +gamma v_z in the theta equation
  (Sec. 7), which makes the conductive state unstable above onset;
* forcing and buoyancy are added at the physical points after restriction;
* products are formed on the Nx*Ny*Nz physical points only.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import fft as dft
from .fcgram import FCGram

BETA_DEFAULT = 16.0 * math.log(10.0)
TWO_P_DEFAULT = 100.0


@dataclass
class Problem:
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    nu: float
    d: int = 5
    C: int = 25
    forcing_x: float = 0.0
    boussinesq: bool = False
    kappa: float = 0.0
    gamma: float = 0.0
    rk_order: int = 2
    filter_beta: float = BETA_DEFAULT
    filter_2p: float = TWO_P_DEFAULT


def _signed(n):
    return dft.signed_index(n)


class Oracle:
    """Plain FP64 implementation of the step; one instance per problem."""

    def __init__(self, prob: Problem):
        p = prob
        if p.nx % 2 or p.ny % 2 or (p.nz + p.C) % 2:
            raise ValueError("nx, ny and nz + C must be even (eq. k)")
        self.p = p
        self.fc = FCGram(p.nz, p.d, p.C, p.lz)
        self.nkx = p.nx // 2 + 1
        self.np_ = self.fc.np_
        self.z = np.arange(p.nz) * self.fc.dz
        # wavenumbers, eq. k (FFT order); *_o: Nyquist zeroed (odd derivatives)
        mx = np.arange(self.nkx, dtype=np.float64)
        my = _signed(p.ny)
        self.kx = 2 * np.pi * mx / p.lx
        self.ky = 2 * np.pi * my / p.ly
        self.kx_o = self.kx.copy()
        self.kx_o[p.nx // 2] = 0.0
        self.ky_o = self.ky.copy()
        self.ky_o[p.ny // 2] = 0.0
        # broadcast shapes for continued arrays [N'][Ny][Nkx]
        self.KX = self.kx_o[None, None, :]
        self.KY = self.ky_o[None, :, None]
        self.KZ = self.fc.kz_odd[:, None, None]
        self.K2_true = (self.kx[None, None, :] ** 2 + self.ky[None, :, None] ** 2
                        + self.fc.kz[:, None, None] ** 2)
        self.K2_odd = self.KX ** 2 + self.KY ** 2 + self.KZ ** 2
        # exponential filter, Sec. 4.3 (eta = 2|m|/N per direction)
        two_p, beta = p.filter_2p, p.filter_beta
        ex = (2.0 * np.abs(mx) / p.nx) ** two_p
        ey = (2.0 * np.abs(my) / p.ny) ** two_p
        ez = (2.0 * np.abs(self.fc.lbar) / self.np_) ** two_p
        self.sigma = np.exp(-beta * (ez[:, None, None] + ey[None, :, None]
                                     + ex[None, None, :]))
        # homogeneous-pressure rate gamma = |k~_h|, Sec. 4.2
        self.gam = np.sqrt(self.kx_o[None, :] ** 2 + self.ky_o[:, None] ** 2)
        self.nf = 3
        self.Vt = None
        self.Tt = None
        self.G = None
        self.phi_last = None
        self.c_last = None

    # -- transforms -----------------------------------------------------------
    def Fxy(self, a):
        return dft.fft(dft.rfft(a, -1), -2)

    def Bxy(self, m):
        return dft.irfft(dft.ifft(m, -2), self.p.nx, -1)

    def Fz(self, m):
        return self.fc.fwd(m)

    def Bz(self, s):
        return self.fc.back(s)

    def to_spec(self, phys):
        return self.Fz(self.Fxy(np.asarray(phys, dtype=np.float64)))

    def to_phys(self, spec):
        return self.Bxy(self.Bz(spec))

    # -- state ----------------------------------------------------------------
    def set_state(self, v, theta=None):
        """V^t = F_z F_xy v; wall pressure gradient G = 0."""
        self.Vt = [self.to_spec(v[i]) for i in range(3)]
        self.Tt = self.to_spec(theta) if self.p.boussinesq else None
        self.G = np.zeros((2, 2, self.p.ny, self.nkx), dtype=np.complex128)
        self.phi_last = None

    def get_state(self):
        """Physical v (3 fields), theta (or None) and p (zero-mean, or None
        before the first stage)."""
        v = np.stack([self.to_phys(V) for V in self.Vt])
        th = self.to_phys(self.Tt) if self.p.boussinesq else None
        pres = None
        if self.phi_last is not None:
            pres = self.Bxy(self.phi_last / self.c_last)
            pres -= pres.mean()
        return v, th, pres

    # -- step 1-2: physical fields and the nonlinear term ----------------------
    def _phys_with_grad(self, W):
        """q, dq/dx, dq/dy, dq/dz at the physical points from continued W."""
        qm = self.Bz(W)
        dzm = self.Bz(1j * self.KZ * W)
        kx = self.kx_o[None, None, :]
        ky = self.ky_o[None, :, None]
        return (self.Bxy(qm), self.Bxy(1j * kx * qm), self.Bxy(1j * ky * qm),
                self.Bxy(dzm))

    def nonlinear(self, W, Th=None):
        """-(v.grad) q for every transported field q (Sec. 4.2: derivatives in
        Fourier space, products in real space).  Returns physical arrays."""
        g = [self._phys_with_grad(Wi) for Wi in W]
        u, v, w = g[0][0], g[1][0], g[2][0]
        out = [-(u * gi[1] + v * gi[2] + w * gi[3]) for gi in g]
        if Th is not None:
            gt = self._phys_with_grad(Th)
            out.append(-(u * gt[1] + v * gt[2] + w * gt[3]))
        return out

    # -- steps 7-11: projection -------------------------------------------------
    def project(self, Vs, c):
        """Pressure projection of a continued field V* (Sec. 4.2 and 4.4 steps
        3-5) in increment units phi = c p.

        Returns (V_new list, G_wall [2 walls][2 comps][Ny][Nkx] (p units,
        mixed space), phi in mixed space).
        """
        nz, lz = self.p.nz, self.p.lz
        KX, KY, KZ, K2 = self.KX, self.KY, self.KZ, self.K2_odd
        div = KX * Vs[0] + KY * Vs[1] + KZ * Vs[2]
        with np.errstate(divide="ignore", invalid="ignore"):
            s = np.where(K2 > 0, div / np.where(K2 > 0, K2, 1.0), 0.0)
        # grad(phi^I) = k~ s, phi^I = -i s (Sec. 4.4 step 3)
        r = self.Bz(Vs[2] - KZ * s)
        b, t = r[0], r[nz - 1]
        gam = self.gam
        pos = gam > 0
        g = np.where(pos, gam, 1.0)
        E = np.exp(-g * lz)
        den = g * (1.0 - E * E)
        A = np.where(pos, (t - b * E) / den, 0.0)
        B = np.where(pos, -(b - t * E) / den, 0.0)
        D = np.where(pos, 0.0, 0.5 * (b + t))
        z = self.z[:, None, None]
        ep = np.where(pos, np.exp(g * (z - lz)), 0.0)
        em = np.where(pos, np.exp(-g * z), 0.0)
        ikx = 1j * self.kx_o[None, None, :]
        iky = 1j * self.ky_o[None, :, None]
        sym = A * ep + B * em
        Hx = ikx * sym
        Hy = iky * sym
        Hz = np.where(pos, gam * (A * ep - B * em), D)
        phiH = np.where(pos, sym, D * z)
        V_new = [Vs[0] - KX * s - self.Fz(Hx),
                 Vs[1] - KY * s - self.Fz(Hy),
                 Vs[2] - KZ * s - self.Fz(Hz)]
        sm = self.Bz(s)
        G = np.empty((2, 2, self.p.ny, self.nkx), dtype=np.complex128)
        for wi, si in ((0, 0), (1, nz - 1)):
            G[wi, 0] = (self.kx_o[None, :] * sm[si] + Hx[si]) / c
            G[wi, 1] = (self.ky_o[:, None] * sm[si] + Hy[si]) / c
        phi = self.Bz(-1j * s) + phiH
        return V_new, G, phi

    # -- one RK stage (Sec. 4.4, steps 1-5) -------------------------------------
    def stage(self, W, Thw, c):
        p = self.p
        nz = p.nz
        NL = self.nonlinear(W, Thw)
        lap = -self.K2_true
        Nh = [self.sigma * self.to_spec(a) for a in NL]
        vs = [self.Bz(self.Vt[i] + c * (Nh[i] + p.nu * lap * W[i]))
              for i in range(3)]
        vs[0][:, 0, 0] += c * p.forcing_x * p.nx * p.ny   # +G x at every point
        if p.boussinesq:
            vs[2] += c * p.gamma * self.Bz(Thw)
            ts = self.Bz(self.Tt + c * (Nh[3] + p.kappa * lap * Thw)) \
                + c * p.gamma * self.Bz(W[2])
            ts[0] = 0.0
            ts[nz - 1] = 0.0
        # BC injection (Sec. 4.4 step 2): v*_par = c grad_par p_prev at walls
        for comp in (0, 1):
            vs[comp][0] = c * self.G[0, comp]
            vs[comp][nz - 1] = c * self.G[1, comp]
        Vs = [self.Fz(a) for a in vs]
        V_new, G, phi = self.project(Vs, c)
        Th_new = self.Fz(ts) if p.boussinesq else None
        return V_new, Th_new, G, phi

    def rk_step(self, dt, nsteps=1):
        o = self.p.rk_order
        for _ in range(nsteps):
            W, Thw = self.Vt, self.Tt
            for j in range(1, o + 1):
                c = dt / (o - j + 1)
                W, Thw, self.G, self.phi_last = self.stage(W, Thw, c)
                self.c_last = c
            self.Vt, self.Tt = W, Thw

    # -- standalone entry points -----------------------------------------------
    def rhs_nonlinear(self, v, theta=None, filtered=False):
        """-(v.grad)v (and -(v.grad)theta) from the continued transform of v."""
        W = [self.to_spec(v[i]) for i in range(3)]
        Th = self.to_spec(theta) if theta is not None else None
        NL = self.nonlinear(W, Th)
        if filtered:
            NL = [self.to_phys(self.sigma * self.to_spec(a)) for a in NL]
        nlv = np.stack(NL[:3])
        nlt = NL[3] if theta is not None else None
        return nlv, nlt

    def pressure_project(self, v_star, c, pressure=False):
        """Project a physical v* (no BC injection).  Returns the physical
        projected velocity and the wall tangential pressure gradient
        [2 walls][2 comps][Ny][Nx] in p units; with ``pressure`` also the
        physical pressure phi / c (phi^I + phi^H of Sec. 4.2) with zero mean."""
        Vs = [self.to_spec(v_star[i]) for i in range(3)]
        V_new, G, phi = self.project(Vs, c)
        v = np.stack([self.to_phys(V) for V in V_new])
        gp = dft.irfft(dft.ifft(G, -2), self.p.nx, -1)
        if not pressure:
            return v, gp
        pres = self.Bxy(phi / c)
        return v, gp, pres - pres.mean()

    # -- diagnostics used by the pins ------------------------------------------
    def divergence(self, V):
        """Physical FC divergence of a continued field."""
        return self.to_phys(1j * (self.KX * V[0] + self.KY * V[1] + self.KZ * V[2]))
