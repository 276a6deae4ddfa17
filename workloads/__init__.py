"""Seeded synthetic inputs shared by the tests, the oracle runs and the bench.

This module builds initial conditions and request streams only: analytic
fields evaluated on the grid with numpy, from a seeded PCG64 generator.  It
holds none of the solver's arithmetic (no FC continuation, no spectral
transform, no projection), so the HIP path and the oracle stay independent.

Workloads (the paper's channel and Rayleigh-Benard set-ups, Sec. 6 and 7,
scaled to the sizes measured here; no dataset is involved):

channel_32x32x33     channel, FP64, box 4pi x 2pi x 2, d=5, C=25, Re=1000
                     (laminar u_max = 1), Poiseuille profile plus divergence-free
                     noise of rms 1e-3, dt=1e-3, 10 steps
channel_256x256x257  channel, box 4pi x 2pi x 2, d=5, C=25, u_tau = 1,
                     nu = 1/180 (Re_tau = 180), forcing 1, Reichardt log-law
                     mean plus divergence-free noise of rms 0.1 U_bulk,
                     dt=2e-4, 100 steps
rb_512x512x257       Rayleigh-Benard, box 2 x 2 x 1, gamma=1, Ra=1e8, Pr=1,
                     nu = kappa = 1e-4, d=5, C=31 (N' = 288), v = 0 and
                     band-limited temperature noise of rms 1e-3 vanishing at
                     the walls, dt=1e-3, 50 steps
serving_stream       64 requests, Poisson arrivals at 20/s, channel or RB
                     (50/50), side in {32,64,96,128,192}, nz = side+1, C=31,
                     Re ~ U[500,5000] or Ra ~ logU[1e4,1e8], 20 steps each,
                     started from the App. A solenoidal no-slip noise
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def grid(nx, ny, nz, lx, ly, lz):
    x = np.arange(nx) * (lx / nx)
    y = np.arange(ny) * (ly / ny)
    z = np.arange(nz) * (lz / (nz - 1))
    return x, y, z


# ----------------------------------------------------------------------------
# analytic fields
# ----------------------------------------------------------------------------
def _mode_list(kmax):
    # (p, q) with p >= 0, and q > 0 when p == 0, excluding (0, 0)
    out = []
    for p in range(0, kmax + 1):
        for q in range(-kmax, kmax + 1):
            if p == 0 and q <= 0:
                continue
            out.append((p, q))
    return out


def solenoidal_noise(nx, ny, nz, lx, ly, lz, kmax, mmax, rms, seed):
    """Divergence-free field vanishing (with its normal derivative) at the
    walls: v = curl Psi, Psi_c = sum a T(x,y) sin(m pi z/Lz) g(z),
    g = (z (Lz - z) / (Lz/2)^2)^2.  Returned as float64 [3][nz][ny][nx],
    scaled to the requested rms (over all components)."""
    r = rng(seed)
    x, y, z = grid(nx, ny, nz, lx, ly, lz)
    X, Y = np.meshgrid(x, y, indexing="xy")  # (ny, nx)
    h = (lz / 2.0) ** 2
    g = (z * (lz - z)) ** 2 / h ** 2
    gp = 2.0 * z * (lz - z) * (lz - 2.0 * z) / h ** 2
    modes = _mode_list(kmax)
    nm = len(modes)
    kx = np.array([2 * np.pi * p / lx for (p, _) in modes])
    ky = np.array([2 * np.pi * q / ly for (_, q) in modes])
    ph = kx[:, None, None] * X[None] + ky[:, None, None] * Y[None]
    H = np.cos(ph).reshape(nm, -1)          # horizontal harmonics (modes, ny*nx)
    S = np.sin(ph).reshape(nm, -1)
    # coefficients drawn in (m, mode, component, cos/sin) order
    ab = r.standard_normal((mmax, nm, 3, 2))
    A, B = ab[..., 0], ab[..., 1]            # (m, mode, c)
    # T_c = sum a cs + b sn; its x and y derivatives, per m and component
    T = np.einsum("mic,ip->mcp", A, H) + np.einsum("mic,ip->mcp", B, S)
    Tx = np.einsum("mic,ip->mcp", B * kx[None, :, None], H) \
        - np.einsum("mic,ip->mcp", A * kx[None, :, None], S)
    Ty = np.einsum("mic,ip->mcp", B * ky[None, :, None], H) \
        - np.einsum("mic,ip->mcp", A * ky[None, :, None], S)
    km = np.arange(1, mmax + 1) * np.pi / lz
    Zm = np.sin(km[:, None] * z[None]) * g[None]                       # (m, nz)
    Zpm = km[:, None] * np.cos(km[:, None] * z[None]) * g[None] + np.sin(km[:, None] * z[None]) * gp[None]
    # v = curl Psi with Psi_c = T_c(x, y) Z(z), summed over m
    v = np.empty((3, nz, ny * nx))
    v[0] = Zm.T @ Ty[:, 2] - Zpm.T @ T[:, 1]
    v[1] = Zpm.T @ T[:, 0] - Zm.T @ Tx[:, 2]
    v[2] = Zm.T @ (Tx[:, 1] - Ty[:, 0])
    v = v.reshape(3, nz, ny, nx)
    cur = math.sqrt(float(np.mean(v ** 2)) * 3.0)
    return v * (rms / cur) if cur > 0 else v


def clamped_beam_lambdas(mmax):
    """lambda_1..lambda_mmax of the Chandrasekhar-Reid functions g_m (App. A):
    the roots of tanh(l/2) + tan(l/2) = 0 (m odd, even functions) and
    coth(l/2) - cot(l/2) = 0 (m even, odd functions), which alternate and lie
    near (m + 1/2) pi; found by bisection in FP64."""
    out = []
    for m in range(1, mmax + 1):
        if m % 2:
            f = lambda l: math.tanh(l / 2) + math.tan(l / 2)
        else:
            f = lambda l: 1.0 / math.tanh(l / 2) - 1.0 / math.tan(l / 2)
        guess = (m + 0.5) * math.pi
        lo, hi = guess - 0.3, guess + 0.3
        flo = f(lo)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            fm = f(mid)
            if (fm < 0) == (flo < 0):
                lo, flo = mid, fm
            else:
                hi = mid
        out.append(0.5 * (lo + hi))
    return out


def _g_cr(m, lam, zp):
    """g_m(z') and g_m'(z') of App. A (z' in [-1/2, 1/2])."""
    if m % 2:
        g = np.cosh(lam * zp) / math.cosh(lam / 2) - np.cos(lam * zp) / math.cos(lam / 2)
        dg = lam * (np.sinh(lam * zp) / math.cosh(lam / 2) + np.sin(lam * zp) / math.cos(lam / 2))
        d2 = lam ** 2 * (np.cosh(lam * zp) / math.cosh(lam / 2) + np.cos(lam * zp) / math.cos(lam / 2))
    else:
        g = np.sinh(lam * zp) / math.sinh(lam / 2) - np.sin(lam * zp) / math.sin(lam / 2)
        dg = lam * (np.cosh(lam * zp) / math.sinh(lam / 2) - np.cos(lam * zp) / math.sin(lam / 2))
        d2 = lam ** 2 * (np.sinh(lam * zp) / math.sinh(lam / 2) + np.sin(lam * zp) / math.sin(lam / 2))
    return g, dg, d2


def curl_eigen_noise(nx, ny, nz, lx, ly, lz, rms, seed, kh2=(4, 25), mrange=(2, 5)):
    """Random solenoidal no-slip field of App. A: q = curl curl(phi z^) +
    curl(psi z^) with phi = sum a exp(i(kx x + ky y)) g_m(z'), psi = sum b
    exp(i(kx x + ky y)) sin(m pi (z' + 1/2)), z' = z/Lz - 1/2, over horizontal
    mode numbers with kh2[0] <= n^2 + l^2 <= kh2[1] and mrange[0] <= m <=
    mrange[1]; random phases, uniform random amplitudes decaying as k^-4 (a)
    and k^-3 (b) with k^2 = kx^2 + ky^2 + (lambda_m / Lz)^2.  The mode numbers
    count the box's fundamental wavenumbers (the paper's box is 2 pi wide).
    Component form: q = (d2 phi/dxdz + dpsi/dy, d2 phi/dydz - dpsi/dx,
    -(d2/dx2 + d2/dy2) phi).  Scaled to the requested rms.

    Evaluated as z profiles times horizontal harmonics: with phase
    ph = kx x + ky y, cos(ph + alpha) = cos(ph) cos(alpha) - sin(ph) sin(alpha),
    so each horizontal mode contributes (profile_c)(z) cos(ph) +
    (profile_s)(z) sin(ph), and the sum over modes is one matrix product."""
    r = rng(seed)
    x, y, z = grid(nx, ny, nz, lx, ly, lz)
    X, Y = np.meshgrid(x, y, indexing="xy")
    zp = z / lz - 0.5
    lams = clamped_beam_lambdas(mrange[1])
    nmax = int(math.isqrt(kh2[1]))
    prof = []    # per horizontal mode: (3 components, cos/sin, nz) profiles
    harm = []    # per horizontal mode: (cos(ph), sin(ph)) flattened
    for n in range(-nmax, nmax + 1):
        for l in range(0, nmax + 1):
            if l == 0 and n < 0:
                continue               # real field: one of each +-(n, l) pair
            if not kh2[0] <= n * n + l * l <= kh2[1]:
                continue
            kx, ky = 2 * math.pi * n / lx, 2 * math.pi * l / ly
            P = np.zeros((3, 2, nz))
            for m in range(mrange[0], mrange[1] + 1):
                lam = lams[m - 1]
                k = math.sqrt(kx * kx + ky * ky + (lam / lz) ** 2)
                amp_a, pha, amp_b, phb = r.random(4)
                a = amp_a * k ** -4
                b = amp_b * k ** -3
                g, dg, _ = _g_cr(m, lam, zp)
                dgz = dg / lz
                sz = np.sin(m * math.pi * (zp + 0.5))
                al, be = 2 * math.pi * pha, 2 * math.pi * phb
                # phi = a cos(ph + al) g(z), psi = b cos(ph + be) sin(m pi (z'+1/2)):
                # u = -a kx sin(ph + al) g' - b ky sin(ph + be) sz,
                # v = -a ky sin(ph + al) g' + b kx sin(ph + be) sz,
                # w = a (kx^2 + ky^2) cos(ph + al) g;
                # sin(ph + t) = sin(ph) cos t + cos(ph) sin t
                for comp, ca, cb in ((0, -a * kx, -b * ky), (1, -a * ky, b * kx)):
                    P[comp, 0] += ca * math.sin(al) * dgz + cb * math.sin(be) * sz
                    P[comp, 1] += ca * math.cos(al) * dgz + cb * math.cos(be) * sz
                aw = a * (kx * kx + ky * ky)
                P[2, 0] += aw * math.cos(al) * g
                P[2, 1] -= aw * math.sin(al) * g
            ph = (kx * X + ky * Y).ravel()
            prof.append(P)
            harm.append((np.cos(ph), np.sin(ph)))
    v = np.zeros((3, nz, ny * nx))
    if prof:
        Hc = np.stack([h[0] for h in harm])          # (modes, ny nx)
        Hs = np.stack([h[1] for h in harm])
        Pr = np.stack(prof)                          # (modes, 3, 2, nz)
        for comp in range(3):
            v[comp] = Pr[:, comp, 0].T @ Hc + Pr[:, comp, 1].T @ Hs
    v = v.reshape(3, nz, ny, nx)
    cur = math.sqrt(float(np.mean(v ** 2)) * 3.0)
    return v * (rms / cur) if cur > 0 else v


def wall_vanishing_noise(nx, ny, nz, lx, ly, lz, kmax, mmax, rms, seed):
    """Scalar band-limited field sum a T(x,y) sin(m pi z / Lz), |p|,|q| <= kmax,
    1 <= m <= mmax, zero at both walls, scaled to the requested rms."""
    r = rng(seed)
    x, y, z = grid(nx, ny, nz, lx, ly, lz)
    X, Y = np.meshgrid(x, y, indexing="xy")
    th = np.zeros((nz, ny, nx))
    modes = _mode_list(kmax)
    phs = [2 * np.pi * p / lx * X + 2 * np.pi * q / ly * Y for (p, q) in modes]
    harm = [(np.cos(ph), np.sin(ph)) for ph in phs]
    for m in range(1, mmax + 1):
        Zm = np.sin(m * np.pi * z / lz)
        P = np.zeros((ny, nx))
        for cs, sn in harm:
            a, b = r.standard_normal(2)
            P += a * cs + b * sn
        P += r.standard_normal()  # horizontally uniform part
        th += Zm[:, None, None] * P[None]
    cur = math.sqrt(float(np.mean(th ** 2)))
    return th * (rms / cur) if cur > 0 else th


def laminar_profile(z, forcing, nu, lz):
    """Plane Poiseuille profile for a body force +forcing x (Sec. 6)."""
    return forcing * z * (lz - z) / (2.0 * nu)


def reichardt_profile(z, lz, nu, u_tau=1.0):
    """Reichardt composite log-law in wall units, symmetric about the centre,
    with eta = z (Lz - z) / Lz as the wall distance."""
    eta = z * (lz - z) / lz
    zp = eta * u_tau / nu
    up = (1.0 / 0.41) * np.log1p(0.41 * zp) + 7.8 * (
        1.0 - np.exp(-zp / 11.0) - (zp / 11.0) * np.exp(-zp / 3.0))
    return u_tau * up


def white_field(shape, seed, scale=1.0):
    return scale * rng(seed).standard_normal(shape)


def smooth_field(nx, ny, nz, lx, ly, lz, seed, kmax=3, zpow=3):
    """Smooth non-periodic-in-z real field (random trig in x, y times a random
    polynomial in z), for single-operation parity tests."""
    r = rng(seed)
    x, y, z = grid(nx, ny, nz, lx, ly, lz)
    X, Y = np.meshgrid(x, y, indexing="xy")
    out = np.zeros((nz, ny, nx))
    zz = z / lz
    for (p, q) in _mode_list(kmax) + [(0, 0)]:
        ph = 2 * np.pi * p / lx * X + 2 * np.pi * q / ly * Y
        a, b = r.standard_normal(2)
        poly = sum(r.standard_normal() * zz ** k for k in range(zpow + 1))
        out += poly[:, None, None] * (a * np.cos(ph) + b * np.sin(ph))[None]
    return out


# ----------------------------------------------------------------------------
# workload definitions
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    nu: float
    d: int
    C: int
    dt: float
    steps: int
    seed: int
    forcing_x: float = 0.0
    boussinesq: bool = False
    kappa: float = 0.0
    gamma: float = 0.0
    kind: str = "channel"
    extra: dict = field(default_factory=dict)

    @property
    def nfields(self):
        return 4 if self.boussinesq else 3

    @property
    def points(self):
        return self.nx * self.ny * self.nz

    def problem_kwargs(self):
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, lx=self.lx, ly=self.ly,
                    lz=self.lz, nu=self.nu, d=self.d, C=self.C,
                    forcing_x=self.forcing_x, boussinesq=self.boussinesq,
                    kappa=self.kappa, gamma=self.gamma)

    def initial_state(self):
        """(v [3][nz][ny][nx], theta [nz][ny][nx] or None), float64."""
        x, y, z = grid(self.nx, self.ny, self.nz, self.lx, self.ly, self.lz)
        if self.kind == "channel":
            prof = self.extra.get("profile", "laminar")
            if prof == "laminar":
                U = laminar_profile(z, self.forcing_x, self.nu, self.lz)
            else:
                U = reichardt_profile(z, self.lz, self.nu)
            ubulk = float(np.mean(U))
            rms = self.extra.get("noise_rms", 1e-3)
            if self.extra.get("noise_rel_bulk"):
                rms = rms * ubulk
            if self.extra.get("perturbation") == "curl_eigen":
                v = curl_eigen_noise(self.nx, self.ny, self.nz, self.lx, self.ly, self.lz, rms,
                                     self.seed)
            else:
                v = solenoidal_noise(self.nx, self.ny, self.nz, self.lx, self.ly, self.lz,
                                     self.extra.get("kmax", 4), self.extra.get("mmax", 4),
                                     rms, self.seed)
            v[0] += U[:, None, None]
            return v, None
        rms = self.extra.get("noise_rms", 1e-3)
        if self.extra.get("perturbation") == "curl_eigen":
            # App. A velocity noise beside the temperature noise (seed + 1)
            v = curl_eigen_noise(self.nx, self.ny, self.nz, self.lx, self.ly, self.lz, rms,
                                 self.seed + 1)
        else:
            v = np.zeros((3, self.nz, self.ny, self.nx))
        th = wall_vanishing_noise(self.nx, self.ny, self.nz, self.lx, self.ly, self.lz,
                                  self.extra.get("kmax", 8), self.extra.get("mmax", 8),
                                  rms, self.seed)
        return v, th


def channel(nx, ny, nz, re, d=5, C=25, dt=1e-3, steps=10, seed=1, name=None,
            noise_rms=1e-3, kmax=4, mmax=4, perturbation="solenoidal"):
    """Laminar-scaled channel: u_max = 1, Re = Lz u_bulk / nu (Sec. 6).
    perturbation: "solenoidal" (curl of a random vector potential with a wall
    envelope) or "curl_eigen" (the App. A noise)."""
    lz = 2.0
    nu = lz * (2.0 / 3.0) / re
    G = 8.0 * nu / lz ** 2
    return Workload(name or f"channel_{nx}x{ny}x{nz}", nx, ny, nz, 4 * np.pi, 2 * np.pi,
                    lz, nu, d, C, dt, steps, seed, forcing_x=G, kind="channel",
                    extra=dict(profile="laminar", noise_rms=noise_rms, kmax=kmax, mmax=mmax,
                               perturbation=perturbation))


def rayleigh_benard(nx, ny, nz, ra, pr=1.0, d=5, C=31, dt=1e-3, steps=50, seed=3,
                    name=None, noise_rms=1e-3, kmax=8, mmax=8, perturbation="none"):
    """Boussinesq box 2 x 2 x 1 with gamma = 1 (Sec. 7, Ra = gamma^2 h^4/(nu kappa)).
    perturbation: "none" (v = 0, temperature noise only) or "curl_eigen" (also
    the App. A velocity noise, same rms)."""
    nu = math.sqrt(pr / ra)
    kappa = nu / pr
    return Workload(name or f"rb_{nx}x{ny}x{nz}", nx, ny, nz, 2.0, 2.0, 1.0, nu, d, C,
                    dt, steps, seed, boussinesq=True, kappa=kappa, gamma=1.0, kind="rb",
                    extra=dict(noise_rms=noise_rms, kmax=kmax, mmax=mmax,
                               perturbation=perturbation))


WORKLOADS = {
    "channel_32x32x33": channel(32, 32, 33, 1000.0, d=5, C=25, dt=1e-3, steps=10, seed=1),
    "channel_256x256x257": Workload(
        "channel_256x256x257", 256, 256, 257, 4 * np.pi, 2 * np.pi, 2.0, 1.0 / 180.0,
        5, 25, 2e-4, 100, 2, forcing_x=1.0, kind="channel",
        extra=dict(profile="reichardt", noise_rms=0.1, noise_rel_bulk=True,
                   kmax=8, mmax=4)),
    "rb_512x512x257": rayleigh_benard(512, 512, 257, 1e8, d=5, C=31, dt=1e-3,
                                      steps=50, seed=3),
}


def get(name, **overrides):
    return replace(WORKLOADS[name], **overrides)


# ----------------------------------------------------------------------------
# serving stream
# ----------------------------------------------------------------------------
SERVING_SIDES = (32, 64, 96, 128, 192)


def stable_dt(w: Workload, cap=1e-3):
    """dt = min(cap, 1/(nu_max k2_max)), k2_max = sum (pi/Delta_i)^2."""
    dx, dy, dz = w.lx / w.nx, w.ly / w.ny, w.lz / (w.nz - 1)
    k2 = (np.pi / dx) ** 2 + (np.pi / dy) ** 2 + (np.pi / dz) ** 2
    numax = max(w.nu, w.kappa)
    return min(cap, 1.0 / (numax * k2))


def serving_stream(n=64, rate=20.0, steps=20, seed=5, sides=SERVING_SIDES, C=31):
    """List of (arrival_time_s, Workload) for the serving workload: Poisson
    arrivals, channel or Rayleigh-Benard with equal odds, side uniform over
    `sides` (nz = side + 1, so N' = side + 32 with C = 31), Re uniform in
    [500, 5000] or Ra log-uniform in [1e4, 1e8].  Every request starts from
    the App. A solenoidal no-slip noise (the paper's initial perturbation),
    plus temperature noise (|k| <= 4) for Rayleigh-Benard."""
    r = rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(r.exponential(1.0 / rate))
        side = int(sides[int(r.integers(len(sides)))])
        if r.random() < 0.5:
            re = float(r.uniform(500.0, 5000.0))
            w = channel(side, side, side + 1, re, d=5, C=C, steps=steps, seed=500 + i,
                        name=f"req{i}_channel_{side}", perturbation="curl_eigen")
        else:
            ra = float(10 ** r.uniform(4.0, 8.0))
            w = rayleigh_benard(side, side, side + 1, ra, d=5, C=C, steps=steps,
                                seed=500 + i, name=f"req{i}_rb_{side}", kmax=4, mmax=4,
                                perturbation="curl_eigen")
        w = replace(w, dt=stable_dt(w))
        out.append((t, w))
    return out
