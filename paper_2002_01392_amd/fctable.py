"""FC-Gram tables for the solver: Gram basis Q_r and blend-to-zero extensions
A_r (App. B), computed once in high precision and stored as text.

Construction (App. B; grid spacing 1, first right matching point at t = 0):
* Gram basis: the monomials 1, t, ..., t^{d-1} on t = 0..d-1 orthonormalised
  for the discrete inner product (g, h) = sum_i g(t_i) h(t_i) by modified
  Gram-Schmidt (with one re-orthogonalisation sweep), positive leading
  coefficients.  Column j of Q_r holds Gram polynomial j at the d points.
* Blend to zero: for each Gram polynomial, the least-squares trigonometric
  polynomial of period 2(C + d) with n_os (d - 1) + 1 samples on [0, d-1]
  (matching the polynomial) and as many on [C + d, C + 2d - 1] (matching 0),
  solved by Householder QR in 60 digits.  Column j of A_r holds its values at
  t = d..d+C-1, the continuation points.
* Oversampling n_os = 20; bandwidth K (cosine/sine pairs) per (d, C) from
  ``BANDWIDTH``: the smallest K whose fit residual is <= 1e-16.

The solver's C ABI takes [Q_r | A_r] (row-major, float64) and forms
M_r = A_r Q_r^T itself.  Run ``python -m paper_2002_01392_amd.fctable`` to
(re)write the stored tables.
"""
from __future__ import annotations

import os

import mpmath as mp
import numpy as np

TABLE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tables")
N_OS = 20
DIGITS = 60
BANDWIDTH = {(5, 15): 23, (5, 25): 20, (5, 31): 19, (7, 33): 23}
STANDARD = [(5, 25), (5, 31), (5, 15), (7, 33)]


def _gram_values(d):
    """d x d matrix of Gram polynomial values and their monomial coefficients."""
    t = [mp.mpf(i) for i in range(d)]
    basis_vals = []   # values of each orthonormal polynomial at the points
    basis_coef = []   # coefficients in the monomial basis
    for k in range(d):
        vals = [ti ** k for ti in t]
        coef = [mp.mpf(0)] * d
        coef[k] = mp.mpf(1)
        for _ in range(2):  # Gram-Schmidt and one re-orthogonalisation
            for qv, qc in zip(basis_vals, basis_coef):
                proj = mp.fsum(a * b for a, b in zip(vals, qv))
                vals = [a - proj * b for a, b in zip(vals, qv)]
                coef = [a - proj * b for a, b in zip(coef, qc)]
        nrm = mp.sqrt(mp.fsum(a * a for a in vals))
        basis_vals.append([a / nrm for a in vals])
        basis_coef.append([a / nrm for a in coef])
    return basis_vals, basis_coef


def _trig_basis(t, K, period):
    row = [mp.mpf(1)]
    for k in range(1, K + 1):
        ang = 2 * mp.pi * k * t / period
        row.append(mp.cos(ang))
        row.append(mp.sin(ang))
    return row


def compute(d, C, K=None, n_os=N_OS):
    """Return (Q_r, A_r) as float64 arrays of shapes (d, d) and (C, d)."""
    if K is None:
        K = BANDWIDTH[(d, C)]
    with mp.workdps(DIGITS):
        period = 2 * (C + d)
        vals, coefs = _gram_values(d)
        npts = n_os * (d - 1) + 1
        left = [mp.mpf(d - 1) * i / (npts - 1) for i in range(npts)]
        right = [mp.mpf(C + d) + x for x in left]
        Amat = mp.matrix([_trig_basis(x, K, period) for x in left + right])
        Q = np.zeros((d, d))
        A = np.zeros((C, d))
        for j in range(d):
            Q[:, j] = [float(v) for v in vals[j]]
            poly = lambda x: mp.fsum(c * x ** k for k, c in enumerate(coefs[j]))  # noqa: E731
            rhs = mp.matrix([poly(x) for x in left] + [mp.mpf(0)] * npts)
            x, _ = mp.qr_solve(Amat, rhs)
            for i in range(C):
                row = _trig_basis(mp.mpf(d + i), K, period)
                A[i, j] = float(mp.fsum(r * x[m] for m, r in enumerate(row)))
        return Q, A


def path(d, C):
    return os.path.join(TABLE_DIR, f"fc_d{d}_C{C}.txt")


def write(d, C):
    Q, A = compute(d, C)
    os.makedirs(TABLE_DIR, exist_ok=True)
    with open(path(d, C), "w") as fh:
        fh.write(f"# FC-Gram table d={d} C={C} K={BANDWIDTH[(d, C)]} n_os={N_OS}: "
                 f"Q_r ({d}x{d}) then A_r ({C}x{d}), row-major\n")
        for v in np.concatenate([Q.ravel(), A.ravel()]):
            fh.write(f"{v:.17e}\n")


def load(d, C):
    """[Q_r | A_r] flattened (float64), generating the table if not stored."""
    p = path(d, C)
    if not os.path.exists(p):
        write(d, C)
    v = np.loadtxt(p, comments="#", dtype=np.float64)
    if v.size != d * d + C * d:
        raise ValueError(f"bad table {p}")
    return v


if __name__ == "__main__":
    for dc in STANDARD:
        write(*dc)
        print("wrote", path(*dc))
