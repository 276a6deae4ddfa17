"""FC-Gram continuation tables, computed in high precision (App. B).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

App. B builds the continuation of a line from two ingredients:

1. a Gram basis: the polynomials of degree < d orthonormal for the discrete
   inner product over the d matching points.  Their values at the matching
   points are the columns of Q, obtained from the QR factorization of the
   d x d Vandermonde matrix of the matching points;
2. for every Gram polynomial, a "blend-to-zero" extension: an oversampled
   least-squares trigonometric polynomial whose period is the interval
   [1 - delta_r, 2b - (1 - delta_r)], which matches the polynomial on the
   right matching interval and vanishes on the left matching interval
   translated by one period b of the continued line.  Its values at the C
   continuation points are the columns of A.

The continuation is then A_r Q_r^T f_r + A_l Q_l^T f_l (App. B, the block form
of the continuation operator).

Units.  The grid spacing is 1 and the first right matching point is t = 0, so
the right matching points are t = 0..d-1, the C continuation points are
t = d..d+C-1, the translated left matching points are t = C+d..C+2d-1 and the
period of the auxiliary trigonometric polynomial is P = 2(C+d).

Readings (the paper leaves these to its reference Amlani & Bruno 2016):
* oversampling: n_os = 20 samples per grid interval on each matching interval;
* bandwidth K (number of cosine/sine pairs): the smallest K whose fit residual
  is <= 1e-16 on every oversampled point; the values found for the tables used
  here are listed in ``K_CHOICE`` (the scan in ``choose_k`` reproduces them);
* arithmetic: 100 significant digits (mpmath), rounded to float64 at the end.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

N_OS = 20
DPS = 100
# (d, C) -> K found by ``choose_k`` (smallest bandwidth with residual <= 1e-16).
K_CHOICE = {(5, 15): 23, (5, 25): 20, (5, 31): 19, (7, 33): 23}


def _gram_basis(d):
    """Gram basis on t = 0..d-1: QR of the Vandermonde matrix (App. B).

    Returns (Q, coef): Q[i, j] is Gram polynomial j at t = i, and
    q_j(t) = sum_k coef[k, j] t**k (coef = R^-1, since V = Q R).
    The sign is fixed so that diag(R) > 0.
    """
    V = mp.matrix(d, d)
    for i in range(d):
        for k in range(d):
            V[i, k] = mp.mpf(i) ** k
    Q, R = mp.qr(V)
    for j in range(d):
        if R[j, j] < 0:
            for i in range(d):
                Q[i, j] = -Q[i, j]
            for k in range(d):
                R[j, k] = -R[j, k]
    return Q, R ** -1


def _trig_row(t, K, P):
    row = [mp.mpf(1)]
    for k in range(1, K + 1):
        w = 2 * mp.pi * k * t / P
        row += [mp.cos(w), mp.sin(w)]
    return row


def _blend_fits(d, C, K, n_os=N_OS):
    """Least-squares blend-to-zero fits of every Gram polynomial.

    Returns (coefs, residuals, Q, Rinv) where coefs[j] are the 2K+1
    trigonometric coefficients (constant, then cos/sin pairs) of T_j.
    """
    P = 2 * (C + d)
    Q, Rinv = _gram_basis(d)
    npts = n_os * (d - 1) + 1
    t_match = [mp.mpf(d - 1) * i / (npts - 1) for i in range(npts)]
    t_zero = [mp.mpf(C + d) + t for t in t_match]
    rows = t_match + t_zero
    Amat = mp.matrix([_trig_row(t, K, P) for t in rows])
    AtA = Amat.T * Amat
    coefs, residuals = [], []
    for j in range(d):
        qj = lambda t: sum(Rinv[k, j] * t ** k for k in range(d))  # noqa: E731
        rhs = mp.matrix([qj(t) for t in t_match] + [0] * npts)
        # normal equations, solved in DPS digits: (A^T A) x = A^T b
        x = mp.lu_solve(AtA, Amat.T * rhs)
        r = Amat * x - rhs
        coefs.append(x)
        residuals.append(max(abs(r[i]) for i in range(r.rows)))
    return coefs, residuals, Q, Rinv


def choose_k(d, C, tol=1e-16, n_os=N_OS):
    """Smallest bandwidth K whose blend fits reach residual <= tol."""
    with mp.workdps(DPS):
        for K in range(d, 2 * (C + d)):
            _, res, _, _ = _blend_fits(d, C, K, n_os)
            if max(res) <= tol:
                return K
    raise ValueError(f"no bandwidth reaches {tol} for d={d}, C={C}")


@functools.lru_cache(maxsize=None)
def fc_tables(d, C, K=None):
    """Return (Q_r, A_r, M_r, K) as float64 arrays.

    Q_r: d x d, column j = Gram polynomial j at the right matching points.
    A_r: C x d, column j = blend-to-zero extension of Gram polynomial j at
         the C continuation points.
    M_r = A_r Q_r^T (C x d), formed in high precision then rounded.
    The left-end operator is the mirror image M_l = J M_r J (J = reversal),
    see ``oracle.fcgram``.
    """
    if K is None:
        K = K_CHOICE.get((d, C)) or choose_k(d, C)
    P = 2 * (C + d)
    with mp.workdps(DPS):
        coefs, _, Q, _ = _blend_fits(d, C, K)
        A = mp.matrix(C, d)
        for j in range(d):
            for i in range(C):
                row = _trig_row(mp.mpf(d + i), K, P)
                A[i, j] = sum(row[m] * coefs[j][m] for m in range(2 * K + 1))
        M = A * Q.T
        to_np = lambda X: np.array([[float(X[i, j]) for j in range(X.cols)]  # noqa: E731
                                    for i in range(X.rows)], dtype=np.float64)
        return to_np(Q), to_np(A), to_np(M), K


@functools.lru_cache(maxsize=None)
def fit_residuals(d, C, K=None):
    """Max fit residual of each Gram polynomial's blend (for the pins)."""
    if K is None:
        K = K_CHOICE.get((d, C)) or choose_k(d, C)
    with mp.workdps(DPS):
        _, res, _, _ = _blend_fits(d, C, K)
        return [float(r) for r in res]
