"""FC-Gram continuation and transforms along the walled direction (Sec. 3).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Conventions
-----------
* A line holds the Nz values f_0..f_{Nz-1} at z_s = s*dz, dz = Lz/(Nz-1)
  (both walls included; Sec. 3 and App. B).
* The continued line has N' = Nz + C points and period Lz' = N' dz (Sec. 3,
  eq. k with N_z + C points in z).
* Continuation (Sec. 3, eq. fc:continuation; App. B, block form of A f): the C
  appended values are M_r f_r + M_l f_l, with f_r the last d values and f_l the
  first d values of the line, M_r = A_r Q_r^T, and M_l = J M_r J (J the
  reversal), the left-end table being the mirror image of the right-end one
  (the row- and column-reversals written in Sec. 3).
* F_z = FFT_{N'} o E (unnormalized), B_z = R o IFFT_{N'} (with 1/N'), R keeps
  the first Nz entries (Sec. 3: the FC-Gram transform and its inverse).
* Wavenumbers in z: k = 2 pi lbar / Lz' in FFT order (eq. k, relabelled);
  odd derivatives zero the Nyquist mode, even ones keep it.
"""
from __future__ import annotations

import numpy as np

from . import fft as dft
from .fc_table import fc_tables


class FCGram:
    """FC-Gram operator for lines of Nz points along axis 0."""

    def __init__(self, nz, d, C, lz=1.0):
        if nz < 2 * d:
            raise ValueError("need nz >= 2d")
        self.nz, self.d, self.C = nz, d, C
        self.np_ = nz + C
        self.dz = lz / (nz - 1)
        self.lzp = self.np_ * self.dz
        _, _, Mr, _ = fc_tables(d, C)
        self.Mr = Mr
        self.Ml = Mr[::-1, ::-1].copy()           # J M_r J
        n = self.np_
        lbar = dft.signed_index(n)                # signed integer index
        self.kz = 2.0 * np.pi * lbar / self.lzp    # true wavenumbers
        self.kz_odd = self.kz.copy()
        if n % 2 == 0:
            self.kz_odd[n // 2] = 0.0              # Nyquist zeroed for odd derivatives
        self.lbar = lbar

    # -- continuation --------------------------------------------------------
    def extend(self, f):
        """E: (Nz, ...) -> (N', ...); the first Nz values are copied."""
        d, nz = self.d, self.nz
        tail = np.tensordot(self.Mr, f[nz - d:], axes=(1, 0)) + \
            np.tensordot(self.Ml, f[:d], axes=(1, 0))
        return np.concatenate([f, tail], axis=0)

    def fwd(self, f):
        """F_z = FFT o E along axis 0 (unnormalized)."""
        return dft.fft(self.extend(f), 0)

    def back(self, fh):
        """B_z = R o IFFT along axis 0."""
        return dft.ifft(fh, 0)[: self.nz]

    def kz_shape(self, ndim, odd=True):
        k = self.kz_odd if odd else self.kz
        return k.reshape((-1,) + (1,) * (ndim - 1))

    def derivative(self, f, order=1):
        """FC spectral derivative of real lines (Sec. 3; Sec. 4.2 'multiplying
        Fourier coefficients by their wavenumber and the imaginary unit').

        order 1 multiplies by i*k~ (Nyquist zeroed), order 2 by -k^2.
        """
        fh = self.fwd(np.asarray(f, dtype=np.float64))
        if order == 1:
            fh = fh * (1j * self.kz_shape(fh.ndim, odd=True))
        elif order == 2:
            fh = fh * (-(self.kz_shape(fh.ndim, odd=False) ** 2))
        else:
            raise ValueError("order must be 1 or 2")
        return self.back(fh).real


def fc_extend_lines(f_lines, d, C):
    """fc_extend over a (nlines, Nz) array: returns (nlines, Nz + C)."""
    f = np.asarray(f_lines, dtype=np.float64)
    op = FCGram(f.shape[1], d, C)
    return op.extend(f.T).T


def fc_derivative_lines(f_lines, d, C, lz, order=1):
    """fc_derivative over a (nlines, Nz) array of real lines."""
    f = np.asarray(f_lines, dtype=np.float64)
    op = FCGram(f.shape[1], d, C, lz)
    return op.derivative(f.T, order).T
