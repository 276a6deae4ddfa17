"""Discrete Fourier transforms of the oracle, written out (no FFT library).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Every transform of the method (the FFTs along the periodic directions and
along the continued wall-normal lines, Sec. 3 and 4.2) is the discrete
Fourier transform

    X_k = sum_{j<N} x_j exp(-2 pi i j k / N),   k = 0..N-1   (unnormalized),

with the inverse x_j = (1/N) sum_k X_k exp(+2 pi i j k / N).

``dft`` evaluates the definition as one matrix product (O(N^2)); ``fft``
evaluates the same sums by the Cooley-Tukey splitting N = r m
(decimation in time): with Y_b the m-point transform of the subsequence
x_{r a + b}, a < m,

    X_{k1 + m k2} = sum_{b<r} exp(-2 pi i b k2 / r) [exp(-2 pi i b k1 / N) Y_b(k1)],

applied recursively with r the largest divisor of N up to 16; lengths up to
16 and prime lengths are evaluated by the definition.  The inverse uses the
same sums with exp(+2 pi i jk/N) and the factor 1/N.  Real transforms
are the complex ones restricted (``rfft`` keeps k <= N/2) or completed by
Hermitian symmetry (``irfft``).
"""
from __future__ import annotations

import functools

import numpy as np


def signed_index(n):
    """The integer frequency of FFT slot k: k for k < n/2 (rounded up), else
    k - n (so the Nyquist slot of an even n is -n/2)."""
    k = np.arange(n, dtype=np.float64)
    return np.where(k < (n + 1) // 2, k, k - n)


@functools.lru_cache(maxsize=None)
def _dft_matrix(n, sign=-1):
    """F[k, j] = exp(sign 2 pi i (j k mod n) / n); the reduced exponent keeps
    the argument of the exponential small."""
    jk = np.outer(np.arange(n), np.arange(n)) % n
    return np.exp(sign * 2j * np.pi * jk / n)


@functools.lru_cache(maxsize=None)
def _twiddle(n, r, sign=-1):
    """exp(sign 2 pi i q k1 / n) for k1 < n/r (rows) and q < r (columns)."""
    m = n // r
    qk = np.outer(np.arange(m), np.arange(r))
    return np.exp(sign * 2j * np.pi * qk / n)


def _radix(n):
    """The split factor r of a length n > 16: its largest divisor r <= 16
    (r < n); n itself where n <= 16 or n is prime (evaluated directly)."""
    if n <= 16:
        return n
    for r in range(16, 1, -1):
        if n % r == 0:
            return r
    return n


def _fft_rows(x, sign=-1):
    """Unnormalized transform (kernel exp(sign 2 pi i jk/N)) along axis 0 of
    a 2-D complex array (N, B)."""
    n = x.shape[0]
    r = _radix(n)
    if r == n:                          # short or prime length: the definition
        return _dft_matrix(n, sign) @ x
    m = n // r
    b = x.shape[1]
    # row a of x.reshape(m, r B) holds x_{r a + q} for q < r side by side, so
    # one call transforms the r decimated subsequences: ys[k1, q] = Y_q(k1)
    ys = _fft_rows(x.reshape(m, r * b), sign).reshape(m, r, b)
    ys *= _twiddle(n, r, sign)[:, :, None]
    # r-point transform over q: out[k1, k2] = X_{k1 + m k2}
    out = np.matmul(_dft_matrix(r, sign), ys)
    return np.ascontiguousarray(out.transpose(1, 0, 2)).reshape(n, b)


def _along(x, axis, fn):
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, 0)
    shape = x.shape
    y = fn(np.ascontiguousarray(x.reshape(shape[0], -1)))
    return np.moveaxis(y.reshape((y.shape[0],) + shape[1:]), 0, axis)


def dft(x, axis=0):
    """Unnormalized forward DFT by its definition (one matrix product)."""
    return _along(x, axis, lambda a: _dft_matrix(a.shape[0]) @ a)


def fft(x, axis=0):
    """Unnormalized forward DFT along ``axis`` (Cooley-Tukey, see above)."""
    return _along(x, axis, _fft_rows)


def ifft(x, axis=0):
    """Inverse DFT with the 1/N factor."""
    n = np.shape(x)[axis]
    y = _along(x, axis, lambda a: _fft_rows(a, +1))
    y /= n
    return y


def rfft(x, axis=-1):
    """Forward DFT of real data, slots k = 0..N/2."""
    n = np.shape(x)[axis]
    X = fft(np.asarray(x, dtype=np.float64), axis)
    return np.take(X, np.arange(n // 2 + 1), axis=axis)


def irfft(X, n, axis=-1):
    """Real inverse of the slots k = 0..n/2 of a Hermitian spectrum (n even):
    the missing slots are X_{n-k} = conj(X_k); the imaginary parts of the
    k = 0 and k = n/2 slots do not contribute to a real result."""
    X = np.moveaxis(np.asarray(X, dtype=np.complex128), axis, 0)
    h = n // 2
    full = np.empty((n,) + X.shape[1:], dtype=np.complex128)
    full[: h + 1] = X[: h + 1]
    full[h + 1:] = np.conj(X[1:n - h][::-1])
    return np.moveaxis(ifft(full, 0).real, 0, axis)
