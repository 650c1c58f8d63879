"""The oracle's own FFT (test infrastructure only; see the package header).

The paper evaluates all derivatives in Fourier space and the nonlinear terms
by collocation (Sec. II-C), so every quantity of the step is built from 2-D
discrete Fourier transforms on a doubly periodic grid.  This module provides
them without any FFT library:

* ``fft`` / ``ifft`` along the last axis: radix-2 Stockham (self-sorting,
  decimation in time).  The forward transform is unnormalised,
  X[m] = sum_n x[n] exp(-2 pi i m n / N); the inverse carries the 1/N.
* ``rfft2``: real (ny, nx) field -> half spectrum (ny, nx//2 + 1),
  m_x in [0, nx/2], m_y in FFT order.
* ``irfft2``: half spectrum -> real field, defined as
  f(x) = (1/N) sum_{half} w_m Re(F_m exp(i k.x)),  w = 1 at m_x in {0, nx/2},
  2 otherwise, N = nx*ny.  This is the inverse of ``rfft2`` on Hermitian
  spectra and a well-defined real-linear map on any half spectrum.

Parity: pinned against brute-force O(N^2) DFT sums, Parseval, the shift
theorem and a numpy.fft cross-check in ``tests/test_oracle_fft.py``.
"""
import numpy as np


def _check_pow2(n):
    if n < 1 or (n & (n - 1)) != 0:
        raise ValueError(f"length {n} is not a power of two")


def _stockham(x, sign):
    """DFT along the last axis with exp(sign * 2 pi i m n / N), no scaling.

    Self-sorting radix-2 decimation in time.  Invariant before a pass with
    sub-length L: A[..., k, s] (shape (..., L, N/L)) is the length-L DFT at
    frequency k of the subsequence x[s], x[s + N/L], x[s + 2N/L], ...
    One pass merges the subsequences s and s + N/(2L) (even and odd samples
    of the length-2L subsequence):
        A2[k]     = A[k, s] + w^k A[k, s + N/(2L)]
        A2[k + L] = A[k, s] - w^k A[k, s + N/(2L)],   w = exp(sign 2 pi i / 2L)
    Starting from L = 1 (A = x) and ending at L = N (A[:, 0] = DFT).
    """
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    _check_pow2(n)
    a = x.reshape(x.shape[:-1] + (1, n))
    L = 1
    while L < n:
        h = n // (2 * L)
        even = a[..., :, :h]
        odd = a[..., :, h:]
        k = np.arange(L)
        ang = sign * 2.0 * np.pi * k / (2 * L)
        w = (np.cos(ang) + 1j * np.sin(ang))[:, None]
        t = w * odd
        a = np.concatenate([even + t, even - t], axis=-2)
        L *= 2
    return a[..., :, 0]


def fft(x, axis=-1):
    """Unnormalised forward DFT along ``axis``."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    return np.moveaxis(_stockham(x, -1.0), -1, axis)


def ifft(x, axis=-1):
    """Inverse DFT along ``axis`` with the 1/N factor."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    n = x.shape[-1]
    return np.moveaxis(_stockham(x, +1.0) / n, -1, axis)


def rfft2(f):
    """Real (..., ny, nx) -> half spectrum (..., ny, nx//2 + 1), unnormalised."""
    f = np.asarray(f, dtype=np.float64)
    nx = f.shape[-1]
    rows = fft(f.astype(np.complex128), axis=-1)[..., : nx // 2 + 1]
    return fft(rows, axis=-2)


def irfft2(F, nx):
    """Half spectrum (..., ny, nx//2 + 1) -> real (..., ny, nx).

    f(x) = (1/N) sum_half w Re(F exp(i k.x)); the columns m_x = 0 and
    m_x = nx/2 contribute their real parts only (weight 1), every other
    column contributes twice its real part (itself and its conjugate image).
    """
    F = np.asarray(F, dtype=np.complex128)
    half = nx // 2 + 1
    if F.shape[-1] != half:
        raise ValueError("half-spectrum width does not match nx")
    cols = ifft(F, axis=-2)  # inverse along y, 1/ny included
    full = np.zeros(F.shape[:-1] + (nx,), dtype=np.complex128)
    full[..., 0] = cols[..., 0].real
    full[..., nx // 2] = cols[..., nx // 2].real
    full[..., 1 : nx // 2] = cols[..., 1 : nx // 2]
    full[..., nx // 2 + 1 :] = np.conj(cols[..., 1 : nx // 2][..., ::-1])
    return ifft(full, axis=-1).real
