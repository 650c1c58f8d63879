"""Pins for the oracle's own FFT (Sec. II-C: all derivatives are taken in
Fourier space, so the transforms are the foundation of every other pin).

Each case is checked against something other than the FFT itself: the
O(N^2) definition of the DFT summed term by term, Parseval's identity, the
shift theorem, and (as a test-only cross-check) numpy.fft.
"""
import numpy as np
import pytest

from oracle import fft as F


def brute_dft(x, sign=-1.0):
    n = x.shape[-1]
    j = np.arange(n)
    M = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
    return x @ M.T


def brute_half_spectrum(f):
    ny, nx = f.shape
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros((ny, nx // 2 + 1), complex)
    for my in range(ny):
        for mx in range(nx // 2 + 1):
            out[my, mx] = np.sum(f * np.exp(-2j * np.pi * (mx * x / nx + my * y / ny)))
    return out


def brute_c2r(Fh, nx):
    ny = Fh.shape[0]
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros((ny, nx))
    for my in range(ny):
        for mx in range(nx // 2 + 1):
            w = 1.0 if mx in (0, nx // 2) else 2.0
            out += w * (Fh[my, mx] * np.exp(2j * np.pi * (mx * x / nx + my * y / ny))).real
    return out / (nx * ny)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64])
def test_1d_against_definition(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    ref = brute_dft(x)
    got = F.fft(x)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
    back = F.ifft(got)
    assert np.max(np.abs(back - x)) <= 1e-14 * n


@pytest.mark.parametrize("ny,nx", [(8, 8), (16, 8), (8, 16), (4, 4)])
def test_rfft2_against_definition(ny, nx):
    f = np.random.default_rng(ny * 100 + nx).standard_normal((ny, nx))
    ref = brute_half_spectrum(f)
    got = F.rfft2(f)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref)) * 10


@pytest.mark.parametrize("ny,nx", [(8, 8), (16, 8), (8, 16), (4, 4)])
def test_irfft2_against_definition(ny, nx):
    rng = np.random.default_rng(7 + ny + nx)
    Fh = rng.standard_normal((ny, nx // 2 + 1)) + 1j * rng.standard_normal((ny, nx // 2 + 1))
    ref = brute_c2r(Fh, nx)
    got = F.irfft2(Fh, nx)
    assert np.max(np.abs(got - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref))) * 10


@pytest.mark.parametrize("ny,nx", [(64, 128), (32, 32), (256, 64)])
def test_round_trip_parseval_shift(ny, nx):
    rng = np.random.default_rng(3)
    f = rng.standard_normal((ny, nx))
    Fh = F.rfft2(f)
    assert np.max(np.abs(F.irfft2(Fh, nx) - f)) < 1e-14 * 50
    w = np.full(nx // 2 + 1, 2.0)
    w[0] = w[-1] = 1.0
    lhs = np.sum(f * f)
    rhs = np.sum(w * np.abs(Fh) ** 2) / (nx * ny)
    assert abs(lhs - rhs) <= 1e-13 * lhs
    sx, sy = 5, 3
    g = np.roll(np.roll(f, sx, axis=1), sy, axis=0)
    mx = np.arange(nx // 2 + 1)[None, :]
    my = np.arange(ny)[:, None]
    phase = np.exp(-2j * np.pi * (mx * sx / nx + my * sy / ny))
    assert np.max(np.abs(F.rfft2(g) - Fh * phase)) <= 1e-12 * np.max(np.abs(Fh))


@pytest.mark.parametrize("ny,nx", [(64, 128), (512, 256), (128, 1024)])
def test_numpy_cross_check(ny, nx):
    f = np.random.default_rng(11).standard_normal((ny, nx))
    ref = np.fft.rfft2(f)
    got = F.rfft2(f)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.max(np.abs(F.irfft2(ref, nx) - np.fft.irfft2(ref, s=(ny, nx)))) <= 1e-15 * 100


def test_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        F.fft(np.zeros(12))
