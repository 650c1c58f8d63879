"""Pins of the LES filter H_full and of the PCC (oracle/les.py):

* the spectral Gaussian equals a brute-force periodic convolution in
  physical space with the Gaussian kernel of variance (delta Delta)^2 / 3
  per axis (the kernel whose transform is exp(-k^2 (delta Delta)^2 / 6)),
  sampled on the coarse grid, for a field band-limited below the cut-off;
* the cut-off keeps a mode just inside pi/Delta_FF and removes one just
  outside, and a kept single mode has the Gaussian's amplitude on the
  coarse grid;
* the PCC equals numpy's correlation coefficient and is +-1 for affine
  relations.
"""
import math

import numpy as np
import pytest

from oracle import les

TWO_PI = 2.0 * math.pi


def band_field(n, kmax, seed):
    rng = np.random.default_rng(seed)
    x = np.arange(n) * TWO_PI / n
    X, Y = np.meshgrid(x, x)
    w = np.zeros((n, n))
    for mx in range(-kmax, kmax + 1):
        for my in range(-kmax, kmax + 1):
            if mx * mx + my * my <= kmax * kmax and (mx, my) != (0, 0):
                w += rng.standard_normal() * np.cos(mx * X + my * Y + rng.uniform(0, TWO_PI))
    return w


@pytest.mark.parametrize("delta", [2, 4])
def test_gaussian_equals_physical_convolution(delta):
    n = 32
    dx = TWO_PI / n
    w = band_field(n, 3, 11)
    var = (delta * dx) ** 2 / 3.0
    # periodic kernel: sum of the Gaussian over the images of the torus
    d = np.arange(n) * dx
    d = np.minimum(d, TWO_PI - d)
    g1 = np.zeros(n)
    for img in range(-3, 4):
        g1 += np.exp(-((np.arange(n) * dx + img * TWO_PI) ** 2) / (2 * var))
    g1 /= g1.sum()
    G = np.outer(g1, g1)
    conv = np.zeros_like(w)
    for sy in range(n):
        for sx in range(n):
            conv += G[sy, sx] * np.roll(np.roll(w, sy, axis=0), sx, axis=1)
    coarse = conv[::delta, ::delta]
    got = les.filter_to(w, TWO_PI, TWO_PI, delta)
    assert got.shape == (n // delta, n // delta)
    # the sampled kernel differs from the continuous one by its k-space images,
    # exp(-(2 pi/dx - k)^2 var / 2) relative: below 1e-9 here
    assert np.max(np.abs(got - coarse)) <= 1e-8 * np.max(np.abs(coarse))


def test_cutoff_edges_and_single_mode_amplitude():
    n, delta = 64, 4
    dx = TWO_PI / n
    kc = math.pi / (delta * dx)          # = 8 for this grid
    x = np.arange(n) * dx
    X, Y = np.meshgrid(x, x)
    inside = np.cos(7 * X + 3 * Y)       # |k| = 7.62 < 8
    outside = np.cos(7 * X + 4 * Y)      # |k| = 8.06 > 8
    assert math.hypot(7, 3) < kc < math.hypot(7, 4)
    out = les.filter_to(outside, TWO_PI, TWO_PI, delta)
    assert np.max(np.abs(out)) < 1e-13
    got = les.filter_to(inside, TWO_PI, TWO_PI, delta)
    amp = math.exp(-(49 + 9) * (delta * dx) ** 2 / 6.0)
    xc = x[::delta]
    Xc, Yc = np.meshgrid(xc, xc)
    assert np.max(np.abs(got - amp * np.cos(7 * Xc + 3 * Yc))) < 1e-13


def test_pcc_against_numpy_and_affine():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((16, 16))
    b = 0.3 * a + rng.standard_normal((16, 16))
    assert abs(les.pcc(a, b) - np.corrcoef(a.ravel(), b.ravel())[0, 1]) < 1e-14
    assert abs(les.pcc(a, 2.5 * a - 7.0) - 1.0) < 1e-14
    assert abs(les.pcc(a, -a + 1.0) + 1.0) < 1e-14
    assert abs(les.pcc(a, b) - les.pcc(b, a)) < 1e-15
