"""Oracle: the filtering of fully-resolved (FR) fields onto the LES grid and
the pattern (Pearson) correlation used to compare fields (Sec. III, the
filter H_full and Sec. IV, Eq. for the PCC).

TEST INFRASTRUCTURE ONLY (see the package header).  FP64 throughout.

H_full = interpolate_{Delta_FF} o H_cut-off o H_Gaussian, with
  H_Gaussian(k) = exp(-k^2 (delta Delta_FR)^2 / 6)   (the printed formula
      lacks the square on the filter width; a Gaussian transfer function is
      quadratic in the width -- reading),
  H_cut-off(k) = 0 for |k| > pi / Delta_FF, Delta_FF = delta Delta_FR
      (radial |k|: the paper writes the wavenumber magnitude -- reading),
  interpolation onto the coarse grid of nx/delta x ny/delta points: every
      retained mode lies below the coarse Nyquist wavenumber, so the
      band-limited field is represented exactly by its coarse samples; the
      coarse Nyquist lines are set to zero.
PCC(X, Y) = <(X - <X>)(Y - <Y>)> / sqrt(<(X - <X>)^2> <(Y - <Y>)^2>), <.> the
grid mean.
"""
import numpy as np

from . import fft as F


def gaussian_cutoff(nx, ny, lx, ly, delta):
    """H_Gaussian * H_cut-off on the half spectrum of the FR grid."""
    mx = np.arange(nx // 2 + 1)[None, :]
    j = np.arange(ny)
    my = np.where(j < ny // 2, j, j - ny)[:, None]
    kx = 2.0 * np.pi * mx / lx
    ky = 2.0 * np.pi * my / ly
    k2 = kx ** 2 + ky ** 2
    dfr = lx / nx
    H = np.exp(-k2 * (delta * dfr) ** 2 / 6.0)
    kc = np.pi / (delta * dfr)
    return np.where(k2 <= kc * kc, H, 0.0)


def filter_to(w, lx, ly, delta):
    """H_full(w): physical FR field (ny, nx) -> physical field on the coarse
    grid (ny/delta, nx/delta)."""
    w = np.asarray(w, np.float64)
    ny, nx = w.shape
    if nx % delta or ny % delta:
        raise ValueError("delta must divide the grid")
    ncx, ncy = nx // delta, ny // delta
    wh = F.rfft2(w) * gaussian_cutoff(nx, ny, lx, ly, delta)
    # coarse half spectrum: modes |m_x| <= ncx/2, |m_y| <= ncy/2 of the FR one
    ch = np.zeros((ncy, ncx // 2 + 1), dtype=complex)
    for jc in range(ncy):
        my = jc if jc < ncy // 2 else jc - ncy
        ch[jc, :] = wh[my % ny, : ncx // 2 + 1]
    ch[:, ncx // 2] = 0.0          # coarse Nyquist lines
    ch[ncy // 2, :] = 0.0
    # the FR transform carries a factor nx*ny, the coarse inverse 1/(ncx*ncy)
    return F.irfft2(ch / (delta * delta), ncx)


def pcc(x, y):
    x = np.asarray(x, np.float64).ravel()
    y = np.asarray(y, np.float64).ravel()
    dx = x - x.mean()
    dy = y - y.mean()
    return float(np.mean(dx * dy) / np.sqrt(np.mean(dx * dx) * np.mean(dy * dy)))
