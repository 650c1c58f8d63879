"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module holds none of the time step's arithmetic: it only builds the
fields a run starts from -- land masks, sponge ramps and initial vorticity --
as float64 NumPy arrays of shape (ny, nx), x contiguous.  Both sides receive
the same arrays (FP32 runs use them rounded to nearest).

Geometry follows the paper's set-ups (Sec. IV-A, IV-B): a circular island
and a coast with a Gaussian cape, each a smoothed 0/1 mask chi_obs (Eq. 2),
and a sponge ramp chi_sponge that is 1 on the boundary and falls linearly to
0 over the sponge thickness (Eq. 3).  The smoothing profile is a tanh of
width eps (two grid cells by default) instead of the paper's Gaussian
filter, as the benchmark configurations specify.
"""
import numpy as np


def grid_xy(nx, ny, lx, ly):
    x = np.arange(nx) * (lx / nx)
    y = np.arange(ny) * (ly / ny)
    return np.meshgrid(x, y)  # X, Y with shape (ny, nx)


def island_mask(nx, ny, lx, ly, xc, yc, radius, eps=None):
    """chi = (1 - tanh((r - R)/eps)) / 2, r = distance to (xc, yc)."""
    if eps is None:
        eps = 2.0 * lx / nx
    X, Y = grid_xy(nx, ny, lx, ly)
    r = np.hypot(X - xc, Y - yc)
    return 0.5 * (1.0 - np.tanh((r - radius) / eps))


def cape_mask(nx, ny, lx, ly, coast=0.2, height=0.6, width=0.3, xc=None, eps=None):
    """Southern coast at y = coast plus a Gaussian cape of the given height and
    width centred at xc; land is the strip -coast <= y' <= y_c(x) in the
    periodic coordinate y' in [-ly/2, ly/2), built from two tanh edges (its
    periodic image is a northern coast at y = ly - coast)."""
    if eps is None:
        eps = 2.0 * lx / nx
    if xc is None:
        xc = 0.5 * lx
    X, Y = grid_xy(nx, ny, lx, ly)
    yp = np.where(Y < 0.5 * ly, Y, Y - ly)
    yc = coast + height * np.exp(-((X - xc) / width) ** 2)
    upper = 0.5 * (1.0 - np.tanh((yp - yc) / eps))
    lower = 0.5 * (1.0 + np.tanh((yp + coast) / eps))
    return upper * lower


def sponge_mask(nx, ny, lx, ly, thickness=None, sides="x", thickness_y=None):
    """chi_s = max(0, 1 - d/d_s), d = distance to the x ends (x = 0 == lx),
    or (sides="xy") to the nearest of the four box edges, with thickness_y
    (default: thickness) along the y edges."""
    if thickness is None:
        thickness = lx / 16.0
    X, Y = grid_xy(nx, ny, lx, ly)
    ramp = np.maximum(0.0, 1.0 - np.minimum(X, lx - X) / thickness)
    if sides == "xy":
        ty = thickness if thickness_y is None else thickness_y
        ramp = np.maximum(ramp, 1.0 - np.minimum(Y, ly - Y) / ty)
    elif sides != "x":
        raise ValueError("sides must be 'x' or 'xy'")
    return ramp


def gaussian_cape_mask(nx, ny, lx, ly, xc, height, length, eps=None):
    """Land below y = height exp(-((x - xc)/length)^2), measured from the
    southern edge: chi = (1 - tanh((y - h(x))/eps))/2 (1 + tanh((y - 2 eps)/eps))/2
    for y in [0, ly), the second factor lifting the land off the periodic
    seam at y = 0 (eps: two grid cells by default)."""
    if eps is None:
        eps = 2.0 * lx / nx
    X, Y = grid_xy(nx, ny, lx, ly)
    h = height * np.exp(-((X - xc) / length) ** 2)
    return 0.25 * (1.0 - np.tanh((Y - h) / eps)) * (1.0 + np.tanh((Y - 2.0 * eps) / eps))


def _wavenumbers(nx, ny, lx, ly):
    kx = 2.0 * np.pi * np.fft.rfftfreq(nx, d=1.0 / nx) / lx
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=1.0 / ny) / ly
    return np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)


def _rms_scaled(f, rms):
    f = f - f.mean()
    s = np.sqrt(np.mean(f * f))
    return f * (rms / s) if s > 0 else f


def bandpass_noise(nx, ny, lx, ly, seed, kmin=2.0, kmax=8.0, rms=0.1):
    """N(0,1) noise from default_rng(seed), band-passed to kmin <= |k| <= kmax
    (physical wavenumber, inclusive) and scaled to the given rms."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((ny, nx))
    zh = np.fft.rfft2(z)
    k = _wavenumbers(nx, ny, lx, ly)
    zh[(k < kmin - 1e-9) | (k > kmax + 1e-9)] = 0.0
    return _rms_scaled(np.fft.irfft2(zh, s=(ny, nx)), rms)


def spectrum_noise(nx, ny, lx, ly, seed, kmin=4.0, rms=0.1):
    """Random-phase vorticity whose energy spectrum falls as k^-3 beyond kmin:
    |omega_hat| ~ 1/|k| on kmin <= |k| and 3|m| < n per axis, phases from the
    FFT of white noise from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((ny, nx))
    zh = np.fft.rfft2(z)
    k = _wavenumbers(nx, ny, lx, ly)
    mx = np.arange(nx // 2 + 1)[None, :]
    j = np.arange(ny)
    my = np.where(j < ny // 2, j, j - ny)[:, None]
    keep = (k >= kmin - 1e-9) & (3 * mx < nx) & (3 * np.abs(my) < ny)
    mag = np.abs(zh)
    ph = np.where(mag > 0, zh / np.where(mag > 0, mag, 1.0), 0.0)
    spec = np.where(keep, ph / np.where(k > 0, k, 1.0), 0.0)
    return _rms_scaled(np.fft.irfft2(spec, s=(ny, nx)), rms)


def smooth_directions(nx, ny, lx, ly, count, seed, kmax=32.0):
    """Random perturbation fields of the resolved scales (1 <= |k| <= kmax)
    with unit rms per grid point, for finite-difference checks."""
    return [bandpass_noise(nx, ny, lx, ly, seed * 1000 + i, 1.0, kmax, 1.0) for i in range(count)]


def random_directions(shape, count, seed):
    """Unit-norm random directions for finite-difference checks."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        d = rng.standard_normal(shape)
        out.append(d / np.linalg.norm(d))
    return out
