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
Ideal SGS forcing Pi_FF (the filtered QG equations of Sec. III): the
commutators of the filter with advection, the Brinkman forcing and the
sponge forcing, evaluated from an FR field; the closure's own Pi at the
filtered field (Pi_FR, the a-priori model term of Sec. IV).
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


# ---------------------------------------------------------------------------
# ideal subgrid-scale forcing (Sec. III, the filtered equations and Pi)
# ---------------------------------------------------------------------------
def advective_forcing(wh, m):
    """G(omega) = D FFT(J) + (1/eta) D curl(chi u) + sigma D FFT(chi_s omega):
    the advection and the two forcings of the QG equation with the signs of
    its left-hand side, in spectral space on grid m (u the total velocity,
    J = u omega_x + v omega_y, products collocated and de-aliased)."""
    g, p = m.g, m.p
    psih = -wh * g.inv_k2
    u = p.u_in + g.phys(-1j * g.ky * psih)
    v = p.v_in + g.phys(1j * g.kx * psih)
    J = u * g.phys(1j * g.kx * wh) + v * g.phys(1j * g.ky * wh)
    G = g.D * g.spec(J)
    if not np.isinf(p.eta):
        G = G + (1.0 / p.eta) * g.D * (1j * g.kx * g.spec(m.chi * v) - 1j * g.ky * g.spec(m.chi * u))
    if p.sponge_sigma:
        G = G + p.sponge_sigma * g.D * g.spec(m.chi_s * g.phys(wh))
    G[0, 0] = 0.0
    return G


def spectral_to_coarse(Gh, g_fr, nx_c, ny_c, delta):
    """H_full on a half spectrum of the FR grid -> half spectrum of the coarse
    grid (same scaling convention as filter_to)."""
    H = gaussian_cutoff(g_fr.nx, g_fr.ny, g_fr.lx, g_fr.ly, delta)
    wh = Gh * H
    ch = np.zeros((ny_c, nx_c // 2 + 1), dtype=complex)
    for jc in range(ny_c):
        my = jc if jc < ny_c // 2 else jc - ny_c
        ch[jc, :] = wh[my % g_fr.ny, : nx_c // 2 + 1]
    ch[:, nx_c // 2] = 0.0
    ch[ny_c // 2, :] = 0.0
    return ch / (delta * delta)


def ideal_sgs(w_fr, m_fr, m_les):
    """Pi_FF on the LES grid (Sec. III, the ideal SGS forcing):
    J(psi_bar, omega_bar) - bar(J(psi, omega)) + bar(F_obs(chi, u))
    - F_obs(chi_bar, u_bar) + bar(F_sponge(chi_s, omega))
    - F_sponge(chi_s_bar, omega_bar) = G_les(omega_bar) - bar(G_fr(omega)).
    Reading: the LES carries only its 2/3 set D, so omega_bar enters the
    LES-grid terms projected onto D and Pi is projected onto D -- the
    forcing that makes the LES tendency on D equal the filtered FR tendency
    (the linear terms commute with the filter).  The LES model's masks must
    be H_full(chi), H_full(chi_s) for the paper's definition.
    Returns (Pi_FF, omega_bar on D), physical on the LES grid."""
    from . import qg
    gf, gl = m_fr.g, m_les.g
    delta = gf.nx // gl.nx
    wh = qg.enter(w_fr, gf)
    Gbar = spectral_to_coarse(advective_forcing(wh, m_fr), gf, gl.nx, gl.ny, delta)
    wbar_d = gl.D * spectral_to_coarse(wh, gf, gl.nx, gl.ny, delta)
    wbar_d[0, 0] = 0.0
    Pi = gl.D * (advective_forcing(wbar_d, m_les) - Gbar)
    Pi[0, 0] = 0.0
    return gl.phys(Pi), gl.phys(wbar_d)


def model_sgs(w_les, m_les):
    """The closure's Pi = C D div(base grad omega) at omega (LES grid, its
    2/3 set), physical."""
    from . import qg
    out = {}
    qg.rhs(qg.enter(w_les, m_les.g), m_les, out)
    if out["Qh"] is None:
        return np.zeros((m_les.g.ny, m_les.g.nx))
    return m_les.g.phys(out["C"] * out["Qh"])
