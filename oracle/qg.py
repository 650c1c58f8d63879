"""Oracle: one pseudo-spectral time step of the beta-plane QG vorticity
equation with eddy-viscosity closures, Brinkman penalization and sponge.

TEST INFRASTRUCTURE ONLY (see the package header).  FP64 throughout.

Notation (paper, Sec. II):
  omega  vorticity, psi streamfunction with omega = lap(psi)        (Eq. 1)
  (u, v) = (-psi_y, psi_x), plus the uniform inflow (U, V) added to the
         zeroth Fourier mode of the velocity as a gauge            (Sec. II-D)
  J(psi, omega) = psi_x omega_y - psi_y omega_x = u omega_x + v omega_y
  d omega/dt + J = (1/Re) lap omega - mu omega - beta psi_x + F      (Eq. 1)
  F_obs   = -curl((1/eta) chi (u - 0))                               (Eq. 2)
  F_sponge = -(1/eta_s) chi_s (omega - omega_s), sigma = 1/eta_s     (Eq. 3)
  Pi = div(nu_e grad omega)                                          (Eq. 8)
  Smagorinsky nu_e = (c Delta)^2 |S|, |S| = sqrt(4 psi_xy^2 + (psi_xx - psi_yy)^2)
                                                                      (Eq. 9)
  Leith       nu_e = (c Delta)^3 |grad omega|                        (Eq. 12)
  dynamic     (c Delta)^p = <H M> / <M^2>, H = J(psi~, omega~) - J(psi, omega)~,
              M = r div(base~ grad omega~) - div(base grad omega)~,
              r = (Delta~/Delta)^p, p = 2 (Smag) or 3 (Leith)  (Eqs. 10-11, 13)

Readings taken where the paper is silent or at odds with the configuration
this oracle serves (each is a parameter, so the other reading stays
selectable where it matters):
  * time scheme: classical RK4 on everything except penalization and sponge;
    those are integrated exactly in a Lie-Trotter sub-step after RK4
    (obstacle first, then sponge, Sec. II-E ordering);
  * B sub-step: exact solution of du/dt = -chi u / eta (u including the
    inflow) is u <- E u with E = exp(-dt chi / eta); its curl by the product
    rule gives omega' = E omega + E_x v - E_y u; then omega'' = S omega' with
    S = exp(-dt sigma chi_s) (omega_s = 0);
  * 2/3 rule: keep 3|m_x| < nx and 3|m_y| < ny (set D), applied to every
    product and to the B output, so the state stays in D; omega_hat(0,0) = 0;
  * test filter T: radial sharp cutoff |k| <= k_max / test_ratio with k_max
    the largest retained wavenumber min over axes; evaluated as an exact
    integer inequality (requires dx = dy);
  * Delta = lx / nx; averages <.> are plain means over the whole grid;
  * clipping: coefficient level C = max(<HM>, 0)/<M^2> (clip_mode 0); the
    pointwise reading (clip_mode 1) clips H at every grid point,
    C = <max(H, 0) M>/<M^2>, with no further clip of the ratio;
  * the dynamic coefficient is recomputed at every RK stage.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from . import fft as F

CLOSURES = ("none", "smag", "leith", "dsmag", "dleith")


@dataclass
class Params:
    """Physical and numerical parameters of one run (Sec. II, Eqs. 1-4, 9-13)."""
    nx: int
    ny: int
    lx: float
    ly: float
    dt: float
    beta: float = 0.0
    re: float = math.inf          # Re; inf disables molecular viscosity
    mu: float = 0.0               # bottom friction
    u_in: float = 0.0             # inflow gauge U (Sec. II-D)
    v_in: float = 0.0
    eta: float = math.inf         # porosity; inf disables the obstacle
    sponge_sigma: float = 0.0     # 1/eta_sponge
    c: float = 0.0                # static c_S or c_L
    closure: str = "none"         # none | smag | leith | dsmag | dleith | const
    test_ratio: int = 2           # Delta~ / Delta
    clip_mode: int = 0            # 0: C = max(<HM>,0)/<M^2>; 1: pointwise H+


class Grid:
    """Wavenumbers, the dealiasing set D, the test set T and Parseval weights
    for an nx-by-ny doubly periodic grid (Sec. II-C)."""

    def __init__(self, nx, ny, lx, ly, test_ratio=2):
        for n in (nx, ny):
            if n < 4 or (n & (n - 1)):
                raise ValueError("grid sizes must be powers of two >= 4")
        self.nx, self.ny, self.lx, self.ly = nx, ny, float(lx), float(ly)
        self.dx, self.dy = lx / nx, ly / ny
        if abs(self.dx - self.dy) > 1e-12 * self.dx:
            raise ValueError("the closures assume dx == dy")
        self.delta = self.dx
        self.N = nx * ny
        mx = np.arange(nx // 2 + 1)
        j = np.arange(ny)
        my = np.where(j < ny // 2, j, j - ny)
        self.mx = mx[None, :]
        self.my = my[:, None]
        self.kx = 2.0 * np.pi * self.mx / lx
        self.ky = 2.0 * np.pi * self.my / ly
        self.k2 = self.kx ** 2 + self.ky ** 2
        self.inv_k2 = np.zeros_like(self.k2)
        nz = self.k2 > 0
        self.inv_k2[nz] = 1.0 / self.k2[nz]
        amx, amy = np.abs(self.mx), np.abs(self.my)
        self.D = ((3 * amx < nx) & (3 * amy < ny)).astype(np.float64)
        Mx, My = (nx - 1) // 3, (ny - 1) // 3
        lim = min(Mx * ny, My * nx) ** 2
        r = int(test_ratio)
        lhs = r * r * (ny * ny * amx.astype(np.int64) ** 2 + nx * nx * amy.astype(np.int64) ** 2)
        self.T = (lhs <= lim).astype(np.float64)
        w = np.full(nx // 2 + 1, 2.0)
        w[0] = 1.0
        w[nx // 2] = 1.0
        self.w = w[None, :]

    # spectral <-> physical -------------------------------------------------
    def phys(self, fh):
        return F.irfft2(fh, self.nx)

    def spec(self, f):
        return F.rfft2(f)

    def mean_product(self, ah, bh):
        """Grid mean of a*b from half spectra (Parseval): (1/N^2) sum w Re(a conj b)."""
        return float(np.sum(self.w * (ah * np.conj(bh)).real)) / self.N ** 2


class Model:
    """Grid + parameters + the once-per-run tables of the B sub-step (row a0)."""

    def __init__(self, p: Params, chi=None, chi_s=None):
        self.p = p
        self.g = Grid(p.nx, p.ny, p.lx, p.ly, p.test_ratio)
        g = self.g
        shape = (p.ny, p.nx)
        self.chi = np.zeros(shape) if chi is None else np.asarray(chi, np.float64)
        self.chi_s = np.zeros(shape) if chi_s is None else np.asarray(chi_s, np.float64)
        self.inv_re = 0.0 if math.isinf(p.re) else 1.0 / p.re
        a = 0.0 if math.isinf(p.eta) else p.dt / p.eta
        chx, chy = mask_gradient(self.chi, g)
        self.E = np.exp(-a * self.chi)
        self.Ex = -a * chx * self.E
        self.Ey = -a * chy * self.E
        self.S = np.exp(-p.dt * p.sponge_sigma * self.chi_s)

    def static_coefficient(self):
        """C = (c Delta)^2 for Smagorinsky (Eq. 9), (c Delta)^3 for Leith (Eq. 12)."""
        p, d = self.p, self.g.delta
        if p.closure == "smag":
            return (p.c * d) ** 2
        if p.closure == "leith":
            return (p.c * d) ** 3
        if p.closure == "const":
            return p.c
        return 0.0


def mask_gradient(chi, g):
    """Spectral gradient of a mask with both Nyquist lines removed (Sec. II-C:
    derivatives in Fourier space).  Returns (chi_x, chi_y) on the grid."""
    ch = F.rfft2(chi)
    ch[:, g.nx // 2] = 0.0
    ch[g.ny // 2, :] = 0.0
    return g.phys(1j * g.kx * ch), g.phys(1j * g.ky * ch)


def enter(w, g):
    """Physical vorticity -> state: D * FFT(omega), mean mode removed (Sec. II-C;
    the mean of omega vanishes on a periodic domain)."""
    wh = g.D * F.rfft2(w)
    wh[0, 0] = 0.0
    return wh


def leave(wh, g):
    return F.irfft2(wh, g.nx)


# -------------------------------------------------------------------------
# right-hand side of the A sub-step (Eq. 1 without F_obs, F_sponge, plus Pi)
# -------------------------------------------------------------------------
def velocity(psih, m):
    """u = U - psi_y, v = V + psi_x (Eq. 1 and the inflow gauge, Sec. II-D)."""
    g, p = m.g, m.p
    u = p.u_in + g.phys(-1j * g.ky * psih)
    v = p.v_in + g.phys(1j * g.kx * psih)
    return u, v


def closure_base(kind, psih, wx, wy, m):
    """|S| (Eq. 9) for Smagorinsky kinds, |grad omega| (Eq. 12) for Leith kinds,
    1 for the constant-viscosity test hook."""
    g = m.g
    if kind in ("smag", "dsmag"):
        pd = g.phys((g.ky ** 2 - g.kx ** 2) * psih)   # psi_xx - psi_yy
        pxy = g.phys(-g.kx * g.ky * psih)             # psi_xy
        return np.sqrt(4.0 * pxy ** 2 + pd ** 2)
    if kind in ("leith", "dleith"):
        return np.sqrt(wx ** 2 + wy ** 2)
    if kind == "const":
        return np.ones_like(wx)
    raise ValueError(kind)


def rhs(wh, m, out=None):
    """R(omega_hat): spectral right-hand side of the A sub-step.

    R = -D FFT(u omega_x + v omega_y) + C D (i kx FFT(h_x) + i ky FFT(h_y))
        - (|k|^2/Re + mu) omega_hat - beta i kx psi_hat,  R(0,0) = 0,
    with h = base * grad(omega) and C the static or dynamic coefficient.
    If ``out`` is a dict, the intermediates are stored in it.
    """
    g, p = m.g, m.p
    psih = -wh * g.inv_k2                                   # omega = lap psi
    u, v = velocity(psih, m)
    wx = g.phys(1j * g.kx * wh)
    wy = g.phys(1j * g.ky * wh)
    J = u * wx + v * wy
    Jh = g.D * g.spec(J)
    R = -Jh - (g.k2 * m.inv_re + p.mu) * wh - p.beta * 1j * g.kx * psih
    C, base, Qh = 0.0, None, None
    if p.closure != "none":
        base = closure_base(p.closure, psih, wx, wy, m)
        hxh = g.spec(base * wx)
        hyh = g.spec(base * wy)
        Qh = g.D * (1j * g.kx * hxh + 1j * g.ky * hyh)      # D div(base grad omega)
        if p.closure in ("dsmag", "dleith"):
            C = dynamic_coefficient(wh, psih, Jh, Qh, m, out)
        else:
            C = m.static_coefficient()
        R = R + C * Qh
    R[0, 0] = 0.0
    if out is not None:
        out.update(psih=psih, u=u, v=v, wx=wx, wy=wy, J=J, Jh=Jh, base=base,
                   Qh=Qh, C=C)
    return R


def dynamic_coefficient(wh, psih, Jh, Qh, m, out=None):
    """Germano identity with Lilly's least squares (Eqs. 10-11 and 13).

    Test-level fields carry the inflow too, so the mean flow cancels in H.
      H_hat = D FFT(J(psi~, omega~)) - T J_hat
      M_hat = r D div(base~ grad omega~)^ - T Q_hat,  r = test_ratio^p
      C = max(<HM>, 0) / <M^2>  (clip_mode 0),  C = 0 if <M^2> = 0.
    """
    g, p = m.g, m.p
    wt = g.T * wh
    pt = g.T * psih
    ut, vt = velocity(pt, m)
    wtx = g.phys(1j * g.kx * wt)
    wty = g.phys(1j * g.ky * wt)
    Jt = ut * wtx + vt * wty
    kind = p.closure
    base_t = closure_base(kind, pt, wtx, wty, m)
    gxh = g.spec(base_t * wtx)
    gyh = g.spec(base_t * wty)
    power = 2 if kind == "dsmag" else 3
    r = float(p.test_ratio) ** power
    Hh = g.D * g.spec(Jt) - g.T * Jh
    Mh = r * g.D * (1j * g.kx * gxh + 1j * g.ky * gyh) - g.T * Qh
    H = g.phys(Hh)
    M = g.phys(Mh)
    MM = float(np.mean(M * M))
    if p.clip_mode == 1:
        HM = float(np.mean(np.maximum(H, 0.0) * M))
        C = HM / MM if MM > 0.0 else 0.0
    else:
        HM = float(np.mean(H * M))
        C = max(HM, 0.0) / MM if MM > 0.0 else 0.0
    if out is not None:
        out.update(Hh=Hh, Mh=Mh, HM=HM, MM=MM, HM_parseval=g.mean_product(Hh, Mh),
                   MM_parseval=g.mean_product(Mh, Mh))
    return C


# -------------------------------------------------------------------------
# time step (Sec. II-E, with the readings listed in the module header)
# -------------------------------------------------------------------------
def rk4(wh, m):
    """Classical RK4 over the A sub-step: omega* = omega + dt/6 (k1+2k2+2k3+k4)."""
    dt = m.p.dt
    k1 = rhs(wh, m)
    k2 = rhs(wh + 0.5 * dt * k1, m)
    k3 = rhs(wh + 0.5 * dt * k2, m)
    k4 = rhs(wh + dt * k3, m)
    return wh + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def b_substep(wh, m):
    """Lie-Trotter B sub-step: exact Brinkman decay of the total velocity in
    curl form, then the sponge relaxation, evaluated pointwise in physical
    space and projected back onto D (Eqs. 2-4)."""
    g = m.g
    psih = -wh * g.inv_k2
    u, v = velocity(psih, m)
    w = g.phys(wh)
    w1 = m.E * w + m.Ex * v - m.Ey * u
    w2 = m.S * w1
    out = g.D * g.spec(w2)
    out[0, 0] = 0.0
    return out


def step_spectral(wh, m):
    return b_substep(rk4(wh, m), m)


def step(w, m):
    """One full step, physical omega_n -> physical omega_{n+1}."""
    return leave(step_spectral(enter(w, m.g), m), m.g)


def run(w, m, nsteps):
    wh = enter(w, m.g)
    for _ in range(nsteps):
        wh = step_spectral(wh, m)
    return leave(wh, m.g)


# -------------------------------------------------------------------------
# diagnostics (row a10)
# -------------------------------------------------------------------------
def diag(w, m):
    """[energy, enstrophy, C, nu_min, nu_mean, nu_max, CFL, nonfinite] at omega.

    energy = 1/2 <|grad psi|^2> (perturbation velocity, inflow excluded),
    enstrophy = 1/2 <omega^2>, both by Parseval on the projected state;
    nu_e = C * base; CFL = max (|u| + |v|) dt / Delta with the total velocity.
    """
    g, p = m.g, m.p
    w = np.asarray(w, np.float64)
    nonfinite = 0.0 if np.all(np.isfinite(w)) else 1.0
    wh = enter(w, g)
    psih = -wh * g.inv_k2
    energy = 0.5 * g.mean_product(np.sqrt(g.k2) * psih, np.sqrt(g.k2) * psih)
    enstrophy = 0.5 * g.mean_product(wh, wh)
    out = {}
    rhs(wh, m, out)
    C = out["C"]
    if out["base"] is None:
        nu = np.zeros((g.ny, g.nx))
    else:
        nu = C * out["base"]
    cfl = float(np.max(np.abs(out["u"]) + np.abs(out["v"]))) * p.dt / g.delta
    vals = [energy, enstrophy, C, float(nu.min()), float(nu.mean()), float(nu.max()),
            cfl, nonfinite]
    return np.array(vals), nu
