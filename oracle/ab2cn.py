"""Oracle: the paper's own time scheme (Sec. II-E, Eq. 4) -- a semi-implicit
Adams-Bashforth / Crank-Nicolson (AB2CN) step for the penalized QG equations,
then the sponge by second-order Adams-Bashforth, as a Lie-Trotter splitting.

TEST INFRASTRUCTURE ONLY (see the package header).  FP64 throughout.

Eq. 4, in the notation of ``qg``:
  omega* = omega^t + dt/2 [ (1/Re) lap(omega* + omega^t) - mu (omega* + omega^t)
                            - beta d/dx (psi* + psi^t) ]
           - dt [ 3/2 J^t - 1/2 J^{t-1} ]
           - curl( (dt/eta) chi (3/2 u^t - 1/2 u^{t-1}) )
  omega^{t+1} = omega* - dt sigma chi_s (3/2 omega* - 1/2 omega**)
with omega** the intermediate field omega* of the previous step and
sigma = 1/eta_sponge.

Readings (where the paper is silent):
  * the linear terms are diagonal in Fourier space: with
    L = -(|k|^2/Re + mu) + i beta kx / |k|^2 (psi_hat = -omega_hat/|k|^2),
    the Crank-Nicolson part is omega_hat* (1 - dt/2 L) = omega_hat^t (1 + dt/2 L) + ...;
  * the eddy-viscosity term Pi of an LES closure (static or dynamic, its
    coefficient at omega^t) is a nonlinear term and goes into the
    Adams-Bashforth part beside J;
  * u is the total velocity (the inflow gauge included), as in the curl of
    the Brinkman term of Eq. 2; chi u is formed by collocation in physical
    space, its curl taken spectrally and truncated to D, like every
    nonlinear term (Sec. II-C);
  * first step (no history): the t-1 terms equal the t terms (forward Euler
    on the explicit parts) and omega** = omega*;
  * omega^{t+1} is projected onto D with its mean removed, as every state.
"""
import numpy as np

from . import qg


def explicit_terms(wh, m):
    """Adams-Bashforth operands at omega_hat: N = -J_hat + C Q_hat (nonlinear
    terms, on D) and the total velocity (u, v) in physical space."""
    out = {}
    qg.rhs(wh, m, out)
    N = -out["Jh"]
    if out["Qh"] is not None:
        N = N + out["C"] * out["Qh"]
    return N, out["u"], out["v"]


def penalty_curl(u, v, m):
    """D curl(chi (u, v)) in spectral space: i kx FFT(chi v) - i ky FFT(chi u)."""
    g = m.g
    ph = g.D * (1j * g.kx * g.spec(m.chi * v) - 1j * g.ky * g.spec(m.chi * u))
    ph[0, 0] = 0.0
    return ph


def linear_symbol(m):
    """L(k) of the Crank-Nicolson part (zero at k = 0)."""
    g, p = m.g, m.p
    L = -(g.k2 * m.inv_re + p.mu) + 1j * p.beta * g.kx * g.inv_k2
    L[0, 0] = 0.0
    return L


def step_spectral(wh, hist, m):
    """One AB2CN + AB2-sponge step.  hist: None (first step) or the dict this
    function returned for the previous step.  Returns (omega_hat^{t+1}, hist)."""
    g, p = m.g, m.p
    dt = p.dt
    N, u, v = explicit_terms(wh, m)
    if hist is None:
        Nm, um, vm = N, u, v
    else:
        Nm, um, vm = hist["N"], hist["u"], hist["v"]
    L = linear_symbol(m)
    rhs = wh * (1.0 + 0.5 * dt * L) + dt * (1.5 * N - 0.5 * Nm)
    if not np.isinf(p.eta):
        rhs = rhs - (dt / p.eta) * penalty_curl(1.5 * u - 0.5 * um, 1.5 * v - 0.5 * vm, m)
    ws_h = rhs / (1.0 - 0.5 * dt * L)
    ws_h[0, 0] = 0.0
    ws = g.phys(ws_h)
    wss = ws if hist is None else g.phys(hist["wstar"])
    a = dt * p.sponge_sigma
    w1 = ws - a * m.chi_s * (1.5 * ws - 0.5 * wss)
    out = g.D * g.spec(w1)
    out[0, 0] = 0.0
    return out, dict(N=N, u=u, v=v, wstar=ws_h)


def run(w, m, nsteps, hist=None):
    """nsteps steps from physical omega; returns (physical omega, hist)."""
    wh = qg.enter(w, m.g)
    for _ in range(nsteps):
        wh, hist = step_spectral(wh, hist, m)
    return qg.leave(wh, m.g), hist
