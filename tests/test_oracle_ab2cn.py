"""Pins of the AB2CN + AB2-sponge oracle (Sec. II-E, Eq. 4) against
closed forms that do not come from the oracle itself:

* Crank-Nicolson on the linear terms: a single Fourier mode (no nonlinear
  term) evolves by the textbook CN factor of the ODE it obeys, and with
  viscosity off its phase advance matches the Rossby-wave dispersion
  relation omega = -beta kx / |k|^2 to second order with |amplification| = 1;
* Adams-Bashforth 2 on advection by the inflow, on the Brinkman term with a
  constant mask and on the sponge with a constant profile: the linear
  recurrences of AB2 (forward-Euler first step) written out by hand;
* global order in time: 2 without the sponge (AB2CN), 1 with it (the
  Lie-Trotter splitting), measured on a nonlinear flow with a closure and an
  island.
"""
import math

import numpy as np
import pytest

from oracle import ab2cn
from oracle import qg

TWO_PI = 2.0 * math.pi


def model(nx=16, ny=16, **kw):
    chi = kw.pop("chi", None)
    chi_s = kw.pop("chi_s", None)
    p = qg.Params(nx=nx, ny=ny, lx=TWO_PI, ly=TWO_PI, **kw)
    return qg.Model(p, chi, chi_s)


def single_mode(m, mx, my, amp=0.3, phase=0.4):
    x = np.arange(m.p.nx) * m.p.lx / m.p.nx
    y = np.arange(m.p.ny) * m.p.ly / m.p.ny
    X, Y = np.meshgrid(x, y)
    return amp * np.cos(mx * X + my * Y + phase)


def mode_value(wh, m, mx, my):
    return wh[my % m.p.ny, mx]


def evolve(m, w0, n):
    wh = qg.enter(w0, m.g)
    hist = None
    out = [wh.copy()]
    for _ in range(n):
        wh, hist = ab2cn.step_spectral(wh, hist, m)
        out.append(wh.copy())
    return out


def only_mode(wh, m, mx, my, tol=1e-13):
    rest = wh.copy()
    rest[my % m.p.ny, mx] = 0.0
    assert np.max(np.abs(rest)) <= tol * max(1.0, np.max(np.abs(wh)))


@pytest.mark.parametrize("re,mu,beta", [(50.0, 0.3, 2.0), (math.inf, 0.0, 3.0), (20.0, 0.0, 0.0)])
def test_crank_nicolson_single_mode(re, mu, beta):
    """d w/dt = lambda w with lambda = -(|k|^2/Re + mu) + i beta kx/|k|^2 for
    one mode (J = 0: psi and omega are parallel); CN: w1 = w0 (1 + lambda dt/2)/(1 - lambda dt/2)."""
    m = model(re=re, mu=mu, beta=beta, dt=0.02)
    mx, my = 2, -1
    kx, ky = float(mx), float(my)
    k2 = kx * kx + ky * ky
    nu = 0.0 if math.isinf(re) else 1.0 / re
    lam = -(nu * k2 + mu) + 1j * beta * kx / k2
    r = (1 + 0.5 * m.p.dt * lam) / (1 - 0.5 * m.p.dt * lam)
    hs = evolve(m, single_mode(m, mx, my), 12)
    w0 = mode_value(hs[0], m, mx, my)
    for n, wh in enumerate(hs):
        only_mode(wh, m, mx, my)
        assert abs(mode_value(wh, m, mx, my) - w0 * r ** n) <= 1e-13 * abs(w0)


def test_rossby_phase_and_modulus():
    """Inviscid beta plane: a plane wave exp(i(k.x - Omega t)) with
    Omega = -beta kx/|k|^2 (Rossby dispersion); CN keeps |w| exactly and
    advances the phase by 2 atan(theta/2), theta = -Omega dt."""
    m = model(beta=4.0, dt=0.05)
    mx, my = 3, 2
    k2 = mx * mx + my * my
    omega_r = -m.p.beta * mx / k2
    hs = evolve(m, single_mode(m, mx, my), 20)
    w0 = mode_value(hs[0], m, mx, my)
    theta = -omega_r * m.p.dt
    for n, wh in enumerate(hs):
        z = mode_value(wh, m, mx, my) / w0
        assert abs(abs(z) - 1.0) < 1e-13
        assert abs(np.angle(z * np.exp(-1j * n * 2 * math.atan(theta / 2)))) < 1e-12
    # second order: per-step phase error against the exact wave is O(dt^3)
    assert abs(2 * math.atan(theta / 2) - theta) < theta ** 3 / 10


def ab2_sequence(w0, a, n):
    """w^{k+1} = w^k + dt (3/2 f^k - 1/2 f^{k-1}) with f = a w (dt folded into a),
    first step forward Euler."""
    seq = [w0, w0 * (1 + a)]
    for _ in range(n - 1):
        seq.append(seq[-1] + 1.5 * a * seq[-1] - 0.5 * a * seq[-2])
    return seq


def test_ab2_advection_by_the_inflow():
    """One mode advected by the uniform inflow: J = U omega_x (the mode's own
    velocity does not advect it), so f = -i U kx w."""
    m = model(u_in=0.7, dt=0.03)
    mx, my = 2, 1
    hs = evolve(m, single_mode(m, mx, my), 10)
    w0 = mode_value(hs[0], m, mx, my)
    ref = ab2_sequence(w0, -1j * m.p.u_in * mx * m.p.dt, 10)
    for wh, r in zip(hs, ref):
        only_mode(wh, m, mx, my)
        assert abs(mode_value(wh, m, mx, my) - r) <= 1e-13 * abs(w0)


def test_ab2_brinkman_constant_mask():
    """chi = c0 everywhere: curl(c0 u) = c0 omega, so the penalization is
    f = -(dt/eta) c0 w under AB2."""
    c0 = 0.7
    m = model(eta=0.2, dt=0.01, chi=np.full((16, 16), c0))
    mx, my = 1, 3
    hs = evolve(m, single_mode(m, mx, my), 10)
    w0 = mode_value(hs[0], m, mx, my)
    ref = ab2_sequence(w0, -m.p.dt / m.p.eta * c0, 10)
    for wh, r in zip(hs, ref):
        only_mode(wh, m, mx, my)
        assert abs(mode_value(wh, m, mx, my) - r) <= 1e-13 * abs(w0)


def test_ab2_sponge_constant_profile():
    """chi_s = 1 everywhere and nothing else: omega* = omega^t each step, so
    omega^{t+1} = omega^t - dt sigma (3/2 omega^t - 1/2 omega^{t-1}), first
    step omega** = omega*."""
    m = model(sponge_sigma=4.0, dt=0.02, chi_s=np.ones((16, 16)))
    mx, my = 2, 2
    hs = evolve(m, single_mode(m, mx, my), 10)
    w0 = mode_value(hs[0], m, mx, my)
    ref = ab2_sequence(w0, -m.p.dt * m.p.sponge_sigma, 10)
    for wh, r in zip(hs, ref):
        only_mode(wh, m, mx, my)
        assert abs(mode_value(wh, m, mx, my) - r) <= 1e-13 * abs(w0)


def convergence_errors(sponge):
    from paper_2508_06678_amd import inputs
    nx = ny = 32
    chi = inputs.island_mask(nx, ny, TWO_PI, TWO_PI, 3.0, 3.0, 0.8)
    chi_s = inputs.sponge_mask(nx, ny, TWO_PI, TWO_PI) if sponge else None
    w0 = inputs.bandpass_noise(nx, ny, TWO_PI, TWO_PI, 7, 1.0, 4.0, 0.5)
    T = 0.08
    sols = []
    for n in (16, 32, 64, 1024):
        m = model(nx, ny, dt=T / n, beta=1.0, re=200.0, u_in=0.5, eta=0.1, closure="smag", c=0.17,
                  chi=chi, chi_s=chi_s, sponge_sigma=3.0 if sponge else 0.0)
        sols.append(ab2cn.run(w0, m, n)[0])
    ref = sols[-1]
    return [float(np.linalg.norm(s - ref)) for s in sols[:-1]]


def test_second_order_without_sponge():
    e = convergence_errors(False)
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 3.2 < r1 < 5.0 and 3.2 < r2 < 5.0, e


def test_first_order_with_sponge_splitting():
    """The splitting error is first order: the ratios fall toward 2."""
    e = convergence_errors(True)
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 1.7 < r2 < 2.7 and r2 <= r1 + 0.05, e
