"""Pins of the LES filter H_full and of the PCC (oracle/les.py):

* the spectral Gaussian equals a brute-force periodic convolution in
  physical space with the Gaussian kernel of variance (delta Delta)^2 / 3
  per axis (the kernel whose transform is exp(-k^2 (delta Delta)^2 / 6)),
  sampled on the coarse grid, for a field band-limited below the cut-off;
* the cut-off keeps a mode just inside pi/Delta_FF and removes one just
  outside, and a kept single mode has the Gaussian's amplitude on the
  coarse grid;
* the PCC equals numpy's correlation coefficient and is +-1 for affine
  relations;
* the ideal SGS forcing against hand-derived closed forms: two modes (the
  Jacobian commutator at the sum and difference frequencies), a single
  mode under one-mode masks (the Brinkman and sponge commutators), constant
  masks (no commutator), and a sum frequency that passes the filter but
  lies outside the LES 2/3 set (the projection);
* the closure's model term against the exact enstrophy identity
  sum omega Pi = -C sum base |grad omega|^2, gradients from numpy's FFT.
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


# ---------------------------------------------------------------------------
# ideal SGS term
# ---------------------------------------------------------------------------
def models(n_fr, delta, **kw):
    from oracle import qg
    chi = kw.pop("chi", None)
    chi_s = kw.pop("chi_s", None)
    pf = qg.Params(nx=n_fr, ny=n_fr, lx=TWO_PI, ly=TWO_PI, dt=1e-3, **kw)
    pl = qg.Params(nx=n_fr // delta, ny=n_fr // delta, lx=TWO_PI, ly=TWO_PI, dt=1e-3, **kw)
    cf = None if chi is None else chi(n_fr)
    cl = None if chi is None else les.filter_to(chi(n_fr), TWO_PI, TWO_PI, delta)
    sf = None if chi_s is None else chi_s(n_fr)
    sl = None if chi_s is None else les.filter_to(chi_s(n_fr), TWO_PI, TWO_PI, delta)
    return qg.Model(pf, cf, sf), qg.Model(pl, cl, sl)


def grid_xy(n):
    x = np.arange(n) * TWO_PI / n
    return np.meshgrid(x, x)


def test_ideal_sgs_two_modes_closed_form():
    """omega = a cos(t1) + b cos(t2), t_i = k_i.x, psi_i = -omega_i/|k_i|^2:
    each mode's self-advection vanishes and the cross terms give
    J = -A sin t1 sin t2 = (A/2)(cos(t1 + t2) - cos(t1 - t2)) with
    A = a b (k1 x k2)(1/|k1|^2 - 1/|k2|^2).  Filtering scales mode k by H(k),
    so Pi = J(psi_bar, omega_bar) - bar(J) carries (H(k1) H(k2) - H(k1 +- k2))
    on each of the two frequencies, sampled on the coarse grid."""
    n, delta = 32, 2
    mf, ml = models(n, delta)
    X, Y = grid_xy(n)
    a, b = 0.7, -0.4
    k1, k2 = (2, 1), (1, -3)
    w = a * np.cos(k1[0] * X + k1[1] * Y) + b * np.cos(k2[0] * X + k2[1] * Y)
    Pi, _ = les.ideal_sgs(w, mf, ml)
    # J(psi, omega) = psi_x omega_y - psi_y omega_x, cross terms only:
    # J(psi1, omega2) = -(a b/q1)(k1 x k2) sin t1 sin t2,
    # J(psi2, omega1) = +(a b/q2)(k1 x k2) sin t1 sin t2
    q1, q2 = k1[0] ** 2 + k1[1] ** 2, k2[0] ** 2 + k2[1] ** 2
    cross = k1[0] * k2[1] - k1[1] * k2[0]          # k1 x k2
    amp = a * b * cross * (1.0 / q1 - 1.0 / q2)
    # -A sin t1 sin t2 = (A/2)(cos(t1 + t2) - cos(t1 - t2))
    dfr = TWO_PI / n

    def H(kx, ky):
        k2_ = kx * kx + ky * ky
        kc = math.pi / (delta * dfr)
        return math.exp(-k2_ * (delta * dfr) ** 2 / 6.0) if k2_ <= kc * kc else 0.0

    sp = (k1[0] + k2[0], k1[1] + k2[1])
    sm = (k1[0] - k2[0], k1[1] - k2[1])
    H1H2 = H(*k1) * H(*k2)
    Xc, Yc = grid_xy(n // delta)
    ref = (0.5 * amp * (H1H2 - H(*sp)) * np.cos(sp[0] * Xc + sp[1] * Yc)
           - 0.5 * amp * (H1H2 - H(*sm)) * np.cos(sm[0] * Xc + sm[1] * Yc))
    assert np.max(np.abs(Pi - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(ref)) > 1e-3      # not vacuous


def test_ideal_sgs_commutators_vanish_for_constant_masks():
    """A constant mask and sponge profile pass the filter unchanged, and their
    forcings are linear in omega: both commutators vanish, and a single mode
    has no Jacobian, so Pi = 0."""
    n, delta = 32, 2
    mf, ml = models(n, delta, eta=0.05, sponge_sigma=3.0,
                    chi=lambda m: np.full((m, m), 0.6), chi_s=lambda m: np.full((m, m), 0.3))
    X, Y = grid_xy(n)
    w = 0.5 * np.cos(3 * X - 2 * Y + 0.2)
    Pi, wbar = les.ideal_sgs(w, mf, ml)
    assert np.max(np.abs(wbar)) > 0.1
    assert np.max(np.abs(Pi)) < 1e-12


def H_of(n, delta):
    dfr = TWO_PI / n
    kc2 = (math.pi / (delta * dfr)) ** 2

    def H(m):
        k2 = m[0] * m[0] + m[1] * m[1]
        return math.exp(-k2 * (delta * dfr) ** 2 / 6.0) if k2 <= kc2 else 0.0
    return H


def test_ideal_sgs_penalty_and_sponge_commutators_closed_form():
    """omega = W cos(k.x + a), chi = c0 + c1 cos(p.x + b), chi_s = s0 +
    s1 cos(q.x + c), uniform inflow (U, V).  A single mode has no Jacobian,
    and the inflow and the constant parts of the masks enter linearly, so
    only the mask modes leave commutators.  With psi = -omega/|k|^2,
    curl(f u) = f omega + f_x v - f_y u gives for f = cos(p.x + b)
      (W/2)(1 + p.k/|k|^2) cos(k.x + a + p.x + b)
      + (W/2)(1 - p.k/|k|^2) cos(k.x + a - p.x - b),
    and chi_s omega splits into (s1 W/2) cos(k.x + a +- (q.x + c)); each
    frequency k +- p picks up (H(p) H(k) - H(k +- p)) in Pi."""
    n, delta = 32, 2
    eta, sigma = 0.05, 3.0
    W, a = 0.8, 0.3
    c0, c1, b = 0.5, 0.3, 0.4
    s0, s1, c = 0.2, 0.15, -0.3
    k, p, q = (2, 1), (1, 2), (-1, 1)
    mf, ml = models(n, delta, eta=eta, sponge_sigma=sigma, u_in=0.4, v_in=-0.2,
                    chi=lambda m: c0 + c1 * np.cos(p[0] * grid_xy(m)[0] + p[1] * grid_xy(m)[1] + b),
                    chi_s=lambda m: s0 + s1 * np.cos(q[0] * grid_xy(m)[0] + q[1] * grid_xy(m)[1] + c))
    X, Y = grid_xy(n)
    w = W * np.cos(k[0] * X + k[1] * Y + a)
    Pi, _ = les.ideal_sgs(w, mf, ml)
    H = H_of(n, delta)
    Xc, Yc = grid_xy(n // delta)
    tk = k[0] * Xc + k[1] * Yc + a
    tp = p[0] * Xc + p[1] * Yc + b
    tq = q[0] * Xc + q[1] * Yc + c
    k2 = k[0] ** 2 + k[1] ** 2
    pk = (p[0] * k[0] + p[1] * k[1]) / k2
    ref = np.zeros_like(Xc)
    for sgn in (1, -1):
        kp = (k[0] + sgn * p[0], k[1] + sgn * p[1])
        kq = (k[0] + sgn * q[0], k[1] + sgn * q[1])
        ref += (1.0 / eta) * c1 * (H(p) * H(k) - H(kp)) * 0.5 * W * (1 + sgn * pk) * np.cos(tk + sgn * tp)
        ref += sigma * s1 * (H(q) * H(k) - H(kq)) * 0.5 * W * np.cos(tk + sgn * tq)
    assert np.max(np.abs(ref)) > 0.1
    assert np.max(np.abs(Pi - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_ideal_sgs_is_projected_on_the_les_two_thirds_set():
    """J of two modes whose sum frequency (6, 0) lies inside the filter's
    cut-off (|k| <= 8) but outside the 16-point grid's 2/3 set (|m| <= 5):
    Pi keeps only the difference frequency."""
    n, delta = 32, 2
    mf, ml = models(n, delta)
    X, Y = grid_xy(n)
    aa, bb = 0.6, 0.5
    k1, k2 = (4, 1), (2, -1)
    w = aa * np.cos(k1[0] * X + k1[1] * Y) + bb * np.cos(k2[0] * X + k2[1] * Y)
    Pi, wbar = les.ideal_sgs(w, mf, ml)
    H = H_of(n, delta)
    q1, q2 = k1[0] ** 2 + k1[1] ** 2, k2[0] ** 2 + k2[1] ** 2
    A = aa * bb * (k1[0] * k2[1] - k1[1] * k2[0]) * (1.0 / q1 - 1.0 / q2)
    sm = (k1[0] - k2[0], k1[1] - k2[1])
    Xc, Yc = grid_xy(n // delta)
    ref = -0.5 * A * (H(k1) * H(k2) - H(sm)) * np.cos(sm[0] * Xc + sm[1] * Yc)
    assert abs(H((6, 0))) > 0.1     # the sum frequency passes the filter
    assert np.max(np.abs(ref)) > 1e-3
    assert np.max(np.abs(Pi - ref)) <= 1e-12 * np.max(np.abs(ref))
    # omega_bar is the filtered field on the LES grid
    ref_w = H(k1) * aa * np.cos(k1[0] * Xc + k1[1] * Yc) + H(k2) * bb * np.cos(k2[0] * Xc + k2[1] * Yc)
    assert np.max(np.abs(wbar - ref_w)) < 1e-14


@pytest.mark.parametrize("closure,power", [("smag", 2), ("leith", 3)])
def test_model_sgs_enstrophy_identity(closure, power):
    """Pi = C div(base grad omega) with omega band-limited: on the grid,
    sum omega Pi = -C sum base |grad omega|^2 exactly (Parseval), with
    C = (c Delta)^p, base = |grad omega| (Leith) or the strain magnitude
    sqrt((psi_xx - psi_yy)^2 + 4 psi_xy^2) (Smagorinsky) -- gradients taken
    here with numpy's FFT, independently of the oracle."""
    from oracle import qg
    n, c = 32, 0.25
    ml = qg.Model(qg.Params(nx=n, ny=n, lx=TWO_PI, ly=TWO_PI, dt=1e-3, closure=closure, c=c), None, None)
    w = band_field(n, 4, 21)
    Pi = les.model_sgs(w, ml)
    m = np.fft.fftfreq(n, 1.0 / n)
    KX, KY = np.meshgrid(m, m)
    wh = np.fft.fft2(w)
    d = lambda fh: np.real(np.fft.ifft2(fh))
    wx, wy = d(1j * KX * wh), d(1j * KY * wh)
    k2 = KX ** 2 + KY ** 2
    k2[0, 0] = 1.0
    ph = -wh / k2
    ph[0, 0] = 0.0
    if closure == "leith":
        base = np.sqrt(wx ** 2 + wy ** 2)
    else:
        pxx, pyy, pxy = d(-KX * KX * ph), d(-KY * KY * ph), d(-KX * KY * ph)
        base = np.sqrt((pxx - pyy) ** 2 + 4 * pxy ** 2)
    C = (c * TWO_PI / n) ** power
    lhs = float(np.sum(w * Pi))
    rhs = -C * float(np.sum(base * (wx ** 2 + wy ** 2)))
    assert rhs < 0
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)
