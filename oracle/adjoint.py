"""Oracle: exact discrete adjoint of one QG time step.

TEST INFRASTRUCTURE ONLY (see the package header).  FP64 throughout.

Inner products.  Physical fields use the plain sum over grid points.  Half
spectra use the weighted product
    <a, b>_w = (1/N) sum_half w Re(conj(a) b),  w = 1 at m_x in {0, nx/2}, else 2,
which equals the physical product of the fields they represent (Parseval).
With these choices the adjoint of irfft2 is rfft2 and the adjoint of rfft2
is irfft2 (exactly, as real-linear maps), diagonal spectral multipliers
adjoin to their conjugates, and the projections D, T and the removal of the
mean mode are self-adjoint.  A pointwise product adjoins to multiplication by
its partner; the square root in |S| and |grad omega| adjoins through its
derivative, taken as 0 where the base vanishes.

The forward map differentiated is exactly ``oracle.qg.step_spectral``: the
RK4 A sub-step over the right-hand side of Eq. 1 with the eddy-viscosity
term of Eq. 8 (Eqs. 9, 12) followed by the B sub-step (Eqs. 2-4, exact
penalization then sponge).  The masks, the inflow and the parameters are
fixed; for the static closures the coefficient c is the one scalar
parameter differentiated (C = (c Delta)^2 or (c Delta)^3).

For the dynamic closures (Eqs. 10-11, 13) the coefficient is itself a
function of the stage input x: C = max(<HM>, 0)/<M^2> (grid means) with
H = D FFT(J(T x)) - T D FFT(J(x)) and M = r D div(g(T x)) - T Q(x).  Its
derivative adds s grad C to the stage's adjoint, s = <lam, Q>_w, where by
the chain rule (C > 0)
    grad C = [J_H^T M + J_M^T (H - 2 C M)] / (N <M^2>),
J_H^T a = T A_J(T x)^T a - A_J(x)^T T a and J_M^T b = r T A_Q(T x)^T b -
A_Q(x)^T T b, with A_J, A_Q the linearizations of y -> D FFT(J(y)) and
y -> D div(base(y) grad y).  Where the clip sets C = 0 the derivative is
zero (the kink at <HM> = 0 is not differentiated).
"""
import numpy as np

from . import qg


def _zero_mean(a):
    a = a.copy()
    a[0, 0] = 0.0
    return a


def dC_dc(m):
    p, d = m.p, m.g.delta
    if p.closure == "smag":
        return 2.0 * p.c * d * d
    if p.closure == "leith":
        return 3.0 * p.c * p.c * d ** 3
    if p.closure == "const":
        return 1.0
    return 0.0


def transport_adjoint(y, cJ, cQ, kind, m):
    """dL/dy (in D) of L = <cJ, D FFT(J(y))>_w + <cQ, D div(base(y) grad y)^>_w,
    J(y) = u omega_x + v omega_y with the total velocity of y; kind is the
    base's family ("smag", "leith", "const") or None for no second term."""
    g = m.g
    psih = -y * g.inv_k2
    u, v = qg.velocity(psih, m)
    wx = g.phys(1j * g.kx * y)
    wy = g.phys(1j * g.ky * y)
    lam_J = g.phys(g.D * cJ)
    lam_u, lam_v = lam_J * wx, lam_J * wy
    lam_wx, lam_wy = lam_J * u, lam_J * v
    lam_psi = np.zeros_like(y)
    if kind is not None:
        base = qg.closure_base(kind, psih, wx, wy, m)
        gx = g.phys(-1j * g.kx * g.D * cQ)
        gy = g.phys(-1j * g.ky * g.D * cQ)
        lam_wx = lam_wx + gx * base
        lam_wy = lam_wy + gy * base
        lam_b = gx * wx + gy * wy
        safe = np.where(base > 0, base, 1.0)
        if kind == "smag":
            pd = g.phys((g.ky ** 2 - g.kx ** 2) * psih)
            pxy = g.phys(-g.kx * g.ky * psih)
            lam_pd = np.where(base > 0, pd / safe, 0.0) * lam_b
            lam_pxy = np.where(base > 0, 4.0 * pxy / safe, 0.0) * lam_b
            lam_psi = lam_psi + (g.ky ** 2 - g.kx ** 2) * g.spec(lam_pd) - g.kx * g.ky * g.spec(lam_pxy)
        elif kind == "leith":
            lam_wx = lam_wx + np.where(base > 0, wx / safe, 0.0) * lam_b
            lam_wy = lam_wy + np.where(base > 0, wy / safe, 0.0) * lam_b
    lam_psi = lam_psi + 1j * g.ky * g.spec(lam_u) - 1j * g.kx * g.spec(lam_v)
    lam_y = -1j * g.kx * g.spec(lam_wx) - 1j * g.ky * g.spec(lam_wy) - g.inv_k2 * lam_psi
    return g.D * lam_y


def dynamic_rhs_adjoint(x, lam, m):
    """Dynamic closures: (dL/dx, 0) for stage input x and lam = dL/dR."""
    g, p = m.g, m.p
    kind = "smag" if p.closure == "dsmag" else "leith"
    lam = _zero_mean(lam)
    fw = {}
    qg.rhs(x, m, fw)
    C = fw["C"]
    lam_x = -(g.k2 * m.inv_re + p.mu) * lam - g.inv_k2 * (1j * p.beta * g.kx) * lam
    lam_x = g.D * lam_x + transport_adjoint(x, -lam, C * lam, kind, m)
    if fw["HM"] > 0.0 and fw["MM"] > 0.0:
        s = g.N * g.mean_product(lam, fw["Qh"])                # <lam, Q>_w = dL/dC
        f = s / (g.N * fw["MM"])
        a = f * fw["Mh"]
        b = f * (fw["Hh"] - 2.0 * C * fw["Mh"])
        r = float(p.test_ratio) ** (2 if p.closure == "dsmag" else 3)
        lam_x = lam_x + g.T * transport_adjoint(g.T * x, a, r * b, kind, m) \
            - transport_adjoint(x, g.T * a, g.T * b, kind, m)
    return g.D * lam_x, 0.0


def rhs_adjoint(x, lam, m):
    """Given stage input x (in D) and lam = dL/dR, return (dL/dx, <lam, dR/dc>_w)."""
    g, p = m.g, m.p
    if p.closure in ("dsmag", "dleith"):
        return dynamic_rhs_adjoint(x, lam, m)
    if p.closure not in ("none", "smag", "leith", "const"):
        raise NotImplementedError(p.closure)
    fw = {}
    qg.rhs(x, m, fw)
    lam = _zero_mean(lam)
    lD = g.D * lam
    C = fw["C"]
    # linear spectral terms: -(k^2/Re + mu) x - i beta kx psi
    lam_x = -(g.k2 * m.inv_re + p.mu) * lam
    lam_psi = (1j * p.beta * g.kx) * lam
    # -D FFT(J):  lam_J = irfft2(-D lam)
    lam_J = g.phys(-lD)
    u, v, wx, wy = fw["u"], fw["v"], fw["wx"], fw["wy"]
    lam_u = lam_J * wx
    lam_v = lam_J * wy
    lam_wx = lam_J * u
    lam_wy = lam_J * v
    dc = 0.0
    if p.closure != "none":
        base = fw["base"]
        gx = g.phys(-1j * g.kx * lD)      # adjoint of D i kx FFT(.)
        gy = g.phys(-1j * g.ky * lD)
        lam_hx, lam_hy = C * gx, C * gy
        lam_wx = lam_wx + lam_hx * base
        lam_wy = lam_wy + lam_hy * base
        lam_b = lam_hx * wx + lam_hy * wy
        dc = dC_dc(m) * float(np.sum(gx * base * wx + gy * base * wy))
        safe = np.where(base > 0, base, 1.0)
        if p.closure == "smag":
            psih = fw["psih"]
            pd = g.phys((g.ky ** 2 - g.kx ** 2) * psih)
            pxy = g.phys(-g.kx * g.ky * psih)
            lam_pd = np.where(base > 0, pd / safe, 0.0) * lam_b
            lam_pxy = np.where(base > 0, 4.0 * pxy / safe, 0.0) * lam_b
            lam_psi = lam_psi + (g.ky ** 2 - g.kx ** 2) * g.spec(lam_pd) \
                - g.kx * g.ky * g.spec(lam_pxy)
        elif p.closure == "leith":
            lam_wx = lam_wx + np.where(base > 0, wx / safe, 0.0) * lam_b
            lam_wy = lam_wy + np.where(base > 0, wy / safe, 0.0) * lam_b
    lam_psi = lam_psi + 1j * g.ky * g.spec(lam_u) - 1j * g.kx * g.spec(lam_v)
    lam_x = lam_x - 1j * g.kx * g.spec(lam_wx) - 1j * g.ky * g.spec(lam_wy)
    lam_x = lam_x - g.inv_k2 * lam_psi
    return g.D * lam_x, dc


def b_adjoint(lam, m):
    """Adjoint of the B sub-step (affine in its input; the inflow drops out)."""
    g = m.g
    l2 = g.phys(g.D * _zero_mean(lam))
    l1 = m.S * l2
    lam_w = m.E * l1
    lam_v = m.Ex * l1
    lam_u = -m.Ey * l1
    lam_psi = 1j * g.ky * g.spec(lam_u) - 1j * g.kx * g.spec(lam_v)
    return g.D * (g.spec(lam_w) - g.inv_k2 * lam_psi)


def step_spectral_adjoint(wh, lam_next, m):
    """Adjoint of qg.step_spectral at wh: returns (dL/dwh, dL/dc from this step)."""
    dt = m.p.dt
    x1 = wh
    k1 = qg.rhs(x1, m)
    x2 = wh + 0.5 * dt * k1
    k2 = qg.rhs(x2, m)
    x3 = wh + 0.5 * dt * k2
    k3 = qg.rhs(x3, m)
    x4 = wh + dt * k3
    lam_s = b_adjoint(lam_next, m)
    lam_w = lam_s.copy()
    lk4 = (dt / 6.0) * lam_s
    lk3 = (dt / 3.0) * lam_s
    lk2 = (dt / 3.0) * lam_s
    lk1 = (dt / 6.0) * lam_s
    dc = 0.0
    l4, d4 = rhs_adjoint(x4, lk4, m)
    lam_w += l4
    lk3 = lk3 + dt * l4
    l3, d3 = rhs_adjoint(x3, lk3, m)
    lam_w += l3
    lk2 = lk2 + 0.5 * dt * l3
    l2, d2 = rhs_adjoint(x2, lk2, m)
    lam_w += l2
    lk1 = lk1 + 0.5 * dt * l2
    l1, d1 = rhs_adjoint(x1, lk1, m)
    lam_w += l1
    dc = d1 + d2 + d3 + d4
    return lam_w, dc


def enter_adjoint(lam, g):
    """Adjoint of qg.enter (D * rfft2, mean removed): physical gradient."""
    return g.phys(g.D * _zero_mean(lam))


def leave_adjoint(lam_phys, g):
    """Adjoint of qg.leave (irfft2) restricted to states in D."""
    return _zero_mean(g.D * g.spec(lam_phys))


def run_adjoint(w0, lam_T, m, nsteps):
    """Gradient of a scalar of omega_T = qg.run(w0, m, nsteps) given
    lam_T = dL/d omega_T (physical).  Returns (dL/d w0, dL/dc)."""
    g = m.g
    states = [qg.enter(w0, g)]
    for _ in range(nsteps - 1):
        states.append(qg.step_spectral(states[-1], m))
    lam = leave_adjoint(lam_T, g)
    dc = 0.0
    for wh in reversed(states):
        lam, d = step_spectral_adjoint(wh, lam, m)
        dc += d
    return enter_adjoint(lam, g), dc


def loss(wT, target):
    """A-posteriori vorticity loss: grid mean of (omega_T - target)^2."""
    d = wT - target
    return float(np.mean(d * d))


def loss_grad(wT, target):
    return 2.0 * (wT - target) / wT.size
