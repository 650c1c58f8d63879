"""Pins for the oracle's discrete adjoint.

Linear pieces (transforms, entry/exit projections, the B sub-step at zero
inflow) pass the dot-product test <A x, y> = <x, A* y> to round-off; the
nonlinear right-hand side, one full step and a multi-step rollout are checked
against central finite differences of the forward oracle, in random
directions and in the closure coefficient c.
"""
import math

import numpy as np
import pytest

from oracle import qg, adjoint as adj
from paper_2508_06678_amd import inputs


def make(closure="smag", c=0.17, nx=32, ny=16, u_in=0.7, **kw):
    lx, ly = 2 * math.pi, math.pi
    chi = inputs.island_mask(nx, ny, lx, ly, 1.5, ly / 2, 0.5)
    chi_s = inputs.sponge_mask(nx, ny, lx, ly)
    kw.setdefault("dt", 2e-3)
    p = qg.Params(nx=nx, ny=ny, lx=lx, ly=ly, beta=1.5, re=300.0, mu=0.05,
                  u_in=u_in, v_in=-0.2, eta=5e-3, sponge_sigma=10.0,
                  closure=closure, c=c, **kw)
    return qg.Model(p, chi, chi_s)


def rstate(m, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return qg.enter(scale * rng.standard_normal((m.g.ny, m.g.nx)), m.g)


def ip(m, a, b):
    return m.g.mean_product(a, b) * m.g.N


def test_transform_adjoints_weighted_product():
    m = make()
    g = m.g
    rng = np.random.default_rng(0)
    f = rng.standard_normal((g.ny, g.nx))
    h = rng.standard_normal((g.ny, g.nx // 2 + 1)) + 1j * rng.standard_normal((g.ny, g.nx // 2 + 1))
    # <spec f, h>_w == <f, phys h>
    assert ip(m, g.spec(f), h) == pytest.approx(np.sum(f * g.phys(h)), rel=1e-13)
    # entry / exit
    wh = rstate(m, 1)
    lam = rng.standard_normal((g.ny, g.nx))
    assert np.sum(qg.enter(lam, g).real * 0) == 0
    assert ip(m, qg.enter(f, g), wh) == pytest.approx(np.sum(f * adj.enter_adjoint(wh, g)), rel=1e-13)
    assert np.sum(qg.leave(wh, g) * lam) == pytest.approx(ip(m, wh, adj.leave_adjoint(lam, g)), rel=1e-13)


def test_b_substep_dot_product():
    m = make(u_in=0.0)
    m.p.v_in = 0.0
    x = rstate(m, 2)
    y = rstate(m, 3)
    lhs = ip(m, qg.b_substep(x, m), y)
    rhs = ip(m, x, adj.b_adjoint(y, m))
    assert lhs == pytest.approx(rhs, rel=1e-13)


@pytest.mark.parametrize("closure", ["none", "smag", "leith", "const"])
def test_rhs_adjoint_central_fd(closure):
    c = {"none": 0.0, "smag": 0.17, "leith": 0.2, "const": 1e-3}[closure]
    m = make(closure=closure, c=c)
    x = rstate(m, 4)
    d = rstate(m, 5)
    lam = rstate(m, 6)
    h = 1e-6
    fd = (ip(m, qg.rhs(x + h * d, m), lam) - ip(m, qg.rhs(x - h * d, m), lam)) / (2 * h)
    la, dc = adj.rhs_adjoint(x, lam, m)
    assert ip(m, d, la) == pytest.approx(fd, rel=1e-8)
    if closure != "none":
        mp = make(closure=closure, c=c + h)
        mm = make(closure=closure, c=c - h)
        fdc = (ip(m, qg.rhs(x, mp), lam) - ip(m, qg.rhs(x, mm), lam)) / (2 * h)
        assert dc == pytest.approx(fdc, rel=1e-7)


@pytest.mark.parametrize("closure", ["smag", "leith"])
def test_rollout_gradient_central_fd(closure):
    c = 0.17 if closure == "smag" else 0.2
    m = make(closure=closure, c=c)
    g = m.g
    w0 = g.phys(rstate(m, 7))
    tgt = g.phys(rstate(m, 8, 0.5))
    n = 4
    wT = qg.run(w0, m, n)
    gw, gc = adj.run_adjoint(w0, adj.loss_grad(wT, tgt), m, n)
    h = 1e-4   # the loss is O(1) and the directional derivatives O(1e-5)
    for k, d in enumerate(inputs.random_directions(w0.shape, 3, 5)):
        lp = adj.loss(qg.run(w0 + h * d, m, n), tgt)
        lm = adj.loss(qg.run(w0 - h * d, m, n), tgt)
        fd = (lp - lm) / (2 * h)
        assert np.sum(gw * d) == pytest.approx(fd, rel=1e-7)
    h = 1e-6
    mp = make(closure=closure, c=c + h)
    mm = make(closure=closure, c=c - h)
    fdc = (adj.loss(qg.run(w0, mp, n), tgt) - adj.loss(qg.run(w0, mm, n), tgt)) / (2 * h)
    assert gc == pytest.approx(fdc, rel=1e-6)


# ---------------------------------------------------------------- dynamic closures
@pytest.mark.parametrize("closure", ["dsmag", "dleith"])
def test_dynamic_rhs_adjoint_central_fd(closure):
    """C = max(<HM>,0)/<M^2> depends on the stage input: the adjoint's s grad C
    term (2% and 13% of this directional derivative) must be exact.  State
    with C > 0, away from the clip."""
    m = make(closure=closure, c=0.0)
    x = rstate(m, 4)
    out = {}
    qg.rhs(x, m, out)
    assert out["C"] > 0.0
    d = rstate(m, 104)
    lam = rstate(m, 204)
    h = 1e-6
    fd = (ip(m, qg.rhs(x + h * d, m), lam) - ip(m, qg.rhs(x - h * d, m), lam)) / (2 * h)
    la, dc = adj.rhs_adjoint(x, lam, m)
    assert dc == 0.0
    assert ip(m, d, la) == pytest.approx(fd, rel=1e-8)


@pytest.mark.parametrize("closure", ["dsmag", "dleith"])
def test_dynamic_rhs_adjoint_clipped(closure):
    """Where <HM> < 0 the clip sets C = 0 in a neighbourhood: the adjoint is
    the closure-free one, and central differences agree."""
    m = make(closure=closure, c=0.0)
    x = rstate(m, 6)
    out = {}
    qg.rhs(x, m, out)
    assert out["HM"] < 0.0 and out["C"] == 0.0
    lam = rstate(m, 206)
    la, _ = adj.rhs_adjoint(x, lam, m)
    m0 = make(closure="none", c=0.0)
    la0, _ = adj.rhs_adjoint(x, lam, m0)
    assert np.max(np.abs(la - la0)) <= 1e-13 * np.max(np.abs(la0))
    d = rstate(m, 106)
    h = 1e-6
    fd = (ip(m, qg.rhs(x + h * d, m), lam) - ip(m, qg.rhs(x - h * d, m), lam)) / (2 * h)
    assert ip(m, d, la) == pytest.approx(fd, rel=1e-8)


@pytest.mark.parametrize("closure", ["dsmag", "dleith"])
def test_dynamic_rollout_gradient_central_fd(closure):
    m = make(closure=closure, c=0.0)
    g = m.g
    w0 = g.phys(rstate(m, 4))
    tgt = g.phys(rstate(m, 8, 0.5))
    n = 3
    wT = qg.run(w0, m, n)
    gw, gc = adj.run_adjoint(w0, adj.loss_grad(wT, tgt), m, n)
    assert gc == 0.0
    h = 1e-4
    for d in inputs.random_directions(w0.shape, 3, 5):
        lp = adj.loss(qg.run(w0 + h * d, m, n), tgt)
        lm = adj.loss(qg.run(w0 - h * d, m, n), tgt)
        assert np.sum(gw * d) == pytest.approx((lp - lm) / (2 * h), rel=1e-7)
