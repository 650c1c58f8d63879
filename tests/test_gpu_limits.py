"""GPU parity at the extremes of the admitted grid sizes: rows and columns
of the maximum length (4096, the run-time-length transform engines and the
row kernel that loops over fields), the smallest grids (32), and the
largest sizes of the options with tighter limits (the pointwise clip and
AB2CN in 64-bit runs: nx = 2048).  One step each against the oracle, to the
per-step tolerances (1e-12 FP64, 1e-5 FP32).

AB2CN's explicit penalty (dt/eta) D curl(chi u) differentiates chi u
spectrally, so the rounding of its transform is multiplied by |k|: taken
literally, the step's relative error is about u_r kappa with u_r the unit
roundoff and kappa = (dt/eta) k_rms |chi u| / |omega*| (k_rms over the 2/3
set).  A mask that covers the whole box makes chi u nearly the constant
inflow, whose curl vanishes while the amplified rounding does not (kappa ~
4e3 at 4096 points a row).  The library forms the curl as
D curl((chi - c) u) + c omega with c the mask's mean, which removes that
near-constant part; the last test checks the FP32 step there against the
ordinary tolerance.
"""
import math

import numpy as np
import pytest

from oracle import ab2cn, qg
from paper_2508_06678_amd import configs, inputs
from tests.bridge import HAVE_GPU, oracle_model, field_err, max_rel, rel_l2, solver_for, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")]

TOL = {64: 1e-12, 32: 1e-5}


def say(*a):
    print(*a, flush=True)


def member(nx, ny, closure, clip=0, scheme="rk4"):
    """An island in a channel whose sides are scaled to the box (dx = dy):
    the island's radius is a fifth of the shorter side."""
    lx, ly = 2 * math.pi, 2 * math.pi * ny / nx
    m = configs.island_member(nx, ny, precision=64, beta=1.5, re=1e3, dt=1e-4, eta=5e-3, xc=0.3 * lx,
                              radius=0.2 * min(lx, ly), closure=closure, seed=3, rms=0.2, lx=lx, ly=ly)
    m.omega0 = inputs.spectrum_noise(nx, ny, lx, ly, 3, 2.0, 0.2)
    m.params["clip_mode"] = clip
    m.params["scheme"] = scheme
    return m


def one_step(m, precision, new_coef=None):
    """One step of member m on the GPU against the oracle's; with new_coef the
    closure coefficient is changed through qg_set_coef after qg_init (and in
    the oracle's parameters)."""
    nx, ny = m.params["nx"], m.params["ny"]
    say("case", nx, ny, precision, m.params["closure"], "clip", m.params["clip_mode"], m.params["scheme"])
    S = solver_for([m], precision)
    if new_coef is not None:
        S.set_coef([new_coef])
        m.params["c"] = new_coef
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    w_in = to_np(om).reshape(ny, nx)
    S.step(om, 1, use_graph=False)
    if m.params["scheme"] == "ab2cn":
        wh, _ = ab2cn.step_spectral(qg.enter(w_in, M.g), None, M)
        ref = qg.leave(wh, M.g)
    else:
        ref = qg.step(w_in, M)
    err = field_err(to_np(om).reshape(ny, nx), ref)
    say("  rel L2", err)
    S.close()
    return err


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("closure", ["smag", "dleith"])
@pytest.mark.parametrize("nx,ny", [(4096, 64), (64, 4096)])
def test_longest_rows_and_columns(nx, ny, closure, precision):
    assert one_step(member(nx, ny, closure), precision) < TOL[precision]


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("closure", ["leith", "dsmag"])
def test_smallest_grid(closure, precision):
    assert one_step(member(32, 32, closure), precision) < TOL[precision]


@pytest.mark.parametrize("nx,precision", [(2048, 64), (4096, 32)])
def test_pointwise_clip_at_its_largest_rows(nx, precision):
    assert one_step(member(nx, 64, "dsmag", clip=1), precision) < TOL[precision]


@pytest.mark.parametrize("nx,precision", [(2048, 64), (4096, 32)])
def test_ab2cn_at_its_largest_rows(nx, precision):
    m = member(nx, 64, "dleith", scheme="ab2cn")
    m.params["eta"] = 2.5 * m.params["dt"]
    say("  kappa", penalty_kappa(m))
    assert one_step(m, precision) < TOL[precision]


def penalty_kappa(m):
    """kappa = (dt/eta) k_rms |chi u| / |omega*| of the first AB2CN step
    (oracle, FP64)."""
    M = oracle_model(m.params, m.chi, m.chi_s)
    g = M.g
    wh = qg.enter(m.omega0, g)
    _, u, v = ab2cn.explicit_terms(wh, M)
    out, _ = ab2cn.step_spectral(wh, None, M)
    inD = g.D != 0
    k_rms = math.sqrt(float(np.sum(g.k2 * inD) / np.sum(inD)))
    chi_u = math.sqrt(float(np.mean((m.chi * u) ** 2 + (m.chi * v) ** 2)))
    w = math.sqrt(float(np.mean(qg.leave(out, g) ** 2)))
    return M.p.dt / M.p.eta * k_rms * chi_u / w


@pytest.mark.parametrize("solid", [1.0, 0.7])
def test_ab2cn_penalty_conditioning_fully_solid_fp32(solid):
    """A mask constant over the whole box (4096 x 64), where the literal
    curl of chi u would lose u_r kappa (kappa > 1e3, u_r = 2^-24) to
    rounding: with the mask's mean split off, the FP32 step meets the
    ordinary 1e-5 against the oracle."""
    m = member(4096, 64, "dleith", scheme="ab2cn")
    m.params["eta"] = 2.5 * m.params["dt"]
    m.chi = np.full_like(m.chi, solid)
    kappa = penalty_kappa(m)
    err = one_step(m, 32)
    say("  kappa", kappa, "u_r kappa", 2.0 ** -24 * kappa)
    assert kappa > 1e3
    assert err < TOL[32]


def test_set_coef_keeps_the_ab2cn_penalty_split():
    """qg_set_coef rebuilds the member constants; the mask mean that qg_init
    split off the AB2CN penalty's curl must survive it, or a fully solid FP32
    box drifts back to the literal form's rounding (u_r kappa ~ 2e-4)."""
    m = member(4096, 64, "smag", scheme="ab2cn")
    m.params["eta"] = 2.5 * m.params["dt"]
    m.chi = np.full_like(m.chi, 1.0)
    err = one_step(m, 32, new_coef=0.13)
    assert err < TOL[32]
