"""GPU parity of the pointwise-clip reading of the dynamic coefficient
(clip_mode 1: C = <max(H, 0) M> / <M^2>, the negative part of H removed at
every grid point before the average) against the oracle, whose clip_mode 1
is pinned by test_oracle_physics.py (2 C <M^2> = <HM> + <|H| M>, oddness,
scale invariance) and test_oracle_mutations.py.

The GPU forms the two grid sums in a pass of its own (H and M back to the
grid, one partial pair per row pair, FP64 accumulation), so these tests cover
every path that takes a dynamic coefficient: the RK4 stages, AB2CN, the
diagnostics, the closure's model term, mixed clip modes in one handle and
every strip width.  Tolerances as for the coefficient-level clip: per step
1e-12 (FP64) and 1e-5 (FP32) relative L2 of the physical vorticity.
"""
import json
import math

import numpy as np
import pytest

from oracle import ab2cn, qg
from oracle import les as oles
from paper_2508_06678_amd import configs, inputs
from tests.bridge import HAVE_GPU, oracle_model, field_err, max_rel, rel_l2, solver_for, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")]

TOL = {64: 1e-12, 32: 1e-5}


def say(*a):
    print(*a, flush=True)


def member(nx, ny, closure, clip=1, seed=3, beta=1.5):
    lx, ly = 2 * math.pi, 2 * math.pi * ny / nx
    m = configs.cape_member(nx, ny, precision=64, beta=beta, re=1e3, dt=1e-3, eta=5e-3,
                            height=0.5, closure=closure, seed=seed, rms=0.2, init="spectrum",
                            lx=lx, ly=ly, u_in=1.0, c=None)
    m.params["clip_mode"] = clip
    return m


def oracle_c(w, M):
    """The oracle's dynamic coefficient at a physical field."""
    out = {}
    qg.rhs(qg.enter(w, M.g), M, out)
    return out["C"]


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("closure", ["dsmag", "dleith"])
def test_rk4_steps(precision, closure):
    """Three RK4 steps at 128x64, compared after each; the two readings of
    the clip must give coefficients that differ well beyond the tolerance,
    so that the test can tell them apart.  (With H clipped at every point
    but M of either sign, <max(H, 0) M> and so C can be negative: the
    reading does not clip the ratio again.)"""
    m = member(128, 64, closure)
    S = solver_for([m], precision)
    M1 = oracle_model(m.params, m.chi, m.chi_s)
    M0 = oracle_model(dict(m.params, clip_mode=0), m.chi, m.chi_s)
    om = S.pack([m.omega0])
    w0 = to_np(om).reshape(64, 128)
    c1, c0 = oracle_c(w0, M1), oracle_c(w0, M0)
    say("clip", closure, precision, "C pointwise", c1, "C coefficient-level", c0)
    assert c1 != 0 and abs(c1 - c0) > 1e-3 * abs(c1)
    worst = 0.0
    for _ in range(3):
        w_n = to_np(om).reshape(64, 128)
        S.step(om, 1, use_graph=False)
        err = field_err(to_np(om).reshape(64, 128), qg.step(w_n, M1))
        worst = max(worst, err)
    say("  worst rel L2 per step", worst)
    assert worst < TOL[precision]
    S.close()


@pytest.mark.parametrize("closure", ["dsmag", "dleith"])
def test_diag_coefficient(closure):
    m = member(256, 128, closure, seed=5)
    S = solver_for([m], 64)
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    out, nu = S.diag(om, want_nu=True)
    out = out.cpu().numpy()[0]
    ref, nu_ref = qg.diag(to_np(om).reshape(128, 256), M)
    say("clip diag", closure, out[2], ref[2])
    assert ref[2] != 0
    np.testing.assert_allclose(out[2], ref[2], rtol=1e-10)
    np.testing.assert_allclose(out[3:7], ref[3:7], rtol=1e-10, atol=1e-14)
    assert field_err(to_np(nu).reshape(128, 256), nu_ref) < 1e-10
    S.close()


def test_graph_replay_and_mixed_clip_modes():
    """One handle with the same closure under both clip modes (two groups)
    and a static member, two steps in one graph replay, each member against
    the oracle."""
    ms = [member(128, 64, "dleith", clip=1, seed=3), member(128, 64, "dleith", clip=0, seed=3),
          member(256, 128, "dsmag", clip=1, seed=4), member(128, 64, "smag", clip=0, seed=6)]
    S = solver_for(ms, 64)
    om = S.pack([m.omega0 for m in ms])
    w_in = [to_np(x) for x in S.unpack(om)]
    S.step(om, 2, use_graph=True)
    got = [to_np(x) for x in S.unpack(om)]
    for m, wi, g in zip(ms, w_in, got):
        M = oracle_model(m.params, m.chi, m.chi_s)
        err = field_err(g, qg.run(wi, M, 2))
        say("  member", m.params["nx"], m.params["closure"], "clip", m.params["clip_mode"], err)
        assert err < 1e-12
    assert rel_l2(got[0], got[1]) > 1e-9     # the two readings differ
    S.close()


@pytest.mark.parametrize("precision", [64, 32])
def test_every_strip_width(tmp_path, precision):
    import torch
    nx, ny = 128, 512
    m = member(nx, ny, "dsmag")
    M = oracle_model(m.params, m.chi, m.chi_s)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = f"{arch}/{nx}x{ny}/fp{precision}/closure3/members1"
    widths = [W for W in (1, 2, 4, 8, 16) if W * ny >= 512 and W * ny <= (2048 if precision == 64 else 4096)]
    ref = None
    for i, W in enumerate(widths):
        Wi = widths[-1 - i]
        cache = tmp_path / f"w{W}_{Wi}.json"
        cache.write_text(json.dumps({key + "/fwd": W, key + "/inv": Wi}))
        S = solver_for([m], precision)
        S.autotune(str(cache))
        assert S.column_widths() == [W] and S.inverse_widths() == [Wi]
        om = S.pack([m.omega0])
        w_in = to_np(om).reshape(ny, nx)
        S.step(om, 1, use_graph=False)
        if ref is None:
            ref = qg.step(w_in, M)
        err = field_err(to_np(om).reshape(ny, nx), ref)
        say("  W", W, "Wi", Wi, err)
        assert err < TOL[precision]
        S.close()


def test_ab2cn_every_step():
    """The paper's AB2CN scheme with the pointwise clip, 10 steps in lockstep."""
    m = configs.ab2cn_island(64, closure="dleith").members[0]
    m.params["clip_mode"] = 1
    m.omega0 = inputs.spectrum_noise(128, 64, 2 * math.pi, math.pi, 7, 2.0, 0.2)
    S = solver_for([m], 64)
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    wh = qg.enter(to_np(om).reshape(64, 128), M.g)
    hist = None
    worst = 0.0
    for n in range(1, 11):
        S.step(om, 1, use_graph=False)
        wh, hist = ab2cn.step_spectral(wh, hist, M)
        worst = max(worst, field_err(to_np(om).reshape(64, 128), qg.leave(wh, M.g)) / n)
    say("AB2CN clip 1 worst rel L2 per step", worst)
    assert worst < 1e-12
    S.close()


@pytest.mark.parametrize("precision", [64, 32])
def test_closure_term(precision):
    """qg_closure_term (C D div(base grad omega) at a field) with the
    pointwise clip, against the oracle's model term.  In 32-bit runs the
    ratio C carries the cancellation of its grid sums, so the term is
    compared in shape (to 1e-5) and C separately, within the first-order
    bound 1e-5 + 1e-6 kappa (kappa_H + kappa_M): kappa = sum |H+ M| /
    |sum H+ M| (H+ = max(H, 0)), kappa_H = (|H| + |T J|) / |H| and kappa_M =
    (|M| + |T Q|) / |M| the cancellations in the sum and in H and M."""
    m = member(256, 128, "dsmag", seed=4)
    S = solver_for([m], precision)
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    w = to_np(om).reshape(128, 256)
    got = to_np(S.closure_term(om)).reshape(128, 256)
    ref = oles.model_sgs(w, M)
    assert np.any(ref)
    if precision == 64:
        e = field_err(got, ref)
        say("closure term clip 1", e)
        assert e < 1e-12
    else:
        out = {}
        qg.rhs(qg.enter(w, M.g), M, out)
        g = M.g
        H, Mf = g.phys(out["Hh"]), g.phys(out["Mh"])
        hp = np.maximum(H, 0.0) * Mf
        kappa = float(np.sum(np.abs(hp)) / abs(np.sum(hp)))
        nrm = np.linalg.norm
        k_h = float((nrm(out["Hh"]) + nrm(g.T * out["Jh"])) / nrm(out["Hh"]))
        k_m = float((nrm(out["Mh"]) + nrm(g.T * out["Qh"])) / nrm(out["Mh"]))
        scale = float(np.dot(got.ravel(), ref.ravel()) / np.dot(ref.ravel(), ref.ravel()))
        e = rel_l2(got / scale, ref)
        bar_c = 1e-5 + 1e-6 * kappa * (k_h + k_m)
        say("closure term clip 1 fp32: shape", e, "C ratio - 1", scale - 1.0, "bar", bar_c)
        assert e < 1e-5 and abs(scale - 1.0) < bar_c
    S.close()


def test_adjoint_is_refused():
    """The adjoint differentiates the coefficient-level clip only: a handle
    with the pointwise clip refuses qg_adjoint_step before any launch."""
    import torch
    m = member(128, 64, "dsmag")
    S = solver_for([m], 64, adj_segment_k=2)
    om = S.pack([m.omega0])
    lam = om.clone()
    grad_c = torch.zeros(1, dtype=torch.float64, device=om.device)
    with pytest.raises(RuntimeError) as e:
        S.adjoint_step(om, lam, 2, grad_c)
    assert "clip_mode" in str(e.value)
    assert torch.equal(lam, om)
    S.close()
