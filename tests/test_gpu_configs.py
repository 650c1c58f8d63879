"""Parity at the full sizes of the five benchmark workloads, in the launch
configuration the benchmark uses (tuned strip widths, graph replay).

Per-step gating: the GPU state after n steps is stepped once by the GPU and
once by the oracle and the two results are compared (relative L2 of the
physical vorticity: 1e-12 in FP64, 1e-5 in FP32).  Long trajectories are
chaotic, so the drift after many steps is reported, not gated.
"""
import math
import os

import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import qg
from paper_2508_06678_amd import configs, inputs
from tests.bridge import HAVE_GPU, oracle_model, rel_l2, solver_for, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")]

TOL = {64: 1e-12, 32: 1e-5}
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)


def per_step_check(S, M, om, shape, precision, steps):
    worst = 0.0
    for _ in range(steps):
        w_n = to_np(om).reshape(shape)
        S.step(om, 1, use_graph=True)
        err = rel_l2(to_np(om).reshape(shape), qg.step(w_n, M))
        worst = max(worst, err)
    return worst


def test_config1_every_step_fp64():
    """Island channel 128x64, static Smagorinsky: all 200 steps gated."""
    m = configs.config1().members[0]
    S = solver_for([m], 64)
    S.autotune()
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    worst = per_step_check(S, M, om, (64, 128), 64, 200)
    say("C1 worst per-step rel L2 over 200 steps", worst)
    assert worst < TOL[64]
    # 100-step drift (reported)
    om2 = S.pack([m.omega0])
    w0 = to_np(om2).reshape(64, 128)
    S.step(om2, 100)
    say("C1 100-step drift rel L2", rel_l2(to_np(om2).reshape(64, 128), qg.run(w0, M, 100)))
    S.close()


@pytest.mark.parametrize("precision", [64, 32])
def test_config2_island_dynamic_smagorinsky(precision):
    """512x256 dynamic Smagorinsky: steps at the start and after 150 GPU steps."""
    m = configs.config2(precision=precision).members[0]
    S = solver_for([m], precision)
    S.autotune()
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    worst = per_step_check(S, M, om, (256, 512), precision, 2)
    S.step(om, 150)
    worst = max(worst, per_step_check(S, M, om, (256, 512), precision, 2))
    say("C2", precision, "worst per-step rel L2", worst)
    assert worst < TOL[precision]
    out, nu = S.diag(om, want_nu=True)
    say("C2 diag", out.cpu().numpy()[0])
    S.close()


def test_config3_cape_dynamic_leith_fp32():
    """1024^2 dynamic Leith FP32: one step from the start and one after 100."""
    m = configs.config3(precision=32).members[0]
    S = solver_for([m], 32)
    S.autotune()
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    worst = per_step_check(S, M, om, (1024, 1024), 32, 1)
    S.step(om, 100)
    worst = max(worst, per_step_check(S, M, om, (1024, 1024), 32, 1))
    say("C3 worst per-step rel L2", worst)
    assert worst < TOL[32]
    S.close()


def test_config4_ensemble_one_launch_fp32():
    """64 members of three sizes and four closures in one graph launch; the
    oracle checks a sample of members (every fourth) one by one."""
    wl = configs.config4(precision=32)
    S = solver_for(wl.members, 32)
    S.autotune()
    om = S.pack([m.omega0 for m in wl.members])
    S.step(om, 20)
    w_n = [to_np(x) for x in S.unpack(om)]
    S.step(om, 1)
    got = [to_np(x) for x in S.unpack(om)]
    worst = 0.0
    for i in range(0, len(wl.members), 4):
        m = wl.members[i]
        M = oracle_model(m.params, m.chi, m.chi_s)
        err = rel_l2(got[i], qg.step(w_n[i], M))
        worst = max(worst, err)
        say("  member", i, m.params["nx"], m.params["ny"], m.params["closure"], err)
    assert worst < TOL[32]
    S.close()


def test_config5_adjoint_vs_oracle_fp64():
    """512x256 static Smagorinsky: the GPU adjoint of 4 steps equals the oracle's."""
    import torch
    m = configs.config5(precision=64).members[0]
    n = 4
    S = solver_for([m], 64, adj_segment_k=n)
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    w0 = to_np(om).reshape(256, 512)
    lamT = inputs.bandpass_noise(512, 256, 2 * math.pi, math.pi, 21, 2, 40, 1.0)
    lam = S.pack([lamT])
    g = torch.zeros(1, dtype=torch.float64, device=om.device)
    S.adjoint_step(om, lam, n, g)
    ref_l, ref_c = oadj.run_adjoint(w0, lamT, M, n)
    err = rel_l2(to_np(lam).reshape(256, 512), ref_l)
    say("C5 adjoint rel", err, "dc", g.item(), ref_c)
    assert err < 1e-11
    assert abs(g.item() - ref_c) <= 1e-10 * abs(ref_c)
    S.close()


def test_resume_from_checkpoint_is_bitwise():
    m = configs.config5(precision=32).members[0]
    S = solver_for([m], 32)
    a = S.pack([m.omega0])
    a, ck = S.step(a, 60, save_every=20)
    b = ck[S.total * 1: S.total * 2].clone()   # omega after 40 steps
    S.step(b, 20)
    assert (a == ck[S.total * 2: S.total * 3]).all().item()
    assert (a == b).all().item()
    S.close()


@pytest.mark.parametrize("precision", [64, 32])
def test_config5_gradients_central_fd(precision):
    """500 steps, checkpoints every 50, loss = mean (omega_T - target)^2 with
    the fine-grid target; gradients w.r.t. omega0 (16 random directions) and
    c by central differences (h = 1e-6 in FP64)."""
    import torch
    from paper_2508_06678_amd.autograd import QGRollout
    path = os.path.join(HERE, "golden", "c5_target_512x256.npy")
    if not os.path.exists(path):
        pytest.skip("target not generated (tests/golden/make_c5_target.py)")
    wl = configs.config5(precision=precision)
    m = wl.members[0]
    nsteps, seg = wl.nsteps, wl.meta["ckpt_every"]
    S = solver_for([m], precision, adj_segment_k=seg)
    S.autotune()
    dtype = S.dtype
    tgt = S.pack([np.load(path)])
    w0 = S.pack([m.omega0]).requires_grad_(True)
    c = torch.tensor([m.params["c"]], dtype=torch.float64, requires_grad=True)

    def loss_of(w, cc):
        wT = QGRollout.apply(w, cc, S, nsteps, seg)
        return torch.mean((wT - tgt) ** 2)

    L = loss_of(w0, c)
    L.backward()
    gw, gc = w0.grad.detach().clone(), c.grad.detach().clone()
    h = 1e-6 if precision == 64 else 1e-2
    worst = 0.0
    with torch.no_grad():
        for d in inputs.random_directions((256, 512), 16, wl.meta["fd_seed"]):
            dd = S.pack([d]).to(dtype)
            lp = loss_of(w0.detach() + h * dd, c.detach()).item()
            lm = loss_of(w0.detach() - h * dd, c.detach()).item()
            fd = (lp - lm) / (2 * h)
            ad = torch.sum(gw * dd).item()
            worst = max(worst, abs(ad - fd) / max(abs(fd), 1e-300))
        hc = 1e-6 if precision == 64 else 1e-3
        fdc = (loss_of(w0.detach(), c.detach() + hc).item() - loss_of(w0.detach(), c.detach() - hc).item()) / (2 * hc)
    errc = abs(gc.item() - fdc) / abs(fdc)
    say("C5", precision, "loss", L.item(), "worst direction rel err", worst, "dc", gc.item(), fdc, errc)
    if precision == 64:
        assert worst < 1e-6
        assert errc < 1e-6
    else:
        assert worst < 0.5 and errc < 0.5
    S.close()
