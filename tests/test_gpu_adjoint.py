"""GPU discrete adjoint (qg_adjoint_step) against the oracle's adjoint and
against central finite differences of the GPU forward step, in FP64."""
import math

import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import qg
from paper_2508_06678_amd import configs, inputs
from tests.bridge import HAVE_GPU, oracle_model, field_err, max_rel, rel_l2, solver_for, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")]


def say(*a):
    print(*a, flush=True)


def island(nx, ny, closure, seed=4):
    return configs.island_member(nx, ny, precision=64, beta=1.5, re=500.0, dt=2e-3, eta=5e-3,
                                 xc=1.5, radius=0.5, closure=closure, seed=seed, rms=0.3,
                                 lx=2 * math.pi, ly=2 * math.pi * ny / nx)


@pytest.mark.parametrize("closure", ["none", "smag", "leith"])
@pytest.mark.parametrize("nx,ny", [(64, 32), (128, 64)])
def test_adjoint_matches_oracle(closure, nx, ny):
    say("adjoint vs oracle", closure, nx, ny)
    import torch
    m = island(nx, ny, closure)
    nsteps = 3
    S = solver_for([m], 64, adj_segment_k=nsteps)
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    w0 = to_np(om).reshape(ny, nx)
    rng = np.random.default_rng(9)
    lamT = rng.standard_normal((ny, nx))
    lam = S.pack([lamT])
    g = torch.zeros(1, dtype=torch.float64, device=om.device)
    S.adjoint_step(om, lam, nsteps, g)
    ref_l, ref_c = oadj.run_adjoint(w0, lamT, M, nsteps)
    err = field_err(to_np(lam).reshape(ny, nx), ref_l)
    say("  lambda rel", err, "dc", g.item(), ref_c)
    assert err < 1e-11
    if closure != "none":
        assert abs(g.item() - ref_c) <= 1e-10 * abs(ref_c)
    else:
        assert g.item() == 0.0
    S.close()


def test_adjoint_central_fd_on_gpu():
    import torch
    nx, ny = 128, 64
    m = island(nx, ny, "smag")
    nsteps = 4
    S = solver_for([m], 64, adj_segment_k=nsteps)
    om0 = S.pack([m.omega0])
    tgt = S.pack([inputs.bandpass_noise(nx, ny, 2 * math.pi, math.pi, 11, 2, 8, 0.3)])

    def loss(om):
        x = om.clone()
        S.step(x, nsteps, use_graph=False)
        return torch.mean((x - tgt) ** 2).item(), x

    L0, wT = loss(om0)
    lam = 2.0 * (wT - tgt) / wT.numel()
    g = torch.zeros(1, dtype=torch.float64, device=om0.device)
    S.adjoint_step(om0, lam, nsteps, g)
    h = 1e-4
    for d in inputs.random_directions((ny, nx), 3, 5):
        dd = S.pack([d])
        fd = (loss(om0 + h * dd)[0] - loss(om0 - h * dd)[0]) / (2 * h)
        ad = torch.sum(lam * dd).item()
        say("  fd", fd, "adjoint", ad)
        assert ad == pytest.approx(fd, rel=1e-6)
    S.close()


@pytest.mark.parametrize("closure,nx,ny,seed", [("dsmag", 64, 32, 4), ("dleith", 64, 32, 8),
                                                ("dsmag", 128, 64, 5), ("dleith", 128, 64, 5)])
def test_dynamic_adjoint_matches_oracle(closure, nx, ny, seed):
    """Dynamic closures: the stage coefficient's dependence on the stage
    input enters the adjoint.  The cases have every stage's <HM> clearly
    away from the clip (normalized correlation >= 2e-4), positive at every
    stage for the first two and clipped at some stages for the others."""
    say("dynamic adjoint vs oracle", closure, nx, ny, seed)
    import torch
    m = island(nx, ny, closure, seed=seed)
    nsteps = 3
    S = solver_for([m], 64, adj_segment_k=nsteps)
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    w0 = to_np(om).reshape(ny, nx)
    rng = np.random.default_rng(9)
    lamT = rng.standard_normal((ny, nx))
    lam = S.pack([lamT])
    g = torch.zeros(1, dtype=torch.float64, device=om.device)
    S.adjoint_step(om, lam, nsteps, g)
    ref_l, ref_c = oadj.run_adjoint(w0, lamT, M, nsteps)
    err = field_err(to_np(lam).reshape(ny, nx), ref_l)
    say("  lambda rel", err, "dc", g.item(), ref_c)
    assert err < 1e-11
    assert g.item() == 0.0 and ref_c == 0.0
    S.close()


def test_dynamic_adjoint_central_fd_on_gpu():
    """Dynamic Leith, 3 steps, every stage with C > 0: the GPU adjoint's
    directional derivatives against central differences of the GPU
    forward run."""
    import torch
    nx, ny = 64, 32
    m = island(nx, ny, "dleith", seed=8)
    nsteps = 3
    S = solver_for([m], 64, adj_segment_k=nsteps)
    om0 = S.pack([m.omega0])
    tgt = S.pack([inputs.bandpass_noise(nx, ny, 2 * math.pi, math.pi, 11, 2, 8, 0.3)])

    def loss(om):
        x = om.clone()
        S.step(x, nsteps, use_graph=False)
        return torch.mean((x - tgt) ** 2).item(), x

    L0, wT = loss(om0)
    lam = 2.0 * (wT - tgt) / wT.numel()
    g = torch.zeros(1, dtype=torch.float64, device=om0.device)
    S.adjoint_step(om0, lam, nsteps, g)
    h = 1e-4
    for d in inputs.random_directions((ny, nx), 3, 5):
        dd = S.pack([d])
        fd = (loss(om0 + h * dd)[0] - loss(om0 - h * dd)[0]) / (2 * h)
        ad = torch.sum(lam * dd).item()
        say("  fd", fd, "adjoint", ad)
        assert ad == pytest.approx(fd, rel=1e-6)
    S.close()


def test_dynamic_rollout_through_autograd():
    """torch.autograd over a dynamic-Leith rollout with two checkpointed
    segments: d loss/d omega0 against central differences; the coefficient
    has no c, so d loss/dc is 0."""
    import torch

    from paper_2508_06678_amd.autograd import QGRollout
    nx, ny = 64, 32
    m = island(nx, ny, "dleith", seed=8)
    seg, nsteps = 2, 4
    S = solver_for([m], 64, adj_segment_k=seg)
    w0 = S.pack([m.omega0]).requires_grad_(True)
    c = torch.tensor([0.0], dtype=torch.float64, requires_grad=True)
    tgt = S.pack([inputs.bandpass_noise(nx, ny, 2 * math.pi, math.pi, 11, 2, 8, 0.3)])

    def loss_of(w):
        return torch.mean((QGRollout.apply(w, c, S, nsteps, seg) - tgt) ** 2)

    L = loss_of(w0)
    L.backward()
    assert c.grad.item() == 0.0
    h = 1e-4
    for d in inputs.random_directions((ny, nx), 2, 7):
        dd = S.pack([d])
        with torch.no_grad():
            fd = (loss_of(w0 + h * dd).item() - loss_of(w0 - h * dd).item()) / (2 * h)
        ad = torch.sum(w0.grad * dd).item()
        say("  autograd fd", fd, "adjoint", ad)
        assert ad == pytest.approx(fd, rel=1e-6)
    S.close()


@pytest.mark.parametrize("closure,seed", [("dsmag", 4), ("dleith", 8)])
def test_dynamic_adjoint_fp32_vs_fp64(closure, seed):
    """The 32-bit dynamic adjoint against the 64-bit one (validated above)
    on the same rounded inputs, 3 steps of 64x32, to the 32-bit step's bar
    of 1e-5 relative (measured: 4e-7)."""
    import torch
    nx, ny = 64, 32
    m = island(nx, ny, closure, seed=seed)
    nsteps = 3
    lamT = np.random.default_rng(9).standard_normal((ny, nx))
    out = {}
    for prec in (64, 32):
        S = solver_for([m], prec, adj_segment_k=nsteps)
        om = S.pack([m.omega0.astype(np.float32).astype(np.float64)])
        lam = S.pack([lamT.astype(np.float32).astype(np.float64)])
        g = torch.zeros(1, dtype=torch.float64, device=om.device)
        S.adjoint_step(om, lam, nsteps, g)
        out[prec] = to_np(lam)
        S.close()
    err = rel_l2(out[32], out[64])
    say("dynamic adjoint fp32 vs fp64", closure, err)
    assert err < 1e-5


@pytest.mark.parametrize("closure,code", [("smag", 1), ("dleith", 4)])
@pytest.mark.parametrize("nx,ny", [(128, 512), (64, 1024)])
def test_adjoint_at_compile_time_column_lengths(closure, code, nx, ny, tmp_path):
    """Columns of 512 and 1024 points at one column per strip (forced
    through the tuning cache): the adjoint's column passes then run their
    compile-time-length engines.  Two steps against the oracle's adjoint.

    The initial field is broadband (k^-3 spectrum beyond |k| = 2): with the
    band-limited noise of the other cases, lying inside the test filter,
    <HM> vanishes identically at the first stage of this grid, which is the
    clip's kink (C = max(<HM>, 0)/<M^2>), whose derivative the adjoint does
    not define; the sign of rounding noise then decides it.  The oracle
    confirms every step starts well away from the kink."""
    import json
    import torch
    say("adjoint, compile-time columns", closure, nx, ny)
    m = island(nx, ny, closure, seed=5)
    m.omega0 = inputs.spectrum_noise(nx, ny, 2 * math.pi, 2 * math.pi * ny / nx, 7, 2.0, 0.3)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = f"{arch}/{nx}x{ny}/fp64/closure{code}/members1"
    cache = tmp_path / "w1.json"
    cache.write_text(json.dumps({key + "/fwd": 1, key + "/inv": 1}))
    nsteps = 2
    S = solver_for([m], 64, adj_segment_k=nsteps)
    S.autotune(str(cache))
    assert S.column_widths() == [1] and S.inverse_widths() == [1]
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    w0 = to_np(om).reshape(ny, nx)
    lamT = np.random.default_rng(9).standard_normal((ny, nx))
    lam = S.pack([lamT])
    g = torch.zeros(1, dtype=torch.float64, device=om.device)
    if closure == "dleith":
        w = w0
        for _ in range(nsteps):
            out = {}
            qg.rhs(qg.enter(w, M.g), M, out)
            assert abs(out["HM"]) > 1e-6, out["HM"]
            w = qg.step(w, M)
    S.adjoint_step(om, lam, nsteps, g)
    ref_l, ref_c = oadj.run_adjoint(w0, lamT, M, nsteps)
    err = field_err(to_np(lam).reshape(ny, nx), ref_l)
    say("  lambda rel", err, "dc", g.item(), ref_c)
    assert err < 1e-11
    if closure == "smag":
        assert abs(g.item() - ref_c) <= 1e-10 * abs(ref_c)
    S.close()


def test_adjoint_of_several_size_groups():
    """One handle with members of two sizes and three closures (three size
    groups, one graph branch each): every member's lambda and dL/dc against
    the oracle's adjoint of that member alone."""
    import torch
    ms = [island(128, 64, "smag", seed=4), island(64, 32, "leith", seed=5), island(128, 64, "smag", seed=6),
          island(64, 32, "dleith", seed=8)]
    nsteps = 2
    S = solver_for(ms, 64, adj_segment_k=nsteps)
    om = S.pack([m.omega0 for m in ms])
    w0 = [to_np(x) for x in S.unpack(om)]
    rng = np.random.default_rng(3)
    lamT = [rng.standard_normal((m.params["ny"], m.params["nx"])) for m in ms]
    lam = S.pack(lamT)
    g = torch.zeros(len(ms), dtype=torch.float64, device=om.device)
    S.adjoint_step(om, lam, nsteps, g)
    got = [to_np(x) for x in S.unpack(lam)]
    for i, m in enumerate(ms):
        M = oracle_model(m.params, m.chi, m.chi_s)
        ref_l, ref_c = oadj.run_adjoint(w0[i], lamT[i], M, nsteps)
        err = field_err(got[i], ref_l)
        say("  member", i, m.params["nx"], m.params["closure"], "lambda rel", err, "dc", g[i].item(), ref_c)
        assert err < 1e-11
        if m.params["closure"] in ("smag", "leith"):
            assert abs(g[i].item() - ref_c) <= 1e-10 * abs(ref_c)
        else:
            assert g[i].item() == 0.0
    S.close()


def test_adjoint_with_shared_penalization_tables(monkeypatch):
    """Three members on one geometry (one device buffer per mask, so they
    read one member's B sub-step tables) and the same members with masks of
    their own: the adjoint's lambda and dL/dc agree bit for bit."""
    import torch
    from paper_2508_06678_amd import solver as solver_mod
    nx, ny, nsteps = 128, 64, 3
    ms = [island(nx, ny, "smag", seed=s) for s in (4, 5, 6)]
    assert all(np.array_equal(m.chi, ms[0].chi) and np.array_equal(m.chi_s, ms[0].chi_s) for m in ms)
    rng = np.random.default_rng(12)
    lamT = [rng.standard_normal((ny, nx)) for _ in ms]
    out = []
    for share in (True, False):
        if not share:
            monkeypatch.setattr(solver_mod, "_one_buffer_per_content", lambda ts: list(ts))
        S = solver_for(ms, 64, adj_segment_k=nsteps)
        om = S.pack([m.omega0 for m in ms])
        lam = S.pack(lamT)
        g = torch.zeros(len(ms), dtype=torch.float64, device=om.device)
        S.adjoint_step(om, lam, nsteps, g)
        out.append((lam.clone(), g.clone()))
        S.close()
    assert (out[0][0] == out[1][0]).all().item()
    assert (out[0][1] == out[1][1]).all().item()
