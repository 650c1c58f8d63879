"""GPU parity: the HIP path through the C ABI against the oracle on the same
seeded inputs, compared point by point.

Tolerances (per step, physical vorticity): 1e-12 in FP64 and 1e-5 in FP32,
as the method's accuracy targets state, applied both to the relative L2
norm of the difference and to the largest pointwise difference relative to
the largest value (``field_err``), so that a mistake confined to one point,
row or strip cannot hide in the norm.  Sizes span several column strips and
row blocks with ragged tails (kx counts that are not multiples of the strip
width).
"""
import itertools
import math

import numpy as np
import pytest

from oracle import qg
from paper_2508_06678_amd import configs, inputs
from tests.bridge import HAVE_GPU, oracle_model, field_err, max_rel, rel_l2, solver_for, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")]

TOL = {64: 1e-12, 32: 1e-5}


def say(*a):
    print(*a, flush=True)


def member(nx, ny, closure, seed=3, init="band", beta=1.5, u_in=1.0, c=None):
    lx, ly = 2 * math.pi, 2 * math.pi * ny / nx
    if init == "band":
        m = configs.island_member(nx, ny, precision=64, beta=beta, re=1e3, dt=1e-3, eta=5e-3,
                                  xc=1.5, radius=0.4, closure=closure, seed=seed, rms=0.2,
                                  lx=lx, ly=ly, u_in=u_in, c=c)
    else:
        m = configs.cape_member(nx, ny, precision=64, beta=beta, re=1e3, dt=1e-3, eta=5e-3,
                                height=0.5, closure=closure, seed=seed, rms=0.2, init="spectrum",
                                lx=lx, ly=ly, u_in=u_in, c=c)
    return m


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("nx,ny", [(64, 32), (128, 64), (32, 256), (512, 128)])
def test_entry_exit_projection(precision, nx, ny):
    say("entry/exit", precision, nx, ny)
    m = member(nx, ny, "none")
    S = solver_for([m], precision)
    rng = np.random.default_rng(1)
    w = rng.standard_normal((ny, nx))
    om = S.pack([w])
    S.step(om, 0, use_graph=False)
    M = oracle_model(m.params, m.chi, m.chi_s)
    ref = qg.leave(qg.enter(w, M.g), M.g)
    got = to_np(om).reshape(ny, nx)
    err = field_err(got, ref)
    say("  rel", err)
    assert err < (1e-14 if precision == 64 else 3e-7)
    S.close()


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("closure", ["none", "smag", "leith", "dsmag", "dleith"])
def test_one_step(precision, closure):
    say("one step", precision, closure)
    m = member(128, 64, closure, init="spectrum")
    S = solver_for([m], precision)
    M = oracle_model(m.params, m.chi, m.chi_s)
    w0 = m.omega0
    om = S.pack([w0])
    S.step(om, 1, use_graph=False)
    got = to_np(om).reshape(64, 128)
    w_in = to_np(S.pack([w0])).reshape(64, 128)   # the input as the GPU saw it
    ref = qg.step(w_in, M)
    err = field_err(got, ref)
    say("  rel", err)
    assert err < TOL[precision]
    S.close()


@pytest.mark.parametrize("precision", [64, 32])
def test_config1_per_step(precision):
    wl = configs.config1()
    m = wl.members[0]
    say("config1 per-step", precision)
    S = solver_for([m], precision)
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    worst = 0.0
    for n in range(5):
        w_n = to_np(om).reshape(64, 128)
        S.step(om, 1, use_graph=False)
        ref = qg.step(w_n, M)
        err = field_err(to_np(om).reshape(64, 128), ref)
        worst = max(worst, err)
    say("  worst", worst)
    assert worst < TOL[precision]
    S.close()


def test_graph_equals_eager_bitwise():
    m = member(128, 64, "dleith", init="spectrum")
    S = solver_for([m], 32)
    a = S.pack([m.omega0])
    b = a.clone()
    S.step(a, 23, use_graph=False)
    S.step(b, 23, use_graph=True)
    assert (a == b).all().item()
    S.close()


@pytest.mark.parametrize("count", [2, 5])
def test_one_group_in_two_branches(count):
    """A handle of one size group of two or five members: its graph runs
    the group as two halves (one and one, two and three members) on branches
    of their own, the eager steps as one chain of launches; the two agree
    bit for bit."""
    ms = [member(128, 64, "dleith", seed=s, init="spectrum") for s in range(11, 11 + count)]
    S = solver_for(ms, 32)
    a = S.pack([m.omega0 for m in ms])
    b = a.clone()
    S.step(a, 12, use_graph=False)
    S.step(b, 12, use_graph=True)
    assert (a == b).all().item()
    S.close()


def test_shared_penalization_tables(monkeypatch):
    """Members with equal masks (one device buffer each, as the binding
    passes them) read one member's B sub-step tables; the same members with
    a buffer of their own each read their own.  Both give the same bits."""
    from paper_2508_06678_amd import solver as solver_mod
    ms = [member(128, 64, "dleith", seed=s, init="spectrum") for s in (21, 22, 23)]
    assert all(np.array_equal(m.chi, ms[0].chi) and np.array_equal(m.chi_s, ms[0].chi_s) for m in ms)
    out = []
    for share in (True, False):
        if not share:
            monkeypatch.setattr(solver_mod, "_one_buffer_per_content", lambda ts: list(ts))
        S = solver_for(ms, 32)
        om = S.pack([m.omega0 for m in ms])
        S.step(om, 7, use_graph=False)
        out.append(om.clone())
        S.close()
    assert (out[0] == out[1]).all().item()


def test_batched_ragged_members():
    ms = [member(64, 32, "smag", seed=5), member(128, 64, "dleith", seed=6, init="spectrum"),
          member(64, 32, "leith", seed=7), member(256, 128, "dsmag", seed=8, init="spectrum"),
          member(128, 64, "none", seed=9)]
    S = solver_for(ms, 64)
    om = S.pack([m.omega0 for m in ms])
    w_in = [to_np(x) for x in S.unpack(om)]
    S.step(om, 2, use_graph=True)
    got = [to_np(x) for x in S.unpack(om)]
    for m, wi, g in zip(ms, w_in, got):
        M = oracle_model(m.params, m.chi, m.chi_s)
        ref = qg.run(wi, M, 2)
        err = field_err(g, ref)
        say("  member", m.params["nx"], m.params["ny"], m.params["closure"], err)
        assert err < 1e-12
    S.close()


@pytest.mark.parametrize("closure", ["smag", "dleith", "dsmag", "none"])
def test_diag(closure):
    m = member(128, 64, closure, init="spectrum")
    S = solver_for([m], 64)
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    out, nu = S.diag(om, want_nu=True)
    out = out.cpu().numpy()[0]
    w_in = to_np(om).reshape(64, 128)
    ref, nu_ref = qg.diag(w_in, M)
    say("diag", closure, out, ref)
    np.testing.assert_allclose(out[:2], ref[:2], rtol=1e-12)
    np.testing.assert_allclose(out[2], ref[2], rtol=1e-10, atol=1e-300)
    np.testing.assert_allclose(out[3:7], ref[3:7], rtol=1e-10, atol=1e-14)
    assert out[7] == 0.0
    assert field_err(to_np(nu).reshape(64, 128), nu_ref) < 1e-10 or np.all(nu_ref == 0)
    bad = om.clone()
    bad[17] = float("nan")
    out2, _ = S.diag(bad)
    assert out2.cpu().numpy()[0][7] == 1.0
    S.close()


@pytest.mark.parametrize("precision", [64, 32])
def test_every_strip_width(tmp_path, precision):
    """The strip widths of the column passes are tuning choices only: every
    admissible forward width W and inverse width Wi (forced through the
    tuning cache) gives the same step to the tolerance."""
    import json
    import torch
    nx, ny = 128, 512
    m = member(nx, ny, "dsmag", init="spectrum")
    M = oracle_model(m.params, m.chi, m.chi_s)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = f"{arch}/{nx}x{ny}/fp{precision}/closure3/members1"
    ref = None
    # admissible widths: one wave at least (W ny >= 512), one tile at most
    widths = [W for W in (1, 2, 4, 8, 16) if W * ny >= 512 and W * ny <= (2048 if precision == 64 else 4096)]
    combos = [(W, widths[-1 - i % len(widths)]) for i, W in enumerate(widths)]
    for W, Wi in combos:
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


@pytest.mark.parametrize("precision", [64, 32])
def test_oversized_dt_cfl_and_nonfinite_flag(precision):
    """Failure detection on the device: the island channel with 50 times its
    time step.  qg_diag's CFL agrees with the oracle's and exceeds 1 at the
    start; the run then grows without bound and the non-finite flag fires
    within 20 steps (the oracle's run blows up within 8)."""
    m = configs.config1().members[0]
    m.params["dt"] = 50 * m.params["dt"]
    S = solver_for([m], precision)
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    out = S.diag(om)[0].cpu().numpy()[0]
    ref, _ = qg.diag(to_np(om).reshape(64, 128), M)
    say("oversized dt", precision, "CFL", out[6], "oracle", ref[6])
    assert out[6] > 1.0 and out[7] == 0.0
    assert abs(out[6] - ref[6]) <= (1e-12 if precision == 64 else 1e-5) * ref[6]
    fired = None
    for n in range(1, 21):
        S.step(om, 1, use_graph=False)
        out = S.diag(om)[0].cpu().numpy()[0]
        say("  step", n, "CFL", out[6], "nonfinite", out[7])
        if out[7] == 1.0:
            fired = n
            break
    assert fired is not None
    S.close()


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("nx,ny,closure", [(1024, 512, "dleith"), (256, 1024, "dsmag")])
def test_every_tuning_choice(tmp_path, precision, nx, ny, closure):
    """Every combination of the tuner's choices for the compile-time engines
    -- row and column pass schedules (1024 = 8 8 8 2 or 8 4 4 8, 512 = 8 8 8
    or 8 4 4 4, 256 = 8 8 4 or 8 4 8; and 8 16 8 for the wave-synchronous
    1024-point rows), one or two row pairs per row block, one or four
    columns per inverse strip, block- or wave-synchronous row transforms --
    forced through the tuning cache, gives the oracle's step to the
    tolerance."""
    import json
    import torch
    m = member(nx, ny, closure, init="spectrum")
    M = oracle_model(m.params, m.chi, m.chi_s)
    code = {"dsmag": 3, "dleith": 4}[closure]
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = f"{arch}/{nx}x{ny}/fp{precision}/closure{code}/members1"
    ref = None
    wmax = min(4, (2048 if precision == 64 else 4096) // ny)   # widest inverse strip of one tile
    for rs, cs, rpb, Wi, wv in itertools.product((0, 1, 2), (0, 1), (1, 2), (1, wmax), (0, 1)):
        if rs == 2 and (wv == 0 or nx != 1024):
            continue
        choice = {"/fwd": 1, "/inv": Wi, "/rsched": rs, "/csched": cs, "/rpb": rpb, "/rwave": wv}
        cache = tmp_path / f"t{rs}{cs}{rpb}{Wi}{wv}.json"
        cache.write_text(json.dumps({key + k: v for k, v in choice.items()}))
        S = solver_for([m], precision)
        S.autotune(str(cache))
        assert S.tuning() == [{"W": 1, "Wi": Wi, "rsched": rs, "csched": cs, "rpb": rpb, "rwave": wv}]
        om = S.pack([m.omega0])
        w_in = to_np(om).reshape(ny, nx)
        S.step(om, 1, use_graph=True)
        if ref is None:
            ref = qg.step(w_in, M)
        err = field_err(to_np(om).reshape(ny, nx), ref)
        say("  rsched", rs, "csched", cs, "rpb", rpb, "Wi", Wi, "rwave", wv, err)
        assert err < TOL[precision]
        S.close()
