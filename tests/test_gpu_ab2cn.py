"""GPU parity of the paper's own time scheme (AB2CN + AB2 sponge, Sec. II-E,
Eq. 4) against the oracle (oracle/ab2cn.py), which is pinned by
test_oracle_ab2cn.py.

The scheme carries history (previous explicit terms and omega**), so the GPU
and the oracle run the same sequence in lockstep from the same start and are
compared after every step (relative L2 of the physical vorticity): FP64 to
1e-12, FP32 to 1e-5 per step elapsed.
"""
import numpy as np
import pytest

from oracle import ab2cn, qg
from paper_2508_06678_amd import configs
from tests.bridge import HAVE_GPU, oracle_model, field_err, max_rel, rel_l2, solver_for, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")]


def say(*a):
    print(*a, flush=True)


def lockstep(S, m, precision, shape, nsteps, use_graph):
    M = oracle_model(m.params, m.chi, m.chi_s)
    om = S.pack([m.omega0])
    wh = qg.enter(to_np(om).reshape(shape), M.g)
    hist = None
    worst = 0.0
    for n in range(1, nsteps + 1):
        S.step(om, 1, use_graph=use_graph)
        wh, hist = ab2cn.step_spectral(wh, hist, M)
        err = field_err(to_np(om).reshape(shape), qg.leave(wh, M.g))
        worst = max(worst, err / n)
    return worst


@pytest.mark.parametrize("closure", ["none", "smag", "leith", "dsmag", "dleith"])
def test_island_fp64_every_step(closure):
    """128x64 island channel, 20 steps, every closure."""
    wl = configs.ab2cn_island(64, closure=closure)
    m = wl.members[0]
    S = solver_for([m], 64)
    worst = lockstep(S, m, 64, (64, 128), 20, use_graph=False)
    say("AB2CN", closure, "fp64 worst rel L2 per step", worst)
    assert worst < 1e-12
    S.close()


@pytest.mark.parametrize("closure", ["smag", "dleith"])
def test_island_fp32_512(closure):
    wl = configs.ab2cn_island(32, 512, 256, closure=closure, dt=5e-4)
    m = wl.members[0]
    S = solver_for([m], 32)
    S.autotune()
    worst = lockstep(S, m, 32, (256, 512), 4, use_graph=True)
    say("AB2CN", closure, "fp32 512x256 worst rel L2 per step", worst)
    assert worst < 1e-5
    S.close()


def test_history_carries_across_calls_and_graphs():
    """The history lives in the handle: 2 + 4 steps in two calls continue the
    sequence of 6 steps in one (equal up to the rounding of the exit/entry
    transforms between the calls); graph replay == eager, bit for bit."""
    m = configs.ab2cn_island(64, closure="dsmag").members[0]
    outs = {}
    for chunks, graph in (((6,), False), ((6,), True), ((2, 4), False), ((3, 3), True)):
        S = solver_for([m], 64)
        om = S.pack([m.omega0])
        for k in chunks:
            S.step(om, k, use_graph=graph)
        outs[(chunks, graph)] = to_np(om)
        S.close()
    ref = outs[((6,), False)]
    assert np.array_equal(outs[((6,), True)], ref)
    # a restart without the history would take a forward-Euler step: O(dt^2)
    # away, far above this bound
    for key in (((2, 4), False), ((3, 3), True)):
        err = field_err(outs[key], ref)
        say("AB2CN chunks", key, "rel L2 vs one call", err)
        assert err < 1e-13


def test_mixed_schemes_in_one_handle():
    """An RK4 and an AB2CN member launched together, each against its own oracle."""
    a = configs.config1(64).members[0]
    b = configs.ab2cn_island(64, closure="leith").members[0]
    S = solver_for([a, b], 64)
    om = S.pack([a.omega0, b.omega0])
    w_a, w_b = (to_np(x).reshape(64, 128) for x in S.unpack(om))
    S.step(om, 3, use_graph=True)
    got_a, got_b = (to_np(x).reshape(64, 128) for x in S.unpack(om))
    Ma = oracle_model(a.params, a.chi, a.chi_s)
    Mb = oracle_model(b.params, b.chi, b.chi_s)
    ea = field_err(got_a, qg.run(w_a, Ma, 3))
    eb = field_err(got_b, ab2cn.run(w_b, Mb, 3)[0])
    say("mixed handle: rk4", ea, "ab2cn", eb)
    assert ea < 1e-12 and eb < 1e-12
    S.close()


@pytest.mark.parametrize("closure,code", [("smag", 1), ("dsmag", 3)])
def test_every_column_width(closure, code, tmp_path):
    """Every strip width the tuner may choose, forced through its cache file:
    the widths whose product strips overflow the product-parallel column
    kernel (W ny = 4096 for three products, W ny >= 2048 for six) take the
    general one, which must carry the AB2CN update too."""
    import json

    import torch
    wl = configs.ab2cn_island(32, 512, 256, closure=closure, dt=5e-4)
    m = wl.members[0]
    M = oracle_model(m.params, m.chi, m.chi_s)
    nsteps = 3
    S0 = solver_for([m], 32)
    w0 = to_np(S0.pack([m.omega0])).reshape(256, 512)
    S0.close()
    wh, hist, refs = qg.enter(w0, M.g), None, []
    for _ in range(nsteps):
        wh, hist = ab2cn.step_spectral(wh, hist, M)
        refs.append(qg.leave(wh, M.g))
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = f"{arch}/512x256/fp32/closure{code}/members1"
    for W in (2, 4, 8, 16):
        path = tmp_path / f"w{W}.json"
        path.write_text(json.dumps({key + "/fwd": W, key + "/inv": 4}))
        S = solver_for([m], 32)
        S.autotune(str(path))
        assert S.column_widths() == [W]
        om = S.pack([m.omega0])
        worst = 0.0
        for n in range(1, nsteps + 1):
            S.step(om, 1, use_graph=False)
            worst = max(worst, field_err(to_np(om).reshape(256, 512), refs[n - 1]) / n)
        say("AB2CN", closure, "W", W, "worst rel L2 per step", worst)
        assert worst < 1e-5
        S.close()


@pytest.mark.parametrize("closure,code", [("smag", 1), ("dleith", 4)])
def test_compile_time_column_lengths(closure, code, tmp_path):
    """Columns of 512 points at one column per strip (forced through the
    tuning cache): AB2CN's penalization, right-hand-side and sponge passes
    then run the compile-time-length column engines.  Three steps in
    lockstep with the oracle, FP64."""
    import json

    import torch
    m = configs.island_member(128, 512, precision=64, beta=1.0, re=1e3, dt=5e-4, eta=1.25e-3, xc=1.5,
                              radius=0.5, closure=closure, seed=2, rms=0.2, lx=2 * np.pi, ly=8 * np.pi)
    m.params["scheme"] = "ab2cn"
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = f"{arch}/128x512/fp64/closure{code}/members1"
    path = tmp_path / "w1.json"
    path.write_text(json.dumps({key + "/fwd": 1, key + "/inv": 1}))
    S = solver_for([m], 64)
    S.autotune(str(path))
    assert S.column_widths() == [1] and S.inverse_widths() == [1]
    worst = lockstep(S, m, 64, (512, 128), 3, use_graph=False)
    say("AB2CN", closure, "compile-time columns, worst rel L2 per step", worst)
    assert worst < 1e-12
    S.close()
