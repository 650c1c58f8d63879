"""Host logic of the island set-up (Sec. IV-A) and of the a-priori analysis:
the constants the paper states, the four-sided sponge ramp and the region
of interest.  CPU only."""
import math

import numpy as np

from paper_2508_06678_amd import experiments, inputs


def test_island_constants_follow_the_paper():
    fr = experiments.island_fr(256, 64, dt=1e-4)
    p = fr.params
    assert p["lx"] == p["ly"] == 8 * math.pi
    assert p["re"] == 200.0 and p["beta"] == 0.0 and p["u_in"] == 2.0
    assert p["eta"] == 1.025e-4 and abs(p["sponge_sigma"] * p["eta"] - 1.0) < 1e-15   # eta_sponge = eta
    assert p["scheme"] == "ab2cn" and p["closure"] == "none"
    # island of diameter 2 pi/5 centred 0.35 Lx, mid-channel: chi = 1/2 on its edge
    dx = p["lx"] / 256
    x = np.arange(256) * dx
    row = fr.chi[128]
    inside = x[row > 0.5]
    assert abs(inside.mean() - 0.35 * p["lx"]) < dx
    assert abs((inside.max() - inside.min() + dx) - 2 * math.pi / 5) < 2 * dx
    # sponge: 1 on every edge, 0 beyond 0.05 Lx
    s = fr.chi_s
    assert s[0, 128] == 1.0 and s[128, 0] == 1.0 and s[128, 128] == 0.0
    w = 0.05 * p["lx"]
    assert np.all(s[128][(x > w) & (x < p["lx"] - w)] == 0.0)
    les = experiments.les_params(p, 2, "dleith")
    assert les["nx"] == 128 and les["closure"] == "dleith" and les["eta"] == p["eta"]


def test_four_sided_sponge_is_the_distance_ramp():
    s = inputs.sponge_mask(64, 32, 2.0, 1.0, thickness=0.25, sides="xy")
    X, Y = inputs.grid_xy(64, 32, 2.0, 1.0)
    d = np.minimum(np.minimum(X, 2.0 - X), np.minimum(Y, 1.0 - Y))
    assert np.allclose(s, np.maximum(0.0, 1.0 - d / 0.25), atol=0, rtol=0)
    sx = inputs.sponge_mask(64, 32, 2.0, 1.0, thickness=0.25)
    assert np.all(sx[:, 32] == 0.0) and np.all(sx[:, 0] == 1.0)


def test_region_of_interest_excludes_sponge_and_filter_width():
    lx = 8 * math.pi
    roi = experiments.region_of_interest(128, lx, 0.05 * lx, 2 * lx / 256)
    roi2 = experiments.region_of_interest(128, lx, 0.125 * lx, 2 * lx / 256, 0.1 * lx)
    x2 = np.arange(128) * lx / 128
    assert np.array_equal(roi2[64], (x2 >= 0.125 * lx + lx / 128) & (x2 <= lx - 0.125 * lx - lx / 128))
    assert np.array_equal(roi2[:, 64], (x2 >= 0.1 * lx + lx / 128) & (x2 <= lx - 0.1 * lx - lx / 128))
    x = np.arange(128) * lx / 128
    edge = 0.05 * lx + 2 * lx / 256
    assert roi.shape == (128, 128)
    assert np.array_equal(roi[64], (x >= edge) & (x <= lx - edge))
    assert np.array_equal(roi[:, 64], roi[64])


def test_cape_set_up():
    fr = experiments.cape_fr(256, 64, dt=1e-4, beta=0.1)
    p = fr.params
    assert p["beta"] == 0.1 and p["scheme"] == "ab2cn" and p["u_in"] == 2.0
    lx = p["lx"]
    dx = lx / 256
    x = np.arange(256) * dx
    ic = int(round(0.2 * lx / dx))
    col = fr.chi[:, ic]
    y = np.arange(256) * dx
    land = y[col > 0.5]
    assert abs(land.max() - 4.0) < 2 * dx          # the cape's tip: height 4 at x = 0.2 Lx
    assert land.min() < 3 * 2 * dx                 # land starts at the southern edge
    far = fr.chi[:, int(round(0.7 * lx / dx))]
    assert far.max() < 0.5                         # no land far from the cape
    # sponge: 0.125 Lx along the x edges, 0.1 Lx along the y edges
    s = fr.chi_s
    assert s[128, int(0.12 * lx / dx)] > 0.0 and s[128, int(0.13 * lx / dx) + 1] == 0.0
    assert s[int(0.09 * lx / dx), 128] > 0.0 and s[int(0.11 * lx / dx) + 1, 128] == 0.0


def test_phase_shift_recovers_a_known_lag():
    """omega_LES(t) = omega_FF(t + 3 dt_s): the argmin of
    ||omega_LES(t - phi) - omega_FF(t)|| is phi = 3 dt_s."""
    import torch
    rng = np.random.default_rng(0)
    n, pts, dts = 60, 50, 0.5
    base = torch.as_tensor(np.cumsum(rng.standard_normal((n + 10, pts)), axis=0))
    ff = base[:n]
    les = base[3:n + 3]
    times = [dts * (i + 1) for i in range(n)]
    assert experiments.phase_shift(les, ff, times, 5.0, 8) == 3 * dts
    assert experiments.phase_shift(ff, ff, times, 5.0, 8) == 0.0
    assert experiments.phase_shift(ff, les, times, 5.0, 8) == -3 * dts


def test_les_run_params_keep_the_eta_rule():
    fr = experiments.island_fr(256, 64, dt=1e-4)
    p = experiments.les_run_params(fr.params, 2, "smag", 1e-3)
    assert p["nx"] == 128 and p["dt"] == 1e-3 and p["scheme"] == "ab2cn"
    assert abs(p["eta"] - 1.025e-3) < 1e-18 and abs(p["sponge_sigma"] * p["eta"] - 1.0) < 1e-15
    assert p["closure"] == "smag" and p["c"] == 0.17


def test_closure_specs():
    assert experiments.parse_closure("smag") == ("smag", 0.17)
    assert experiments.parse_closure("leith:0.15") == ("leith", 0.15)
    fr = experiments.island_fr(256, 64)
    assert experiments.les_run_params(fr.params, 2, "smag:0.3", 1e-3)["c"] == 0.3
    import pytest
    with pytest.raises(ValueError):
        experiments.parse_closure("smagorinsky")
