"""The phase-stamp debug build (libqg_stamps.so, QG_STAMPS): its stamp run
computes the same steps as the ordinary library (the stamps only read a
counter and write to the caller's buffer), and every wave of the four
right-hand-side kernels records its phases in order, for a wave count that
matches the kernel's grid."""
import math

import numpy as np
import pytest

from paper_2508_06678_amd import configs, inputs, stamps
from paper_2508_06678_amd._lib import STAMPS_LIB_PATH
from tests.bridge import HAVE_GPU, solver_for, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")]


def say(*a):
    print(*a, flush=True)


def cape(n, closure="dleith", seed=4):
    m = configs.cape_member(n, n, precision=32, beta=5.0, re=2e4, dt=2.5e-4, eta=1e-4, height=0.6,
                            closure=closure, seed=seed, rms=0.1, init="spectrum", lx=2 * math.pi,
                            ly=2 * math.pi)
    m.omega0 = inputs.spectrum_noise(n, n, 2 * math.pi, 2 * math.pi, seed, 2.0, 0.3)
    return m


@pytest.mark.parametrize("n", [256, 1024])
def test_stamp_run_equals_the_ordinary_step_and_stamps_are_ordered(n):
    say(f"stamps: FP32 {n}x{n} dynamic Leith, 2 steps")
    m = cape(n)
    S = solver_for([m], 32)
    om = S.pack([m.omega0])
    S.step(om, 2, use_graph=False)
    ref = to_np(om)
    S.close()
    T = solver_for([m], 32, lib_path=STAMPS_LIB_PATH)
    om2 = T.pack([m.omega0])
    st = T.stamp_steps(om2, 2)
    got = to_np(om2)
    assert np.array_equal(got, ref)
    for kind, (name, labels) in stamps.KINDS.items():
        t, hw = stamps.waves_of(st, kind)
        # the column-forward pass is stamped on its one-column path only
        # (strip width 1, the tuner's choice at 1024; the default width at
        # 256 is wider)
        if kind == 2 and T.column_widths()[0] != 1:
            assert len(t) == 0
            continue
        assert len(t) > 0, name
        assert np.all(np.diff(t, axis=1) >= 0), name
        # every wave sits on one of the eight XCDs, and spans under a second
        assert np.all(((hw >> 32) & 0xf) < 8), name
        assert (t[:, -1] - t[:, 0]).max() < 100_000_000, name
    # the row pass stamps every wave of its grid: one block per row pair and
    # level, 1024 threads' worth of transforms per block at most
    t_row, _ = stamps.waves_of(st, 0)
    assert len(t_row) % (n // 2 * 2) == 0
    text = stamps.report(st, "test")
    assert "row pass" in text and "combine" in text
    T.close()
