"""The C ABI without Python: the C99 program paper_2508_06678_amd/qg_example
(built beside libqg.so) allocates with hipMalloc, runs 20 RK4 steps of the
128x64 island channel through qg_init / qg_step / qg_diag and writes its
inputs and result.  The same inputs through the Python binding must give
the same field bit for bit (same library, same launches), and the oracle's
20 steps agree to the 64-bit bar."""
import math
import os
import subprocess

import numpy as np
import pytest

from oracle import qg
from tests.bridge import HAVE_GPU, oracle_model, field_err, max_rel, rel_l2, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")]

PKG = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2508_06678_amd")
PARAMS = dict(nx=128, ny=64, lx=2 * math.pi, ly=math.pi, beta=1.0, re=1000.0, mu=0.0, u_in=1.0, v_in=0.0,
              eta=1e-3, sponge_sigma=10.0, dt=2e-3, c=0.17, closure="smag", precision=64, test_ratio=2,
              clip_mode=0, fp64_lowk=8, scheme="rk4")


def test_c_program_matches_binding_and_oracle(tmp_path):
    exe = os.path.join(PKG, "qg_example")
    assert os.path.exists(exe), "qg_example is built with the library"
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0
    rd = lambda n: np.fromfile(tmp_path / f"{n}.f64", dtype=np.float64).reshape(64, 128)  # noqa: E731
    chi, chs, w0, w20 = rd("chi"), rd("chi_s"), rd("omega0"), rd("omega20")
    from paper_2508_06678_amd.solver import Solver
    S = Solver([PARAMS], [chi], [chs])
    om = S.pack([w0])
    S.step(om, 20)
    got = to_np(om).reshape(64, 128)
    S.close()
    assert np.array_equal(got, w20)
    M = oracle_model(PARAMS, chi, chs)
    ref = qg.run(w0, M, 20)
    err = field_err(w20, ref)
    print("C program vs oracle, 20 steps:", err, flush=True)
    assert err < 20 * 1e-12
