"""The allocation-free entry point qg_step_noalloc (one member, the library's
static device workspace) against qg_step of a handle on the same input, on
two calls in a row (the second with a smaller grid, so the array's earlier
contents must not leak into it), in both precisions, to the per-step
tolerances; members too large for the array are refused."""
import math

import pytest

from paper_2508_06678_amd import configs
from tests.bridge import HAVE_GPU, field_err, max_rel, rel_l2, solver_for, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")]

TOL = {64: 1e-12, 32: 1e-5}


def say(*a):
    print(*a, flush=True)


def member(nx, ny, closure, seed):
    lx, ly = 2 * math.pi, 2 * math.pi * ny / nx
    return configs.cape_member(nx, ny, precision=64, beta=1.5, re=1e3, dt=1e-3, eta=5e-3, height=0.5,
                               closure=closure, seed=seed, rms=0.2, init="spectrum", lx=lx, ly=ly)


def device_field(a, precision):
    import torch
    dt = torch.float64 if precision == 64 else torch.float32
    return torch.tensor(a, dtype=dt, device="cuda").contiguous().reshape(-1)


@pytest.mark.parametrize("precision", [64, 32])
def test_noalloc_matches_qg_step_on_two_calls(precision):
    import torch
    from paper_2508_06678_amd.solver import step_noalloc
    cases = [(member(512, 256, "dleith", 4), 3), (member(128, 64, "smag", 5), 2)]
    for m, n in cases:
        nx, ny = m.params["nx"], m.params["ny"]
        S = solver_for([m], precision)
        ref = S.pack([m.omega0])
        om = ref.clone()
        S.step(ref, n, use_graph=False)
        params = dict(m.params, precision=precision)
        say("noalloc", precision, nx, ny, m.params["closure"], n, "steps")
        step_noalloc(params, device_field(m.chi, precision), device_field(m.chi_s, precision), om, n)
        torch.cuda.synchronize()
        got, want = to_np(om).reshape(ny, nx), to_np(ref).reshape(ny, nx)
        err = field_err(got, want)
        say("  rel L2", rel_l2(got, want), "max-norm rel", max_rel(got, want))
        assert err < TOL[precision]
        S.close()


def test_noalloc_refuses_members_beyond_the_array():
    from paper_2508_06678_amd import _lib
    from paper_2508_06678_amd.solver import step_noalloc
    m = member(1024, 1024, "dleith", 6)
    params = dict(m.params, precision=32)
    om = device_field(m.omega0, 32)
    with pytest.raises(_lib.QGError) as e:
        step_noalloc(params, device_field(m.chi, 32), device_field(m.chi_s, 32), om, 1)
    assert e.value.code == _lib.QG_EUNSUPPORTED and "static scratch" in str(e.value)
