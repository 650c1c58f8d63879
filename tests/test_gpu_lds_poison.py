"""The LDS-poison debug build (libqg_ldspoison.so, QG_LDS_POISON): every
kernel sets its LDS to NaN before use and every transform pass poisons its
buffer before writing its outputs, so that a read of an LDS element nothing
has written -- a position a pass fails to write, a padding slot read by a
wrong index, or a read that runs ahead of the write it depends on -- carries
NaN into the result.  Each case runs the same input through the ordinary
library and the poisoned one: the poisoned result must be finite and equal
the ordinary one to the per-step tolerance (1e-12 FP64, 1e-5 FP32); in
practice the two agree bit for bit.  The cases cover every transform engine
(compile-time lengths 256..1024 under each pass schedule and row
synchronisation, the run-time single-vector and batched engines, rows of
4096 points), every kind of pass (right-hand side of each closure, B
sub-step, AB2CN's penalization and sponge, pointwise clip, diagnostics,
adjoint, SGS analysis) in both precisions.
"""
import json
import math

import numpy as np
import pytest

from paper_2508_06678_amd import configs, inputs
from paper_2508_06678_amd._lib import POISON_LIB_PATH
from tests.bridge import HAVE_GPU, field_err, solver_for, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")]

TOL = {64: 1e-12, 32: 1e-5}


def say(*a):
    print(*a, flush=True)


def island(nx, ny, closure, seed=3, clip=0, scheme="rk4"):
    lx, ly = 2 * math.pi, 2 * math.pi * ny / nx
    m = configs.island_member(nx, ny, precision=64, beta=1.5, re=1e3, dt=1e-4, eta=5e-3, xc=0.3 * lx,
                              radius=0.2 * min(lx, ly), closure=closure, seed=seed, rms=0.2, lx=lx, ly=ly)
    m.omega0 = inputs.spectrum_noise(nx, ny, lx, ly, seed, 2.0, 0.2)
    m.params["clip_mode"] = clip
    m.params["scheme"] = scheme
    if scheme == "ab2cn":
        m.params["eta"] = 2.5 * m.params["dt"]
    return m


def both(members, precision, run, tuning=None, tmp_path=None, adj=0):
    """run(S, om) -> list of arrays, on the ordinary and the poisoned
    library; returns the worst error of the poisoned results."""
    out = []
    for lib in (None, POISON_LIB_PATH):
        S = solver_for(members, precision, adj_segment_k=adj, lib_path=lib)
        if tuning is not None:
            import torch
            arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
            p = members[0].params
            code = {"none": 0, "smag": 1, "leith": 2, "dsmag": 3, "dleith": 4}[p["closure"]]
            key = f"{arch}/{p['nx']}x{p['ny']}/fp{precision}/closure{code}/members{len(members)}"
            cache = tmp_path / "tuning.json"
            cache.write_text(json.dumps({key + k: v for k, v in tuning.items()}))
            S.autotune(str(cache))
        om = S.pack([m.omega0 for m in members])
        out.append([to_np(x) for x in run(S, om)])
        S.close()
    worst = 0.0
    for a, b in zip(out[0], out[1]):
        assert np.all(np.isfinite(a)), "the case itself is not finite"
        assert np.all(np.isfinite(b)), "NaN from the poisoned LDS"
        worst = max(worst, field_err(b, a) if np.any(a) else float(np.max(np.abs(b))))
    bitwise = all(np.array_equal(a, b) for a, b in zip(out[0], out[1]))
    return worst, bitwise


def steps(n):
    def run(S, om):
        S.step(om, n, use_graph=False)
        return [om]
    return run


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("tuning", [
    {"/fwd": 1, "/inv": 4, "/rsched": 1, "/csched": 1, "/rpb": 1, "/rwave": 0},
    {"/fwd": 1, "/inv": 1, "/rsched": 0, "/csched": 0, "/rpb": 2, "/rwave": 1},
    {"/fwd": 2, "/inv": 2, "/rsched": 0, "/csched": 1, "/rpb": 1, "/rwave": 1},
    {"/fwd": 1, "/inv": 4, "/rsched": 2, "/csched": 1, "/rpb": 1, "/rwave": 1},
])
def test_compile_time_engines_dynamic_leith(tmp_path, precision, tuning):
    """1024 x 512 dynamic Leith (compile-time rows of 1024 and columns of
    512, grid and test levels, B sub-step) under four tunings."""
    say("poison 1024x512 dleith", precision, tuning)
    err, bit = both([island(1024, 512, "dleith")], precision, steps(2), tuning, tmp_path)
    say("  err", err, "bitwise", bit)
    assert err < TOL[precision]


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("rwave", [0, 1])
def test_columns_of_1024_dynamic_leith(tmp_path, precision, rwave):
    """512 x 1024 dynamic Leith: the two-half forward column pass over
    1024-point columns, block-synchronous or (FP32, rwave 1) one wave per
    transform with radix-16 passes."""
    tuning = {"/fwd": 1, "/inv": 2, "/rsched": 1, "/csched": 1, "/rpb": 1, "/rwave": rwave}
    say("poison 512x1024 dleith", precision, tuning)
    err, bit = both([island(512, 1024, "dleith")], precision, steps(2), tuning, tmp_path)
    say("  err", err, "bitwise", bit)
    assert err < TOL[precision]


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("nx,ny,closure", [(256, 256, "dsmag"), (128, 64, "smag"), (4096, 64, "leith"),
                                           (64, 1024, "none"), (32, 32, "dleith")])
def test_other_engines(precision, nx, ny, closure):
    """Compile-time 256, the run-time single-vector engines (128 x 64), rows
    of 4096 points (the field-looping row kernel), columns of 1024 with
    short rows, and the smallest grid."""
    say("poison", nx, ny, closure, precision)
    err, bit = both([island(nx, ny, closure)], precision, steps(2))
    say("  err", err, "bitwise", bit)
    assert err < TOL[precision]


@pytest.mark.parametrize("precision", [32, 64])
def test_ab2cn_and_pointwise_clip(precision):
    """AB2CN (penalization, right-hand side, sponge passes) with the
    pointwise clip (its two-field grid pass), three steps."""
    say("poison ab2cn clip", precision)
    err, bit = both([island(256, 128, "dsmag", clip=1, scheme="ab2cn")], precision, steps(3))
    say("  err", err, "bitwise", bit)
    assert err < TOL[precision]


def test_diagnostics_and_closure_term():
    def run(S, om):
        out, nu = S.diag(om, want_nu=True)
        return [out, nu, S.closure_term(om)]
    say("poison diag")
    err, bit = both([island(256, 128, "dleith", clip=1)], 64, run)
    say("  err", err, "bitwise", bit)
    assert err < TOL[64]


@pytest.mark.parametrize("closure", ["smag", "dleith"])
def test_adjoint(closure):
    """The adjoint sweep of a 3-step segment (its recompute, the reverse
    passes and, for the dynamic closure, the two-level passes)."""
    import torch

    def run(S, om):
        lam = S.pack([np.random.default_rng(9).standard_normal((64, 128))])
        g = torch.zeros(1, dtype=torch.float64, device=om.device)
        S.adjoint_step(om, lam, 3, g)
        return [lam, g]
    say("poison adjoint", closure)
    err, bit = both([island(128, 64, closure)], 64, run, adj=3)
    say("  err", err, "bitwise", bit)
    assert err < TOL[64]


@pytest.mark.parametrize("precision", [32, 64])
def test_sgs_analysis(precision):
    """Ideal SGS forcing, model term and PCC, FR 256^2 -> LES 128^2 (static
    Leith model: its term is nonzero, so the PCC is defined)."""
    from tests.bridge import solver_for as sf
    out = []
    for lib in (None, POISON_LIB_PATH):
        fr, les = configs.config3(precision=64, n=256), configs.config3(precision=64, n=128)
        for m in fr.members + les.members:
            m.params["closure"], m.params["c"] = "leith", 0.2
        F = sf(fr.members, precision, lib_path=lib)
        L = sf(les.members, precision, lib_path=lib)
        omf = F.pack([m.omega0 for m in fr.members])
        pi, model, wbar = F.ideal_sgs(L, omf)
        pcc = L.pcc(pi, model)
        out.append([to_np(pi), to_np(model), to_np(wbar), to_np(pcc)])
        F.close()
        L.close()
    worst = 0.0
    for a, b in zip(*out):
        assert np.all(np.isfinite(a)) and np.all(np.isfinite(b))
        worst = max(worst, field_err(b, a))
    say("poison sgs", precision, worst)
    assert worst < TOL[precision]
