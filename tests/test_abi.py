"""C ABI checks that need no GPU: the library loads, exports every function
include/qg.h declares, and rejects invalid parameters with the documented
status codes (qg_workspace_bytes validates exactly as qg_init does)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2508_06678_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "qg.h")) as f:
        txt = f.read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qg_[a-z_]+)\s*\(", txt)))


@pytest.mark.parametrize("path", [None, _lib.POISON_LIB_PATH, _lib.STAMPS_LIB_PATH],
                         ids=["libqg", "libqg_ldspoison", "libqg_stamps"])
def test_every_declared_symbol_is_exported(path):
    """The library and its debug builds (LDS poison, phase stamps) load and
    export every function include/qg.h declares."""
    L = _lib.lib(path)
    names = declared_functions()
    assert {"qg_workspace_bytes", "qg_init", "qg_step", "qg_adjoint_step", "qg_diag"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTS)


def good(**kw):
    d = dict(nx=128, ny=64, lx=2 * math.pi, ly=math.pi, beta=1.0, re=1e3, mu=0.0, u_in=1.0,
             v_in=0.0, eta=1e-3, sponge_sigma=10.0, dt=2e-3, c=0.17, closure="smag",
             precision=64, test_ratio=2, clip_mode=0, fp64_lowk=8)
    d.update(kw)
    return d


def ws(params, adj=0):
    L = _lib.lib()
    arr = (_lib.QGParams * len(params))(*[_lib.make_params(p) for p in params])
    size = ctypes.c_size_t(0)
    rc = L.qg_workspace_bytes(arr, len(params), adj, ctypes.byref(size))
    return rc, size.value


def test_ab2cn_workspace_holds_its_history():
    rc, b_rk4 = ws([good()])
    rc2, b_ab = ws([good(scheme="ab2cn", eta=5e-3)])
    assert rc == 0 and rc2 == 0 and b_ab > b_rk4


def test_workspace_bytes_valid_and_monotone():
    rc, b1 = ws([good()])
    assert rc == 0 and b1 > 0
    rc, b2 = ws([good(), good(nx=256, ny=128, closure="dleith")])
    assert rc == 0 and b2 > b1
    rc, b3 = ws([good()], adj=50)
    assert rc == 0 and b3 > b1
    rc, b4 = ws([good(precision=32)])
    assert rc == 0 and b4 < b1
    # the pointwise clip keeps the H and M spectra of a stage
    rc, b5 = ws([good(closure="dsmag")])
    rc6, b6 = ws([good(closure="dsmag", clip_mode=1)])
    assert rc == 0 and rc6 == 0 and b6 > b5


@pytest.mark.parametrize("bad,code", [
    (dict(nx=96), _lib.QG_EUNSUPPORTED),
    (dict(nx=16, ny=16, lx=2 * math.pi, ly=2 * math.pi), _lib.QG_EUNSUPPORTED),
    (dict(ly=2.0), _lib.QG_EUNSUPPORTED),
    (dict(dt=0.0), _lib.QG_EINVAL),
    (dict(dt=-1.0), _lib.QG_EINVAL),
    (dict(closure=7), _lib.QG_EINVAL),
    (dict(precision=16), _lib.QG_EINVAL),
    (dict(clip_mode=1, closure="dsmag", nx=32, ny=32, lx=2 * math.pi, ly=2 * math.pi), _lib.QG_EUNSUPPORTED),
    (dict(clip_mode=1, closure="dleith", nx=4096, ny=2048), _lib.QG_EUNSUPPORTED),
    (dict(clip_mode=2), _lib.QG_EINVAL),
    (dict(closure="dsmag", test_ratio=2.5), _lib.QG_EUNSUPPORTED),
    (dict(eta=0.0), _lib.QG_EINVAL),
    (dict(eta=-1.0), _lib.QG_EINVAL),
    (dict(beta=float("nan")), _lib.QG_EINVAL),
    (dict(sponge_sigma=-1.0), _lib.QG_EINVAL),
    (dict(scheme=2), _lib.QG_EINVAL),
    (dict(scheme="ab2cn", nx=32, ny=32, lx=2 * math.pi, ly=2 * math.pi), _lib.QG_EUNSUPPORTED),
    (dict(scheme="ab2cn", nx=4096, ny=2048, lx=2 * math.pi, ly=math.pi), _lib.QG_EUNSUPPORTED),
    # explicit penalization of the paper's scheme needs eta > dt (Sec. II-E)
    (dict(scheme="ab2cn", eta=2e-3, dt=2e-3), _lib.QG_EINVAL),
    (dict(scheme="ab2cn", eta=1e-3, dt=2e-3), _lib.QG_EINVAL),
])
def test_invalid_parameters_are_rejected(bad, code):
    rc, _ = ws([good(**bad)])
    assert rc == code
    msg = _lib.lib().qg_last_error().decode()
    assert msg.startswith("member 0")


def test_null_arguments():
    L = _lib.lib()
    assert L.qg_workspace_bytes(None, 1, 0, None) == _lib.QG_EINVAL
    rc, _ = ws([])
    assert rc == _lib.QG_EINVAL
    h = ctypes.c_void_p()
    assert L.qg_init(None, 0, None, None, None, 0, 0, None, ctypes.byref(h)) == _lib.QG_EINVAL
    assert L.qg_step(None, None, 1, 0, None, 1, None) == _lib.QG_EINVAL
    assert L.qg_diag(None, None, None, None, None) == _lib.QG_EINVAL
    assert L.qg_adjoint_step(None, None, None, 1, None, None) == _lib.QG_EINVAL
    assert L.qg_filter_les(None, None, None, None, None) == _lib.QG_EINVAL
    assert L.qg_ideal_sgs(None, None, None, None, None, None, None) == _lib.QG_EINVAL
    assert L.qg_pcc(None, None, None, None, None) == _lib.QG_EINVAL
    assert L.qg_closure_term(None, None, None, None) == _lib.QG_EINVAL
    assert L.qg_profile_steps(None, None, 1, 0, None, 0, None, None) == _lib.QG_EINVAL
    assert L.qg_step_noalloc(None, None, None, None, 1, None) == _lib.QG_EINVAL
    # the stamp run exists in the stamp build only
    assert L.qg_stamp_steps(None, None, 1, None, 0, None) == _lib.QG_EUNSUPPORTED
    S = _lib.lib(_lib.STAMPS_LIB_PATH)
    assert S.qg_stamp_steps(None, None, 1, None, 0, None) == _lib.QG_EINVAL
    L.qg_destroy(None)


def test_init_rejects_small_or_missing_workspace():
    L = _lib.lib()
    params = [good()]
    arr = (_lib.QGParams * 1)(*[_lib.make_params(p) for p in params])
    dummy = (ctypes.c_void_p * 1)(ctypes.c_void_p(256))
    h = ctypes.c_void_p()
    assert L.qg_init(arr, 1, dummy, dummy, None, 1 << 20, 0, None, ctypes.byref(h)) == _lib.QG_EWORKSPACE
    assert L.qg_init(arr, 1, dummy, dummy, ctypes.c_void_p(4096), 16, 0, None, ctypes.byref(h)) == _lib.QG_EWORKSPACE
    assert L.qg_init(arr, 1, dummy, dummy, ctypes.c_void_p(4097), 1 << 40, 0, None, ctypes.byref(h)) == _lib.QG_EWORKSPACE


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library the product path raises: there is no
    CPU fallback to take its place."""
    monkeypatch.setattr(_lib, "_libs", {})
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libqg.so"))
    with pytest.raises(ImportError, match="missing"):
        _lib.lib()
    from paper_2508_06678_amd.solver import Solver
    m = good()
    chi = np.zeros((m["ny"], m["nx"]))
    with pytest.raises(ImportError, match="missing"):
        Solver([m], [chi], [chi], device="cpu")


def test_stamp_report_from_synthetic_stamps():
    """The stamp report's host logic on hand-made stamps: two waves of the
    row pass on one SIMD, phases of 1..5 ticks."""
    from paper_2508_06678_amd import stamps
    st = np.zeros((4, 8192, 8), dtype=np.uint64)
    for w, base in ((0, 100), (1, 103)):
        st[0, w, :6] = base + np.cumsum([0, 1, 2, 3, 4, 5])
        st[0, w, 7] = (np.uint64(2) << np.uint64(32)) | np.uint64(0x0123)   # XCC 2, CU 1, SIMD 2
    t, hw = stamps.waves_of(st, 0)
    assert t.shape == (2, 6)
    xcc, cu, simd = stamps.placement(hw)
    assert set(xcc.tolist()) == {2} and len(set(simd.tolist())) == 1
    text = stamps.report(st, "synthetic")
    assert "2 waves, span 0.18 us" in text      # (103 + 15) - 100 ticks of 10 ns
    assert "column-inverse pass: no stamps" in text
