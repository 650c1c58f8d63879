"""Python front end of libqg.so: device memory and streams from torch, every
step of the computation in the HIP library.

``Solver`` holds one handle for a batch of members (one or many grids).
Fields are passed as flat device tensors (all members concatenated, each
row-major (ny, nx)), or as lists of (ny, nx) tensors via ``pack``/``unpack``.
"""
import ctypes

import numpy as np
import torch

from . import _lib

_DTYPES = {32: torch.float32, 64: torch.float64}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Solver:
    """A batch of QG members on one GPU (see include/qg.h for the semantics)."""

    def __init__(self, params, chi, chi_sponge, device="cuda:0", adj_segment_k=0, lib_path=None):
        if isinstance(params, dict):
            params, chi, chi_sponge = [params], [chi], [chi_sponge]
        self.L = _lib.lib(lib_path)
        self.device = torch.device(device)
        self.params = [dict(p) for p in params]
        precs = {int(p.get("precision", 64)) for p in self.params}
        if len(precs) != 1:
            raise ValueError("the Python front end takes one precision per Solver")
        self.precision = precs.pop()
        self.dtype = _DTYPES[self.precision]
        self.n = len(self.params)
        self.shapes = [(int(p["ny"]), int(p["nx"])) for p in self.params]
        self.sizes = [a * b for a, b in self.shapes]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self.total = int(self.offsets[-1])
        arr = (_lib.QGParams * self.n)(*[_lib.make_params(p) for p in self.params])
        self._arr = arr
        size = ctypes.c_size_t()
        self._check(self.L.qg_workspace_bytes(arr, self.n, int(adj_segment_k), ctypes.byref(size)))
        self.ws_bytes = size.value
        raw = torch.empty(size.value + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self.ws = raw[off:off + size.value]
        # members with equal masks get the same device buffers: qg_init
        # then lets them read one copy of the B sub-step's tables
        masks = _one_buffer_per_content([self._dev(c) for c in chi])
        smasks = _one_buffer_per_content([self._dev(c) for c in chi_sponge])
        cp = (ctypes.c_void_p * self.n)(*[m.data_ptr() for m in masks])
        sp = (ctypes.c_void_p * self.n)(*[m.data_ptr() for m in smasks])
        h = ctypes.c_void_p()
        self._check(self.L.qg_init(arr, self.n, cp, sp, _ptr(self.ws), self.ws_bytes,
                                  int(adj_segment_k), _stream(self.device), ctypes.byref(h)))
        self.h = h
        self.adj_segment_k = int(adj_segment_k)

    def _check(self, rc):
        _lib.check(rc, self.L)

    # -------------------------------------------------------------- fields
    def _dev(self, a):
        if isinstance(a, torch.Tensor):
            return a.to(device=self.device, dtype=self.dtype).contiguous()
        return torch.as_tensor(np.asarray(a), dtype=self.dtype, device=self.device).contiguous()

    def pack(self, fields):
        """List of (ny, nx) arrays/tensors -> flat device tensor."""
        return torch.cat([self._dev(f).reshape(-1) for f in fields])

    def unpack(self, flat):
        return [flat[self.offsets[i]:self.offsets[i + 1]].view(*self.shapes[i]) for i in range(self.n)]

    def _check_flat(self, t, name):
        if not isinstance(t, torch.Tensor) or t.dtype != self.dtype or t.device != self.device:
            raise TypeError(f"{name} must be a {self.dtype} tensor on {self.device}")
        if not t.is_contiguous() or t.numel() < self.total:
            raise ValueError(f"{name} must be contiguous with {self.total} elements")

    # -------------------------------------------------------------- calls
    def step(self, omega, nsteps, save_every=0, ckpt=None, use_graph=True):
        """Advance in place; returns omega.  ckpt: flat tensor of
        (nsteps // save_every) * total elements when save_every > 0."""
        self._check_flat(omega, "omega")
        cptr = None
        if save_every:
            nsave = nsteps // save_every
            if ckpt is None:
                ckpt = torch.empty(max(nsave, 1) * self.total, dtype=self.dtype, device=self.device)
            self._check_flat(ckpt, "ckpt")
            if ckpt.numel() < nsave * self.total:
                raise ValueError("ckpt too small")
            cptr = _ptr(ckpt)
        self._check(self.L.qg_step(self.h, _ptr(omega), int(nsteps), int(save_every), cptr,
                                  1 if use_graph else 0, _stream(self.device)))
        return (omega, ckpt) if save_every else omega

    def adjoint_step(self, omega_ckpt, lam, nsteps, grad_c):
        """lam: dL/d omega at the segment end -> at the segment start (in place);
        grad_c: float64 device tensor (n,), dL/dc added."""
        self._check_flat(omega_ckpt, "omega_ckpt")
        self._check_flat(lam, "lambda")
        if grad_c.dtype != torch.float64 or grad_c.device != self.device or grad_c.numel() < self.n:
            raise TypeError("grad_c must be a float64 device tensor with one entry per member")
        self._check(self.L.qg_adjoint_step(self.h, _ptr(omega_ckpt), _ptr(lam), int(nsteps),
                                          _ptr(grad_c), _stream(self.device)))
        return lam

    def diag(self, omega, want_nu=False):
        """Returns (n, 8) float64 [E, Z, C, nu_min, nu_mean, nu_max, CFL, nonfinite]
        and, if asked, the flat nu_e field."""
        self._check_flat(omega, "omega")
        out = torch.zeros(self.n * 8, dtype=torch.float64, device=self.device)
        nu = torch.empty(self.total, dtype=self.dtype, device=self.device) if want_nu else None
        self._check(self.L.qg_diag(self.h, _ptr(omega), _ptr(out),
                                  _ptr(nu) if nu is not None else None, _stream(self.device)))
        return out.view(self.n, 8), nu

    def filter_les(self, les, omega_fr):
        """H_full of every member's fully-resolved field onto the grids of
        the solver `les` (same members, coarsened grids).  Returns the flat
        filtered fields in `les`'s layout."""
        self._check_flat(omega_fr, "omega_fr")
        out = torch.empty(les.total, dtype=les.dtype, device=les.device)
        self._check(self.L.qg_filter_les(self.h, les.h, _ptr(omega_fr), _ptr(out), _stream(self.device)))
        return out

    def ideal_sgs(self, les, omega_fr, model=True, bar=True):
        """Ideal SGS forcing of every member pair (this solver: the
        fully-resolved grids, `les`: the coarsened ones) at the FR fields
        omega_fr.  Returns (pi_ff, pi_model or None, omega_bar or None), flat
        fields in `les`'s layout."""
        self._check_flat(omega_fr, "omega_fr")
        new = lambda: torch.empty(les.total, dtype=les.dtype, device=les.device)
        pi_ff = new()
        pi_m = new() if model else None
        wbar = new() if bar else None
        self._check(self.L.qg_ideal_sgs(self.h, les.h, _ptr(omega_fr), _ptr(pi_ff),
                                       _ptr(pi_m) if pi_m is not None else None,
                                       _ptr(wbar) if wbar is not None else None, _stream(self.device)))
        return pi_ff, pi_m, wbar

    def closure_term(self, omega):
        """The closure's term C D div(base grad omega) of every member at the
        flat fields omega (a new flat tensor)."""
        self._check_flat(omega, "omega")
        out = torch.empty(self.total, dtype=self.dtype, device=self.device)
        self._check(self.L.qg_closure_term(self.h, _ptr(omega), _ptr(out), _stream(self.device)))
        return out

    def pcc(self, a, b):
        """Pattern correlation of two flat fields, one float64 per member."""
        self._check_flat(a, "a")
        self._check_flat(b, "b")
        out = torch.zeros(self.n, dtype=torch.float64, device=self.device)
        self._check(self.L.qg_pcc(self.h, _ptr(a), _ptr(b), _ptr(out), _stream(self.device)))
        return out

    def set_coef(self, c):
        """Closure coefficient c per member (sequence of floats)."""
        c = [float(x) for x in c]
        if len(c) != self.n:
            raise ValueError("one coefficient per member")
        arr = (ctypes.c_double * self.n)(*c)
        self._check(self.L.qg_set_coef(self.h, arr, _stream(self.device)))
        for p, v in zip(self.params, c):
            p["c"] = v

    def autotune(self, cache_path=None):
        self._check(self.L.qg_autotune(self.h, cache_path.encode() if cache_path else None,
                                      _stream(self.device)))

    def profile_steps(self, omega, nsteps, kind, max_launches=4096):
        """qg_step without graphs, with the dispatch of every launch of one
        kind of step kernel timed by HIP events bound to it (profiling);
        returns the launch durations in milliseconds."""
        self._check_flat(omega, "omega")
        ms = (ctypes.c_float * max_launches)()
        n = ctypes.c_int32(0)
        self._check(self.L.qg_profile_steps(self.h, _ptr(omega), int(nsteps), int(kind), ms, max_launches,
                                           ctypes.byref(n), _stream(self.device)))
        return list(ms[:n.value])

    def stamp_steps(self, omega, nsteps):
        """qg_step without graphs, with per-wave phase stamps of the four
        right-hand-side kernels (the stamp build libqg_stamps.so only);
        returns them as a (4, 8192, 8) uint64 array on the host."""
        self._check_flat(omega, "omega")
        buf = torch.zeros(4 * 8192 * 8, dtype=torch.int64, device=self.device)
        self._check(self.L.qg_stamp_steps(self.h, _ptr(omega), int(nsteps), _ptr(buf), buf.numel() * 8,
                                         _stream(self.device)))
        return buf.cpu().numpy().view(np.uint64).reshape(4, 8192, 8)

    def tuning(self):
        """Launch configuration per member: dicts with W, Wi, rsched, csched, rpb, rwave."""
        t = (ctypes.c_int32 * (6 * self.n))()
        self._check(self.L.qg_tuning(self.h, t))
        keys = ("W", "Wi", "rsched", "csched", "rpb", "rwave")
        return [dict(zip(keys, t[6 * i: 6 * i + 6])) for i in range(self.n)]

    def column_widths(self):
        """Strip width of the column-forward pass per member."""
        w = (ctypes.c_int32 * self.n)()
        self._check(self.L.qg_info(self.h, None, None, w, None))
        return list(w)

    def inverse_widths(self):
        """Strip width of the column-inverse pass per member."""
        w = (ctypes.c_int32 * self.n)()
        self._check(self.L.qg_info(self.h, None, None, None, w))
        return list(w)

    def close(self):
        if getattr(self, "h", None):
            torch.cuda.current_stream(self.device).synchronize()
            self.L.qg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _one_buffer_per_content(ts):
    """The list with every tensor equal to an earlier one replaced by that
    earlier tensor."""
    out = []
    for t in ts:
        same = next((u for u in out if u.shape == t.shape and u.dtype == t.dtype and torch.equal(u, t)), None)
        out.append(t if same is None else same)
    return out


def step_noalloc(params, chi, chi_sponge, omega, nsteps):
    """qg_step_noalloc: advance one member's omega (a device tensor of its
    precision, ny * nx elements) in place by nsteps steps with the library's
    static workspace -- no handle, no allocation.  chi and chi_sponge are
    device tensors of the same shape and type."""
    L = _lib.lib()
    dtype = _DTYPES[int(params.get("precision", 64))]
    for t, name in ((omega, "omega"), (chi, "chi"), (chi_sponge, "chi_sponge")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous() or t.dtype != dtype:
            raise TypeError(f"{name} must be a contiguous {dtype} device tensor")
        if t.numel() != int(params["nx"]) * int(params["ny"]):
            raise ValueError(f"{name} must hold ny * nx elements")
    prm = _lib.make_params(params)
    _lib.check(L.qg_step_noalloc(ctypes.byref(prm), _ptr(chi), _ptr(chi_sponge), _ptr(omega), int(nsteps),
                                 _stream(omega.device)))
    return omega
