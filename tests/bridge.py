"""Test helpers: build oracle models and GPU solvers from the same member
definitions, and compare fields.  (Tests only; the product never imports the
oracle.)"""
import math

import numpy as np

from oracle import qg

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    torch = None
    HAVE_GPU = False


def oracle_model(params, chi, chi_s):
    p = {k: v for k, v in params.items() if k in qg.Params.__dataclass_fields__}
    p["closure"] = params.get("closure", "none")
    p["test_ratio"] = int(params.get("test_ratio", 2))
    p["re"] = params.get("re", math.inf)
    if p["re"] is None or p["re"] <= 0:
        p["re"] = math.inf
    return qg.Model(qg.Params(**p), chi, chi_s)


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_rel(a, b):
    """Largest pointwise difference relative to the largest value of the
    reference, max |a - b| / max |b|.  A mistake confined to one point, one
    row or one strip moves the L2 norm by the square root of its share of
    the grid; here it shows at full size."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def field_err(a, b):
    """Error of a field against its reference for a gate: the larger of the
    relative L2 norm and the pointwise (max-norm) relative error."""
    return max(rel_l2(a, b), max_rel(a, b))


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def solver_for(members, precision, adj_segment_k=0, lib_path=None):
    from paper_2508_06678_amd.solver import Solver
    params = []
    for m in members:
        p = dict(m.params)
        p["precision"] = precision
        params.append(p)
    dt = np.float32 if precision == 32 else np.float64
    chi = [m.chi.astype(dt) for m in members]
    chs = [m.chi_s.astype(dt) for m in members]
    return Solver(params, chi, chs, adj_segment_k=adj_segment_k, lib_path=lib_path)
