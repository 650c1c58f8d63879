"""Named workloads: parameter sets plus the recipe for their seeded inputs.

A workload is one or more members; each member is a parameter dict whose keys
match the fields of the C ``qg_params`` struct, plus its masks and initial
vorticity from ``inputs``.  Values follow the benchmark definitions of the
method (flow past a circular island, a coast with a cape, a batched ensemble
of uneven grids, a differentiable island run); constants that those
definitions leave open are fixed here and listed in the design notes.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from . import inputs

CLOSURE_IDS = {"none": 0, "smag": 1, "leith": 2, "dsmag": 3, "dleith": 4}
STATIC_C = {"smag": 0.17, "leith": 0.2, "dsmag": 0.0, "dleith": 0.0, "none": 0.0}


def base_params(nx, ny, lx, ly, **kw):
    p = dict(nx=nx, ny=ny, lx=lx, ly=ly, beta=0.0, re=math.inf, mu=0.0,
             u_in=0.0, v_in=0.0, eta=math.inf, sponge_sigma=0.0, dt=1e-3,
             c=0.0, closure="none", precision=64, test_ratio=2, clip_mode=0,
             fp64_lowk=8)
    p.update(kw)
    return p


@dataclass
class Member:
    params: dict
    chi: np.ndarray
    chi_s: np.ndarray
    omega0: np.ndarray
    meta: dict = field(default_factory=dict)


@dataclass
class Workload:
    name: str
    members: list
    nsteps: int
    meta: dict = field(default_factory=dict)

    @property
    def points(self):
        return sum(m.params["nx"] * m.params["ny"] for m in self.members)


def island_member(nx, ny, *, precision, beta, re, dt, eta, xc, radius, closure,
                  seed, rms, u_in=1.0, c=None, lx=2 * math.pi, ly=math.pi,
                  sigma=10.0, eps=None):
    p = base_params(nx, ny, lx, ly, beta=beta, re=re, dt=dt, eta=eta, u_in=u_in,
                    sponge_sigma=sigma, closure=closure, precision=precision,
                    c=STATIC_C[closure] if c is None else c)
    chi = inputs.island_mask(nx, ny, lx, ly, xc, ly / 2, radius, eps=eps)
    chi_s = inputs.sponge_mask(nx, ny, lx, ly)
    w0 = inputs.bandpass_noise(nx, ny, lx, ly, seed, 2.0, 8.0, rms)
    return Member(p, chi, chi_s, w0, dict(geometry="island", radius=radius, seed=seed))


def cape_member(nx, ny, *, precision, beta, re, dt, eta, height, closure, seed,
                rms, init="band", u_in=1.0, c=None, lx=2 * math.pi, ly=math.pi,
                sigma=10.0):
    p = base_params(nx, ny, lx, ly, beta=beta, re=re, dt=dt, eta=eta, u_in=u_in,
                    sponge_sigma=sigma, closure=closure, precision=precision,
                    c=STATIC_C[closure] if c is None else c)
    chi = inputs.cape_mask(nx, ny, lx, ly, coast=0.2, height=height, width=0.3,
                           xc=math.pi)
    chi_s = inputs.sponge_mask(nx, ny, lx, ly)
    if init == "spectrum":
        w0 = inputs.spectrum_noise(nx, ny, lx, ly, seed, 4.0, rms)
    else:
        w0 = inputs.bandpass_noise(nx, ny, lx, ly, seed, 2.0, 8.0, rms)
    return Member(p, chi, chi_s, w0, dict(geometry="cape", height=height, seed=seed))


def config1(precision=64, nx=128, ny=64):
    """Island channel, static Smagorinsky c=0.17, 200 RK4 steps of 2e-3."""
    m = island_member(nx, ny, precision=precision, beta=1.0, re=1e3, dt=2e-3,
                      eta=1e-3, xc=1.5, radius=0.3, closure="smag", seed=0, rms=0.1)
    return Workload("C1 island 128x64 smag", [m], 200)


def config2(precision=64, nx=512, ny=256):
    """Flow past a circular island, dynamic Smagorinsky, 2000 steps of 5e-4."""
    m = island_member(nx, ny, precision=precision, beta=2.0, re=5e3, dt=5e-4,
                      eta=1e-4, xc=1.2, radius=0.25, closure="dsmag", seed=1,
                      rms=0.05)
    return Workload(f"C2 island {nx}x{ny} dsmag", [m], 2000)


def config3(precision=32, n=1024, seed=2):
    """Coast with a Gaussian cape on 2pi x 2pi, dynamic Leith, 1000 steps."""
    m = cape_member(n, n, precision=precision, beta=5.0, re=2e4, dt=2.5e-4,
                    eta=1e-4, height=0.6, closure="dleith", seed=seed, rms=0.1,
                    init="spectrum", lx=2 * math.pi, ly=2 * math.pi)
    return Workload(f"C3 cape {n}x{n} dleith", [m], 1000)


def ab2cn_island(precision=64, nx=128, ny=64, closure="smag", dt=2e-3):
    """The island channel of config 1 under the paper's own time scheme
    (AB2CN + AB2 sponge, Sec. II-E): explicit penalization needs eta > dt,
    so eta = 2.5 dt."""
    m = island_member(nx, ny, precision=precision, beta=1.0, re=1e3, dt=dt,
                      eta=2.5 * dt, xc=1.5, radius=0.3, closure=closure, seed=0, rms=0.1)
    m.params["scheme"] = "ab2cn"
    return Workload(f"AB2CN island {nx}x{ny} {closure}", [m], 200)


def config4(precision=32, sizes=((256, 128, 32), (512, 256, 24), (1024, 512, 8))):
    """Batched ensemble of uneven grids, closures drawn uniformly, 500 steps."""
    rng = np.random.default_rng(4)
    kinds = ["smag", "leith", "dsmag", "dleith"]
    members = []
    idx = 0
    for nx, ny, count in sizes:
        for _ in range(count):
            geom = "island" if rng.random() < 0.5 else "cape"
            size = float(rng.uniform(0.2, 0.5))
            beta = float(rng.uniform(1.0, 5.0))
            closure = kinds[int(rng.integers(0, 4))]
            if geom == "island":
                m = island_member(nx, ny, precision=precision, beta=beta, re=5e3,
                                  dt=5e-4, eta=1e-4, xc=1.5, radius=size,
                                  closure=closure, seed=100 + idx, rms=0.05)
            else:
                m = cape_member(nx, ny, precision=precision, beta=beta, re=5e3,
                                dt=5e-4, eta=1e-4, height=size, closure=closure,
                                seed=100 + idx, rms=0.05)
            members.append(m)
            idx += 1
    return Workload("C4 ensemble", members, 500)


def config5(precision=64, nx=512, ny=256):
    """Differentiable island run (as C2 with static Smagorinsky c=0.17), 500
    steps with checkpoints every 50."""
    m = island_member(nx, ny, precision=precision, beta=2.0, re=5e3, dt=5e-4,
                      eta=1e-4, xc=1.2, radius=0.25, closure="smag", seed=1,
                      rms=0.05)
    return Workload(f"C5 island {nx}x{ny} smag adjoint", [m], 500,
                    dict(ckpt_every=50, fd_directions=16, fd_seed=5))


def batched1024(precision=32, members=8):
    """Eight 1024^2 dynamic-Leith cape members (seeds 2..9) in one launch."""
    ms = [config3(precision, 1024, seed=2 + i).members[0] for i in range(members)]
    return Workload("B1024 cape 8x1024^2 dleith", ms, 200)
