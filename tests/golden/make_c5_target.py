"""Write tests/golden/c5_target_512x256.npy: the loss target of the
differentiable island run.

The target is the oracle run at twice the resolution (1024 x 512, same
physics, masks rebuilt on the fine grid with the coarse grid's smoothing
width) from the zero-padded, exactly band-limited initial vorticity of the
512 x 256 run, advanced 500 steps, then truncated spectrally to the modes of
the 512 x 256 grid (|m_x| < 256, |m_y| < 128) and rescaled for the
unnormalised transform.  Only the oracle is called.

Usage: python tests/golden/make_c5_target.py [--steps 500]
"""
import argparse
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import qg  # noqa: E402
from oracle import fft as F  # noqa: E402
from paper_2508_06678_amd import configs, inputs  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--out", default=os.path.join(HERE, "c5_target_512x256.npy"))
    a = ap.parse_args()
    coarse = configs.config5(precision=64).members[0]
    pc = coarse.params
    nxc, nyc = pc["nx"], pc["ny"]
    nxf, nyf = 2 * nxc, 2 * nyc
    lx, ly = pc["lx"], pc["ly"]
    eps = 2.0 * lx / nxc
    chi = inputs.island_mask(nxf, nyf, lx, ly, 1.2, ly / 2, 0.25, eps=eps)
    chi_s = inputs.sponge_mask(nxf, nyf, lx, ly)
    p = {k: v for k, v in pc.items() if k in qg.Params.__dataclass_fields__}
    p.update(nx=nxf, ny=nyf)
    M = qg.Model(qg.Params(**p), chi, chi_s)
    # zero-pad the coarse initial spectrum onto the fine grid (exact: band-limited)
    wc = F.rfft2(coarse.omega0)
    wf = np.zeros((nyf, nxf // 2 + 1), complex)
    scale = (nxf * nyf) / (nxc * nyc)
    for my in range(-nyc // 2 + 1, nyc // 2):
        wf[my % nyf, : nxc // 2] = wc[my % nyc, : nxc // 2] * scale
    w0 = F.irfft2(wf, nxf)
    wh = qg.enter(w0, M.g)
    t0 = time.time()
    for n in range(a.steps):
        wh = qg.step_spectral(wh, M)
        if (n + 1) % 25 == 0:
            print(f"step {n + 1}/{a.steps}  {time.time() - t0:.0f} s", flush=True)
    # truncate to the coarse grid's modes and rescale
    tc = np.zeros((nyc, nxc // 2 + 1), complex)
    for my in range(-nyc // 2 + 1, nyc // 2):
        tc[my % nyc, : nxc // 2] = wh[my % nyf, : nxc // 2] / scale
    target = F.irfft2(tc, nxc)
    np.save(a.out, target)
    print("wrote", a.out, target.shape, float(np.sqrt(np.mean(target ** 2))))


if __name__ == "__main__":
    main()
