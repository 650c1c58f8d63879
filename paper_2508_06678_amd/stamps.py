"""Where the right-hand-side kernels of one step spend their time, from the
per-wave phase stamps of the debug build libqg_stamps.so (qg_stamp_steps):
the spread of each phase over the waves, the kernel's span, and how the
waves were placed on XCDs, compute units and SIMDs (from the hardware ids
each wave records).

    python -m paper_2508_06678_amd.stamps [--members 1|8] [--precision 32|64] [--steps 3] [--tune-cache PATH]

runs the 1024 x 1024 dynamic-Leith cape workload (one member, or the
8-member ensemble, whose member 0 is stamped) and prints a Markdown report.
Times are the GPU's 100 MHz real-time counter (10 ns ticks); the stamps'
own waits lengthen the kernels a little.
"""
import argparse
import collections

import numpy as np

KINDS = {
    0: ("row pass", ["loads in", "c2r done", "products formed", "r2c done", "stores complete"]),
    1: ("column-inverse pass", ["fields formed", "transform done", "stores complete"]),
    2: ("column-forward pass", ["loads in", "transform done", "mode stores complete", "partial sums stored"]),
    3: ("combine", ["loads in", "coefficient formed", "stores complete"]),
}
TICK_NS = 10.0
PCT = (0, 10, 50, 90, 100)


def waves_of(stamps, kind):
    """The waves of `kind` that recorded every slot: (times int64 [n, slots],
    hardware ids uint64 [n])."""
    ns = len(KINDS[kind][1]) + 1
    raw = stamps[kind]
    t = raw[:, :ns].astype(np.int64)
    ok = np.all(t > 0, axis=1)
    return t[ok], raw[ok, 7]


def placement(hw):
    """XCD, compute-unit and SIMD keys of each wave from HW_ID / XCC_ID."""
    hid = (hw & 0xffffffff).astype(np.int64)
    xcc = ((hw >> 32) & 0xf).astype(np.int64)
    simd = (hid >> 4) & 3
    cu = (hid >> 8) & 15
    sh = (hid >> 12) & 1
    se = (hid >> 13) & 7
    cukey = ((xcc * 8 + se) * 2 + sh) * 16 + cu
    return xcc, cukey, cukey * 4 + simd


def report(stamps, title):
    """Markdown tables of one stamp run."""
    out = [f"## {title}", ""]
    for kind, (name, labels) in KINDS.items():
        t, hw = waves_of(stamps, kind)
        if len(t) == 0:
            out += [f"### {name}: no stamps", ""]
            continue
        ns = len(labels) + 1
        t0 = t[:, 0].min()
        span = (t[:, ns - 1].max() - t0) * TICK_NS
        out += [f"### {name}: {len(t)} waves, span {span / 1e3:.2f} us", "",
                "| phase (us) | " + " | ".join(f"p{p}" for p in PCT) + " |",
                "|---|" + "---:|" * len(PCT)]

        def row(label, a):
            return f"| {label} | " + " | ".join(f"{np.percentile(a, p) * TICK_NS / 1e3:.2f}" for p in PCT) + " |"

        out.append(row("start (after the first wave's)", t[:, 0] - t0))
        for i, lab in enumerate(labels):
            out.append(row(f"-> {lab}", t[:, i + 1] - t[:, i]))
        out.append(row("wave lifetime", t[:, ns - 1] - t[:, 0]))
        out.append(row("end (after the first wave's start)", t[:, ns - 1] - t0))
        xcc, cukey, simdkey = placement(hw)
        per_xcd = collections.Counter(xcc.tolist())
        per_cu = collections.Counter(cukey.tolist())
        ends = collections.defaultdict(list)
        for k, e in zip(simdkey.tolist(), (t[:, ns - 1] - t0).tolist()):
            ends[k].append(e)
        by_n = collections.defaultdict(list)
        for es in ends.values():
            by_n[len(es)].append(max(es))
        out += ["", f"Waves per XCD: {dict(sorted(per_xcd.items()))}; compute units used {len(per_cu)}, "
                f"waves per compute unit: {dict(sorted(collections.Counter(per_cu.values()).items()))}.", "",
                "| waves on the SIMD | SIMDs | its last wave ends (median us) | (max us) |", "|---:|---:|---:|---:|"]
        for n, es in sorted(by_n.items()):
            out.append(f"| {n} | {len(es)} | {np.median(es) * TICK_NS / 1e3:.2f} | {max(es) * TICK_NS / 1e3:.2f} |")
        out.append("")
    return "\n".join(out)


def main(argv=None):
    import json
    import torch
    from . import configs
    from ._lib import STAMPS_LIB_PATH
    from .solver import Solver

    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--members", type=int, default=1, choices=(1, 8))
    ap.add_argument("--precision", type=int, default=32, choices=(32, 64))
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--tune-cache", default=None, help="the autotuner's cache (tunes and writes it when absent)")
    a = ap.parse_args(argv)
    wl = configs.config3(precision=a.precision) if a.members == 1 else configs.batched1024(a.precision)
    dt = np.float32 if a.precision == 32 else np.float64
    params, chi, chs = [], [], []
    for m in wl.members:
        p = dict(m.params)
        p["precision"] = a.precision
        params.append(p)
        chi.append(m.chi.astype(dt))
        chs.append(m.chi_s.astype(dt))
    S = Solver(params, chi, chs, lib_path=STAMPS_LIB_PATH)
    try:
        S.autotune(a.tune_cache)
        om = S.pack([m.omega0 for m in wl.members])
        stamps = S.stamp_steps(om, a.steps)
        torch.cuda.synchronize()
        title = (f"FP{a.precision} 1024x1024 cape, dynamic Leith, {len(wl.members)} member(s) "
                 f"(member 0 stamped), tuning {json.dumps(S.tuning()[0])}")
        print(report(stamps, title), flush=True)
    finally:
        S.close()


if __name__ == "__main__":
    main()
