#!/usr/bin/env python3
"""Benchmark of the QG step on one MI355X.

Metric: grid-point-steps per second at 1024^2 for the coast-with-cape
workload (dynamic Leith, RK4 + penalization/sponge sub-step), in FP32
(``value``), FP64 and FP32 batched (8 members of 1024^2 in one graph
launch), the same step under the paper's own AB2CN scheme, plus the
adjoint/forward time ratio of the differentiable island run (512x256,
static Smagorinsky, one 50-step checkpoint segment).

Inputs are synthetic and seeded (masks, sponge ramps, k^-3 random-phase
initial vorticity) and resident in HBM before timing.  Every leg is timed
with HIP events on the launch stream between synchronisations, as the
median of five windows of graph replays.  The roofline entry is for the
kernel with the largest share of the step: its average launch duration
comes from HIP events bound to each of its dispatches (begin and end of the
dispatch itself) over a run of eager steps of the same workload, and its
bytes are the algorithmic bytes of one launch (mixed-layout fields at the
2/3-pruned width and the state on the 2/3 set).  ``cpu_baseline`` is the
FP64 NumPy oracle (the correctness reference, not a tuned CPU code) on a few
steps of the same 1024^2 workload on one host thread; the oracle at the
other workloads' sizes and the 64-member ensemble over a process pool are
reported beside it.  The host legs run before the GPU is touched.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
PHASE_NAMES = ["colinv_rhs", "row_rhs", "colfwd_rhs", "combine_dyn", "colinv_b", "row_b", "colfwd_b"]
PHASE_LAUNCHES = [4, 4, 4, 4, 1, 1, 1]


def kernel_names(nx, ny, tuning):
    """Names of the kernels behind each phase (as the profiler lists them,
    with every template argument): compile-time transform lengths for
    256..1024 with the tuned pass schedules, row pairs per block and row
    synchronisation, the single-column forward kernel when the forward strip
    width is 1 (the two-half one for the dynamic closures' right-hand side
    at the compile-time lengths)."""
    lx = int(math.log2(nx)) if nx in (256, 512, 1024) else 0
    ly = int(math.log2(ny)) if ny in (256, 512, 1024) else 0
    lf = ly if tuning["W"] == 1 else 0
    cs = tuning["csched"]
    row = f"{tuning['rsched'] if lx else 0}, {'true' if tuning['rwave'] and lx else 'false'}, {tuning['rpb'] if lx else 1}"
    return {
        "colinv_rhs": f"k_colinv<float, 0, 4, {ly}, {cs if ly else 0}>",
        "row_rhs": f"k_rowp<float, 0, 4, {lx}, {row}>",
        "colfwd_rhs": (f"k_colfwdd<float, 4, {lf}, {cs}>" if lf else "k_colfwdp<float, 0, 4, 0, 0>"),
        "combine_dyn": "k_combine<float>",
        "colinv_b": f"k_colinv<float, 1, 0, {ly}, {cs if ly else 0}>",
        "row_b": f"k_rowp<float, 1, 0, {lx}, {row}>",
        "colfwd_b": f"k_colfwdp<float, 1, 0, {lf}, {cs if lf else 0}>",
    }


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(nx, ny, word, closure="dleith", test_ratio=2):
    """Bytes each kernel of one step must move for one member (see the
    module docstring): fields and products cross HBM once in the mixed
    layout of ny * kxn complex values (the test-filtered fields of the
    dynamic closures only over the test_kx columns that hold their modes);
    spectral quantities live on the 2/3 set of kxn * kyn complex values;
    physical tables are nx * ny reals."""
    kxn = (nx - 1) // 3 + 1
    kyn = 2 * ((ny - 1) // 3) + 1
    c = 2 * word
    nM = ny * kxn * c
    nD = kxn * kyn * c
    dyn = closure in ("dsmag", "dleith")
    nb = {"none": 4, "smag": 6, "leith": 4, "dsmag": 6, "dleith": 4}[closure]
    test_kx = 0
    if dyn:
        lim = min(((nx - 1) // 3) * ny, ((ny - 1) // 3) * nx) ** 2
        while test_kx <= nx // 2 and test_ratio ** 2 * ny * ny * test_kx * test_kx <= lim:
            test_kx += 1
    F = nb + (nb * min(test_kx, kxn) / kxn if dyn else 0)     # full-width field equivalents
    P = {"none": 1, "smag": 3, "leith": 3, "dsmag": 6, "dleith": 6}[closure]
    per = {
        "colinv_rhs": nD + F * nM,
        "row_rhs": F * nM + P * nM,
        "colfwd_rhs": P * nM + (2 * nD if dyn else 4 * nD),
        "combine_dyn": 7 * nD if dyn else 0,
        "colinv_b": nD + 3 * nM,
        "row_b": 3 * nM + 3 * nx * ny * word + nM,
        "colfwd_b": nM + nD,
    }
    step = sum(per[k] * n for k, n in zip(PHASE_NAMES, PHASE_LAUNCHES))
    return per, step


WINDOWS = 5


def time_steps(S, om, steps, warmup, torch, windows=WINDOWS):
    """Median over `windows` windows of `steps` graph-replayed steps, HIP
    events on the launch stream (the torch current stream); returns seconds
    per window and the wall clock of all windows."""
    S.step(om, warmup, use_graph=True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    times = []
    t0 = time.perf_counter()
    for _ in range(windows):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        S.step(om, steps, use_graph=True)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    wall = time.perf_counter() - t0
    return float(np.median(times)), wall


def time_kernels(S, om, nsteps, kinds=range(len(PHASE_NAMES))):
    """Average dispatch duration (ms) of each kind of step kernel: HIP events
    bound to every dispatch of that kind over `nsteps` eager steps
    (qg_profile_steps), on the launch stream."""
    out = {}
    for k in kinds:
        ms = S.profile_steps(om, nsteps, k)
        out[PHASE_NAMES[k]] = (float(np.mean(ms)) if ms else 0.0, len(ms))
    return out


def full_width_bytes_per_point(closure, word):
    """Byte model with every inverse field and product at full width: per
    grid-point-step 4 [2/3 2 (F + P) + 4/3 (RK state) + 16/9 (dynamic
    split)] + 10 words (B sub-step), F inverse fields and P forward products
    per right-hand side (388 B for dynamic Leith in FP32)."""
    F = {"none": 4, "smag": 6, "leith": 4, "dsmag": 12, "dleith": 8}[closure]
    P = {"none": 1, "smag": 3, "leith": 3, "dsmag": 6, "dleith": 6}[closure]
    dyn = 16.0 / 9.0 if closure in ("dsmag", "dleith") else 0.0
    return (4 * (2.0 / 3.0 * 2 * (F + P) + 4.0 / 3.0 + dyn) + 10) * word


TUNE_CACHE = None
HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(HERE, "profiles", "traffic.json")


KERNEL_SOURCES = ("qg_fft.hpp", "qg_internal.hpp", "qg_kernels.hip")


def kernel_sources_digest():
    """SHA-256 over the kernel sources (device code and the launch
    arguments it reads; the host runtime is not part of it), to tell whether
    counters taken earlier still describe the kernels that run now."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "paper_2508_06678_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE counters, each scaled by the factor a plain device copy of
    known size gives; None if there are none for this kernel or the sources
    changed since they were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("sources_sha256") != kernel_sources_digest():
        return None
    # the main entry, or the same counters for the kernel's other form
    # (the tuner's other row synchronisation)
    e = t if t.get("kernel") == kernel else t.get("alternates", {}).get(kernel)
    if e is None:
        return None
    return 1024.0 * (e["fetch_kib"] * e["fetch_factor"] + e["write_kib"] * e["write_factor"])


def make_solver(workload, precision, adj=0, tune=True):
    from paper_2508_06678_amd.solver import Solver
    params, chi, chs = [], [], []
    dt = np.float32 if precision == 32 else np.float64
    for m in workload.members:
        p = dict(m.params)
        p["precision"] = precision
        params.append(p)
        chi.append(m.chi.astype(dt))
        chs.append(m.chi_s.astype(dt))
    S = Solver(params, chi, chs, adj_segment_k=adj)
    if tune:
        S.autotune(TUNE_CACHE)
        log(f"  strip widths fwd {sorted(set(S.column_widths()))} inv {sorted(set(S.inverse_widths()))}")
    om = S.pack([m.omega0 for m in workload.members])
    return S, om


def _oracle_model(m):
    from oracle import qg
    p = {k: v for k, v in m.params.items() if k in qg.Params.__dataclass_fields__}
    return qg.Model(qg.Params(**p), m.chi, m.chi_s)


def oracle_rate(member, nsteps):
    """Oracle grid-point-steps/s of one member on this thread: median of
    nsteps single steps after one warm-up step (first touch of the tables)."""
    from oracle import qg
    M = _oracle_model(member)
    w = qg.step(member.omega0, M)
    times = []
    for _ in range(nsteps):
        t0 = time.perf_counter()
        w = qg.step(w, M)
        times.append(time.perf_counter() - t0)
    pts = member.params["nx"] * member.params["ny"]
    return pts / float(np.median(times)), float(np.sum(times))


_POOL_MEMBERS = None


def _pool_init():
    global _POOL_MEMBERS
    from paper_2508_06678_amd import configs
    _POOL_MEMBERS = configs.config4(precision=64).members


def _pool_member_step(i):
    from oracle import qg
    m = _POOL_MEMBERS[i]
    return qg.step(m.omega0, _oracle_model(m)).shape


def cpu_baseline(args):
    """The oracle on the host: the 1024^2 workload of `value` (one thread,
    the line's cpu_baseline), the single-member workloads C1 and C2 and the
    64-member ensemble, one step of every member over a process pool on the
    host's cores.  Runs before anything touches the GPU (the pool forks)."""
    import multiprocessing as mp
    from paper_2508_06678_amd import configs
    c3 = configs.config3(precision=64).members[0]
    v3, t3 = oracle_rate(c3, args.cpu_steps)
    base = {"value": v3, "unit": "grid-pt-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"median of {args.cpu_steps} single steps (after one warm-up step) of the 1024x1024 cape "
                      f"workload, FP64 NumPy oracle with its own radix-2 FFT on 1 host thread "
                      f"({os.cpu_count()} cores on the host), {t3:.1f} s"}
    extra = {}
    for name, m in (("C1 128x64 island, static Smagorinsky", configs.config1().members[0]),
                    ("C2 512x256 island, dynamic Smagorinsky", configs.config2(precision=64).members[0])):
        v, t = oracle_rate(m, 3)
        extra[name] = {"value": v, "unit": "grid-pt-steps/s", "cores": 1, "seconds": t}
    n = len(configs.config4(precision=64).members)
    cores = max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("fork")
    with ctx.Pool(cores, initializer=_pool_init) as pool:
        pool.map(_pool_member_step, range(cores))         # workers started, modules imported
        t0 = time.perf_counter()
        pool.map(_pool_member_step, range(n))
        tp = time.perf_counter() - t0
    pts = configs.config4(precision=64).points
    extra["C4 64-member ensemble, one step of every member, process pool"] = {
        "value": pts / tp, "unit": "grid-pt-steps/s", "cores": cores, "seconds": tp}
    base["other_workloads"] = extra
    return base


def roofline_of(S, om, nx, ny, closure, nsteps, names, members=1):
    """Dominant kernel by time share over nsteps eager steps, its average
    dispatch duration from events bound to its dispatches, and its
    algorithmic bytes per launch (all members of the launch)."""
    per, _ = algorithmic_bytes(nx, ny, 4, closure)
    kt = time_kernels(S, om, nsteps)
    share = {k: kt[k][0] * PHASE_LAUNCHES[i] for i, k in enumerate(PHASE_NAMES)}
    dom = max(PHASE_NAMES, key=lambda k: share[k])
    avg_ms, nl = kt[dom]
    b = per[dom] * members
    ach = b / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": measured_traffic(names[dom]) if members == 1 else None,
            "kernel": names[dom], "bytes_per_launch": b, "avg_launch_us": avg_ms * 1e3,
            "launches_timed": nl,
            "timing": f"HIP events bound to each dispatch (begin, end), {nsteps} eager steps"}, kt, per


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--prof-steps", type=int, default=20,
                    help="eager steps whose kernel dispatches are timed for the roofline entry")
    ap.add_argument("--skip", default="", help="comma list of: fp64,batched,ensemble,ab2cn,clip,sgs,adjoint,cpu,phases")
    ap.add_argument("--tune-cache", default=None,
                    help="tuning cache file: read if it holds the workload, else written after tuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB elementwise device copy (scale reference for HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(ensemble members shard across GPUs without communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    skip = set(s for s in args.skip.split(",") if s)
    global TUNE_CACHE
    TUNE_CACHE = args.tune_cache
    cpu = None
    if "cpu" not in skip:
        cpu = cpu_baseline(args)
        log(f"cpu oracle: {cpu['value']:.4g} pt-steps/s (1 thread, 1024^2); "
            + "; ".join(f"{k}: {v['value']:.4g} on {v['cores']}" for k, v in cpu["other_workloads"].items()))
    import torch
    from paper_2508_06678_amd import configs

    K, W = args.steps, args.warmup
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)     # a plain streaming kernel: 256 MiB read, 256 MiB written
        torch.cuda.synchronize()
        log("copy calibration: 3 elementwise copies (negation) of 268435456 bytes")
        del src, dst
    wl = configs.config3(precision=32)
    nx, ny = wl.members[0].params["nx"], wl.members[0].params["ny"]
    pts = nx * ny
    bpp32 = full_width_bytes_per_point("dleith", 4)

    # ---- FP32, one 1024^2 member (value)
    S, om = make_solver(wl, 32)
    tuned = S.tuning()[0]
    names = kernel_names(nx, ny, tuned)
    sec, wall = time_steps(S, om, K, W, torch)
    value = pts * K / sec
    log(f"fp32 1024^2 dleith: {sec / K * 1e3:.4f} ms/step (median of {WINDOWS} windows of {K}), "
        f"{value:.4g} pt-steps/s (wall {wall:.3f} s)")
    per, step_bytes = algorithmic_bytes(nx, ny, 4, "dleith")
    roof = kt = None
    if "phases" not in skip:
        roof, kt, per = roofline_of(S, om, nx, ny, "dleith", args.prof_steps, names)
        for i, name in enumerate(PHASE_NAMES):
            avg, nl = kt[name]
            gbs = per[name] / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
            log(f"  {name:12s} {avg * 1e3:8.2f} us/dispatch x{PHASE_LAUNCHES[i]}  {avg * PHASE_LAUNCHES[i] * 1e3:8.1f}"
                f" us/step  {gbs:7.0f} GB/s algorithmic  ({nl} dispatches timed)")
    S.close()
    step_gbs = step_bytes / (sec / K) / 1e9

    result = {
        "metric": "grid-pt-steps/s at 1024^2: FP64 vs FP32 vs batched; adjoint/forward time ratio",
        "value": value,
        "unit": "grid-pt-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": sec / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded masks, sponge and k^-3 random-phase vorticity)",
        "config": {"workload": "coast with Gaussian cape, 1024x1024, 2pi x 2pi, dynamic Leith, "
                               "beta=5, Re=2e4, U=1, eta=1e-4, RK4 dt=2.5e-4, FP32",
                   "grid": [ny, nx], "members": 1, "parallelism": "single GPU"},
        "timing": f"median of {WINDOWS} windows of K graph-replayed steps, HIP events on the launch stream",
        "step_algorithmic_GBps": step_gbs,
        "step_roofline_frac": step_gbs / HBM_PEAK_GBS,
        "step_roofline_frac_388B": bpp32 * pts / (sec / K) / 1e9 / HBM_PEAK_GBS,
    }
    result["tuning"] = tuned
    if roof:
        result["roofline"] = roof
        result["kernels_us_per_dispatch"] = {k: v[0] * 1e3 for k, v in kt.items()}

    # ---- FP64, one member
    if "fp64" not in skip:
        S, om = make_solver(wl, 64)
        k64 = max(10, K // 2)
        sec64, _ = time_steps(S, om, k64, W, torch)
        S.close()
        _, b64 = algorithmic_bytes(nx, ny, 8, "dleith")
        result["fp64"] = {"value": pts * k64 / sec64, "ms_per_step": sec64 / k64 * 1e3, "steps": k64,
                          "step_roofline_frac": b64 / (sec64 / k64) / 1e9 / HBM_PEAK_GBS,
                          "step_roofline_frac_777B": full_width_bytes_per_point("dleith", 8) * pts / (sec64 / k64)
                          / 1e9 / HBM_PEAK_GBS}
        log(f"fp64 1024^2 dleith: {sec64 / k64 * 1e3:.4f} ms/step")

    # ---- FP32 batched: 8 x 1024^2 in one graph
    if "batched" not in skip:
        bw = configs.batched1024(32)
        S, om = make_solver(bw, 32)
        kb = max(10, K // 4)
        secb, _ = time_steps(S, om, kb, W // 2 + 1, torch)
        nb = len(bw.members)
        ptsb = bw.points
        result["batched"] = {"value": ptsb * kb / secb, "ms_per_step": secb / kb * 1e3, "steps": kb,
                             "members": nb,
                             "step_roofline_frac": nb * step_bytes / (secb / kb) / 1e9 / HBM_PEAK_GBS,
                             "step_roofline_frac_388B": bpp32 * ptsb / (secb / kb) / 1e9 / HBM_PEAK_GBS,
                             "tuning": S.tuning()[0]}
        if "phases" not in skip:
            bnames = kernel_names(nx, ny, S.tuning()[0])
            broof, bkt, _ = roofline_of(S, om, nx, ny, "dleith", max(5, args.prof_steps // 4), bnames, members=nb)
            result["batched"]["roofline_dominant"] = broof
            result["batched"]["kernels_us_per_dispatch"] = {k: v[0] * 1e3 for k, v in bkt.items()}
        S.close()
        log(f"batched 8x1024^2: {secb / kb * 1e3:.4f} ms/step, {ptsb * kb / secb:.4g} pt-steps/s")

    # ---- the ragged FP32 ensemble of the batched workload: 64 members of
    # three sizes (32 x 256x128, 24 x 512x256, 8 x 1024x512), closures drawn
    # over all four, one graph
    if "ensemble" not in skip:
        we = configs.config4(precision=32)
        S, om = make_solver(we, 32)
        ke = max(10, K // 4)
        sece, _ = time_steps(S, om, ke, W // 2 + 1, torch)
        S.close()
        ebytes = sum(algorithmic_bytes(m.params["nx"], m.params["ny"], 4, m.params["closure"])[1]
                     for m in we.members)
        result["ensemble_ragged"] = {
            "value": we.points * ke / sece, "ms_per_step": sece / ke * 1e3, "steps": ke,
            "members": len(we.members),
            "step_roofline_frac": ebytes / (sece / ke) / 1e9 / HBM_PEAK_GBS,
            "workload": "64 members: 32 x 256x128, 24 x 512x256, 8 x 1024x512, island or cape, "
                        "closures drawn over the four, FP32"}
        log(f"ragged ensemble (64 members): {sece / ke * 1e3:.4f} ms/step, {we.points * ke / sece:.4g} pt-steps/s")

    # ---- the paper's own scheme (AB2CN + AB2 sponge) on the same workload,
    # with eta = 2.5 dt (explicit penalization needs eta > dt)
    if "ab2cn" not in skip:
        wa = configs.config3(precision=32)
        for m in wa.members:
            m.params["scheme"] = "ab2cn"
            m.params["eta"] = 2.5 * m.params["dt"]
        S, om = make_solver(wa, 32)
        ka = max(10, K // 2)
        seca, _ = time_steps(S, om, ka, W, torch)
        S.close()
        result["ab2cn"] = {"value": pts * ka / seca, "ms_per_step": seca / ka * 1e3, "steps": ka,
                           "workload": "as value, AB2CN + AB2 sponge, eta = 2.5 dt"}
        log(f"ab2cn 1024^2 dleith: {seca / ka * 1e3:.4f} ms/step")

    # ---- the pointwise clip of the dynamic coefficient (clip_mode 1) on the
    # same workload: one two-field inverse pass more per stage
    if "clip" not in skip:
        wc = configs.config3(precision=32)
        for m in wc.members:
            m.params["clip_mode"] = 1
        S, om = make_solver(wc, 32)
        kc = max(10, K // 2)
        secc, _ = time_steps(S, om, kc, W, torch)
        S.close()
        result["clip_pointwise"] = {"value": pts * kc / secc, "ms_per_step": secc / kc * 1e3, "steps": kc,
                                    "workload": "as value, C = <max(H,0) M>/<M^2> (clip_mode 1)"}
        log(f"pointwise clip 1024^2 dleith: {secc / kc * 1e3:.4f} ms/step")

    # ---- a-priori SGS analysis: FR 1024^2 -> LES 512^2 (delta = 2), ideal
    # Pi_FF, the Dynamic Leith model term at the filtered field, their PCC
    if "sgs" not in skip:
        frw = configs.config3(precision=32)
        lesw = configs.config3(precision=32, n=512)
        F, omf = make_solver(frw, 32, tune=False)
        L, _ = make_solver(lesw, 32, tune=False)
        for _ in range(3):
            F.ideal_sgs(L, omf)
        torch.cuda.synchronize()
        ks = max(10, K // 4)
        stream = torch.cuda.current_stream()
        times = []
        for _ in range(WINDOWS):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(ks):
                pi, model, _ = F.ideal_sgs(L, omf)
                pcc = L.pcc(pi, model)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
        secs = float(np.median(times))
        F.close()
        L.close()
        result["sgs"] = {"value": pts * ks / secs, "unit": "FR grid-pts/s", "ms_per_analysis": secs / ks * 1e3,
                         "analyses": ks, "pcc_a_priori": float(pcc[0]),
                         "workload": "ideal SGS Pi_FF + Dynamic Leith model term + PCC, FR 1024^2 -> "
                                     "LES 512^2 (delta 2), FP32; LES masks sampled on the LES grid"}
        log(f"sgs analysis 1024^2 -> 512^2: {secs / ks * 1e3:.3f} ms per analysis")

    # ---- adjoint / forward on the differentiable island run: one segment of
    # `seg` steps (recompute + reverse sweep) against `seg` forward steps,
    # both graph replays, median of five each
    if "adjoint" not in skip:
        w5 = configs.config5(precision=64)
        seg = w5.meta["ckpt_every"]
        w5d = configs.config5(precision=64)
        for m in w5d.members:   # the same run with the dynamic Leith closure
            m.params["closure"] = "dleith"
        ratios = {}
        stream = torch.cuda.current_stream()
        for prec, wl5, tag in ((64, w5, ""), (32, w5, ""), (64, w5d, "_dleith")):
            S, om = make_solver(wl5, prec, adj=seg)
            w0 = om.clone()
            tf, _ = time_steps(S, om, seg, 5, torch)
            lam0 = torch.randn_like(om) * 1e-3
            g = torch.zeros(1, dtype=torch.float64, device=om.device)
            S.adjoint_step(w0, lam0.clone(), seg, g)
            torch.cuda.synchronize()
            times = []
            for _ in range(WINDOWS):
                lam = lam0.clone()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                S.adjoint_step(w0, lam, seg, g)
                e1.record(stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1) / 1e3)
            ta = float(np.median(times))
            S.close()
            ratios[f"fp{prec}{tag}"] = ta / tf
            log(f"adjoint/forward fp{prec}{tag}: {ta / tf:.3f} ({ta * 1e3:.2f} ms / {tf * 1e3:.2f} ms, {seg} steps)")
        result["adjoint_forward_ratio"] = ratios

    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
