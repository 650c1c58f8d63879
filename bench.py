#!/usr/bin/env python3
"""Benchmark of the QG step on one MI355X.

Metric: grid-point-steps per second at 1024^2 for the coast-with-cape
workload (dynamic Leith, RK4 + penalization/sponge sub-step), in FP32
(``value``), FP64 and FP32 batched (8 members of 1024^2 in one graph
launch), the same step under the paper's own AB2CN scheme, plus the
adjoint/forward time ratio of the differentiable island run (512x256,
static Smagorinsky, one 50-step checkpoint segment).

Inputs are synthetic and seeded (masks, sponge ramps, k^-3 random-phase
initial vorticity) and resident in HBM before timing.  Steps are timed with
HIP events on the launch stream between synchronisations.  The roofline
entry is for the kernel with the largest share of the step, timed live
with HIP events on its stream; its bytes are the algorithmic bytes of one
launch (what the method must move: mixed-layout fields at the 2/3-pruned
width and the state on the 2/3 set).  ``cpu_baseline`` is the FP64 NumPy
oracle (the correctness reference, not a tuned CPU code) on one step of the
same 1024^2 workload, on the host.

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


def kernel_names(nx, ny, fwd_width):
    """Names of the kernels behind each phase (as the profiler lists them):
    compile-time transform lengths for 256..1024, the single-column forward
    kernel when the forward strip width is 1."""
    lx = int(math.log2(nx)) if nx in (256, 512, 1024) else 0
    ly = int(math.log2(ny)) if ny in (256, 512, 1024) else 0
    lf = ly if fwd_width == 1 else 0
    return {
        "colinv_rhs": f"k_colinv<float, 0, 4, {ly}>",
        "row_rhs": f"k_rowp<float, 0, 4, {lx}>",
        "colfwd_rhs": f"k_colfwdp<float, 0, 4, {lf}>",
        "combine_dyn": "k_combine<float>",
        "colinv_b": f"k_colinv<float, 1, 0, {ly}>",
        "row_b": f"k_rowp<float, 1, 0, {lx}>",
        "colfwd_b": f"k_colfwdp<float, 1, 0, {lf}>",
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


def time_steps(S, om, steps, warmup, torch):
    S.step(om, warmup, use_graph=True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    S.step(om, steps, use_graph=True)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def time_phases(S, torch, reps=20):
    """Average duration of each kernel of the step, HIP events on the stream
    the kernels are launched on (the torch current stream)."""
    stream = torch.cuda.current_stream()
    out = {}
    for ph, name in enumerate(PHASE_NAMES):
        S.run_phase(ph, stage=2, reps=2)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        S.run_phase(ph, stage=2, reps=reps)
        e1.record(stream)
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / reps
    return out


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
    if t.get("kernel") != kernel or t.get("sources_sha256") != kernel_sources_digest():
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_factor"] + t["write_kib"] * t["write_factor"])


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


def cpu_baseline(workload, nsteps):
    from oracle import qg
    m = workload.members[0]
    p = {k: v for k, v in m.params.items() if k in qg.Params.__dataclass_fields__}
    M = qg.Model(qg.Params(**p), m.chi, m.chi_s)
    w = m.omega0
    qg.step(w, M)  # warm-up (first-touch of the tables)
    t0 = time.perf_counter()
    for _ in range(nsteps):
        w = qg.step(w, M)
    dt = time.perf_counter() - t0
    pts = m.params["nx"] * m.params["ny"]
    return {"value": pts * nsteps / dt, "unit": "grid-pt-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{nsteps} step(s) of the {m.params['nx']}x{m.params['ny']} cape workload, "
                      f"FP64 NumPy oracle with its own radix-2 FFT on 1 host thread "
                      f"({os.cpu_count()} cores on the host), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--skip", default="", help="comma list of: fp64,batched,ensemble,ab2cn,clip,sgs,adjoint,cpu,phases")
    ap.add_argument("--tune-cache", default=None,
                    help="strip-width cache file: read if it holds the workload, else written after tuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (scale reference for HBM counters)")
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
    import torch
    from paper_2508_06678_amd import configs

    K, W = args.steps, args.warmup
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of 268435456 bytes")
        del src, dst
    wl = configs.config3(precision=32)
    nx, ny = wl.members[0].params["nx"], wl.members[0].params["ny"]
    pts = nx * ny

    # ---- FP32, one 1024^2 member (value)
    S, om = make_solver(wl, 32)
    names = kernel_names(nx, ny, S.column_widths()[0])
    sec, wall = time_steps(S, om, K, W, torch)
    value = pts * K / sec
    log(f"fp32 1024^2 dleith: {sec / K * 1e3:.3f} ms/step, {value:.4g} pt-steps/s (wall {wall:.3f} s)")
    per, step_bytes = algorithmic_bytes(nx, ny, 4, "dleith")
    phases = None
    if "phases" not in skip:
        phases = time_phases(S, torch)
        for name in PHASE_NAMES:
            share = phases[name] * PHASE_LAUNCHES[PHASE_NAMES.index(name)]
            gbs = per[name] / (phases[name] * 1e-3) / 1e9 if phases[name] > 0 else 0.0
            log(f"  {name:12s} {phases[name] * 1e3:8.1f} us/launch x{PHASE_LAUNCHES[PHASE_NAMES.index(name)]}"
                f"  {share * 1e3:8.1f} us/step  {gbs:7.0f} GB/s algorithmic")
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
        "step_algorithmic_GBps": step_gbs,
        "step_roofline_frac": step_gbs / HBM_PEAK_GBS,
    }
    if phases:
        dom = max(PHASE_NAMES, key=lambda n: phases[n] * PHASE_LAUNCHES[PHASE_NAMES.index(n)])
        ach = per[dom] / (phases[dom] * 1e-3) / 1e9
        result["roofline"] = {"bound": "hbm", "kernel": names[dom], "achieved": ach,
                              "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                              "traffic": measured_traffic(names[dom]), "bytes_per_launch": per[dom],
                              "avg_launch_us": phases[dom] * 1e3}
        result["kernels_us_per_launch"] = {k: v * 1e3 for k, v in phases.items()}

    # ---- FP64, one member
    if "fp64" not in skip:
        S, om = make_solver(wl, 64)
        k64 = max(10, K // 2)
        sec64, _ = time_steps(S, om, k64, W, torch)
        S.close()
        _, b64 = algorithmic_bytes(nx, ny, 8, "dleith")
        result["fp64"] = {"value": pts * k64 / sec64, "ms_per_step": sec64 / k64 * 1e3, "steps": k64,
                          "step_roofline_frac": b64 / (sec64 / k64) / 1e9 / HBM_PEAK_GBS}
        log(f"fp64 1024^2 dleith: {sec64 / k64 * 1e3:.3f} ms/step")

    # ---- FP32 batched: 8 x 1024^2 in one graph
    if "batched" not in skip:
        bw = configs.batched1024(32)
        S, om = make_solver(bw, 32)
        kb = max(10, K // 4)
        secb, _ = time_steps(S, om, kb, W // 2 + 1, torch)
        S.close()
        ptsb = bw.points
        result["batched"] = {"value": ptsb * kb / secb, "ms_per_step": secb / kb * 1e3, "steps": kb,
                             "members": len(bw.members),
                             "step_roofline_frac": len(bw.members) * step_bytes / (secb / kb) / 1e9
                             / HBM_PEAK_GBS}
        log(f"batched 8x1024^2: {secb / kb * 1e3:.3f} ms/step, {ptsb * kb / secb:.4g} pt-steps/s")

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
        log(f"ragged ensemble (64 members): {sece / ke * 1e3:.3f} ms/step, {we.points * ke / sece:.4g} pt-steps/s")

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
        log(f"ab2cn 1024^2 dleith: {seca / ka * 1e3:.3f} ms/step")

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
        log(f"pointwise clip 1024^2 dleith: {secc / kc * 1e3:.3f} ms/step")

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
        t0 = time.perf_counter()
        for _ in range(ks):
            pi, model, _ = F.ideal_sgs(L, omf)
            pcc = L.pcc(pi, model)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        F.close()
        L.close()
        result["sgs"] = {"value": pts * ks / secs, "unit": "FR grid-pts/s", "ms_per_analysis": secs / ks * 1e3,
                         "analyses": ks, "pcc_a_priori": float(pcc[0]),
                         "workload": "ideal SGS Pi_FF + Dynamic Leith model term + PCC, FR 1024^2 -> "
                                     "LES 512^2 (delta 2), FP32; LES masks sampled on the LES grid"}
        log(f"sgs analysis 1024^2 -> 512^2: {secs / ks * 1e3:.3f} ms per analysis")

    # ---- adjoint / forward on the differentiable island run
    if "adjoint" not in skip:
        w5 = configs.config5(precision=64)
        seg = w5.meta["ckpt_every"]
        w5d = configs.config5(precision=64)
        for m in w5d.members:   # the same run with the dynamic Leith closure
            m.params["closure"] = "dleith"
        ratios = {}
        for prec, wl, tag in ((64, w5, ""), (32, w5, ""), (64, w5d, "_dleith")):
            S, om = make_solver(wl, prec, adj=seg)
            w0 = om.clone()
            S.step(om, 5, use_graph=True)
            torch.cuda.synchronize()
            f0 = time.perf_counter()
            S.step(om, seg, use_graph=True)
            torch.cuda.synchronize()
            tf = time.perf_counter() - f0
            lam = torch.randn_like(om) * 1e-3
            g = torch.zeros(1, dtype=torch.float64, device=om.device)
            S.adjoint_step(w0, lam.clone(), seg, g)
            torch.cuda.synchronize()
            a0 = time.perf_counter()
            S.adjoint_step(w0, lam, seg, g)
            torch.cuda.synchronize()
            ta = time.perf_counter() - a0
            S.close()
            ratios[f"fp{prec}{tag}"] = ta / tf
            log(f"adjoint/forward fp{prec}{tag}: {ta / tf:.2f} ({ta * 1e3:.1f} ms / {tf * 1e3:.1f} ms, {seg} steps)")
        result["adjoint_forward_ratio"] = ratios

    if "cpu" not in skip:
        result["cpu_baseline"] = cpu_baseline(configs.config3(precision=64), args.cpu_steps)
        log(f"cpu oracle: {result['cpu_baseline']['value']:.4g} pt-steps/s")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
