"""The paper's flows past a circular island (Sec. IV-A) and past an
idealized cape (Sec. IV-B) as runnable set-ups, and the a-priori analysis of
its Tables I and III: a fully-resolved (FR) run sampled at regular
snapshots; at each snapshot the ideal SGS forcing Pi_FF on the LES grid,
each closure's model term at the filtered field, and their pattern
correlation (PCC); the PCCs averaged over the snapshots.

    python -m paper_2508_06678_amd.experiments island|cape [--beta B]
        [--n 1024] [--steps 1000000] [--every 5000] [--precision 64]

Constants the paper states: Lx = Ly = 8 pi; inflow 2; Re = 200;
eta = 1.025 dt and eta_sponge = eta; dt = 1e-4; FR grid 1024^2; delta = 2;
T = 100 (10^6 steps) with snapshots every 5000 steps; the AB2CN scheme.
Island: diameter 2 pi/5 centred 0.35 Lx from the western edge,
mid-channel; beta = 0; a sponge of width 0.05 Lx on all four edges.  Cape:
land below y = 4 exp(-((x - 0.2 Lx)/1)^2); beta in {0, 0.1, 1}; sponge
parameters 0.125 Lx and 0.1 Lx.

Left open by the paper and fixed here: the land edges (tanh over two FR
cells; the cape measured from the southern edge and lifted off the
periodic seam by two smoothing widths), the cape's sponge (read as
thickness 0.125 Lx along the x edges and 0.1 Lx along the y edges), the
start (rest plus a 1e-3 rms perturbation at 1 <= |k| <= 8 that breaks the
symmetry), the averaging window (all snapshots, and those with t >= 20,
after the spin-up the paper describes) and the region of interest (the PCC
is reported over the whole box and over the box inside the sponge layers
less one filter width).  The LES masks are H_full of the FR masks.

The a-posteriori mode (--mode posteriori) steps one LES per closure (and
one without closure) from the filtered FR start with dt_LES = 1e-3 (eta =
1.025 dt_LES, as the paper uses for every run; c the default static
coefficients, the paper's tuned values not being stated) and reports
PCC(omega_LES, omega_FF), PCC(Pi_LES, Pi_FF) per snapshot and the phase
shift phi = argmin ||omega_LES(t - phi) - omega_FF(t)|| over snapshot lags
(Sec. IV-A, Table II).

Besides the PCC of the whole Pi_FF, each snapshot reports it over open
water (the region of interest where the filtered land mask is below 0.05)
and the PCC of the advection commutator alone (the analysis handles built
without penalization and sponge), to show which part of Pi_FF sets it.

Every field operation runs in the HIP library (steps, filtering, Pi_FF,
model terms, whole-box PCC); the masked PCCs are diagnostics formed here
from those fields.
"""
import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import configs, inputs
from .solver import Solver

CLOSURES = ("smag", "leith", "dsmag", "dleith")


def island_fr(n=1024, precision=64, dt=1e-4, seed=0):
    """The FR member of the island application (Sec. IV-A)."""
    lx = ly = 8.0 * math.pi
    eta = 1.025 * dt
    p = configs.base_params(n, n, lx, ly, beta=0.0, re=200.0, dt=dt, eta=eta, u_in=2.0,
                            sponge_sigma=1.0 / eta, closure="none", precision=precision)
    p["scheme"] = "ab2cn"
    chi = inputs.island_mask(n, n, lx, ly, 0.35 * lx, 0.5 * ly, math.pi / 5.0)
    chi_s = inputs.sponge_mask(n, n, lx, ly, thickness=0.05 * lx, sides="xy")
    w0 = inputs.bandpass_noise(n, n, lx, ly, seed, 1.0, 8.0, 1e-3)
    return configs.Member(p, chi, chi_s, w0, dict(geometry="island", seed=seed, lx=lx,
                                                  sponge_x=0.05 * lx, sponge_y=0.05 * lx))


def cape_fr(n=1024, precision=64, dt=1e-4, beta=0.0, seed=0):
    """The FR member of the cape application (Sec. IV-B)."""
    lx = ly = 8.0 * math.pi
    eta = 1.025 * dt
    p = configs.base_params(n, n, lx, ly, beta=beta, re=200.0, dt=dt, eta=eta, u_in=2.0,
                            sponge_sigma=1.0 / eta, closure="none", precision=precision)
    p["scheme"] = "ab2cn"
    chi = inputs.gaussian_cape_mask(n, n, lx, ly, 0.2 * lx, 4.0, 1.0)
    chi_s = inputs.sponge_mask(n, n, lx, ly, thickness=0.125 * lx, sides="xy", thickness_y=0.1 * lx)
    w0 = inputs.bandpass_noise(n, n, lx, ly, seed, 1.0, 8.0, 1e-3)
    return configs.Member(p, chi, chi_s, w0, dict(geometry="cape", seed=seed, lx=lx,
                                                  sponge_x=0.125 * lx, sponge_y=0.1 * lx))


def les_params(fr_params, delta, closure, dt=1e-3):
    """The LES member on the grid coarsened by delta: same physics, the
    closure's default coefficient (the PCC does not depend on it)."""
    p = dict(fr_params)
    p.update(nx=fr_params["nx"] // delta, ny=fr_params["ny"] // delta, closure=closure,
             c=configs.STATIC_C[closure], dt=dt, scheme="rk4")
    return p


def filtered_masks(fr, fr_solver, delta):
    """H_full of the FR masks on the LES grid, through the library's filter
    (which drops the mean mode of a state; H(0) = 1, so the mean is added
    back)."""
    lp = les_params(fr.params, delta, "none")
    zero = np.zeros((lp["ny"], lp["nx"]))
    tmp = Solver([lp], [zero], [zero], device=fr_solver.device)
    out = []
    for m in (fr.chi, fr.chi_s):
        flat = fr_solver.pack([m])
        bar = fr_solver.filter_les(tmp, flat) + float(np.mean(m))
        out.append(tmp.unpack(bar)[0].clone())
    tmp.close()
    return out


def region_of_interest(n_les, lx, sponge_x, delta_ff, sponge_y=None):
    """Boolean (ny, nx) mask of the (square) LES grid inside the sponge
    layers less one filter width."""
    x = np.arange(n_les) * (lx / n_les)
    sy = sponge_x if sponge_y is None else sponge_y
    inner_x = (x >= sponge_x + delta_ff) & (x <= lx - sponge_x - delta_ff)
    inner_y = (x >= sy + delta_ff) & (x <= lx - sy - delta_ff)
    return np.logical_and.outer(inner_y, inner_x)


def masked_pcc(a, b, mask):
    x = a[mask].double()
    y = b[mask].double()
    dx = x - x.mean()
    dy = y - y.mean()
    return float((dx * dy).mean() / torch.sqrt((dx * dx).mean() * (dy * dy).mean()))


def a_priori(fr, nsteps, every, delta=2, closures=CLOSURES, log=print, t_avg=20.0):
    """Run the FR member for nsteps, analysing every `every` steps; returns
    the per-snapshot records and the averages."""
    p = fr.params
    F = Solver([p], [fr.chi], [fr.chi_s])
    om = F.pack([fr.omega0])
    chi_bar, chs_bar = filtered_masks(fr, F, delta)
    les = {c: Solver([les_params(p, delta, c)], [chi_bar], [chs_bar]) for c in closures}
    # the same analysis with the advection commutator alone
    pj = dict(p, eta=math.inf, sponge_sigma=0.0, scheme="rk4")
    FJ = Solver([pj], [fr.chi], [fr.chi_s])
    lesj = {c: Solver([les_params(pj, delta, c)], [chi_bar], [chs_bar]) for c in closures}
    lx = fr.meta.get("lx", p["lx"])
    n_les = p["nx"] // delta
    roi = torch.as_tensor(region_of_interest(n_les, lx, fr.meta["sponge_x"], delta * lx / p["nx"],
                                             fr.meta["sponge_y"]), device=om.device)
    sea = roi & (chi_bar.view(n_les, n_les) < 0.05)
    records = []
    t0 = time.perf_counter()
    for k in range(nsteps // every):
        F.step(om, every)
        d = F.diag(om)[0][0].cpu().numpy()
        rec = dict(step=(k + 1) * every, t=(k + 1) * every * p["dt"], energy=float(d[0]),
                   enstrophy=float(d[1]), cfl=float(d[6]), nonfinite=bool(d[7] != 0))
        if rec["nonfinite"]:
            log(json.dumps(rec))
            raise RuntimeError(f"non-finite FR state at step {rec['step']}")
        for c, L in les.items():
            pi, model, _ = F.ideal_sgs(L, om, bar=False)
            rec[f"pcc_{c}"] = float(L.pcc(pi, model)[0])
            rec[f"pcc_roi_{c}"] = masked_pcc(pi.view(n_les, n_les), model.view(n_les, n_les), roi)
            rec[f"pcc_sea_{c}"] = masked_pcc(pi.view(n_les, n_les), model.view(n_les, n_les), sea)
            pij, _, _ = FJ.ideal_sgs(lesj[c], om, model=False, bar=False)
            rec[f"pcc_J_{c}"] = float(lesj[c].pcc(pij, model)[0])
            rec[f"pcc_J_sea_{c}"] = masked_pcc(pij.view(n_les, n_les), model.view(n_les, n_les), sea)
            if c == closures[0]:
                a = pi.view(n_les, n_les)
                rec["pi_rms_sea_over_land"] = float(a[sea].double().pow(2).mean().sqrt()
                                                    / a[~sea].double().pow(2).mean().sqrt())
            if c in ("dsmag", "dleith"):
                rec[f"C_{c}"] = float(L.diag(F.filter_les(L, om))[0][0, 2])
        rec["wall_s"] = round(time.perf_counter() - t0, 2)
        records.append(rec)
        log(json.dumps(rec))
    F.close()
    FJ.close()
    for L in list(les.values()) + list(lesj.values()):
        L.close()
    summary = {}
    for key in [k for k in records[0] if k.startswith("pcc_") or k.startswith("pi_rms")]:
        vals = np.array([r[key] for r in records], dtype=np.float64)
        late = np.array([r[key] for r in records if r["t"] >= t_avg], dtype=np.float64)
        summary[key] = {"mean_all": float(np.nanmean(vals)) if np.isfinite(vals).any() else None,
                        f"mean_t_ge_{t_avg:g}": (float(np.nanmean(late)) if late.size and np.isfinite(late).any()
                                                 else None)}
    return records, summary


def parse_closure(spec):
    """'smag' -> ('smag', default c); 'smag:0.15' -> ('smag', 0.15)."""
    name, _, c = spec.partition(":")
    if name not in configs.STATIC_C:
        raise ValueError(f"unknown closure {name!r}")
    return name, (float(c) if c else configs.STATIC_C[name])


def les_run_params(fr_params, delta, closure, les_dt, scheme=None):
    """An LES member that is stepped: time step les_dt, with the FR run's
    ratio eta/dt (the paper uses eta = 1.025 dt for every simulation) and
    eta_sponge = eta; the FR run's scheme unless `scheme` is given.
    closure: a name, or 'name:c' for a coefficient other than the default."""
    closure, c = parse_closure(closure)
    p = les_params(fr_params, delta, closure, dt=les_dt)
    p["c"] = c
    eta = fr_params["eta"] * les_dt / fr_params["dt"]
    p.update(eta=eta, sponge_sigma=1.0 / eta, scheme=scheme or fr_params.get("scheme", "rk4"))
    return p


def phase_shift(les_series, ff_series, times, t_min, max_lag):
    """phi = argmin over snapshot lags of the mean over t >= t_min of
    ||omega_LES(t - phi) - omega_FF(t)||_2^2 (the paper's phase shift), in
    time units; les_series, ff_series: (snapshots, points) tensors."""
    dts = float(times[1] - times[0])
    best, best_lag = None, 0
    n = len(times)
    for lag in range(-max_lag, max_lag + 1):
        ts = [i for i in range(n) if times[i] >= t_min and 0 <= i - lag < n]
        if not ts:
            continue
        idx = torch.as_tensor(ts, device=ff_series.device)
        d = les_series[idx - lag] - ff_series[idx]
        e = float((d.double() ** 2).sum(dim=1).mean())
        if best is None or e < best:
            best, best_lag = e, lag
    return best_lag * dts


def a_posteriori(fr, nsteps, every, delta=2, closures=("none",) + CLOSURES, les_dt=1e-3, log=print,
                 t_avg=20.0, max_lag=20, les_scheme=None):
    """The FR run and one LES run per closure (grid coarsened by delta, time
    step les_dt) from the filtered FR start; at every snapshot
    PCC(omega_LES, omega_FF) and PCC(Pi_LES, Pi_FF) (Pi_LES the closure's
    term at omega_LES; Pi_FF the full ideal forcing and the advection
    commutator alone); at the end the phase shift of each LES against the
    filtered field.  An LES that turns non-finite stops there: its PCCs are
    NaN from then on, its phase shift None, and the summary gives the time
    (``diverged_<closure>``)."""
    p = fr.params
    ratio = int(round(les_dt / p["dt"]))
    if ratio < 1 or every % ratio:
        raise ValueError("every must be a multiple of les_dt / dt")
    F = Solver([p], [fr.chi], [fr.chi_s])
    om = F.pack([fr.omega0])
    chi_bar, chs_bar = filtered_masks(fr, F, delta)
    # analysis handles on the LES grid (Pi_FF with the FR run's physics)
    La = Solver([les_params(p, delta, "none")], [chi_bar], [chs_bar])
    pj = dict(p, eta=math.inf, sponge_sigma=0.0, scheme="rk4")
    FJ = Solver([pj], [fr.chi], [fr.chi_s])
    LJ = Solver([les_params(pj, delta, "none")], [chi_bar], [chs_bar])
    les = {c: Solver([les_run_params(p, delta, c, les_dt, les_scheme)], [chi_bar], [chs_bar]) for c in closures}
    ff0 = F.filter_les(La, om)
    w = {c: ff0.clone() for c in closures}
    ff_hist, w_hist, times, records = [], {c: [] for c in closures}, [], []
    diverged = {}
    t0 = time.perf_counter()
    for k in range(nsteps // every):
        F.step(om, every)
        t = (k + 1) * every * p["dt"]
        for c, L in les.items():
            if c not in diverged:
                L.step(w[c], every // ratio)
        ff = F.filter_les(La, om)
        pi_ff, _, _ = F.ideal_sgs(La, om, model=False, bar=False)
        pi_j, _, _ = FJ.ideal_sgs(LJ, om, model=False, bar=False)
        rec = dict(step=(k + 1) * every, t=t)
        for c, L in les.items():
            if c not in diverged and L.diag(w[c])[0][0, 7].item() != 0:
                diverged[c] = t          # an LES that blew up: no further steps, NaN from here on
                w[c].fill_(float("nan"))
            if c in diverged:
                rec[f"pcc_w_{c}"] = float("nan")
                if not c.startswith("none"):
                    rec[f"pcc_sgs_{c}"] = rec[f"pcc_sgs_J_{c}"] = float("nan")
                w_hist[c].append(w[c].clone())
                continue
            rec[f"pcc_w_{c}"] = float(L.pcc(w[c], ff)[0])
            if not c.startswith("none"):
                pi_les = L.closure_term(w[c])
                rec[f"pcc_sgs_{c}"] = float(L.pcc(pi_les, pi_ff)[0])
                rec[f"pcc_sgs_J_{c}"] = float(L.pcc(pi_les, pi_j)[0])
            w_hist[c].append(w[c].clone())
        ff_hist.append(ff)
        times.append(t)
        rec["wall_s"] = round(time.perf_counter() - t0, 2)
        records.append(rec)
        log(json.dumps(rec))
    ffs = torch.stack(ff_hist)
    summary = {}
    for key in [k for k in records[0] if k.startswith("pcc_")]:
        late = np.array([r[key] for r in records if r["t"] >= t_avg], dtype=np.float64)
        summary[key] = float(np.nanmean(late)) if late.size and np.isfinite(late).any() else None
    for c in closures:
        summary[f"phase_{c}"] = (None if c in diverged
                                 else phase_shift(torch.stack(w_hist[c]), ffs, times, t_avg, max_lag))
        if c in diverged:
            summary[f"diverged_{c}"] = diverged[c]
    for S in [F, La, FJ, LJ] + list(les.values()):
        S.close()
    return records, summary


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("case", choices=["island", "cape"])
    ap.add_argument("--beta", type=float, default=0.0, help="cape only")
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--precision", type=int, default=64, choices=[32, 64])
    ap.add_argument("--dt", type=float, default=1e-4)
    ap.add_argument("--steps", type=int, default=1_000_000)
    ap.add_argument("--every", type=int, default=5000)
    ap.add_argument("--delta", type=int, default=2)
    ap.add_argument("--mode", choices=["priori", "posteriori"], default="priori")
    ap.add_argument("--les-dt", type=float, default=1e-3)
    ap.add_argument("--les-scheme", choices=["ab2cn", "rk4"], default=None,
                    help="time scheme of the LES runs (default: the FR run's)")
    ap.add_argument("--closures", default=None,
                    help="comma list of LES closures for --mode posteriori, each 'name' or 'name:c' "
                         "(default: none and the four closures at their default c)")
    args = ap.parse_args(argv)
    if args.case == "island":
        fr = island_fr(args.n, args.precision, args.dt)
    else:
        fr = cape_fr(args.n, args.precision, args.dt, args.beta)
    log = lambda s: print(s, flush=True)  # noqa: E731
    if args.mode == "priori":
        records, summary = a_priori(fr, args.steps, args.every, args.delta, log=log)
    else:
        kw = {} if not args.closures else {"closures": tuple(args.closures.split(","))}
        records, summary = a_posteriori(fr, args.steps, args.every, args.delta, les_dt=args.les_dt, log=log,
                                        les_scheme=args.les_scheme, **kw)
    print(json.dumps({"summary": summary, "mode": args.mode, "les_scheme": args.les_scheme,
                      "case": args.case, "beta": fr.params["beta"],
                      "n": args.n,
                      "precision": args.precision,
                      "dt": args.dt, "steps": args.steps, "every": args.every, "delta": args.delta}),
          flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
