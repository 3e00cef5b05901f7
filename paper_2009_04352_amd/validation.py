"""Mean-profile validation of a channel run against the wall law (Sec. 3.2):
the L2 error norm of Eq. 19 against Spalding's law (Eq. 16) in the buffer
layer, the logarithmic layer and the whole half channel, and the log-law
intercept b of Eq. 20.

profile_metrics works on the FP64 plane statistics of a run; run() drives a
channel on the GPU (develop, then sample) and returns the metrics:

python -m paper_2009_04352_amd.validation --workload c3 --store f16 --bc wfb \
    --collision mrt --van-driest 26 --develop 400000 --sample 400000

The workload is a benchmark channel (c3, ...) or one of Table 1's cases
(A20, A40, B40, B80).
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from .channel import spalding_uplus


def profile_metrics(mean_ux, u_tau, nu0, y1=1.0, kappa=0.41, B=5.5, split=100.0):
    """Metrics of a mean streamwise profile mean_ux[y] (y = 0 .. ny - 1, walls
    below 0 and above ny - 1): the two halves are folded onto the distance
    d = y + y1 from the nearer wall (the first-layer rule), u+ = <u_x> / u_tau,
    y+ = d u_tau / nu0.  Returns the layers' y+, u+ and Spalding's u+, the
    Eq. 19 norms for y+ < split (buffer), y+ >= split (logarithmic) and all
    layers, and b = mean of u+ - ln(y+) / kappa over the logarithmic layers
    (the least-squares intercept of Eq. 20 at fixed kappa)."""
    u = np.asarray(mean_ux, dtype=np.float64)
    half = len(u) // 2
    fold = 0.5 * (u[:half] + u[::-1][:half])
    yp = (np.arange(half) + y1) * u_tau / nu0
    up = fold / u_tau
    us = np.array([spalding_uplus(v, kappa, B) for v in yp])

    def eps(mask):
        if not np.any(mask):
            return None
        return float(math.sqrt(((up[mask] - us[mask]) ** 2).sum() / (us[mask] ** 2).sum()))

    buf, log = yp < split, yp >= split
    b = float((up[log] - np.log(yp[log]) / kappa).mean()) if np.any(log) else None
    return dict(yplus=yp.tolist(), uplus=up.tolist(), spalding=us.tolist(), eps_buffer=eps(buf), eps_log=eps(log),
                eps_all=eps(np.ones_like(buf)), b=b)


def mass_check(ch, steps):
    """Appendix B (Eq. B-1, Table B-1) over `steps` single steps of a channel:
    before each step, the change of the population sum that its WFB correction
    makes at every wall cell, from the device (the step's own arithmetic).
    Returns the fraction of steps whose wall-averaged change (Eq. B-1, both
    walls) is not zero and the largest |change| over the mean population
    f_a = rho / 19 of the wall cells, and the same two figures per cell."""
    hits = cell_hits = cells = 0
    worst = cell_worst = 0.0
    for _ in range(steps):
        ds, rho = ch.wall_mass_change()
        fbar = float(rho.mean()) / 19.0
        df = float(ds.mean())
        hits += df != 0.0
        worst = max(worst, abs(df) / fbar)
        cell_hits += int(np.count_nonzero(ds))
        cells += ds.size
        cell_worst = max(cell_worst, float(np.max(np.abs(ds) / (rho / 19.0))))
        ch.step(1)
    return dict(steps=steps, rate_nonzero=hits / max(steps, 1), max_over_fbar=worst,
                cell_rate_nonzero=cell_hits / max(cells, 1), cell_max_over_fbar=cell_worst)


def run(workload="c3", store="f16", bc="wfb", collision="mrt", van_driest=26.0, develop=400000, sample=400000,
        stats_every=20, report_every=50000, pdf_bins=40, pdf_range=4.0, mass_steps=0, mrt_rates=None,
        wall_nodes=False, out=sys.stderr):
    """Develop the channel from its Spalding initial state, then sample the
    plane statistics every stats_every steps; progress lines every
    report_every steps, at which the sampling phase also takes a snapshot of
    the first-layer y+ distribution (pdf_bins bins over +-pdf_range standard
    deviations).  mrt_rates: dict of MRT rates overriding the defaults
    (keys s_e, s_eps, s_q, s_pi, s_m).  With mass_steps > 0, the Appendix B
    mass check runs over
    that many steps between the two phases.  wall_nodes: the wall grid as a
    lattice node (LBM_P_WALL_NODES 1 or 2: the stress from the first layer's
    velocity of the previous or of the same step); the channel then has ny - 1 fluid layers
    between wall nodes ny spacings apart, so that D = ny / 2 and the
    parameters are those of the halfway channel of ny layers.  Returns the
    metrics with the run's parameters and the sampled mean profile."""
    import torch

    from . import Channel
    from . import workloads as W
    p = W.params(workload)
    nx, ny, nz = p["grid"]
    tiles = W.launch_tiles(workload, store, collision) if workload in W.LAUNCH_TILES else None
    if wall_nodes:
        ny -= 1
        tiles = None
    ch = Channel(nx, ny, nz, p["tau0"], cs=p["cs"], fx=p["fx"], store=store, bc=bc,
                 tiles=tiles, collision=collision, van_driest=van_driest, mrt_rates=mrt_rates, wall_nodes=wall_nodes)
    ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
    T = (p["grid"][1] / 2.0) / p["u_tau"]  # D / u_tau in steps
    t0 = time.time()
    done = 0
    pdf_counts, pdf_mean, pdf_std, pdf_snaps = None, 0.0, 0.0, 0
    mass = None
    for phase, n in (("develop", develop), ("sample", sample)):
        if phase == "sample" and mass_steps > 0:
            mass = mass_check(ch, mass_steps)
            done += mass_steps
            print("[validation] mass check over %d steps: %s" % (mass_steps, mass), file=out, flush=True)
        if phase == "sample":
            ch.set_param(3, stats_every)   # LBM_P_STATS_EVERY
            ch.stats_reset()
        while n > 0:
            k = min(n, report_every)
            ch.step(k)
            st, first = ch.sync()
            n -= k
            done += k
            print("[validation] %s %s %s %s: step %d (%.2f T), %.0f s, status %d"
                  % (workload, store, bc, collision, done, done / T, time.time() - t0, st), file=out, flush=True)
            if st != 0:
                return dict(status=st, first_bad_step=first, steps=done)
            if phase == "sample":
                # Fig. 7: first-layer y+ normalised per snapshot, counts summed over snapshots
                c, edges, mu, sd = ch.wall_yplus_pdf(pdf_bins, -pdf_range, pdf_range)
                pdf_counts = c if pdf_counts is None else pdf_counts + c
                pdf_mean += mu
                pdf_std += sd
                pdf_snaps += 1
    m, nsamp = {}, 0
    if sample > 0:
        stats, nsamp = ch.stats()
        m = profile_metrics(stats[:, 0], p["u_tau"], p["nu0"])
        m.update(mean_ux=stats[:, 0].tolist(), mean_uxuy=stats[:, 6].tolist(), mean_ux2=stats[:, 3].tolist())
    m.update(workload=workload, grid=[nx, ny, nz], store=store, bc=bc, collision=collision,
             van_driest_aplus=van_driest, re_tau=W.case(workload)["re_tau"], u_tau=p["u_tau"], tau0=p["tau0"],
             fx=p["fx"], wall_nodes=int(wall_nodes), develop_steps=develop, sample_steps=sample,
             stats_every=stats_every, develop_T=develop / T, sample_T=sample / T, sampled_steps=nsamp, status=0,
             seconds=time.time() - t0)
    if mass is not None:
        m.update(mass_check=mass)
    if pdf_snaps:
        m.update(yplus_pdf_counts=pdf_counts.tolist(), yplus_pdf_edges=np.linspace(-pdf_range, pdf_range,
                 pdf_bins + 1).tolist(), yplus_mean=pdf_mean / pdf_snaps, yplus_std=pdf_std / pdf_snaps,
                 yplus_snapshots=pdf_snaps)
    ch.close()
    torch.cuda.empty_cache()
    return m


def main():
    ap = argparse.ArgumentParser(description="Wall-law validation run: develop the channel, sample plane "
                                 "statistics, report the Eq. 19 errors against Spalding's law and the Eq. 20 "
                                 "intercept as one JSON record.")
    ap.add_argument("--workload", default="c3", help="a Table 1 case (A20, A40, B40, B80) or a benchmark workload")
    ap.add_argument("--store", default="f16", help="population store: f64, f32, f16 or bf16")
    ap.add_argument("--bc", default="wfb", help="wall boundary: wfb, bb or freeslip")
    ap.add_argument("--collision", default="mrt", help="bgk or mrt")
    ap.add_argument("--van-driest", type=float, default=26.0, help="van Driest A+ (0: no damping)")
    ap.add_argument("--develop", type=int, default=400000, help="steps of development before sampling")
    ap.add_argument("--sample", type=int, default=400000, help="steps over which statistics are sampled")
    ap.add_argument("--stats-every", type=int, default=20, help="sample the plane statistics every k steps")
    ap.add_argument("--report-every", type=int, default=50000, help="progress line every k steps")
    ap.add_argument("--mass-steps", type=int, default=0, help="also run the Appendix B mass check over this many "
                                                              "steps (0: off)")
    ap.add_argument("--mrt-rates", default="", help="e.g. s_e=1.19,s_q=1.2 (MRT rates to override)")
    ap.add_argument("--wall-nodes", type=int, nargs="?", const=1, default=0, choices=(0, 1, 2),
                    help="the wall grid as a lattice node (LBM_P_WALL_NODES): 1 = stress of the previous step, "
                         "2 = of the same step")
    ap.add_argument("--out", default="", help="also write the record to this JSON file")
    a = ap.parse_args()
    rates = {k: float(v) for k, v in (kv.split("=") for kv in a.mrt_rates.split(",") if kv)} or None
    m = run(a.workload, a.store, a.bc, a.collision, a.van_driest, a.develop, a.sample, a.stats_every,
            a.report_every, mass_steps=a.mass_steps, mrt_rates=rates, wall_nodes=a.wall_nodes)
    if rates:
        m.update(mrt_rates=rates)
    m.update(command=" ".join(["python -m paper_2009_04352_amd.validation"] + sys.argv[1:]))
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(m, fh, indent=1)
    print(json.dumps(m))


if __name__ == "__main__":
    main()
