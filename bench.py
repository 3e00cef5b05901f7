"""Benchmark: MLUPS and HBM-roofline fraction of the fused WFB LBM-LES step on
one MI355X: the plain FP64 store (the headline) and the FP32 / FP16 / BF16
stores beside it, each reduced store with its accuracy stated against the FP64
GPU run after the workload's own step count.

Workloads (synthetic inputs generated on the device, see workloads.py):
  c5 (default)  2048 x 512 x 1024 channel (1.07G cells), Re_tau 2003, WFB
                walls, Smagorinsky Cs = 0.1, Spalding profile + 5 % seeded
                noise; accuracy after 500 steps;
  c5s           256 x 512 x 1024 (134M cells): one GPU's x-slab of c5 split over
                8 GPUs, at its real shape (periodic in x; no halo exchange);
  c3            512 x 128 x 256 channel (16.8M cells), same physics; 2,000 steps;
  c2            128 x 64 x 64 channel, Re_tau 640, FP32 with WFB and with
                bounce-back walls; 10,000 steps (40 MB of populations: it lives
                in the 256 MB Infinity Cache, so its "HBM" figures are flagged
                as cache-resident);
  c4            64 independent channels in one launch per step (FP32 store).
One step is one launch of the fused kernel over every cell (odd and even AA
kernels alternate).  Per store: W untimed warm-up steps, then K steps
bracketed by synchronisation with a HIP event recorded on the library's stream
after every launch (per-kernel durations for the roofline), then untimed
steps up to the workload's step count, after which the velocity field (on the
device) is compared with the FP64 run's.  Prints one JSON line.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5|c5s|c3|c2|c4]
                [--stores f64,f32,f16,bf16] [--no-cpu-baseline]
                [--collision bgk|mrt] [--van-driest A+]
                [--no-autotune] [--tune-steps N]
Before each store's run the library's autotuner picks the launch shapes
(timed on the run's own allocation, N steps per candidate); --no-autotune
keeps the fixed launch table of workloads.py.
The headline line is the BGK step (the default); --collision mrt with
--van-driest 26 measures the paper's LES collision on the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % of HBM roofline at 1 GPU, FP16/FP32-store vs FP64, at stated ε_u+"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
STORE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
DTYPE = {"f64": "f64", "f32": "f32", "f16": "f32", "bf16": "f32"}   # arithmetic of each store
# per workload: headline store, default timed steps and warm-up
DEFAULTS = {"c5": ("f64", 100, 20), "c5s": ("f64", 200, 20), "c3": ("f64", 1000, 200), "c2": ("f32", 2000, 200),
            "c4": ("f32", 1000, 100)}
CACHE_RESIDENT = {"c2"}        # populations fit the 256 MB Infinity Cache


def kernel_source_hash():
    """Hash of the device sources (every kernel file and header of csrc/)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2009_04352_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")) and f != "lbm_capi.hip":
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, store, kernel, name=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source and (name given) for the same
    kernel ("k_step" or "k_odd_rows"); else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source") != kernel_source_hash():
        return None
    rec = t.get("stores", {}).get(store, {}).get(kernel)
    if not rec or (name is not None and rec.get("kernel") != name):
        return None
    return rec.get("bytes_per_launch")


def timed_steps(torch, stepper, stream, steps, warmup, first_step):
    """Runs warm-up steps, then `steps` timed steps with an event after each
    launch; returns (total ms, mean odd-kernel ms, mean even-kernel ms, the
    per-step times in ms)."""
    import numpy as np
    if warmup:
        stepper(warmup)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(steps):
        stepper(1)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    total = ev[0].elapsed_time(ev[steps])
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    t_index = first_step + warmup + np.arange(steps)      # 1-based step numbers; odd ones run the odd kernel
    odd = float(per[t_index % 2 == 1].mean()) if np.any(t_index % 2 == 1) else float("nan")
    even = float(per[t_index % 2 == 0].mean()) if np.any(t_index % 2 == 0) else float("nan")
    return total, odd, even, per


def collision_kw(args):
    return dict(collision=args.collision, van_driest=args.van_driest)


def step_profile(per, first_step):
    """Per-step times summarised: the first 8 timed steps and the mean of each
    tenth of the timed region, by kernel (a cold start shows as a trend)."""
    import numpy as np
    idx = first_step + np.arange(len(per))
    out = {"first_ms": [round(float(v), 5) for v in per[:8]]}
    for name, sel in (("odd", idx % 2 == 1), ("even", idx % 2 == 0)):
        v = per[sel]
        if len(v) >= 10:
            out[name + "_tenths_ms"] = [round(float(c.mean()), 5) for c in np.array_split(v, 10)]
    return out


def run_store(P, W, name, store, bc, steps, warmup, coll, acc_steps, ref, tune_steps):
    """Times one store on one workload, then continues (untimed) to the
    workload's own step count and compares the velocity field on the device
    with the FP64 run's (ref; None for the FP64 run itself, whose fields it
    returns).  The launch shapes start from the measured table of workloads.py;
    with tune_steps > 0 the library's autotuner (lbm_autotune) then searches
    from there, timing each candidate over tune_steps steps, and the timed run
    uses its choice."""
    import torch
    p = W.params(name)
    nx, ny, nz = p["grid"]
    n = nx * ny * nz
    table = W.launch_tiles(name, store, coll["collision"])
    ch = P.Channel(nx, ny, nz, p["tau0"], cs=p["cs"], fx=p["fx"], store=store, bc=bc, tiles=table, graph_steps=0,
                   **coll)
    t0 = time.perf_counter()
    launch = ch.autotune(steps=tune_steps) if tune_steps > 0 else None
    tune_s = time.perf_counter() - t0
    if launch is None:
        from paper_2009_04352_amd import _lib as L
        launch = dict(tile_odd=int(ch.get_param(L.LBM_P_TILE_ODD)), tile_even=int(ch.get_param(L.LBM_P_TILE_EVEN)),
                      vector=int(ch.get_param(L.LBM_P_VECTOR)), brick=int(ch.get_param(L.LBM_P_BRICK)),
                      spread=int(ch.get_param(L.LBM_P_SPREAD)), odd_rows=int(ch.get_param(L.LBM_P_ODD_BY_ROWS)),
                      cached=0, xcd_chunk=int(ch.get_param(L.LBM_P_XCD_CHUNK)))
    launch.update(source="autotuned from the measured table" if tune_steps > 0 else "measured table",
                  table=list(table), tune_seconds=round(tune_s, 2))
    ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
    total_ms, odd_ms, even_ms, per = timed_steps(torch, ch.step, ch.stream, steps, warmup, 1)
    out = dict(ms_per_step=total_ms / steps, mlups=n * steps / (total_ms * 1e-3) / 1e6,
               odd_kernel_ms=odd_ms, even_kernel_ms=even_ms, odd_by_rows=int(ch.get_param(17)),
               steps_profile=step_profile(per, 1 + warmup), launch=launch)
    done = warmup + steps
    # the accuracy figures belong to the workload's own step count, whatever K and W were
    ch.set_param(8, 32)                      # LBM_P_GRAPH_STEPS: the untimed remainder runs in graphs
    if done > acc_steps:
        ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
        done = 0
    ch.step(acc_steps - done)
    status, first_bad = ch.sync()
    out.update(status=int(status), first_bad_step=int(first_bad), accuracy_steps=acc_steps)
    fields = None
    if status == 0:
        fields = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]
        ch.moments_device(None, *fields)
        torch.cuda.synchronize()
        # plane-averaged streamwise velocity per layer (FP64)
        out["profile"] = fields[0].view(nz, ny, nx).mean(dim=(0, 2)).cpu().numpy()
    ch.close()
    del ch
    torch.cuda.empty_cache()
    if fields is not None and ref is not None:
        du = 0.0
        for a, b in zip(fields, ref["fields"]):
            du = max(du, float((a - b).abs_().max()))
        prof, prof_ref = out["profile"] / p["u_tau"], ref["profile"] / p["u_tau"]
        out["max_du_over_utau_vs_f64"] = du / p["u_tau"]
        out["eps_uplus_vs_f64"] = float(math.sqrt(((prof - prof_ref) ** 2).sum() / (prof_ref ** 2).sum()))
        fields = None
        torch.cuda.empty_cache()
    return out, fields, p


def copy_probe_gbs(P, nbytes=4 << 30, reps=10):
    """HBM bandwidth of the library's copy kernel (lbm_copy_probe): bytes read
    plus bytes written per second, between two buffers and in place on one
    (the AA step's access form)."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    s = torch.cuda.current_stream()
    out = []
    for d in (dst, src):
        P.copy_probe(d, src, nbytes, s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            P.copy_probe(d, src, nbytes, s)
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out.append(2.0 * nbytes / (ms * 1e-3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return out


def _oracle_rate(O, p, grid, okw, budget_s):
    """MLUPS of the oracle on a channel of this grid from the workload's initial
    state: one untimed step, then as many steps as fit the budget."""
    nx, ny, nz = grid
    o = O.Oracle(O.make_params(nx, ny, nz, p["tau0"], cs=p["cs"], fx=p["fx"], bc=O.WFB, **okw))
    o.init_spalding(p["u_tau"], p["noise"], p["seed"])
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter() - t0
    k = max(1, min(200, int(budget_s / max(t1, 1e-6))))
    t0 = time.perf_counter()
    o.step(k)
    dt = time.perf_counter() - t0
    del o
    return nx * ny * nz * k / dt / 1e6, k, dt


def cpu_baseline(W, name, coll, budget_s=20.0, budget_1core_s=8.0):
    """The FP64 CPU oracle on this host's cores: a bounded sample of the same
    workload (the same grid from the same initial state, or a z-slab of it when
    the grid does not fit the host twice), on all cores and on one core."""
    from oracle import oracle as O
    okw = dict(collision=O.MRT if coll["collision"] == "mrt" else O.BGK, vd_aplus=coll["van_driest"])
    if name == "c4":
        ens = W.ensemble()
        o_list = []
        for e in ens:
            o = O.Oracle(O.make_params(e["nx"], e["ny"], e["nz"], e["tau"], cs=e["cs"], fx=e["fx"],
                                       bc=O.WFB if e["bc"] == "wfb" else O.BB, **okw))
            o.init_spalding(e["u_tau"], 0.05, e["seed"])
            o_list.append(o)
        cells = sum(e["nx"] * e["ny"] * e["nz"] for e in ens)
        t0 = time.perf_counter()
        for o in o_list:
            o.step(1)
        t1 = time.perf_counter() - t0
        k = max(1, min(200, int(budget_s / max(t1, 1e-6))))
        t0 = time.perf_counter()
        for o in o_list:
            o.step(k)
        dt = time.perf_counter() - t0
        return dict(value=cells * k / dt / 1e6, unit="MLUPS", cores=O.threads(), kind="oracle",
                    sample="the 64 ensemble channels, FP64, %d steps each after one untimed step (%.1f s)" % (k, dt))
    p = W.params(name)
    nx, ny, nz = p["grid"]
    slab = nx * ny * nz > (64 << 20)          # a z-slab of the large channel fits the host
    grid = (nx, ny, 16 if slab else nz)
    cores = O.threads()
    rate, k, dt = _oracle_rate(O, p, grid, okw, budget_s)
    grid1 = (nx, ny, 2 if slab else nz)
    O.set_threads(1)
    try:
        rate1, k1, dt1 = _oracle_rate(O, p, grid1, okw, budget_1core_s)
    finally:
        O.set_threads(cores)
    sample = ("%dx%dx%d channel%s, WFB, FP64, %d steps after one untimed step (%.1f s) on %d threads; "
              "one core: %dx%dx%d, %d steps (%.1f s)" % (grid + (" (z-slab of the workload)" if slab else "",
                                                                 k, dt, cores) + grid1 + (k1, dt1)))
    return dict(value=rate, unit="MLUPS", cores=cores, kind="oracle", sample=sample, value_1core=rate1)


def roofline(per, kernel_key, n_cells, workload, collision="bgk"):
    kern = per["dominant_kernel"]
    # the committed counter summaries were taken with the BGK kernels
    name = "k_odd_rows" if (kern == "odd" and per.get("odd_by_rows")) else "k_step"
    traffic = measured_traffic(workload, kernel_key, kern, name) if collision == "bgk" else None
    r = dict(bound="hbm", achieved=per["kernel_gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
             frac=per["kernel_gbs"] / HBM_PEAK_GBS, traffic=traffic,
             kernel=(("k_odd_rows odd (one wavefront per row; pull/push with wall reflections)"
                      if per.get("odd_by_rows") else "k_step odd (pull/push with wall reflections)")
                     if kern == "odd" else "k_step even (local)"),
             kernel_ms=per[kern + "_kernel_ms"], algorithmic_bytes_per_launch=per["bytes_per_cell"] * n_cells)
    if workload in CACHE_RESIDENT:
        r["cache_resident"] = True
    return r


def store_record(r, s, n, copy_gbs):
    bytes_cell = 38 * STORE_BYTES[s]
    kern = "odd" if r["odd_kernel_ms"] >= r["even_kernel_ms"] else "even"
    gbs = bytes_cell * n / (r[kern + "_kernel_ms"] * 1e-3) / 1e9
    d = dict(mlups=r["mlups"], ms_per_step=r["ms_per_step"], bytes_per_cell=bytes_cell,
             odd_kernel_ms=r["odd_kernel_ms"], even_kernel_ms=r["even_kernel_ms"], dominant_kernel=kern,
             kernel_gbs=gbs, hbm_frac=gbs / HBM_PEAK_GBS, odd_by_rows=r.get("odd_by_rows", 0),
             step_gbs=bytes_cell * n / (r["ms_per_step"] * 1e-3) / 1e9, status=r["status"])
    for k in ("first_bad_step", "accuracy_steps", "max_du_over_utau_vs_f64", "eps_uplus_vs_f64", "steps_profile",
              "launch"):
        if k in r:
            d[k] = r[k]
    if copy_gbs:
        d["copy_frac"] = gbs / copy_gbs
    return d


def bench_single(P, W, args, copy_gbs):
    stores = args.stores.split(",")
    if "f64" not in stores:
        stores = ["f64"] + stores
    stores = ["f64"] + [s for s in stores if s != "f64"]     # the reference runs first
    wl = W.WORKLOADS[args.workload]
    nx, ny, nz = wl["grid"]
    n = nx * ny * nz
    acc_steps = wl["steps"]
    head = DEFAULTS[args.workload][0]
    bcs = wl["bcs"]
    per_bc = {}
    for bc in bcs:
        ref = None
        per_store = {}
        for s in stores:
            r, fields, p = run_store(P, W, args.workload, s, bc, args.steps, args.warmup, collision_kw(args),
                                     acc_steps, ref, 0 if args.no_autotune else args.tune_steps)
            if s == "f64":
                ref = dict(fields=fields, profile=r.get("profile")) if fields is not None else None
            print("[bench] %s %s: %.1f MLUPS, odd %.4f ms, even %.4f ms, status %d, max|du|/u_tau %s after %d steps"
                  % (bc, s, r["mlups"], r["odd_kernel_ms"], r["even_kernel_ms"], r["status"],
                     r.get("max_du_over_utau_vs_f64"), acc_steps), file=sys.stderr, flush=True)
            d = store_record(r, s, n, copy_gbs)
            per_store[s] = d
        for s in stores:
            per_store[s]["mlups_gain_vs_f64"] = per_store[s]["mlups"] / per_store["f64"]["mlups"]
        per_bc[bc] = per_store
        ref = None
        import torch
        torch.cuda.empty_cache()
    per_store = per_bc[bcs[0]]
    if head not in per_store:
        head = stores[0]
    hd = per_store[head]
    config = {"workload": "%s: %s; %d steps timed per store after %d warm-up steps, accuracy after %d steps"
                          % (args.workload, wl["desc"], args.steps, args.warmup, acc_steps),
              "grid": [nx, ny, nz], "store": head, "boundary": bcs[0], "re_tau": wl["re_tau"], "tau0": p["tau0"],
              "fx": p["fx"], "launch": hd["launch"],
              "collision": args.collision, "van_driest_aplus": args.van_driest, "parallelism": "single GPU",
              "timed_steps": args.steps, "accuracy_steps": acc_steps}
    if args.workload in CACHE_RESIDENT:
        config["cache_resident"] = True
    roof = roofline(hd, head, n, args.workload, args.collision)
    extra = {"per_boundary": per_bc} if len(bcs) > 1 else {}
    return hd, per_store, config, roof, DTYPE[head], extra


def bench_ensemble(P, W, args, copy_gbs):
    import torch
    ens = W.ensemble(W.ENSEMBLE["n"])
    store = W.ENSEMBLE["store"]
    n = sum(e["nx"] * e["ny"] * e["nz"] for e in ens)
    b = P.Batch(ens, store=store, graph_steps=0, **collision_kw(args))
    tiles = None if args.no_autotune else b.autotune(steps=6)   # None: the library's default shapes
    launch = list(tiles) if tiles else "library default"
    b.init_spalding([e["u_tau"] for e in ens], 0.05, seeds=[e["seed"] for e in ens])
    total_ms, odd_ms, even_ms, per = timed_steps(torch, b.step, b.stream, args.steps, args.warmup, 1)
    status, first, inst = b.sync()
    r = dict(ms_per_step=total_ms / args.steps, mlups=n * args.steps / (total_ms * 1e-3) / 1e6,
             odd_kernel_ms=odd_ms, even_kernel_ms=even_ms, status=int(status))
    # the same work through captured graphs, the production path
    b2 = P.Batch(ens, store=store, tiles=tiles, graph_steps=50, **collision_kw(args))
    b2.init_spalding([e["u_tau"] for e in ens], 0.05, seeds=[e["seed"] for e in ens])
    b2.step(100)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g_steps = args.steps - args.steps % 50 if args.steps >= 50 else 50
    e0.record(b2.stream)
    b2.step(g_steps)
    e1.record(b2.stream)
    torch.cuda.synchronize()
    graph_mlups = n * g_steps / (e0.elapsed_time(e1) * 1e-3) / 1e6
    print("[bench] ensemble: %.1f MLUPS eager, %.1f MLUPS graphs, odd %.4f ms, even %.4f ms, tiles %s"
          % (r["mlups"], graph_mlups, odd_ms, even_ms, tiles), file=sys.stderr, flush=True)
    d = store_record(r, store, n, copy_gbs)
    d["graph_mlups"] = graph_mlups
    d["launch"] = launch
    config = {"workload": "c4: %s; %d steps timed after %d warm-up steps" % (W.ENSEMBLE["desc"], args.steps,
                                                                              args.warmup),
              "instances": len(ens), "cells": n, "store": store, "launch": launch, "parallelism": "single GPU",
              "timed_steps": args.steps}
    b.close()
    b2.close()
    config.update(collision=args.collision, van_driest_aplus=args.van_driest)
    return d, {store: d}, config, roofline(d, store, n, "c4", args.collision), "f32", {}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps per store (default per workload)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed warm-up steps (default per workload)")
    ap.add_argument("--workload", default="c5", choices=("c5", "c5s", "c3", "c2", "c4"))
    ap.add_argument("--stores", default=None, help="comma list (default f64,f32,f16,bf16; c2: f64,f32)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="time the measured launch table as it is")
    ap.add_argument("--tune-steps", type=int, default=4, help="steps timed per autotuner candidate")
    ap.add_argument("--collision", default="bgk", choices=("bgk", "mrt"),
                    help="collision operator (mrt: the paper's LES collision)")
    ap.add_argument("--van-driest", type=float, default=0.0, help="van Driest A+ (0: no damping)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the channel step runs on a single MI355X here; "
              "the multi-GPU slab decomposition is not implemented (--gpus %d refused)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    _, k_def, w_def = DEFAULTS[args.workload]
    args.steps = k_def if args.steps is None else args.steps
    args.warmup = w_def if args.warmup is None else args.warmup
    if args.stores is None:
        args.stores = "f64,f32" if args.workload == "c2" else "f64,f32,f16,bf16"
    if args.steps < 2:
        print("--steps must be >= 2 (one odd and one even kernel)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2009_04352_amd as P
    from paper_2009_04352_amd import workloads as W

    torch.cuda.set_device(0)
    copies = None if args.no_copy_probe else copy_probe_gbs(P)
    copy_gbs = max(copies) if copies else None     # the better of the two forms: the ceiling for copy_frac
    if args.workload == "c4":
        hd, per_store, config, roof, dtype, extra = bench_ensemble(P, W, args, copy_gbs)
    else:
        hd, per_store, config, roof, dtype, extra = bench_single(P, W, args, copy_gbs)
    line = {
        "metric": METRIC,
        "value": hd["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hd["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": config,
        "roofline": roof,
        "per_store": per_store,
        "copy_probe_gbs": {"two_buffers": copies[0], "in_place": copies[1]} if copies else None,
        "kernel_source": kernel_source_hash(),
    }
    line.update(extra)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(W, args.workload, collision_kw(args))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
