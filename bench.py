"""Benchmark: MLUPS and HBM-roofline fraction of the fused WFB LBM-LES step on
one MI355X, FP16 / FP32 / BF16 stores against the plain FP64 store, with the
accuracy of each reduced store stated against the FP64 GPU run.

Workloads (synthetic inputs generated on the device, see workloads.py):
  c3 (default)  512 x 128 x 256 channel (16.8M cells), Re_tau 2003, WFB walls,
                Smagorinsky Cs = 0.1, Spalding profile + 5 % seeded noise;
  c5            2048 x 512 x 1024 channel (1.07B cells), same physics;
  c4            64 independent channels in one launch per step (FP32 store).
One step is one launch of the fused kernel over every cell (odd and even AA
kernels alternate).  Timing: W untimed warm-up steps (default 200: in a
fresh process the first ~100 odd steps of the 2-byte stores run up to 30 %
slower, on MI355X, than the steady state a long run sees), then K steps
bracketed by synchronisation, a HIP event recorded on the library's stream
after every launch (per-kernel durations for the roofline).  Prints one
JSON line.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c4|c5]
                [--stores f64,f32,f16,bf16] [--no-cpu-baseline]
                [--collision bgk|mrt] [--van-driest A+]
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
HEADLINE = "f16"
FULL_FIELD_LIMIT = 64 << 20    # cells; larger grids compare sampled cells


def kernel_source_hash():
    """Hash of the device sources (every kernel file and header of csrc/)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2009_04352_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")) and f != "lbm_capi.hip":
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, store, kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source") != kernel_source_hash():
        return None
    rec = t.get("stores", {}).get(store, {}).get(kernel)
    return rec.get("bytes_per_launch") if rec else None


def timed_steps(torch, stepper, stream, steps, warmup, first_step):
    """Runs warm-up steps, then `steps` timed steps with an event after each
    launch; returns (total ms, mean odd-kernel ms, mean even-kernel ms)."""
    import numpy as np
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
    return total, odd, even


def collision_kw(args):
    return dict(collision=args.collision, van_driest=args.van_driest)


def run_store(P, W, name, store, steps, warmup, coll):
    import numpy as np
    import torch
    p = W.params(name)
    nx, ny, nz = p["grid"]
    n = nx * ny * nz
    ch = P.Channel(nx, ny, nz, p["tau0"], cs=p["cs"], fx=p["fx"], store=store, bc="wfb",
                   tiles=W.launch_tiles(name, store, coll["collision"]), graph_steps=0, **coll)
    ch.init_spalding(p["u_tau"], p["noise"], p["seed"])
    total_ms, odd_ms, even_ms = timed_steps(torch, ch.step, ch.stream, steps, warmup, 1)
    status, first_bad = ch.sync()
    out = dict(ms_per_step=total_ms / steps, mlups=n * steps / (total_ms * 1e-3) / 1e6,
               odd_kernel_ms=odd_ms, even_kernel_ms=even_ms, status=int(status), first_bad_step=int(first_bad),
               odd_by_rows=int(ch.get_param(17)))
    acc = None
    if status == 0:
        cells = W.sample_cells(p["grid"], 200000, seed=7)
        if n <= FULL_FIELD_LIMIT:
            rho, ux, uy, uz = ch.moments()
            fields = (ux, uy, uz)
        else:
            m = ch.moments_cells(cells)
            fields = (m[:, 1], m[:, 2], m[:, 3])
        # plane-averaged streamwise profile: one further (untimed) step sampled into the FP64 statistics
        ch.set_param(3, 1)
        ch.stats_reset()
        ch.step(1)
        st, _ = ch.stats()
        acc = dict(fields=fields, profile=st[:, 0])
    ch.close()
    del ch
    torch.cuda.empty_cache()
    return out, acc, p


def copy_probe_gbs(P, nbytes=4 << 30, reps=10):
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    s = torch.cuda.current_stream()
    P.copy_probe(dst, src, nbytes, s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        P.copy_probe(dst, src, nbytes, s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(W, name, coll, budget_s=20.0):
    """The FP64 CPU oracle on this host's cores: a bounded sample of the same
    workload (the same grid from the same initial state, a few steps)."""
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
        sample = "the 64 ensemble channels, FP64, %d steps each after one untimed step (%.1f s)" % (k, dt)
    else:
        p = W.params(name)
        nx, ny, nz = p["grid"]
        if nx * ny * nz > FULL_FIELD_LIMIT:   # a z-slab of the large channel fits the host
            nz = 16
        cells = nx * ny * nz
        o = O.Oracle(O.make_params(nx, ny, nz, p["tau0"], cs=p["cs"], fx=p["fx"], bc=O.WFB, **okw))
        o.init_spalding(p["u_tau"], p["noise"], p["seed"])
        t0 = time.perf_counter()
        o.step(1)
        t1 = time.perf_counter() - t0
        k = max(1, min(200, int(budget_s / max(t1, 1e-6))))
        t0 = time.perf_counter()
        o.step(k)
        dt = time.perf_counter() - t0
        sample = "%dx%dx%d channel, WFB, FP64, %d steps after one untimed step (%.1f s)" % (nx, ny, nz, k, dt)
        del o
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=cells * k / dt / 1e6, unit="MLUPS", cores=cores, kind="oracle", sample=sample)


def roofline(per, kernel_key, n_cells, workload, collision="bgk"):
    kern = per["dominant_kernel"]
    # the committed counter summaries were taken with the BGK kernels
    traffic = measured_traffic(workload, kernel_key, kern) if collision == "bgk" else None
    return dict(bound="hbm", achieved=per["kernel_gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                frac=per["kernel_gbs"] / HBM_PEAK_GBS, traffic=traffic,
                kernel=(("k_odd_rows odd (one wavefront per row; pull/push with wall reflections)"
                         if per.get("odd_by_rows") else "k_step odd (pull/push with wall reflections)")
                        if kern == "odd" else "k_step even (local)"),
                kernel_ms=per[kern + "_kernel_ms"], algorithmic_bytes_per_launch=per["bytes_per_cell"] * n_cells)


def store_record(r, s, n, copy_gbs):
    bytes_cell = 38 * STORE_BYTES[s]
    kern = "odd" if r["odd_kernel_ms"] >= r["even_kernel_ms"] else "even"
    gbs = bytes_cell * n / (r[kern + "_kernel_ms"] * 1e-3) / 1e9
    d = dict(mlups=r["mlups"], ms_per_step=r["ms_per_step"], bytes_per_cell=bytes_cell,
             odd_kernel_ms=r["odd_kernel_ms"], even_kernel_ms=r["even_kernel_ms"], dominant_kernel=kern,
             kernel_gbs=gbs, hbm_frac=gbs / HBM_PEAK_GBS, odd_by_rows=r.get("odd_by_rows", 0),
             step_gbs=bytes_cell * n / (r["ms_per_step"] * 1e-3) / 1e9, status=r["status"])
    if copy_gbs:
        d["copy_frac"] = gbs / copy_gbs
    return d


def bench_single(P, W, args, copy_gbs):
    import numpy as np
    stores = args.stores.split(",")
    if "f64" not in stores:
        stores = ["f64"] + stores
    wl = W.WORKLOADS[args.workload]
    nx, ny, nz = wl["grid"]
    n = nx * ny * nz
    res, acc = {}, {}
    for s in stores:
        r, a, p = run_store(P, W, args.workload, s, args.steps, args.warmup, collision_kw(args))
        print("[bench] %s: %.1f MLUPS, odd %.4f ms, even %.4f ms, status %d"
              % (s, r["mlups"], r["odd_kernel_ms"], r["even_kernel_ms"], r["status"]), file=sys.stderr, flush=True)
        res[s], acc[s] = r, a
    u_tau = p["u_tau"]
    ref = acc.get("f64")
    per_store = {}
    for s in stores:
        d = store_record(res[s], s, n, copy_gbs)
        if ref is not None and acc[s] is not None:
            du = max(float(np.abs(a - b).max()) for a, b in zip(acc[s]["fields"], ref["fields"]))
            prof, prof_ref = acc[s]["profile"] / u_tau, ref["profile"] / u_tau
            d["max_du_over_utau_vs_f64"] = du / u_tau
            d["eps_uplus_vs_f64"] = float(math.sqrt(((prof - prof_ref) ** 2).sum() / (prof_ref ** 2).sum()))
        d["mlups_gain_vs_f64"] = res[s]["mlups"] / res["f64"]["mlups"]
        per_store[s] = d
    head = HEADLINE if HEADLINE in per_store else stores[-1]
    hd = per_store[head]
    config = {"workload": "%s: %s" % (args.workload, wl["desc"]), "grid": [nx, ny, nz], "store": head,
              "boundary": "wfb", "re_tau": wl["re_tau"], "tau0": p["tau0"], "fx": p["fx"],
              "launch": list(W.launch_tiles(args.workload, head, args.collision)), "collision": args.collision,
              "van_driest_aplus": args.van_driest, "parallelism": "single GPU"}
    roof = roofline(hd, head, n, args.workload, args.collision)
    return hd, per_store, config, roof, "f32" if head != "f64" else "f64"


def bench_ensemble(P, W, args, copy_gbs):
    import torch
    ens = W.ensemble(W.ENSEMBLE["n"])
    store = W.ENSEMBLE["store"]
    n = sum(e["nx"] * e["ny"] * e["nz"] for e in ens)
    b = P.Batch(ens, store=store, graph_steps=0, **collision_kw(args))
    tiles = b.autotune(steps=6)
    b.init_spalding([e["u_tau"] for e in ens], 0.05, seeds=[e["seed"] for e in ens])
    total_ms, odd_ms, even_ms = timed_steps(torch, b.step, b.stream, args.steps, args.warmup, 1)
    status, first, inst = b.sync()
    r = dict(ms_per_step=total_ms / args.steps, mlups=n * args.steps / (total_ms * 1e-3) / 1e6,
             odd_kernel_ms=odd_ms, even_kernel_ms=even_ms, status=int(status))
    # the same work through captured graphs, the production path
    b2 = P.Batch(ens, store=store, tiles=tiles, graph_steps=50, **collision_kw(args))
    b2.init_spalding([e["u_tau"] for e in ens], 0.05, seeds=[e["seed"] for e in ens])
    b2.step(100)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(b2.stream)
    b2.step(args.steps - args.steps % 50 if args.steps >= 50 else 50)
    e1.record(b2.stream)
    torch.cuda.synchronize()
    g_steps = args.steps - args.steps % 50 if args.steps >= 50 else 50
    graph_mlups = n * g_steps / (e0.elapsed_time(e1) * 1e-3) / 1e6
    print("[bench] ensemble: %.1f MLUPS eager, %.1f MLUPS graphs, odd %.4f ms, even %.4f ms, tiles %s"
          % (r["mlups"], graph_mlups, odd_ms, even_ms, tiles), file=sys.stderr, flush=True)
    d = store_record(r, store, n, copy_gbs)
    d["graph_mlups"] = graph_mlups
    d["launch"] = list(tiles)
    config = {"workload": "c4: " + W.ENSEMBLE["desc"], "instances": len(ens), "cells": n, "store": store,
              "launch": list(tiles), "parallelism": "single GPU"}
    b.close()
    b2.close()
    config.update(collision=args.collision, van_driest_aplus=args.van_driest)
    return d, {store: d}, config, roofline(d, store, n, "c4", args.collision), "f32"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="c3", choices=("c3", "c4", "c5"))
    ap.add_argument("--stores", default="f64,f32,f16,bf16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--collision", default="bgk", choices=("bgk", "mrt"),
                    help="collision operator (mrt: the paper's LES collision)")
    ap.add_argument("--van-driest", type=float, default=0.0, help="van Driest A+ (0: no damping)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the channel step runs on a single MI355X here; "
              "the multi-GPU slab decomposition is not implemented (--gpus %d refused)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2009_04352_amd as P
    from paper_2009_04352_amd import workloads as W

    torch.cuda.set_device(0)
    copy_gbs = None if args.no_copy_probe else copy_probe_gbs(P)
    if args.workload == "c4":
        hd, per_store, config, roof, dtype = bench_ensemble(P, W, args, copy_gbs)
    else:
        hd, per_store, config, roof, dtype = bench_single(P, W, args, copy_gbs)
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
        "copy_probe_gbs": copy_gbs,
        "kernel_source": kernel_source_hash(),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(W, args.workload, collision_kw(args))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
