"""The benchmark's command-line contract that holds without a GPU: more than
one GPU is refused with a message, the options parse, the kernel source hash
covers the device sources, and committed traffic summaries are used only for
the kernel sources they were taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_the_options():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for opt in ("--steps", "--warmup", "--workload", "--stores", "--collision", "--van-driest", "--no-autotune",
                "--tune-steps"):
        assert opt in r.stdout
    for wl in ("c5", "c5s", "c3", "c2", "c4"):
        assert wl in r.stdout


def test_every_single_channel_workload_has_defaults_and_a_launch_table():
    import bench
    from paper_2009_04352_amd import workloads as W
    for wl in ("c5", "c5s", "c3", "c2"):
        store, steps, warmup = bench.DEFAULTS[wl]
        assert store in W.WORKLOADS[wl]["stores"] or store == "f64"
        assert steps >= 2 and warmup >= 0
        for s in ("f64", "f32", "f16", "bf16"):
            odd, even, v = W.launch_tiles(wl, s)
            assert odd in (64, 128, 256, 512) and even in (64, 128, 256, 512) and v in (1, 2, 4)
    assert bench.DEFAULTS["c5"][0] == "f64"          # the headline store


def test_traffic_used_only_for_its_kernel_sources(tmp_path, monkeypatch):
    import bench
    h = bench.kernel_source_hash()
    assert len(h) == 16
    for wl in ("c3", "c5"):
        path = os.path.join(ROOT, "profiles", "traffic_%s.json" % wl)
        with open(path) as fh:
            t = json.load(fh)
        if t["kernel_source"] == h:
            rec = t["stores"]["f16"]["odd"]
            assert bench.measured_traffic(wl, "f16", "odd") == rec["bytes_per_launch"]
            assert bench.measured_traffic(wl, "f16", "odd", rec["kernel"]) == rec["bytes_per_launch"]
            # a record of the other odd kernel is not used for this one
            other = "k_step" if rec["kernel"] == "k_odd_rows" else "k_odd_rows"
            assert bench.measured_traffic(wl, "f16", "odd", other) is None
            # a traffic figure within 3 % of the algorithmic bytes: no re-reads
            assert abs(rec["bytes_per_launch"] / rec["algorithmic"] - 1.0) <= 0.03
    # a summary taken on other sources is ignored
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("c3", "f16", "odd") is None


def test_roofline_is_algorithmic_bytes_over_the_dominant_kernel_time():
    """The line's roofline object: the dominant (slower) kernel's algorithmic
    bytes (38 x cells x store bytes) over its measured time, against the
    8 TB/s HBM peak; traffic only from the BGK counter records."""
    import bench
    n = 2048 * 512 * 1024
    r = dict(mlups=20000.0, ms_per_step=52.0, odd_kernel_ms=52.5, even_kernel_ms=51.0, status=0)
    d = bench.store_record(r, "f64", n, 6500.0)
    assert d["dominant_kernel"] == "odd" and d["bytes_per_cell"] == 38 * 8
    roof = bench.roofline(d, "f64", n, "c5")
    want = 38 * 8 * n / 52.5e-3 / 1e9
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert abs(roof["achieved"] - want) <= 1e-9 * want and abs(roof["frac"] - want / 8000.0) <= 1e-12
    assert roof["algorithmic_bytes_per_launch"] == 38 * 8 * n and roof["kernel_ms"] == 52.5
    assert abs(d["copy_frac"] - want / 6500.0) <= 1e-12
    # the even kernel dominates when it is the slower one; MRT runs report no traffic
    r2 = dict(r, odd_kernel_ms=50.0)
    d2 = bench.store_record(r2, "f16", n, None)
    assert d2["dominant_kernel"] == "even" and "copy_frac" not in d2
    assert bench.roofline(d2, "f16", n, "c5", collision="mrt")["traffic"] is None
