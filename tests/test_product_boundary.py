"""Host-side checks of the product boundary (no GPU needed)."""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2108_02991_amd")


def test_product_never_imports_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith(".py"):
                tree = ast.parse(open(os.path.join(dirpath, f)).read())
                for node in ast.walk(tree):
                    if isinstance(node, ast.Import):
                        assert all(a.name.split(".")[0] != "oracle" for a in node.names), f
                    if isinstance(node, ast.ImportFrom):
                        assert (node.module or "").split(".")[0] != "oracle", f
            if f.endswith((".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_library_build_flags_disable_packed_fp32():
    from paper_2108_02991_amd import build
    flags = " ".join(build.FLAGS)
    assert "-packed-fp32-ops" in flags and "gfx950" in flags


def test_bench_clock_sampler_never_holds_the_run():
    """Without a reachable device the shader-clock sampler reports why and gives
    no figure; stop() returns at once."""
    import time
    sys.path.insert(0, ROOT)
    import bench
    c = bench.EngineClock(period_s=0.01).start(0)
    t0 = time.perf_counter()
    c.stop(wait_s=5.0)
    assert time.perf_counter() - t0 < 5.0
    if c.result() is None:
        assert c.error


def test_bench_traffic_record_is_tied_to_the_sweep_variant():
    sys.path.insert(0, ROOT)
    import bench
    w, prec = "c3_fp32_comp_8p4M", "fp32_comp"
    assert bench.recorded_traffic(w, prec, energy=False) is None
    assert bench.recorded_traffic(w, prec, kernel="log") is None
    assert bench.recorded_traffic("c5_loop", prec) is None
    assert bench.recorded_traffic(w, prec, pairs_per_launch=12345.0) is None
