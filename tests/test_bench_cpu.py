"""bench.py on the CPU: the one-GPU contract and the committed profile
records it reads (no GPU, nothing timed)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_committed_traffic_records_match_the_kernel_source():
    """The HBM byte records under profiles/ were taken on the current kernel
    source, so the bench line carries them (a kernel change without new
    counters makes the bench report traffic as null)."""
    bench = _bench()
    digest = bench.kernel_digest()
    rec = bench.traffic_record(bench.TRAFFIC_FILE, "k_pr_iter_slots<2, true, true>")
    assert rec is not None, f"profiles/ sweep record is not for kernel source {digest}"
    assert rec["bytes_per_launch"] > 0 and rec["fetch_factor"] > 1.5
    loop = bench.traffic_record(bench.LOOP_TRAFFIC_FILE, "+".join(bench.LOOP_KERNELS))
    assert loop is not None and loop["bytes_per_loop"] > 0
