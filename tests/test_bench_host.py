"""Host logic of bench.py (no GPU): the one-GPU guard, the traffic lookup
that only trusts counters taken on the current kernel sources, and the
oracle baseline's record."""
import json
import os
import subprocess
import sys

ROOT = os.path.join(os.path.dirname(__file__), "..")
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_traffic_is_used_only_for_the_profiled_sources(tmp_path, monkeypatch):
    with open(os.path.join(ROOT, "profiles", "step_fp32_8192_traffic.json")) as fh:
        prof = json.load(fh)
    assert bench.traffic_from_profiles("step_fp32_8192") == (
        prof["bytes_per_launch"] if prof["kernel_hash"] == bench.kernel_hash() else None)
    # a profile of other sources, or of another workload, is not used
    (tmp_path / "profiles").mkdir()
    stale = dict(prof, kernel_hash="0" * 16)
    (tmp_path / "profiles" / "step_fp32_8192_traffic.json").write_text(json.dumps(stale))
    current = bench.kernel_hash()
    monkeypatch.setattr(bench, "kernel_hash", lambda: current)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profiles("step_fp32_8192") is None
    assert bench.traffic_from_profiles("step_fp64_8192") is None


def test_kernel_hash_follows_code_not_comments(tmp_path, monkeypatch):
    """The sources hash that keys the counter record changes with the code of
    the step kernel's sources and not with their comments or layout."""
    src = tmp_path / "k.hip"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["k.hip"])

    def h(text):
        src.write_text(text)
        return bench.kernel_hash()

    base = h("// step\nint f(int x) {\n  return x + 1;  // one\n}\n")
    assert h("/* the step,\n   reworded */\nint f(int x) {\n    return x + 1;\n}\n") == base
    assert h("// step\nint f(int x) {\n  return x + 2;  // one\n}\n") != base
    assert h("// step\nint f(int x) {\n  return x - 1;  // one\n}\n") != base


def test_cpu_baseline_record():
    """The oracle on every host core (the threads it used are `cores`), with
    the single-thread rate beside it."""
    r = bench.cpu_baseline(seconds=0.6)
    assert r["kind"] == "oracle" and r["unit"] == "MLUPS"
    assert r["cores"] == bench.host_cores() >= 1
    assert r["value"] > 0 and r["single_thread_mlups"] > 0 and "128x128" in r["sample"]


def test_d3q19_line_reports_the_flop_roofline():
    """The D3Q19 workload is bound by its vector arithmetic: its roofline
    object is its FP32 flops per site over the kernel time against the
    unpacked FP32 vector peak (78.6 TFLOP/s), with the HBM fraction of its
    152 algorithmic bytes per site beside it."""
    class Lat:
        def __init__(self, p, stream=None):
            pass

        def step(self, n):
            pass

        def sync(self):
            pass

        def profile(self, on):
            pass

        def kernel_time(self):
            return 10.0, 10  # 1 ms per launch

    class F:
        FP32_SHIFTED = 1
        Lattice3 = Lat

        @staticmethod
        def make_params3(*a, **k):
            return None

    class Torch:
        class cuda:
            @staticmethod
            def current_stream():
                return None

    r = bench.run_d3q19(F, Torch, steps=10, warmup=1, n=64)
    rf, hb = r["roofline"], r["hbm"]
    assert abs(bench.FP32_VECTOR_PEAK - 78.6432e12) < 1e6
    tflops = bench.D3Q19_FLOPS_PER_SITE * 64 ** 3 / 1e-3 / 1e12
    assert rf["bound"] == "alu" and rf["unit"] == "TFLOP/s" and rf["peak"] == 78.6
    assert abs(rf["achieved"] - tflops) < 0.01
    assert abs(rf["frac"] - tflops / 78.6432) < 1e-3
    assert abs(hb["achieved"] - 152 * 64 ** 3 / 1e-3 / 1e9) < 0.1
