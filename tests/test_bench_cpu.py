"""Host-side contract of bench.py (no GPU): the one-GPU refusal, the kernel
table behind the profile hashes, and the traffic lookup."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_every_variant_is_described_and_hashed():
    b = load_bench()
    for v, (name, prefix, srcs) in b.KERNELS.items():
        assert name.startswith("k_sweep") and prefix
        for f in srcs:
            assert os.path.exists(os.path.join(ROOT, "paper_2009_04619_amd", "csrc", f)), f
        assert len(b.kernel_source_sha(v)) == 16
        assert isinstance(b.describe((v, 1, 16, 64)), str)


def test_traffic_lookup_follows_the_kernel_hash():
    """A committed traffic summary is used only while its kernel hash matches
    the sources, and a listed tile instance takes precedence."""
    b = load_bench()
    p = os.path.join(ROOT, "profiles", "traffic_sweep_512cube_w20_f32.json")
    t = json.load(open(p))
    got = b.measured_traffic("512cube_w20_f32", 0.0, 1, tile=(1, 16))
    if t["kernel_sha"] == b.kernel_source_sha(1):
        inst = t["instances"].get("1,16")
        want = inst["hbm_bytes_per_launch"] if inst else t["hbm_bytes_per_launch"]
        assert got == float(want)
    else:
        assert got is None
    assert b.measured_traffic("7cube_w1_f32", 0.0, 1) is None
