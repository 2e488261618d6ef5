"""Host checks of the measurement logic of bench.py (no GPU): the roofline
object, the choice of the roofline kernel, the committed HBM-traffic
records and the one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_roofline_kernel_is_the_slowest_single_kernel_class():
    stats = {
        "jacobi_svd": {"ms": 900.0},  # a whole routine, not one kernel
        "jacobi_cross": {"ms": 600.0},
        "zgemm": {"ms": 400.0},
        "jacobi_svds": {"ms": 0.0},  # an event counter
        "qr_fallbacks": {"ms": 0.0},
    }
    assert bench.dominant(stats) == "jacobi_cross"
    assert not (bench.COUNTERS & set(bench.KERNEL_BOUND))


@pytest.mark.parametrize("name,bound,peak,unit", [
    ("jacobi_cross", "alu", bench.PEAK_F64_TFLOPS, "TFLOP/s"),
    ("zgemm", "mfma", bench.PEAK_F64_TFLOPS, "TFLOP/s"),
    ("zgemm_fp16x3", "mfma", bench.PEAK_F16_TFLOPS, "TFLOP/s"),
    ("zgemm_fp32", "mfma", bench.PEAK_F32_TFLOPS, "TFLOP/s"),
    ("gather_left", "hbm", bench.PEAK_HBM_GBS, "GB/s"),
])
def test_roofline_object(name, bound, peak, unit):
    # 2,000 launches, 10 ms in all, 1.572e11 flops and 4e9 bytes
    kd = {"ms": 10.0, "flops": 1.572e11, "bytes": 4e9, "launches": 2000}
    r = bench.roofline(name, kd, with_traffic=False)
    assert r["bound"] == bound and r["peak"] == peak and r["unit"] == unit and r["kernel"] == name
    want = 4e9 / 0.01 / 1e9 if bound == "hbm" else 1.572e11 / 0.01 / 1e12
    assert r["achieved"] == pytest.approx(want)
    assert r["frac"] == pytest.approx(want / peak)
    assert r["avg_launch_us"] == pytest.approx(5.0)
    assert r["algorithmic_flops_per_launch"] == pytest.approx(1.572e11 / 2000)
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(4e9 / 2000)
    assert r["traffic"] is None
    assert set(r) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}


def test_traffic_records_name_their_summaries():
    """Every committed traffic record names an existing source and profile
    summary that quotes its per-launch figure; bench.py reports the record
    only while the source hash matches."""
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        recs = json.load(fh)
    assert recs
    for name, rec in recs.items():
        assert name in bench.KERNEL_BOUND
        assert os.path.exists(os.path.join(ROOT, rec["source"]))
        summary = os.path.join(ROOT, rec["summary"])
        assert os.path.exists(summary)
        assert rec["bytes_per_launch"] > 0
        kib = f"{rec['bytes_per_launch'] / 1024:.1f} KiB"
        with open(summary) as fh:
            assert kib in fh.read(), (name, kib)
        got = bench.traffic_per_launch(name)
        assert got is None or got == rec["bytes_per_launch"]
    assert bench.traffic_per_launch("no_such_kernel") is None


def test_profile_commands_run_committed_files_only():
    """Every command quoted in a profile summary (indented lines starting
    with rocprofv3 or python3) runs scripts, modules and test files of this
    repository that exist, and gives the summary's output directory under
    gpurun_out/ rather than a path outside the repository."""
    import glob
    import re

    pdir = os.path.join(ROOT, "profiles")
    summaries = sorted(glob.glob(os.path.join(pdir, "*.md")))
    assert summaries
    for path in summaries:
        commands = 0
        with open(path) as fh:
            for line in fh:
                if not re.match(r"^    (rocprofv3|python3?) ", line):
                    continue
                commands += 1
                for mod in re.findall(r"-m (paper_2403_04946_amd\.[a-z_0-9]+)", line):
                    assert os.path.exists(os.path.join(ROOT, *mod.split(".")) + ".py"), (path, mod)
                for script in re.findall(r"(?<![\w/.-])([\w/]+\.py)\b", line):
                    assert os.path.exists(os.path.join(ROOT, script)), (path, script)
                assert "/root/" not in line and "_work/" not in line, (path, line)
        assert commands >= 1, f"{path} quotes no command that made it"
