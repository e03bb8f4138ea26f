"""Host logic of the benchmark: algorithmic bytes, the committed counter
summaries it reads (and refuses once the kernel sources change), the VALU
bound, and the single-GPU guard."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1710_01758_amd import inputs as gen  # noqa: E402


def test_apply_bytes_is_eight_bytes_per_element_of_x_maps_and_y():
    spec = gen.SliceSpec(256, 256, 12, 4.0, 24, wavelet="db4", levels=3)
    assert bench.apply_bytes([spec]) == 8 * 256 * 256 * 14
    assert bench.apply_bytes([spec] * bench.ROOFLINE_BATCH) == 939_524_096
    ragged = [gen.SliceSpec(128, 128, 8, 3.0, 8), gen.SliceSpec(320, 320, 32, 6.0, 16)]
    assert bench.apply_bytes(ragged) == 8 * (128 * 128 * 10 + 320 * 320 * 34)


def test_committed_summaries_match_the_kernel_sources():
    f = bench.profile_fields(bench.TRAFFIC_PROFILE)
    assert f is not None, "the traffic summary no longer matches the operator kernel's sources"
    t = bench.measured_traffic()
    assert t == int(f["traffic_bytes_per_launch"])
    # a counted figure in the plausible range: at least the algorithmic bytes,
    # at most twice them
    alg = bench.apply_bytes([gen.SliceSpec(256, 256, 12, 4.0, 24)] * bench.ROOFLINE_BATCH)
    assert alg <= t <= 2 * alg
    v = bench.valu_roofline(261e-6)
    assert v is not None and v["bound"] == "alu"
    floor = v["valu_wave_instr_per_launch"] * 4 / (bench.SIMDS * bench.PEAK_CLOCK_HZ)
    assert v["floor_us_at_peak_clock"] == pytest.approx(floor * 1e6, abs=0.01)
    assert v["frac"] == pytest.approx(floor / 261e-6, abs=1e-4)


def test_summary_is_refused_after_a_source_change(tmp_path):
    src = bench.TRAFFIC_PROFILE
    dst = tmp_path / os.path.basename(src)
    txt = open(src).read()
    f = bench.profile_fields(src)
    dst.write_text(txt.replace(f["kernel_source_sha256"].strip(), "0" * 64))
    assert bench.profile_fields(str(dst)) is None
    shutil.copy(src, dst)
    assert bench.profile_fields(str(dst)) is not None
    assert bench.profile_fields(str(tmp_path / "missing.md")) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_all_cores_oracle_baseline_sums_the_workers():
    """Two single-threaded oracle workers, each at least one full
    reconstruction: the reported rate is the sum of the workers' rates."""
    r = bench.cpu_baseline_all_cores(2, seconds=0.1)
    assert r["cores"] == 2 and r["count"] >= 2
    assert 0 < r["value"] <= r["count"] / min(0.1, r["seconds"]) and r["unit"] == "recons/s"


def test_reconstruction_bytes_per_pixel():
    """The whole-step byte model at the headline slice: 5023 bytes per pixel
    with no PCG iteration (build 116, initialisation 200, first set-up 188,
    19 later set-ups 1444, 20 shrink passes 3075) and 228 per iteration."""
    spec = gen.SliceSpec(256, 256, 12, 4.0, 24, wavelet="db4", levels=3)
    N = 256 * 256
    assert bench.reconstruction_bytes(spec, 0) == 5023 * N
    assert bench.reconstruction_bytes(spec, 10) - bench.reconstruction_bytes(spec, 0) == 2280 * N
    assert bench.reconstruction_bytes(spec, 0, n_outer=1) == (116 + 200 + 188 + 153.75) * N
