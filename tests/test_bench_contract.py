"""Host-side logic of bench.py (no GPU): the one-GPU refusal and the rule that PMC traffic is
reported only while the plane-pass source is the one the counters were taken for."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _write_profile(path, sha, nbytes):
    with open(path, "w") as f:
        f.write("# PMC summary\n\n")
        f.write(f"traffic: kernel=k_plane_stage kernel_sha={sha} bytes_per_launch={nbytes}\n")


def test_traffic_only_for_the_profiled_source(tmp_path, monkeypatch):
    prof = tmp_path / "plane_stage_fp64_traffic.md"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(prof))
    assert bench.read_traffic("fp64") is None                       # no profile
    _write_profile(prof, bench.kernel_hash(), 123456789)
    assert bench.read_traffic("fp64") == 123456789.0                # profile of this source
    _write_profile(prof, "0" * 16, 123456789)
    assert bench.read_traffic("fp64") is None                       # profile of another source
    mixed = tmp_path / "plane_stage_mixed_traffic.md"
    _write_profile(mixed, bench.kernel_hash(), 987)
    assert bench.read_traffic("mixed") == 987.0                     # the mixed file beside it


def test_kernel_hash_follows_the_plane_pass_source(tmp_path, monkeypatch):
    src = open(bench.KERNEL_SOURCE).read()
    assert bench.PLANE_BEGIN in src and bench.PLANE_END in src
    h0 = bench.kernel_hash()
    i = src.find(bench.PLANE_BEGIN) + len(bench.PLANE_BEGIN)
    inside = tmp_path / "inside.hip"
    inside.write_text(src[:i] + "\n// edit inside the plane pass\n" + src[i:])
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(inside))
    assert bench.kernel_hash() != h0
    j = src.find(bench.PLANE_END) + len(bench.PLANE_END)
    outside = tmp_path / "outside.hip"
    outside.write_text(src[:j] + "\n// edit after the plane pass\n" + src[j:])
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(outside))
    assert bench.kernel_hash() == h0


@pytest.mark.parametrize("name", sorted(os.listdir(os.path.join(ROOT, "profiles"))))
def test_profiles_give_their_command(name):
    text = open(os.path.join(ROOT, "profiles", name)).read()
    assert "rocprofv3" in text
    for line in text.splitlines():
        if "rocprofv3 " in line and " -- " in line:
            prog = line.split(" -- ", 1)[1].split()
            assert prog[0] in ("python3", "python")
            assert os.path.exists(os.path.join(ROOT, prog[1])), prog[1]
