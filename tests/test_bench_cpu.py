"""Host logic of bench.py that needs no GPU: reading the committed rocprofv3
counter summaries, and dropping their traffic once the kernel source they
were taken on has changed."""
import os

import pytest

import bench

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def write_profile(tmp_path, text):
    d = tmp_path / "profiles"
    d.mkdir(exist_ok=True)
    (d / "frame_kernel_x_acc_counters.txt").write_text(text)
    return d


PROFILE = """# comment: a line with a colon that is skipped
kernel_source_hash: {h}
fetch_kib_per_dispatch: 100.0
write_kib_per_dispatch: 50.0
leg_fetch_kib_per_dispatch: 10.0
leg_write_kib_per_dispatch: 4.0
fetch_scale: 2.0
write_scale: 1.0
"""


def test_counter_bytes_scaled_per_launch(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    write_profile(tmp_path, PROFILE.format(h="abc"))
    assert bench.measured_traffic("x", True) == (100.0 * 2.0 + 50.0) * 1024.0
    assert bench.measured_leg_traffic("frame_kernel_x_acc_counters.txt", "leg") == (10.0 * 2.0 + 4.0) * 1024.0
    assert bench.measured_leg_traffic("frame_kernel_x_acc_counters.txt", "other") is None
    assert bench.measured_traffic("x", False) is None  # no such file


def test_counters_of_another_kernel_source_are_dropped(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    write_profile(tmp_path, PROFILE.format(h="def"))
    assert bench.measured_traffic("x", True) is None
    assert bench.measured_leg_traffic("frame_kernel_x_acc_counters.txt", "leg") is None


def test_kernel_source_hash_follows_the_sources(tmp_path, monkeypatch):
    h0 = bench.kernel_source_hash()
    assert len(h0) == 16
    src = tmp_path / "paper_2305_07083_amd" / "csrc"
    src.mkdir(parents=True)
    for name in bench.KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2305_07083_amd", "csrc", name), "rb") as fh:
            (src / name).write_bytes(fh.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == h0
    (src / bench.KERNEL_SOURCES[0]).write_bytes((src / bench.KERNEL_SOURCES[0]).read_bytes() + b"\n")
    assert bench.kernel_source_hash() != h0


@pytest.mark.parametrize("name", sorted(f for f in os.listdir(os.path.join(ROOT, "profiles"))
                                        if f.endswith("_counters.txt")))
def test_committed_counter_summaries_parse(name):
    """Every committed counter summary states the kernel source it was taken
    on and the two scale factors."""
    kv = {}
    for line in open(os.path.join(ROOT, "profiles", name)):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    assert len(kv["kernel_source_hash"]) == 16
    assert float(kv["fetch_scale"]) > 0 and float(kv["write_scale"]) > 0
    assert any(k.endswith("fetch_kib_per_dispatch") for k in kv)


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert not r.stdout.lstrip().startswith("{")  # no JSON line
