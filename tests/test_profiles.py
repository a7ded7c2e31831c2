"""The committed rocprofv3 summaries and the bench's reader of them (host
logic only, no GPU): every summary names the command that made it and the
kernel sources it was taken on; the HBM traffic per launch of every solver
stage is within 1 % of the algorithmic 16 B per point (one read and one
write of the FP64 field); and a reading taken on other kernel sources is
not used."""
import os

import pytest

import bench
from paper_1802_10323_amd import profiling

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")
POINTS = {"channel": 512 * 256 * 192, "cube": 512 ** 3}


@pytest.mark.parametrize("name", ["kernel_trace_channel.txt", "kernel_trace_cube.txt",
                                  "kernel_trace_taylor_green.txt",
                                  "traffic_channel.txt", "traffic_cube.txt"])
def test_summary_names_its_command_and_sources(name):
    text = open(os.path.join(PROFILES, name)).read()
    assert "rocprofv3 " in text and " -- python3 bench.py" in text
    assert "kernel sources " in text or "kernel_source_hash " in text


@pytest.mark.parametrize("workload", sorted(POINTS))
def test_traffic_per_stage_is_the_algorithmic_16_bytes_per_point(workload):
    src, per_stage = profiling.read_traffic(os.path.join(PROFILES, f"traffic_{workload}.txt"))
    assert src is not None and len(src) == 16
    assert sorted(per_stage) == sorted(bench.STAGES)
    algorithmic = bench.BYTES_PER_POINT_FP64 * POINTS[workload]
    for stage, measured in per_stage.items():
        assert abs(measured / algorithmic - 1.0) < 0.01, (stage, measured, algorithmic)


def _write_summary(folder, workload, src_hash, value):
    os.makedirs(os.path.join(folder, "profiles"), exist_ok=True)
    with open(os.path.join(folder, "profiles", f"traffic_{workload}.txt"), "w") as fh:
        fh.write("# test summary\n")
        fh.write(f"kernel_source_hash {src_hash}\n")
        fh.write(f"stage tridiag kernel k launches 8 fetch_KiB 1 write_KiB 1 "
                 f"bytes_per_launch {value}\n")


def test_bench_uses_a_reading_only_on_the_kernels_it_was_taken_on(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.stored_traffic("channel", "tridiag") is None          # no summary
    _write_summary(str(tmp_path), "channel", profiling.kernel_source_hash(), 123.0)
    assert bench.stored_traffic("channel", "tridiag") == 123.0
    assert bench.stored_traffic("channel", "fwd_t1") is None           # stage not in it
    _write_summary(str(tmp_path), "channel", "0" * 16, 123.0)
    assert bench.stored_traffic("channel", "tridiag") is None          # other sources
