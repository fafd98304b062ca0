"""Host logic of bench.py, on the CPU: the refusal of more than one GPU, the byte model of the
operator passes (fields of one real scalar per voxel, F, plus the 2-byte grain id where a pass
reads it) and the gate that reports the stored HBM counter traffic only for the kernel sources
it was taken on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
VOXELS_256 = 256 ** 3


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_pass_byte_model():
    # stress pass: six strain half-spectra in, six stress half-spectra out, the grain id
    assert bench.pass_bytes_per_voxel("x_stress", 4) == 12 * 4 + 2
    assert bench.pass_bytes_per_voxel("x_stress", 8) == 12 * 8 + 2
    # the whole operator apply: 62 field passes and two grain-id reads
    assert sum(bench.OPERATOR_PASS_FIELDS.values()) == 62
    assert bench.operator_bytes_per_voxel(8) == 62 * 8 + 4 == 500
    assert bench.operator_bytes_per_voxel(4) == 62 * 4 + 4 == 252


def test_counter_traffic_is_reported_only_for_its_sources(monkeypatch):
    algorithmic = {"fp32": bench.pass_bytes_per_voxel("x_stress", 4) * VOXELS_256,
                   "fp64": bench.pass_bytes_per_voxel("x_stress", 8) * VOXELS_256}
    for label, want in algorithmic.items():
        t = bench.pmc_traffic("x_stress", label, 256)
        if bench.sources_sha16() == bench.PMC_SOURCES_SHA16:
            # the counters were taken on these sources: the pass moves its algorithmic bytes
            assert t is not None and abs(t / want - 1.0) < 0.01, (label, t, want)
        else:
            assert t is None
        # another grid, or other sources, report no traffic
        assert bench.pmc_traffic("x_stress", label, 512) is None
    monkeypatch.setattr(bench, "PMC_SOURCES_SHA16", "0" * 16)
    assert bench.pmc_traffic("x_stress", "fp32", 256) is None
    assert bench.pmc_traffic("z_strain", "fp32", 256) is None
