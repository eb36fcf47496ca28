"""Host-side parts of the benchmark script (no GPU): the one-GPU guard, the
roofline decomposition and the bookkeeping of the committed counters."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_counters_belong_to_the_committed_sources():
    """The HBM traffic and instruction mix that bench.py reports were taken
    on the kernel sources as they stand (else it reports them as null)."""
    assert bench.COUNTER_TRAFFIC["source_sha256"] == bench.kernel_sources_sha256()
    assert bench.counter_traffic() is not None


@pytest.mark.parametrize("kernel_ms", [0.0595, 0.0667])
def test_roofline_decomposition_multiplies_to_the_fraction(kernel_ms):
    """clock x mix x issue equals the flop-based roofline fraction for any
    kernel time; the FP64 pipe fraction counts the FP64 instructions."""
    flops = bench.FLOPS_PER_EVENT
    v = bench.valu_issue(kernel_ms, flops)
    frac = flops * bench.N_EVENTS / (kernel_ms * 1e-3) / (bench.FP64_PEAK_TFLOPS * 1e12)
    assert v["decomposition"]["product"] == pytest.approx(frac, rel=1e-12)
    cls = v["classes_per_event"]
    lane_ops = (cls["fp64"] + cls["fp64_trans"]) * bench.N_EVENTS / (kernel_ms * 1e-3)
    assert v["fp64_pipe_frac"] == pytest.approx(lane_ops / (256 * 4 * 16 * 2.4e9), rel=1e-12)
    # the classes account for every VALU instruction the counters read
    assert sum(cls.values()) == pytest.approx(v["valu_insts_per_event"], abs=0.1)


def test_traffic_close_to_the_algorithmic_bytes():
    """The counters' HBM bytes per launch stay within a few per cent of the
    algorithmic 27 B per event: no wasted re-reads."""
    ratio = bench.counter_traffic() / (bench.BYTES_PER_EVENT * bench.N_EVENTS)
    assert 1.0 <= ratio < 1.05

