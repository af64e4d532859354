"""The committed rocprofv3 summaries describe the code in the tree.

bench.py reports the counter-measured HBM traffic of the power-series kernel
only while the counter summary was taken on the current kernels and factor
packing (otherwise it reports null); these checks keep the summaries, the
sources and the bench in step, and check that the profiler's average kernel
duration agrees with the HIP-event mean of the bench line recorded in the
same run.  The power-series step of the apply (k_series) and the bare E_s
product of the Arnoldi setup (k_es) are separate kernels, so each average is
over one launch population.
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROF = os.path.join(ROOT, "profiles")
TRACE = os.path.join(PROF, "k_series_lap3d64_kernel_trace.txt")
PMC = os.path.join(PROF, "k_series_lap3d64_pmc.txt")


def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _kv(path):
    return dict(line.split(" = ", 1) for line in open(path).read().splitlines() if " = " in line)


def test_counter_summary_used_only_for_its_sources():
    bench = _bench()
    kv = _kv(PMC)
    traffic = bench.measured_traffic()
    if kv.get("source_sha256_16", "").strip() != bench.kernel_hash():
        # taken on other kernels: the bench must not report it
        assert traffic is None
        return
    alg = int(kv["algorithmic_bytes_per_launch"])
    assert traffic == float(kv["bytes_per_launch"])
    # every factor entry is read once: counter traffic within 10% of the algorithmic bytes
    assert abs(traffic / alg - 1.0) < 0.10, (traffic, alg)
    # the dispatch counts of both counter runs are stated and cover only k_series launches
    assert int(kv["fetch_dispatches"]) > 0 and int(kv["write_dispatches"]) > 0


def test_trace_average_agrees_with_events():
    kv = _kv(TRACE)
    prof_us = float(kv["k_series_fp64_avg_us"])
    event_us = 1e3 * float(kv["bench_mean_launch_ms"])
    # same launches, two clocks: the profiler's dispatch timestamps and the HIP
    # events stamped at the kernel by the bench
    assert abs(event_us - prof_us) <= 0.05 * prof_us, (prof_us, event_us)
    frac = float(kv["k_series_fp64_hbm_fraction"])
    assert abs(frac - float(kv["k_series_algorithmic_bytes"]) / (prof_us * 1e-6) / 8e12) < 1e-3


@pytest.mark.parametrize("path", [TRACE, PMC], ids=["trace", "pmc"])
def test_summaries_state_their_commands(path):
    text = open(path).read()
    assert "rocprofv3" in text and "bench.py" in text
