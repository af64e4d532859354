"""The committed rocprofv3 summaries describe the code in the tree.

bench.py reports the counter-measured HBM traffic of the power-series kernel
only while the counter summary was taken on the current kernels and factor
packing; these checks keep the summaries and the sources in step, and check
that the profiler's average kernel duration agrees with the HIP-event mean of
the bench line recorded in the same run.
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROF = os.path.join(ROOT, "profiles")


def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_counter_summary_matches_sources():
    bench = _bench()
    traffic = bench.measured_traffic()
    assert traffic is not None, "profiles/k_series_lap3d64_pmc.txt was taken on other sources"
    kv = dict(line.split(" = ", 1) for line in open(os.path.join(PROF, "k_series_lap3d64_pmc.txt"))
              if " = " in line)
    alg = re.search(r"algorithmic: (\d+) bytes", open(os.path.join(PROF, "k_series_lap3d64_pmc.txt")).read())
    assert alg is not None
    # every factor entry read once: counter traffic within 5% of the algorithmic bytes
    assert abs(traffic / float(alg.group(1)) - 1.0) < 0.05
    assert float(kv["bytes_per_launch"]) == traffic


def test_trace_average_agrees_with_events():
    text = open(os.path.join(PROF, "k_series_lap3d64_kernel_trace.txt")).read()
    m = re.search(r"k_series<double, 1, false> \(the 64\^3 power-series step\) averages ([\d.]+) us", text)
    e = re.search(r"mean_launch_ms ([\d.]+)", text)
    assert m and e
    prof_us, event_us = float(m.group(1)), 1e3 * float(e.group(1))
    # the event interval also spans the dispatch and the end-of-kernel release
    assert 0.0 <= event_us - prof_us <= 0.15 * prof_us, (prof_us, event_us)


@pytest.mark.parametrize("name", ["k_series_lap3d64_kernel_trace.txt", "k_series_lap3d64_pmc.txt"])
def test_summaries_state_their_commands(name):
    text = open(os.path.join(PROF, name)).read()
    assert "rocprofv3" in text and "bench.py" in text
