"""The committed rocprofv3 summaries describe the code in the tree.

bench.py reports the counter-measured HBM traffic of the power-series step
only while the counter summary was taken on the current kernels and factor
packing (otherwise it reports null); these checks keep the summaries, the
sources and the bench in step, and check that the profiler's clock and the
bench's HIP events agree on the duration of the same steps.  With one
right-hand side a power-series step is six back-to-back launches (the team
solves of B_i and then of C_i: subtree lower solves, top groups, subtree
upper solves); the k_team_* kernels of mode 0 run in these steps only.
"""
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROF = os.path.join(ROOT, "profiles")
TRACE = os.path.join(PROF, "series_step_lap3d64_kernel_trace.txt")
PMC = os.path.join(PROF, "series_step_lap3d64_pmc.txt")


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
    # the counters see every algorithmic byte, and the excess the summary
    # accounts for (top right-hand sides formed per row block, records and
    # indices) stays below a quarter
    assert 1.0 <= traffic / alg < 1.25, (traffic, alg)
    # both counter runs cover the six launches of every step of both forms
    assert int(kv["fetch_dispatches"]) > 0 and int(kv["fetch_dispatches"]) % 6 == 0
    assert int(kv["write_dispatches"]) == int(kv["fetch_dispatches"])


def test_trace_span_agrees_with_events():
    kv = _kv(TRACE)
    span_us = float(kv["step_fp64_trace_span_us"])
    event_us = 1e3 * float(kv["bench_mean_launch_ms"])
    # same steps, two clocks: the profiler's dispatch timestamps (first launch
    # start to last launch end) and the HIP events the bench records around them
    assert abs(event_us - span_us) <= 0.05 * span_us, (span_us, event_us)
    # the launches run back to back: the span exceeds the sum of the six
    # kernels' averages by the five gaps only
    ksum = float(kv["step_fp64_kernel_sum_us"])
    assert ksum <= span_us <= ksum + 5 * 2.0, (ksum, span_us)
    frac = float(kv["series_step_fp64_hbm_fraction"])
    assert abs(frac - float(kv["series_step_algorithmic_bytes"]) / (span_us * 1e-6) / 8e12) < 1e-3


@pytest.mark.parametrize("path", [TRACE, PMC], ids=["trace", "pmc"])
def test_summaries_state_their_commands(path):
    text = open(path).read()
    assert "rocprofv3" in text and "bench.py" in text
