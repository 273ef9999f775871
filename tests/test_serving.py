"""The continuous-batching scheduler on the CPU, with a simulated device
and clock: admission by HBM budget, rejection, FIFO order, overlap of
parameter sets, continuous admission, and the per-op baseline server."""

import numpy as np
import pytest

from paper_1908_06972_amd.serving import (PsetPolicy, Request, Scheduler, SimClock, SimExecutor, Stats,
                                          poisson_trace)


def _run(trace, policies, budget, cost, continuous=True):
    clock = SimClock()
    ex = SimExecutor(clock, cost)
    stats = Scheduler(ex, policies, budget, clock=clock, continuous=continuous).run(trace)
    return stats, ex


def test_budget_limits_batch_and_rest_waits():
    pol = {"A": PsetPolicy(bytes_per_request=100, max_batch=8)}
    trace = [Request(i, "A", 0.0, i, 10) for i in range(5)]
    stats, ex = _run(trace, pol, budget=300, cost=lambda p, n: 1.0)
    assert [len(b) for _, _, b in ex.log] == [3, 2]
    assert ex.log[1][0] >= 1.0                      # second batch waits for the first
    assert stats.completed == 5 and stats.rejected == 0
    assert all(r.result == ("result", r.rid) for r in trace)


def test_oversized_request_rejected():
    pol = {"A": PsetPolicy(100, 4), "B": PsetPolicy(1000, 4)}
    trace = [Request(0, "B", 0.0, 0, 1), Request(1, "A", 0.0, 0, 1)]
    stats, _ = _run(trace, pol, budget=500, cost=lambda p, n: 0.1)
    assert trace[0].rejected and not trace[1].rejected
    assert stats.rejected == 1 and stats.completed == 1


def test_fifo_within_a_set_and_max_batch():
    pol = {"A": PsetPolicy(1, 2)}
    trace = [Request(i, "A", 0.001 * i, i, 1) for i in range(5)]
    _, ex = _run(trace, pol, budget=10 ** 9, cost=lambda p, n: 0.5)
    order = [rid for _, _, b in ex.log for rid in b]
    assert order == [0, 1, 2, 3, 4]
    assert all(len(b) <= 2 for _, _, b in ex.log)


def test_sets_overlap_and_late_arrivals_join_next_batch():
    pol = {"A": PsetPolicy(1, 8), "B": PsetPolicy(1, 8)}
    trace = [Request(0, "A", 0.0, 0, 1), Request(1, "B", 0.0, 0, 1),
             Request(2, "A", 0.2, 0, 1), Request(3, "A", 0.3, 0, 1)]
    stats, ex = _run(trace, pol, budget=10 ** 9, cost=lambda p, n: 1.0)
    starts = {tuple(b): (t, p) for t, p, b in ex.log}
    assert starts[(0,)][0] == starts[(1,)][0] == 0.0   # both sets in flight at once
    assert (2, 3) in starts and 1.0 <= starts[(2, 3)][0] < 1.01
    assert stats.batches == 3


def test_per_op_server_is_serial_in_arrival_order():
    pol = {"A": PsetPolicy(1, 8), "B": PsetPolicy(1, 8)}
    trace = [Request(0, "A", 0.0, 0, 1), Request(1, "B", 0.01, 0, 1), Request(2, "A", 0.02, 0, 1)]
    stats, ex = _run(trace, pol, budget=10 ** 9, cost=lambda p, n: 1.0, continuous=False)
    assert [b for _, _, b in ex.log] == [[0], [1], [2]]
    t = [t for t, _, _ in ex.log]
    assert t[1] >= 1.0 and t[2] >= 2.0
    assert stats.completed == 3


def test_batching_beats_per_op_under_load():
    pol = {"A": PsetPolicy(1, 16)}
    trace = poisson_trace(5, 400, 200.0, {"A": 1}, {"A": 8}, {"A": [10] * 8})
    cost = lambda p, n: 0.004 + 0.001 * n  # noqa: E731  (fixed launch cost + per-request cost)
    cont, _ = _run(trace, pol, 10 ** 9, cost)
    trace2 = poisson_trace(5, 400, 200.0, {"A": 1}, {"A": 8}, {"A": [10] * 8})
    serial, _ = _run(trace2, pol, 10 ** 9, cost, continuous=False)
    assert cont.percentile(99) < serial.percentile(99)
    assert cont.summary()["req_per_s"] >= serial.summary()["req_per_s"] * 0.99


def test_percentiles():
    s = Stats(latencies=[0.001 * i for i in range(1, 101)], makespan=1.0, completed=100)
    assert s.percentile(50) == pytest.approx(0.051, abs=1e-9) or s.percentile(50) == pytest.approx(0.050, abs=1e-9)
    assert s.percentile(99) == pytest.approx(0.099, abs=1e-9) or s.percentile(99) == pytest.approx(0.100, abs=1e-9)
    assert s.summary()["req_per_s"] == 100


def test_poisson_trace_rate_and_mix():
    tr = poisson_trace(505, 20000, 200.0, {"a": 3, "b": 2, "c": 1}, {"a": 4, "b": 4, "c": 4},
                       {k: [1, 2, 3, 4] for k in "abc"})
    gaps = np.diff([0.0] + [r.arrival for r in tr])
    assert abs(gaps.mean() - 1 / 200.0) < 0.05 / 200
    frac = {k: sum(r.pset == k for r in tr) / len(tr) for k in "abc"}
    assert abs(frac["a"] - 0.5) < 0.02 and abs(frac["b"] - 1 / 3) < 0.02 and abs(frac["c"] - 1 / 6) < 0.02


def test_retained_scratch_counts_against_the_budget():
    """A set's context keeps the scratch of its largest batch allocated; that
    scratch counts against the HBM budget while other sets admit work, so
    the sum over sets of max(in-flight working set, retained scratch) stays
    within the budget."""
    pol = {"A": PsetPolicy(100, 8), "B": PsetPolicy(100, 8)}
    trace = [Request(i, "A", 0.0, 0, 1) for i in range(4)] + [Request(4 + i, "B", 2.0, 0, 1) for i in range(3)]
    clock = SimClock()
    ex = SimExecutor(clock, lambda p, n: 1.0, retain=lambda p, n: 100 * n)
    stats = Scheduler(ex, pol, 500, clock=clock).run(trace)
    assert stats.completed == 7
    sizes = [(p, len(b)) for _, p, b in ex.log]
    assert sizes[0] == ("A", 4)
    # A keeps 400 bytes after its batch: B fits one request at a time
    assert [n for p, n in sizes if p == "B"] == [1, 1, 1]
    # without retained scratch the three B requests go as one batch
    clock2 = SimClock()
    ex2 = SimExecutor(clock2, lambda p, n: 1.0)
    trace2 = [Request(i, "A", 0.0, 0, 1) for i in range(4)] + [Request(4 + i, "B", 2.0, 0, 1) for i in range(3)]
    Scheduler(ex2, pol, 500, clock=clock2).run(trace2)
    assert [len(b) for _, p, b in ex2.log if p == "B"] == [3]
