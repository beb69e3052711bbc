"""Host-side logic of the serving driver (no GPU)."""
import importlib.util
import os
import sys

import numpy as np
import pytest


def _serve():
    if importlib.util.find_spec("torch") is None:
        pytest.skip("torch not importable")
    from paper_1701_01607_amd import serve
    return serve


def rec(sub, queue, done, status=0):
    return {"t_submit": sub, "queue_s": queue, "t_done": done, "latency_s": done - sub, "status": status}


def test_busy_fraction_merges_overlapping_solves():
    serve = _serve()
    recs = [rec(0.0, 0.0, 2.0), rec(1.0, 0.0, 3.0), rec(5.0, 1.0, 8.0)]
    # running intervals [0,2] u [1,3] u [6,8] = 3 + 2 = 5 of [0, 8]
    assert serve.busy_fraction(recs, 0.0, 8.0) == pytest.approx(5.0 / 8.0)


def test_summary_percentiles_and_rate():
    serve = _serve()
    recs = [rec(float(i), 0.0, float(i) + 1.0 + (i % 3)) for i in range(10)]
    out = serve.summarize(recs)
    lat = np.array([1.0 + (i % 3) for i in range(10)])
    assert out["p50_s"] == pytest.approx(np.percentile(lat, 50))
    assert out["converged"] == 10
    assert out["atmospheres_per_hr"] == pytest.approx(3600.0 * 10 / (max(r["t_done"] for r in recs)))


def test_expected_run_time_weights_sizes_and_atoms():
    serve = _serve()
    times = [(1.0, 3.0), (2.0, 10.0)]
    # 0.75 * (1 + 3) / 2 + 0.25 * (2 + 10) / 2
    assert serve.expected_run_time(times, [0.75, 0.25]) == pytest.approx(0.75 * 2.0 + 0.25 * 6.0)


def test_requests_follow_the_mix_and_are_reproducible():
    serve = _serve()
    rng1, rng2 = np.random.default_rng(7), np.random.default_rng(7)
    sizes, probs = serve.SIZES[:2], np.array([0.5, 0.5])
    a = [serve.make_request(j, rng1, [(8, 8, 9), (16, 16, 17)], probs)[3] for j in range(6)]
    b = [serve.make_request(j, rng2, [(8, 8, 9), (16, 16, 17)], probs)[3] for j in range(6)]
    assert a == b and {t[0] for t in a} <= {"two-level", "six-level"}
    assert len(sizes) == 2


def test_stream_parts_do_not_depend_on_the_stream_length():
    serve = _serve()
    probs = np.array(serve.SIZE_P)
    d10, g10 = serve.draw_stream(10, serve.SIZES, probs)
    d30, g30 = serve.draw_stream(30, serve.SIZES, probs)
    assert d10 == d30[:10] and np.array_equal(g10, g30[:10])
    assert [d[0] for d in d30] == [10000 + j for j in range(30)]
    t = serve.arrival_times(g30[10:20], 0.5)
    assert t[0] == 0.0 and np.allclose(np.diff(t), g30[11:20] / 0.5)


def test_combined_parts_pool_latencies_and_add_makespans():
    serve = _serve()
    a = [rec(0.0, 0.0, 2.0), rec(1.0, 0.5, 4.0)]          # makespan 4, busy [0,4] = 4
    b = [rec(100.0, 0.0, 101.0), rec(105.0, 0.0, 106.0)]   # makespan 6, busy 2
    out = serve.combine([a, b])
    lat = np.array([2.0, 3.0, 1.0, 1.0])
    assert out["requests"] == 4 and out["parts"] == 2
    assert out["makespan_s"] == pytest.approx(10.0)
    assert out["atmospheres_per_hr"] == pytest.approx(3600.0 * 4 / 10.0)
    assert out["p99_s"] == pytest.approx(np.percentile(lat, 99))
    assert out["device_busy_fraction"] == pytest.approx((4.0 + 2.0) / 10.0)


def test_a_failing_request_builder_stops_the_stream_with_its_error():
    serve = _serve()

    class NoDevice:
        def serve_config(self, n):
            pass

        def serve_batching(self, n):
            pass

    def broken():
        raise ValueError("atmosphere generator failed")

    with pytest.raises(ValueError, match="generator failed"):
        serve.run_stream(NoDevice(), [broken], [0.0])
