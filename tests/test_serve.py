"""Scheduler policy of the serving loop, on the CPU with a deterministic fake device."""
import numpy as np
import pytest

from paper_2601_15401_amd import serve

SETS = {13: (3, 1, 3), 14: (8, 2, 4), 15: (16, 4, 4), 16: (32, 8, 4)}


def reqs_at(times, mix):
    return [serve.Request(i, ln, k, lv, t) for i, ((ln, k, lv), t) in enumerate(zip(mix, times))]


def inflight_bytes_at(reqs, t):
    return sum(r.nbytes for r in reqs if r.start <= t < r.done)


def test_every_request_completes_once_after_its_arrival():
    mix = serve.request_mix(300, 1, SETS)
    rs = reqs_at(serve.poisson_arrivals(300, 2000.0, 3), mix)
    st = serve.Server(serve.FakeExecutor(), budget=10 ** 9).run(rs)
    assert sorted(r.rid for r in st.completed) == list(range(300))
    for r in rs:
        assert r.arrival <= r.start < r.done


def test_budget_never_exceeded_and_binds():
    mix = serve.request_mix(200, 2, SETS)
    ex = serve.FakeExecutor(n_streams=3)
    rs = reqs_at([0.0] * 200, mix)
    budget = 3 * max(ex.bytes_fn(r) for r in rs)
    st = serve.Server(ex, budget=budget).run(rs)
    assert len(st.completed) == 200
    assert st.peak_bytes <= budget
    for r in rs:  # checked from the schedule itself, not the server's counter
        assert inflight_bytes_at(rs, r.start) <= budget
    # the budget, not the request count, limited the micro-batches
    assert max(len(b[3]) for b in ex.launched) < 200


def test_resident_state_counts_against_budget():
    with pytest.raises(ValueError):
        serve.Server(serve.FakeExecutor(), budget=100, resident=100)
    rs = reqs_at([0.0], [(16, 12, 32)])
    ex = serve.FakeExecutor()
    with pytest.raises(ValueError):
        serve.Server(ex, budget=ex.bytes_fn(rs[0]) + 10, resident=20).run(rs)


def test_fifo_admission():
    mix = serve.request_mix(400, 4, SETS)
    rs = reqs_at(serve.poisson_arrivals(400, 5000.0, 5), mix)
    ex = serve.FakeExecutor()
    budget = 5 * max(ex.bytes_fn(r) for r in rs)
    serve.Server(ex, budget=budget).run(rs)
    order = sorted(rs, key=lambda r: (r.arrival, r.rid))
    starts = [r.start for r in order]
    assert starts == sorted(starts)


def test_stream_slots_bound_concurrency():
    mix = serve.request_mix(300, 6, SETS)
    rs = reqs_at(serve.poisson_arrivals(300, 20000.0, 7), mix)
    ex = serve.FakeExecutor(n_streams=2)
    st = serve.Server(ex, budget=10 ** 12, max_batch=16).run(rs)
    assert max(len(b[3]) for b in ex.launched) <= 16
    # groups on one stream never overlap in time
    for slot in range(2):
        iv = sorted((s, e) for sl, s, e, _ in ex.launched if sl == slot)
        assert all(a[1] <= b[0] for a, b in zip(iv, iv[1:]))
    assert st.micro_batches >= 300 // 16


def test_light_group_completes_before_heavy_in_same_micro_batch():
    # one micro-batch with a small-N request and a heavy N = 2^16 request
    mix = [(16, 12, 32), (13, 2, 3)]
    rs = reqs_at([0.0, 0.0], mix)
    ex = serve.FakeExecutor(n_streams=1, cost_fn=lambda g: 1e-3 * sum(r.k * (r.log_n - 12) for r in g))
    serve.Server(ex, budget=10 ** 9).run(rs)
    assert ex.launched[0][3] == [1] and ex.launched[1][3] == [0]
    assert rs[1].done < rs[0].done


def test_idle_server_serves_each_request_at_once():
    mix = [(13, 2, 3)] * 5
    rs = reqs_at([0.1 * i for i in range(5)], mix)
    ex = serve.FakeExecutor(cost_fn=lambda g: 1e-3)
    serve.Server(ex, budget=10 ** 9).run(rs)
    for r in rs:
        assert r.done - r.arrival == pytest.approx(1e-3, abs=5e-5)


def test_batches_grow_with_load():
    mix = serve.request_mix(1000, 8, SETS)
    sizes = []
    for rate in (500.0, 50000.0):
        ex = serve.FakeExecutor(cost_fn=lambda g: 2e-4 + 2e-5 * len(g))
        serve.Server(ex, budget=10 ** 12).run(reqs_at(serve.poisson_arrivals(1000, rate, 9), mix))
        sizes.append(np.mean([len(b[3]) for b in ex.launched]))
    assert sizes[1] > 4 * sizes[0]


def test_poisson_rate_and_mix():
    t = np.array(serve.poisson_arrivals(20000, 1000.0, 10))
    assert np.all(np.diff(t) > 0)
    assert abs(20000 / t[-1] - 1000.0) < 30.0
    mix = serve.request_mix(20000, 11, SETS)
    heavy = sum(1 for ln, k, lv in mix if ln == 16 and k == 12)
    # 10% heavy plus the ordinary draws that land on N = 2^16, k = 12: 0.1 + 0.9 / 4 / 11
    assert abs(heavy / 20000 - (0.1 + 0.9 / 44)) < 0.01
    for ln, k, lv in mix:
        L = SETS[ln][0]
        assert 2 <= k <= min(12, L) and k <= lv <= L
    assert {ln for ln, _, _ in mix} == set(SETS)
