"""Host-side policy of the continuous-batching loop (no device)."""
import pytest

from paper_2305_03284_amd.serve import Request, Scheduler, poisson_requests


def _req(t, key, i, last=False):
    return Request(t, key, i, last)


def test_admission_by_budget_in_arrival_order():
    s = Scheduler(budget_bytes=100, max_batch=8)
    s.arrive(_req(0.0, "a", 0), 60)
    s.arrive(_req(0.1, "b", 0), 50)
    s.arrive(_req(0.2, "c", 0), 30)
    # a fits; b does not fit next to a and blocks c behind it (no overtaking)
    assert s.admit(0.05) == ["a"] and s.used == 60
    assert s.streams["a"].queue[0].t_admit == 0.05
    assert [r.key for r in s.next_batch()] == ["a"]
    s.arrive(_req(0.3, "a", 1), 60)
    assert s.streams["a"].queue[0].t_admit == 0.3  # admitted stream: service starts at arrival


def test_retirement_frees_budget_and_admits_waiting():
    s = Scheduler(budget_bytes=100, max_batch=8)
    s.arrive(_req(0.0, "a", 0, last=True), 60)
    s.arrive(_req(0.1, "b", 0, last=True), 50)
    assert s.admit() == ["a"]
    batch = s.next_batch()
    assert s.admit() == []
    assert s.complete(batch, 1.0) == ["a"] and s.used == 0
    assert batch[0].t_done == 1.0
    assert s.admit() == ["b"]
    assert s.complete(s.next_batch(), 2.0) == ["b"] and s.idle()


def test_one_frame_per_stream_per_launch_in_order():
    s = Scheduler(budget_bytes=1000, max_batch=8)
    for i in range(3):
        s.arrive(_req(0.01 * i, "a", i), 10)
    s.arrive(_req(0.005, "b", 0), 10)
    s.admit()
    b1 = s.next_batch()
    assert [(r.key, r.index) for r in b1] == [("a", 0), ("b", 0)]
    b2 = s.next_batch()  # the next launch may take a's next frame while b1 is in flight
    assert [(r.key, r.index) for r in b2] == [("a", 1)]
    assert s.streams["a"].in_flight == 2
    s.complete(b1, 1.0)
    s.complete(b2, 2.0)
    assert [(r.key, r.index) for r in s.next_batch()] == [("a", 2)]


def test_max_batch_takes_oldest_first():
    s = Scheduler(budget_bytes=1000, max_batch=2)
    s.arrive(_req(0.3, "a", 0), 10)
    s.arrive(_req(0.1, "b", 0), 10)
    s.arrive(_req(0.2, "c", 0), 10)
    s.admit()
    assert [r.key for r in s.next_batch()] == ["b", "c"]
    assert [r.key for r in s.next_batch()] == ["a"]


def test_plain_loop_is_arrival_order():
    s = Scheduler(budget_bytes=1000, max_batch=1)
    s.arrive(_req(0.2, "a", 0), 10)
    s.arrive(_req(0.1, "b", 0), 10)
    s.arrive(_req(0.15, "b", 1), 10)
    s.admit()
    order = []
    while True:
        b = s.next_batch()
        if not b:
            break
        order.append((b[0].key, b[0].index))
        s.complete(b, 0.0)
    assert order == [("b", 0), ("b", 1), ("a", 0)]


def test_rejections():
    s = Scheduler(budget_bytes=100, max_batch=4)
    with pytest.raises(ValueError):
        s.arrive(_req(0.0, "big", 0), 101)
    s.arrive(_req(0.0, "a", 1), 10)  # frame 1 before frame 0
    s.admit()
    with pytest.raises(ValueError):
        s.next_batch()
    s2 = Scheduler(budget_bytes=100, max_batch=4)
    s2.arrive(_req(0.0, "a", 0, last=True), 10)
    s2.admit()
    s2.next_batch()
    with pytest.raises(ValueError):
        s2.arrive(_req(0.1, "a", 1), 10)
    with pytest.raises(ValueError):
        Scheduler(0, 1)


def test_poisson_requests_shape():
    reqs = poisson_requests(list(range(8)), rate_hz=2000.0, frames_per_stream=50, seed=3, start_spread_s=0.01)
    assert len(reqs) == 400
    for k in range(8):
        mine = [r for r in reqs if r.key == k]
        assert [r.index for r in mine] == list(range(50)) and mine[-1].last and not any(r.last for r in mine[:-1])
        ts = [r.t_arrival for r in mine]
        assert all(b > a for a, b in zip(ts, ts[1:]))
    # aggregate rate close to 2 kHz while all streams are live
    span = max(r.t_arrival for r in reqs) - min(r.t_arrival for r in reqs)
    assert 1500 < len(reqs) / span < 2700
    assert poisson_requests([0, 1], 100.0, 5, seed=1)[0].t_arrival == poisson_requests([0, 1], 100.0, 5, seed=1)[0].t_arrival
