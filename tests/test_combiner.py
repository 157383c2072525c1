"""The arrival-rate combining policy (Sec. 3.1) through the C-ABI: pure host logic, injected clock.

Expected decisions are worked out by hand from the rule: at a poll, max_size waiting requests are
combined if that many wait; otherwise all waiting ones are once the time since the last arrival
exceeds twice the largest interval seen between consecutive arrivals.
"""
import pytest

import paper_2008_05712_amd as gc


def test_full_batches_leave_in_max_size_chunks():
    c = gc.Combiner(4)
    c.arrive(0.0, 10)
    assert c.poll(0.0) == (4, 1)
    assert c.poll(0.0) == (4, 1)
    assert c.poll(0.0) == (0, 0)  # 2 wait, no time has passed since the arrival
    assert c.state()["waiting"] == 2
    c.destroy()


def test_idle_trigger_at_twice_the_largest_interval():
    c = gc.Combiner(100)
    for t in (0.0, 1.0, 2.0):
        c.arrive(t)
    assert c.state()["max_interval"] == 1.0
    assert c.poll(3.9) == (0, 0)      # 1.9 since the last arrival, not above 2 x 1.0
    assert c.poll(4.0) == (0, 0)      # exactly 2 x max_interval: not above
    assert c.poll(4.01) == (3, 2)
    assert c.poll(10.0) == (0, 0)     # nothing waits
    s = c.state()
    assert (s["waiting"], s["n_full"], s["n_idle"]) == (0, 0, 1)
    c.destroy()


def test_max_interval_is_a_running_maximum():
    c = gc.Combiner(100)
    c.arrive(0.0)
    c.arrive(0.5)
    c.arrive(3.0)           # interval 2.5
    c.arrive(3.25, 2)       # interval 0.25 (and 0 between the two)
    assert c.state()["max_interval"] == 2.5
    assert c.poll(8.0) == (0, 0)      # 4.75 < 5.0
    assert c.poll(8.3) == (5, 2)
    c.destroy()


def test_first_arrival_has_no_interval():
    c = gc.Combiner(8)
    c.arrive(5.0, 3)
    assert c.poll(5.0) == (0, 0)      # no time has passed
    assert c.poll(5.0 + 1e-9) == (3, 2)
    c.destroy()


def test_full_rule_takes_precedence_and_keeps_the_rest_waiting():
    c = gc.Combiner(3)
    c.arrive(0.0, 2)
    c.arrive(1.0, 2)                  # max_interval 1.0, 4 waiting
    assert c.poll(50.0) == (3, 1)     # idle too, but a full batch goes first
    assert c.poll(50.0) == (1, 2)     # the remaining one: idle rule
    c.destroy()


def test_invalid_arguments_leave_the_state_unchanged():
    with pytest.raises(gc.GcError):
        gc.Combiner(0)
    c = gc.Combiner(2)
    c.arrive(1.0)
    with pytest.raises(gc.GcError):
        c.arrive(0.5)                 # time went backwards
    with pytest.raises(gc.GcError):
        c.arrive(2.0, 0)              # no request
    with pytest.raises(gc.GcError):
        c.poll(0.9)
    assert c.state() == {"waiting": 1, "max_interval": 0.0, "n_full": 0, "n_idle": 0}
    c.destroy()


def test_every_request_leaves_exactly_once():
    # a bursty stream: every request is taken once, never more than max_size per launch
    import numpy as np
    rng = np.random.default_rng(7)
    c = gc.Combiner(16)
    gaps = [float(rng.exponential(0.01 if step % 50 < 40 else 0.2)) for step in range(400)]
    times = np.cumsum(gaps)
    arrived, taken, sizes = 0, 0, []
    for i, t in enumerate(times):
        k = int(rng.integers(1, 6))
        c.arrive(float(t), k)
        arrived += k
        nxt = times[i + 1] if i + 1 < len(times) else t + 1.0
        for tp in (float(t), float(0.5 * (t + nxt))):  # polls between arrivals, in time order
            n, why = c.poll(tp)
            if n:
                sizes.append(n)
                taken += n
    t = float(times[-1]) + 1.0
    n, why = c.poll(t + 1e6)
    taken += n
    assert taken == arrived
    assert max(sizes) <= 16
    assert c.state()["waiting"] == 0
    c.destroy()
