"""Host logic of the request server: the admission policy (FIFO with bounded
overtaking under a slot count and a device-memory budget), run on a virtual
clock through the library's own simulation entry point and checked against
an independent statement of the policy and its invariants.  No GPU."""
import numpy as np
import pytest

from paper_1607_03777_amd import sdg


def reference_policy(arrival, service, nbytes, slots, budget, bypass):
    """The policy restated: at every event time, repeatedly start the oldest
    waiting request if it fits (slots and bytes); otherwise, at most `bypass`
    times per head, the oldest later request that fits."""
    n = len(arrival)
    order = sorted(range(n), key=lambda i: (arrival[i], i))
    start = [None] * n
    waiting, running = [], []  # running: (end, i)
    t, nxt, skips = (arrival[order[0]] if n else 0.0), 0, 0
    while sum(s is not None for s in start) < n:
        while nxt < n and arrival[order[nxt]] <= t:
            waiting.append(order[nxt])
            nxt += 1
        while waiting and len(running) < slots:
            used = sum(nbytes[i] for _, i in running)
            if used + nbytes[waiting[0]] <= budget:
                pick, skips = 0, 0
            elif skips < bypass:
                pick = next((j for j in range(1, len(waiting)) if used + nbytes[waiting[j]] <= budget), None)
                if pick is None:
                    break
                skips += 1
            else:
                break
            i = waiting.pop(pick)
            start[i] = t
            running.append((t + service[i], i))
        if all(s is not None for s in start):
            break
        running.sort()
        t_arr = arrival[order[nxt]] if nxt < n else np.inf
        if running and running[0][0] <= t_arr:
            t = max(t, running.pop(0)[0])
        else:
            t = max(t, t_arr)
    return np.array(start, dtype=float)


def check_invariants(arrival, service, nbytes, slots, budget, start):
    assert np.all(start >= arrival)
    ev = sorted(set(start.tolist()))
    for t in ev:
        live = (start <= t) & (start + service > t)
        assert live.sum() <= slots
        assert nbytes[live].sum() <= budget


def trace(seed, n, slots_budget):
    rng = np.random.default_rng(seed)
    arrival = np.cumsum(rng.exponential(5.0, n))
    service = rng.uniform(5.0, 60.0, n)
    nbytes = rng.integers(1, slots_budget + 1, n).astype(np.uint64)
    return arrival, service, nbytes


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("slots,budget,bypass", [(1, 100, 0), (4, 100, 8), (3, 40, 2), (8, 60, 0)])
def test_admission_matches_policy(seed, slots, budget, bypass):
    arrival, service, nbytes = trace(seed, 60, min(budget, 40))
    start = sdg.sdg_admission_simulate(arrival, service, nbytes, slots, budget, bypass)
    ref = reference_policy(arrival, service, nbytes, slots, budget, bypass)
    assert np.array_equal(start, ref)
    check_invariants(arrival, service, nbytes, slots, budget, start)


def test_fifo_when_everything_fits():
    arrival = np.array([0.0, 1.0, 2.0, 3.0])
    service = np.array([10.0, 10.0, 10.0, 10.0])
    start = sdg.sdg_admission_simulate(arrival, service, np.ones(4, np.uint64), 1, 10, 4)
    assert start.tolist() == [0.0, 10.0, 20.0, 30.0]
    start = sdg.sdg_admission_simulate(arrival, service, np.ones(4, np.uint64), 2, 10, 4)
    assert start.tolist() == [0.0, 1.0, 10.0, 11.0]


def test_overtaking_is_bounded():
    # request 1 (big) cannot start while request 0 runs; small ones overtake
    # it at most `bypass` times
    arrival = np.array([0.0, 1.0, 2.0, 3.0, 4.0, 5.0])
    service = np.array([100.0, 10.0, 1.0, 1.0, 1.0, 1.0])
    nbytes = np.array([60, 60, 10, 10, 10, 10], np.uint64)
    s0 = sdg.sdg_admission_simulate(arrival, service, nbytes, 4, 100, 0)
    assert s0[1] == 100.0 and np.all(s0[2:] >= 100.0)  # strict FIFO
    s2 = sdg.sdg_admission_simulate(arrival, service, nbytes, 4, 100, 2)
    assert s2[2] == 2.0 and s2[3] == 3.0  # two overtakes
    assert s2[1] == 100.0 and s2[4] >= 100.0 and s2[5] >= 100.0


def test_request_over_budget_is_rejected():
    with pytest.raises(sdg.SDGError) as e:
        sdg.sdg_admission_simulate([0.0], [1.0], np.array([11], np.uint64), 1, 10, 0)
    assert e.value.code == sdg.ERR_NOMEM
