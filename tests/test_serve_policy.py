"""Serving policy on the host: chunking, priority, LDS and HBM budgets.

A fake executor replays the scheduler's decisions with modelled chunk
durations (no GPU): every request must finish, chunks of one request stay
in order, the LDS budget is never exceeded by co-running requests, and the
priority behaves as documented (FIFO at aging 0, shortest remaining work
first at large aging)."""
import math
import types

import numpy as np
import pytest

pytest.importorskip("torch")
sv = pytest.importorskip("paper_1707_09683_amd.serve")


def test_chunk_ranges_cover_the_order():
    rng = np.random.default_rng(3)
    lens = np.sort(rng.integers(20, 3000, size=5000))[::-1]
    cum = np.concatenate(([0], np.cumsum(lens)))
    for M, cc in ((30, 1e8), (400, 1e8), (2000, 3e8), (400, float("inf"))):
        ch = sv.chunk_ranges(cum, len(lens), M, cc)
        assert ch[0][0] == 0 and sum(c for _, c in ch) == len(lens)
        assert all(a + c == b for (a, c), (b, _) in zip(ch[:-1], ch[1:]))
        assert all(c > 0 for _, c in ch)
        if math.isfinite(cc):
            cells = [M * int(cum[a + c] - cum[a]) for a, c in ch]
            assert len(ch) >= int(M * cum[-1] // cc) - 1
            assert max(cells) <= cc + M * lens.max()
    assert sv.chunk_ranges(cum, 0, 400, 1e8) == [(0, 0)]


def _req(rid, t, remaining, lds):
    return types.SimpleNamespace(rid=rid, t_arrival=t, remaining=remaining, lds=lds)


def test_priority_fifo_and_shortest_first():
    a = _req(1, 0.0, 1e12, 1000)
    b = _req(2, 0.5, 1e9, 1000)
    assert sv.pick_next([a, b], {}, 160 * 1024, 0.0, 2e13) is a          # FIFO
    assert sv.pick_next([a, b], {}, 160 * 1024, 1e9, 2e13) is b          # SRPT
    # aging 1: b overtakes only while a has not waited longer than its run
    assert sv.pick_next([a, b], {}, 160 * 1024, 1.0, 2e13) is a          # 0+0.05 < 0.5+5e-5
    c = _req(3, 0.01, 1e9, 1000)
    assert sv.pick_next([a, c], {}, 160 * 1024, 1.0, 2e13) is c


def test_lds_budget_blocks_co_residence():
    big = _req(1, 0.0, 1e12, 100 * 1024)
    other = _req(2, 0.1, 1e9, 80 * 1024)
    small = _req(3, 0.2, 1e9, 40 * 1024)
    running = {id(big): big.lds}
    # other does not fit beside big; small does; big itself may always continue
    assert sv.pick_next([other, small], running, 160 * 1024, 1e9, 2e13) is small
    assert sv.pick_next([other], running, 160 * 1024, 1e9, 2e13) is None
    assert sv.pick_next([big, other], running, 160 * 1024, 1e9, 2e13) is big
    assert sv.pick_next([other], {}, 160 * 1024, 1e9, 2e13) is other


def test_hbm_budget_slots():
    assert sv.slots_for_budget(2 << 30, 5 << 20, 8) == 8
    assert sv.slots_for_budget(12 << 20, 5 << 20, 8) == 2
    assert sv.slots_for_budget(1 << 20, 5 << 20, 8) == 1          # always one


def test_fake_executor_replay():
    """Drive pick_next with modelled chunk times: 40 requests, 3 chunks in
    flight, random LDS sizes.  Every request completes, chunk order holds
    per request, and co-running LDS never exceeds the budget."""
    rng = np.random.default_rng(8)
    lens = rng.integers(20, 2000, size=3000)
    cum = np.concatenate(([0], np.cumsum(lens)))
    rate, budget, depth = 2e13, 160 * 1024, 3
    reqs = []
    for i in range(40):
        M = int(rng.integers(30, 2000))
        r = _req(i, float(i) * 1e-4, 0, int(rng.choice([20, 40, 70, 100])) * 1024)
        r.chunks = sv.chunk_ranges(cum, len(lens), M, 2e9)
        r.cost = [M * int(cum[a + c] - cum[a]) for a, c in r.chunks]
        r.remaining = sum(r.cost)
        r.next = 0
        r.done = 0
        reqs.append(r)
    now, active, inflight, order = 0.0, [], [], []
    pending = list(reqs)
    while pending or active or inflight:
        while pending and pending[0].t_arrival <= now:
            active.append(pending.pop(0))
        while len(inflight) < depth and active:
            running = {id(r): r.lds for r, _, _ in inflight}
            assert sum(running.values()) <= budget or len(running) == 1
            r = sv.pick_next(active, running, budget, 1.0, rate)
            if r is None:
                break
            ci = r.next
            r.next += 1
            r.remaining -= r.cost[ci]
            start = max([now] + [e for x, _, e in inflight if x is r])
            inflight.append((r, ci, start + r.cost[ci] / rate + 1e-6))
            order.append((r.rid, ci))
            if r.next == len(r.chunks):
                active.remove(r)
        if not inflight:
            now = pending[0].t_arrival if pending else now
            continue
        inflight.sort(key=lambda t: t[2])
        r, ci, now = inflight.pop(0)
        r.done += 1
    assert all(r.done == len(r.chunks) for r in reqs)
    for r in reqs:
        mine = [ci for rid, ci in order if rid == r.rid]
        assert mine == list(range(len(r.chunks)))
