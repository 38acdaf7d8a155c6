"""Scheduler logic of the serving loop, on the CPU with a fake executor."""
import numpy as np
import pytest

import synth
from paper_2508_05343_amd.serving import FakeExecutor, Job, Scheduler, serve


class VClock:
    """Virtual clock: every read advances time a little; sleep jumps."""

    def __init__(self, dt=2e-4):
        self.t, self.dt = 0.0, dt

    def __call__(self):
        self.t += self.dt
        return self.t

    def sleep(self, s):
        self.t += s


def trace(n=120, qps=400.0, seed=3, sizes=(1000, 5000, 20000)):
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1 / qps, n))
    res = [(64, 64), (128, 96), (256, 256)]
    jobs = []
    for i in range(n):
        w, h = res[int(rng.integers(3))]
        cam = synth.pinhole_camera(w, h, 60.0, (0, 0, -3), (0, 0, 0))
        jobs.append(Job(i, int(rng.integers(len(sizes))), cam, float(t[i])))
    return jobs, sizes


def test_all_requests_complete_in_fifo_batches_within_budget():
    jobs, sizes = trace()
    clk = VClock()
    ex = FakeExecutor(clk, n_streams=2, scene_sizes=sizes)
    budget = 8 * ex.bytes_for(jobs[:1], [200000])
    sch = Scheduler(sizes, budget, max_slots=16, max_batch=8, max_inflight=2)
    st = serve(jobs, ex, sch, clock=clk, sleep=clk.sleep)
    assert st.requests == len(jobs) and len(st.latencies_ms) == len(jobs)
    assert st.max_bytes_in_use <= budget
    assert 0 < st.peak_bytes_measured <= budget
    assert sch.slots_used == 0
    order = [r for b in ex.submitted for r in b]
    assert order == sorted(order), "admission is FIFO"
    assert all(len(b) <= 8 for b in ex.submitted)
    assert all(j.done_s >= j.arrival_s for j in jobs)
    assert st.max_inflight_jobs <= 16
    s = st.summary()
    assert s["batches"] == len(ex.submitted) and s["host_ms_per_batch_p50"] == 0.0


def test_requests_arriving_during_a_batch_join_the_next_one():
    jobs, sizes = trace(n=60, qps=5000.0)
    clk = VClock()
    ex = FakeExecutor(clk, n_streams=1, fixed_s=0.01, scene_sizes=sizes)
    sch = Scheduler(sizes, 1 << 40, max_slots=64, max_batch=64, max_inflight=1)
    serve(jobs, ex, sch, clock=clk, sleep=clk.sleep)
    # with one stream busy for 10 ms, later arrivals accumulate into large batches
    assert max(len(b) for b in ex.submitted) > 5
    assert sum(len(b) for b in ex.submitted) == 60


def test_small_budget_defers_but_never_overcommits():
    """Budget for about one and a half of the largest jobs: the held bytes
    (buffers kept per stream between batches) never exceed it, idle streams
    give theirs back so the next batch fits, and the work spreads over many
    small batches."""
    jobs, sizes = trace(n=40)
    clk = VClock()
    ex = FakeExecutor(clk, n_streams=4, scene_sizes=sizes)
    sch0 = Scheduler(sizes, 1 << 40)
    one = max(ex.bytes_for([j], sch0.estimates([j])) for j in jobs)
    budget = int(one * 1.5)
    sch = Scheduler(sizes, budget, max_slots=16, max_batch=16, max_inflight=4)
    st = serve(jobs, ex, sch, clock=clk, sleep=clk.sleep)
    assert st.requests == 40
    assert st.max_bytes_in_use <= budget and st.peak_bytes_measured <= budget
    # the budget holds at most a couple of jobs: work is spread over many batches
    assert st.batches >= 20


def test_request_larger_than_budget_is_rejected():
    jobs, sizes = trace(n=3)
    clk = VClock()
    sch = Scheduler(sizes, 1000)
    with pytest.raises(ValueError):
        serve(jobs, FakeExecutor(clk, scene_sizes=sizes), sch, clock=clk, sleep=clk.sleep)


def test_sequential_baseline_is_one_job_per_batch():
    jobs, sizes = trace(n=30)
    clk = VClock()
    ex = FakeExecutor(clk, n_streams=1, scene_sizes=sizes)
    sch = Scheduler(sizes, 1 << 40, max_slots=1, max_batch=1, max_inflight=1)
    st = serve(jobs, ex, sch, clock=clk, sleep=clk.sleep)
    assert all(len(b) == 1 for b in ex.submitted) and st.batches == 30


def test_pair_overflow_is_retried_with_grown_buffers_within_budget():
    """A batch whose pair count outgrew its buffer is run again with larger
    pair buffers once they fit; every request still completes and the held
    bytes stay within the budget."""
    jobs, sizes = trace(n=50)
    clk = VClock()
    ex = FakeExecutor(clk, n_streams=2, scene_sizes=sizes, overflow_every=3)
    sch0 = Scheduler(sizes, 1 << 40)
    one = max(ex.bytes_for([j], [2 * e + 4096 for e in sch0.estimates([j])]) for j in jobs)
    budget = 6 * one
    sch = Scheduler(sizes, budget, max_slots=16, max_batch=4, max_inflight=2)
    st = serve(jobs, ex, sch, clock=clk, sleep=clk.sleep)
    assert st.requests == 50 and len(st.latencies_ms) == 50
    assert st.retries >= 1
    assert st.peak_bytes_measured <= budget and st.max_bytes_in_use <= budget
    assert sch.slots_used == 0


def test_idle_buffers_are_released_only_when_needed():
    """Buffers stay with their stream between batches (no reallocation per
    batch) until a batch on another stream needs the memory."""
    sizes = [1000, 1000]
    cam = synth.pinhole_camera(64, 64, 60.0, (0, 0, -3), (0, 0, 0))
    clk = VClock()
    ex = FakeExecutor(clk, n_streams=2, scene_sizes=sizes)
    sch = Scheduler(sizes, 1 << 40)
    j = [Job(0, 0, cam, 0.0)]
    need = ex.bytes_for(j, sch.estimates(j))
    h = ex.submit(j, sch.estimates(j), 0)
    ex.release(h)
    assert ex.bytes_held() == need  # kept for the next batch on stream 0
    roomy = Scheduler(sizes, 3 * need)
    assert roomy.fits(ex, 1, j, sch.estimates(j)) and ex.bytes_held() == need
    tight = Scheduler(sizes, need + need // 2)
    assert tight.fits(ex, 1, j, sch.estimates(j)) and ex.bytes_held() == 0


def test_arena_frees_a_buffer_before_growing_it(monkeypatch):
    """When a buffer of a DeviceArena grows, the old one has lost its last
    reference before the new one is allocated, so the two never coexist
    (the bytes the serving scheduler charges are then the allocator's peak)."""
    import weakref

    import torch

    from paper_2508_05343_amd.rasterize import DeviceArena
    ar = DeviceArena(device="cpu")
    small = ar.take("vals", (100,), torch.int32)
    old = weakref.ref(ar.bufs["vals"])
    del small
    seen = []
    real_empty = torch.empty

    def empty(*a, **kw):
        seen.append(old() is None)
        return real_empty(*a, **kw)
    monkeypatch.setattr(torch, "empty", empty)
    big = ar.take("vals", (1000,), torch.int32)
    assert seen == [True] and big.numel() == 1000 and ar.allocations == 2
    again = ar.take("vals", (500,), torch.int32)  # fits: reused, no allocation
    assert seen == [True] and ar.allocations == 2 and again.data_ptr() == big.data_ptr()
    assert ar.nbytes() == 4096 and ar.nbytes_after({"vals": ((2000,), torch.int32)}) == 8192


def test_idle_loop_never_sleeps_into_the_next_arrival():
    """While idle the loop sleeps only until spin_s before the next arrival
    (a sleep may overshoot) and polls from there, so a request is picked up
    at most one poll after it arrives."""
    jobs, sizes = trace(n=40, qps=50.0)
    clk = VClock(dt=1e-6)
    arrivals = sorted(j.arrival_s for j in jobs)
    spin = 3e-4
    ends = []

    def sleep(s):
        assert s > 0
        clk.sleep(s)
        ends.append(clk.t)

    ex = FakeExecutor(clk, n_streams=1, fixed_s=1e-4, per_mpix_s=0.0, scene_sizes=sizes)
    sch = Scheduler(sizes, 1 << 40, max_slots=1, max_batch=1, max_inflight=1)
    st = serve(jobs, ex, sch, clock=clk, sleep=sleep, spin_s=spin)
    assert st.requests == len(jobs) and ends
    for t in ends:  # serve's clock starts near 0: times here are arrival times
        nxt = min((a for a in arrivals if a >= t - 1e-5), default=None)
        assert nxt is None or t <= nxt - spin + 1e-5
    # picked up promptly: a one-at-a-time batch starts within a few polls of
    # its arrival (the batch itself takes fixed_s)
    assert max(st.latencies_ms) < 1e3 * (1e-4 + 1e-3)
