"""Continuous-batching render server.

Several scenes stay resident in HBM.  Render requests (scene, camera,
resolution) arrive over time; the scheduler admits every arrived request for
which a job slot is free and whose buffers fit the HBM budget, packs the
admitted requests into one batch and launches it as ONE launch per stage
(preprocess, bin sort, blend) over all of the batch's jobs.  Up to
`max_inflight` batches run at once on separate HIP streams, so a batch admitted
while another is still on the GPU overlaps with it; when a batch's completion
event fires its slots and memory are released and the next batch is formed
from whatever has arrived meanwhile.

Memory is accounted in the bytes the executor really holds: each stream owns a
device arena whose buffers are reused (and grown only when a batch outgrows
them), and a batch is admitted only while every stream's arena, after serving
it, fits the budget.  Idle streams give their buffers back when that is what
it takes to admit the next batch.

The scheduler (admission, slots, budget) is plain host logic and is written
against an executor interface, so it can be tested on the CPU with a fake
executor; `GpuExecutor` drives the HIP kernels through the C ABI.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

TILE = 16


@dataclass
class Job:
    rid: int
    scene: int
    camera: object
    arrival_s: float
    admitted_s: float = -1.0
    done_s: float = -1.0
    bytes: int = 0


@dataclass
class ServeStats:
    latencies_ms: List[float]
    wall_s: float
    requests: int
    pixels: int
    batches: int
    max_inflight_jobs: int
    max_bytes_in_use: int
    retries: int = 0
    # device bytes actually allocated for the jobs' buffers at their peak
    # (the allocator's count, resident scenes excluded), or -1 if not measured
    peak_bytes_measured: int = -1
    host_ms: List[float] = field(default_factory=list)  # host time to build and launch each batch

    def summary(self) -> Dict[str, float]:
        lat = sorted(self.latencies_ms)

        def pct(v, p):
            if not v:
                return float("nan")
            i = min(len(v) - 1, max(0, int(math.ceil(p / 100.0 * len(v))) - 1))
            return v[i]
        host = sorted(self.host_ms)
        return dict(p50_ms=pct(lat, 50), p99_ms=pct(lat, 99), mean_ms=sum(lat) / max(1, len(lat)),
                    throughput_rps=self.requests / self.wall_s if self.wall_s > 0 else float("nan"),
                    mpix_s=self.pixels / self.wall_s / 1e6 if self.wall_s > 0 else float("nan"),
                    batches=self.batches, max_inflight_jobs=self.max_inflight_jobs,
                    max_bytes_in_use=self.max_bytes_in_use, peak_bytes_measured=self.peak_bytes_measured,
                    host_ms_per_batch_p50=pct(host, 50), host_ms_per_batch_mean=sum(host) / max(1, len(host)),
                    retries=self.retries)


# --------------------------------------------------------------- estimates
class PairEstimator:
    """Pairs per job, learned online per scene: the largest pairs-per-pixel
    ratio seen so far times a safety factor, starting from a generous prior
    (an underestimate costs a retry of that batch's binning, an overestimate
    only admission headroom)."""

    def __init__(self, prior_pairs_per_pixel=8.0, safety=1.5):
        self.ppp: Dict[int, float] = {}
        self.prior = prior_pairs_per_pixel
        self.safety = safety

    def estimate(self, scene: int, pixels: int, n_items: int) -> int:
        r = self.ppp.get(scene, self.prior)
        return int(max(4096, self.safety * r * pixels, 0.05 * n_items))

    def observe(self, scene: int, pixels: int, pairs: int):
        r = pairs / max(1, pixels)
        old = self.ppp.get(scene)
        self.ppp[scene] = max(r, self.prior / 4) if old is None else max(r, old)


# --------------------------------------------------------------- scheduler
class Scheduler:
    """Admission and batching policy (host logic only).  Memory is charged
    as the executor's own count of the device bytes it holds for job buffers
    (its per-stream buffers, reused from batch to batch), so what is admitted
    is what is allocated: a batch is formed for a free stream only while the
    bytes every stream would then hold fit the budget."""

    def __init__(self, scene_sizes: Sequence[int], budget_bytes: int, max_slots: int = 16,
                 max_batch: int = 16, max_inflight: int = 2, k: int = 4):
        self.scene_sizes = list(scene_sizes)
        self.budget = int(budget_bytes)
        self.max_slots = max_slots
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.k = k
        self.est = PairEstimator()
        self.slots_used = 0
        self.max_in_use = 0
        self.max_slots_used = 0

    def estimates(self, jobs: Sequence[Job]) -> List[int]:
        return [self.est.estimate(j.scene, j.camera.width * j.camera.height, self.scene_sizes[j.scene])
                for j in jobs]

    def fits(self, executor, stream, jobs: Sequence[Job], estimates: Sequence[int]) -> bool:
        """Would a batch of these jobs on `stream` keep every stream's held
        bytes within the budget?  Frees the buffers of idle streams first if
        that is what it takes."""
        def total():
            return executor.bytes_held(exclude=stream) + executor.bytes_after(stream, jobs, estimates)
        if total() <= self.budget:
            return True
        executor.release_idle()
        return total() <= self.budget

    def note_in_use(self, executor):
        self.max_in_use = max(self.max_in_use, executor.bytes_held())

    def form_batch(self, queue: deque, now: float, inflight_batches: int, executor, stream) -> List[Job]:
        """Pop arrived jobs (FIFO) that fit the free slots and the budget."""
        if inflight_batches >= self.max_inflight or stream is None:
            return []
        batch: List[Job] = []
        while queue and len(batch) < self.max_batch and self.slots_used < self.max_slots:
            job = queue[0]
            if job.arrival_s > now:
                break
            cand = batch + [job]
            if not self.fits(executor, stream, cand, self.estimates(cand)):
                if not batch and executor.bytes_for([job], self.estimates([job])) > self.budget:
                    raise ValueError(f"request {job.rid} needs more than the whole budget")
                break  # head-of-line waits for memory (FIFO, no starvation)
            queue.popleft()
            job.admitted_s = now
            batch.append(job)
        self.slots_used += len(batch)
        self.max_slots_used = max(self.max_slots_used, self.slots_used)
        return batch

    def release(self, batch: Sequence[Job]):
        self.slots_used -= len(batch)
        assert self.slots_used >= 0


def serve(requests: Sequence[Job], executor, scheduler: Scheduler, clock=time.perf_counter,
          keep_results=False, sleep=time.sleep, spin_s=3e-4) -> ServeStats:
    """Run the request trace in real time (arrival_s relative to the start).
    While idle it sleeps until spin_s before the next arrival and polls from
    there: a sleep overshoots by tens of microseconds, which would be added
    to that request's latency."""
    queue = deque(sorted(requests, key=lambda j: (j.arrival_s, j.rid)))
    inflight = []  # [handle, jobs, pair capacities of a pending retry or None]
    t0 = clock()
    lat, pixels, batches, retries = [], 0, 0, 0
    max_jobs = 0
    results = {}
    executor.start_measuring()
    while queue or inflight:
        now = clock() - t0
        # completions first: they free slots and memory
        still = []
        for h, jobs, retry in inflight:
            if retry is not None:
                # a batch whose pairs overflowed waits until its larger buffers fit
                if scheduler.fits(executor, executor.stream_of(h), jobs, retry):
                    executor.resubmit(h, retry)
                    scheduler.note_in_use(executor)
                    retry = None
                elif not executor.others_busy(h):
                    raise RuntimeError("a batch's pair buffers do not fit the budget even alone")
                still.append([h, jobs, retry])
                continue
            if executor.poll(h):
                done = clock() - t0
                if executor.overflowed(h):
                    retries += 1
                    still.append([h, jobs, executor.grown_estimates(h)])
                    continue
                for j in jobs:
                    j.done_s = done
                    lat.append(1e3 * (done - j.arrival_s))
                    pixels += j.camera.width * j.camera.height
                for j, pairs in zip(jobs, executor.pairs(h)):
                    scheduler.est.observe(j.scene, j.camera.width * j.camera.height, pairs)
                if keep_results:
                    for j, img in zip(jobs, executor.images(h)):
                        results[j.rid] = img
                executor.release(h)
                scheduler.release(jobs)
            else:
                still.append([h, jobs, retry])
        inflight = still
        stream = executor.free_stream()
        batch = scheduler.form_batch(queue, now, len(inflight), executor, stream)
        if batch:
            h = executor.submit(batch, scheduler.estimates(batch), stream)
            scheduler.note_in_use(executor)
            inflight.append([h, batch, None])
            batches += 1
            max_jobs = max(max_jobs, sum(len(b) for _, b, _ in inflight))
            continue
        if not inflight and queue:
            # idle until the next arrival
            wait = queue[0].arrival_s - (clock() - t0)
            if wait > spin_s:
                sleep(min(wait - spin_s, 0.001))
    wall = clock() - t0
    st = ServeStats(lat, wall, len(requests), pixels, batches, max_jobs, scheduler.max_in_use, retries,
                    executor.peak_bytes_measured(), list(executor.host_ms))
    st.results = results
    return st


# ---------------------------------------------------------------- executors
class GpuExecutor:
    """Runs a batch as one RenderPlan (one launch per stage over all jobs) on
    one of a pool of HIP streams (all at the default priority).  Each stream
    keeps its device buffers (a DeviceArena) and its pinned readback slots
    from batch to batch; a batch's plan takes its buffers from its stream's
    arena, so building a batch allocates only when it outgrows them."""

    def __init__(self, device_scenes, n_streams: int = 2):
        import torch
        from .rasterize import DeviceArena
        self.torch = torch
        self.scenes = list(device_scenes)
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.arenas = [DeviceArena() for _ in range(n_streams)]
        self.flags = [torch.zeros(1, dtype=torch.int32).pin_memory() for _ in range(n_streams)]
        self.pairs_host = [torch.zeros(1, dtype=torch.int64).pin_memory() for _ in range(n_streams)]
        self.events = [torch.cuda.Event() for _ in range(n_streams)]
        self.free_streams = list(range(n_streams))
        self.live = {}
        self.next_id = 0
        self.host_ms: List[float] = []
        self.base_bytes = 0
        # per batch: bytes its plan's buffers take, bytes its stream's arena holds
        self.batch_bytes: List[tuple] = []

    # ----- memory accounting (bytes of the job buffers, resident scenes excluded)
    def _specs(self, jobs, estimates):
        from .rasterize import plan_buffer_specs
        used = set(j.scene for j in jobs)
        items = sum(self.scenes[j.scene].n for j in jobs)
        pix = sum(j.camera.width * j.camera.height for j in jobs)
        tiles = sum(((j.camera.width + TILE - 1) // TILE) * ((j.camera.height + TILE - 1) // TILE) for j in jobs)
        return plan_buffer_specs(self.scenes[0].k, items, pix, tiles, len(jobs), len(used), int(sum(estimates)))

    def bytes_for(self, jobs, estimates) -> int:
        from .rasterize import specs_block_bytes
        return specs_block_bytes(self._specs(jobs, estimates))

    def bytes_after(self, stream, jobs, estimates) -> int:
        return self.arenas[stream].nbytes_after(self._specs(jobs, estimates))

    def bytes_held(self, exclude=None) -> int:
        return sum(a.nbytes() for i, a in enumerate(self.arenas) if i != exclude)

    def release_idle(self):
        for i in self.free_streams:
            self.arenas[i].release()

    def start_measuring(self):
        torch = self.torch
        torch.cuda.synchronize()
        self.base_bytes = torch.cuda.memory_allocated() - self.bytes_held()
        torch.cuda.reset_peak_memory_stats()

    def peak_bytes_measured(self) -> int:
        return int(self.torch.cuda.max_memory_allocated() - self.base_bytes)

    # ----- batches
    def free_stream(self):
        return self.free_streams[0] if self.free_streams else None

    def stream_of(self, h):
        return self.live[h]["stream"]

    def others_busy(self, h) -> bool:
        return len(self.live) > 1

    def _launch(self, h):
        torch = self.torch
        rec = self.live[h]
        st = rec["stream"]
        s = self.streams[st]
        with torch.cuda.stream(s):
            plan = rec["plan"]
            plan.preprocess(s)
            plan.bin_sort(s)
            plan.render_fwd(s)
            self.flags[st].copy_(plan.overflow, non_blocking=True)
            self.pairs_host[st].copy_(plan.num_pairs, non_blocking=True)
            self.events[st].record(s)

    def submit(self, jobs: Sequence[Job], pair_estimates: Sequence[int], stream):
        from .rasterize import RenderPlan, specs_nbytes
        t = time.perf_counter()
        self.free_streams.remove(stream)
        h = self.next_id
        self.next_id += 1
        used = sorted(set(j.scene for j in jobs))
        remap = {sidx: i for i, sidx in enumerate(used)}
        with self.torch.cuda.stream(self.streams[stream]):
            plan = RenderPlan([self.scenes[u] for u in used], [j.camera for j in jobs],
                              [remap[j.scene] for j in jobs], pair_capacity=int(sum(pair_estimates)),
                              arena=self.arenas[stream])
        self.live[h] = dict(jobs=list(jobs), stream=stream, plan=plan)
        self._launch(h)
        # bookkeeping after the launches, off the batch's latency
        self.batch_bytes.append((specs_nbytes(plan.buffer_specs()), self.arenas[stream].nbytes()))
        self.host_ms.append(1e3 * (time.perf_counter() - t))
        return h

    def poll(self, h) -> bool:
        return self.events[self.live[h]["stream"]].query()

    def overflowed(self, h) -> bool:
        return bool(int(self.flags[self.live[h]["stream"]][0]))

    def grown_estimates(self, h) -> List[int]:
        """Pair capacities (per job, by pixel share) that hold the pairs the
        overflowed binning counted, with headroom."""
        rec = self.live[h]
        need = int(int(self.pairs_host[rec["stream"]][0]) * 1.25) + 4096
        pix = [j.camera.width * j.camera.height for j in rec["jobs"]]
        return [need * p // sum(pix) + 1 for p in pix]

    def resubmit(self, h, estimates):
        rec = self.live[h]
        with self.torch.cuda.stream(self.streams[rec["stream"]]):
            rec["plan"]._alloc_pairs(int(sum(estimates)))
        self._launch(h)

    def pairs(self, h) -> List[int]:
        # pairs are counted per batch; attribute them to jobs by pixel share
        rec = self.live[h]
        tot = int(self.pairs_host[rec["stream"]][0])
        pix = [j.camera.width * j.camera.height for j in rec["jobs"]]
        sp = sum(pix)
        return [int(tot * p / sp) for p in pix]

    def images(self, h):
        plan = self.live[h]["plan"]
        return [plan.view_image(v).clone() for v in range(len(self.live[h]["jobs"]))]

    def release(self, h):
        rec = self.live.pop(h)
        self.free_streams.append(rec["stream"])


class FakeExecutor:
    """CPU stand-in for scheduler tests: a batch completes after a modelled
    duration (fixed cost + cost per pixel), overlapped up to n_streams; its
    buffers are modelled as bytes per primitive, pixel and pair, held per
    stream (grow-only, released when idle) like the GPU executor's."""

    def __init__(self, clock, n_streams=2, fixed_s=0.002, per_mpix_s=0.001, scene_sizes=(), overflow_every=0):
        self.clock = clock
        self.fixed, self.per = fixed_s, per_mpix_s
        self.live = {}
        self.next_id = 0
        self.n_streams = n_streams
        self.held = [0] * n_streams
        self.free_streams = list(range(n_streams))
        self.scene_sizes = list(scene_sizes)
        self.overflow_every = overflow_every  # every n-th first launch reports a pair overflow
        self.submitted: List[List[int]] = []
        self.host_ms: List[float] = []
        self.peak = 0

    def bytes_for(self, jobs, estimates):
        items = sum(self.scene_sizes[j.scene] for j in jobs) if self.scene_sizes else 0
        pix = sum(j.camera.width * j.camera.height for j in jobs)
        return 100 * items + 20 * pix + 24 * int(sum(estimates)) + 4096

    def bytes_after(self, stream, jobs, estimates):
        return max(self.held[stream], self.bytes_for(jobs, estimates))

    def bytes_held(self, exclude=None):
        return sum(b for i, b in enumerate(self.held) if i != exclude)

    def release_idle(self):
        for i in self.free_streams:
            self.held[i] = 0

    def start_measuring(self):
        self.peak = 0

    def peak_bytes_measured(self):
        return self.peak

    def free_stream(self):
        return self.free_streams[0] if self.free_streams else None

    def stream_of(self, h):
        return self.live[h]["stream"]

    def others_busy(self, h):
        return len(self.live) > 1

    def _hold(self, stream, jobs, estimates):
        self.held[stream] = self.bytes_after(stream, jobs, estimates)
        self.peak = max(self.peak, sum(self.held))

    def submit(self, jobs, pair_estimates, stream):
        if stream not in self.free_streams:
            raise RuntimeError("stream busy")
        self.free_streams.remove(stream)
        self._hold(stream, jobs, pair_estimates)
        h = self.next_id
        self.next_id += 1
        mp = sum(j.camera.width * j.camera.height for j in jobs) / 1e6
        over = self.overflow_every > 0 and h % self.overflow_every == 0
        self.live[h] = dict(jobs=list(jobs), stream=stream, t_done=self.clock() + self.fixed + self.per * mp,
                            over=over, est=list(pair_estimates))
        self.submitted.append([j.rid for j in jobs])
        self.host_ms.append(0.0)
        return h

    def poll(self, h):
        return self.clock() >= self.live[h]["t_done"]

    def overflowed(self, h):
        return self.live[h]["over"]

    def grown_estimates(self, h):
        return [2 * e + 4096 for e in self.live[h]["est"]]

    def resubmit(self, h, estimates):
        rec = self.live[h]
        self._hold(rec["stream"], rec["jobs"], estimates)
        rec.update(over=False, est=list(estimates), t_done=self.clock() + self.fixed)

    def pairs(self, h):
        return [j.camera.width * j.camera.height for j in self.live[h]["jobs"]]

    def images(self, h):
        return [None for _ in self.live[h]["jobs"]]

    def release(self, h):
        rec = self.live.pop(h)
        self.free_streams.append(rec["stream"])
