"""Continuous-batching render server.

Several scenes stay resident in HBM.  Render requests (scene, camera,
resolution) arrive over time; the scheduler admits every arrived request for
which a job slot is free and whose scratch estimate fits the HBM budget, packs
the admitted requests into one batch and launches it as ONE launch per stage
(preprocess, bin sort, blend) over all of the batch's jobs.  Up to
`max_inflight` batches run at once on separate HIP streams, so a batch admitted
while another is still on the GPU overlaps with it; when a batch's completion
event fires its slots and memory are released and the next batch is formed
from whatever has arrived meanwhile.

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

    def summary(self) -> Dict[str, float]:
        lat = sorted(self.latencies_ms)

        def pct(p):
            if not lat:
                return float("nan")
            i = min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))
            return lat[i]
        return dict(p50_ms=pct(50), p99_ms=pct(99), mean_ms=sum(lat) / max(1, len(lat)),
                    throughput_rps=self.requests / self.wall_s if self.wall_s > 0 else float("nan"),
                    mpix_s=self.pixels / self.wall_s / 1e6 if self.wall_s > 0 else float("nan"),
                    batches=self.batches, max_inflight_jobs=self.max_inflight_jobs,
                    max_bytes_in_use=self.max_bytes_in_use, retries=self.retries)


# --------------------------------------------------------------- estimates
def scratch_bytes(n_items: int, pixels: int, pairs: int, k: int = 4) -> int:
    """Device scratch of one job: per-item geometry (record + depth + rect +
    tiles), pair buffers (values, two key/value ping-pong buffers, per-partition
    counts) and the image, transmittance and contribution-count outputs."""
    rec = 4 * ((12 + 3 * k + 3) // 4 * 4)  # gabsplat_record_floats(k)
    per_item = rec + 4 + 8 + 4 + 4 * 5 + 1024 * 4 // 4096
    per_pair = 4 * 4 + 256 * 4 * 4 // 4096 + 4
    per_pixel = 12 + 4 + 4
    return per_item * n_items + per_pair * pairs + per_pixel * pixels + 4096


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
    """Admission and batching policy (host logic only)."""

    def __init__(self, scene_sizes: Sequence[int], budget_bytes: int, max_slots: int = 16,
                 max_batch: int = 16, max_inflight: int = 2, k: int = 4):
        self.scene_sizes = list(scene_sizes)
        self.budget = int(budget_bytes)
        self.max_slots = max_slots
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.k = k
        self.est = PairEstimator()
        self.in_use = 0
        self.slots_used = 0
        self.max_in_use = 0
        self.max_slots_used = 0

    def job_bytes(self, job: Job) -> int:
        pix = job.camera.width * job.camera.height
        n = self.scene_sizes[job.scene]
        return scratch_bytes(n, pix, self.est.estimate(job.scene, pix, n), self.k)

    def form_batch(self, queue: deque, now: float, inflight_batches: int) -> List[Job]:
        """Pop arrived jobs (FIFO) that fit the free slots and budget."""
        if inflight_batches >= self.max_inflight:
            return []
        batch: List[Job] = []
        while queue and len(batch) < self.max_batch and self.slots_used < self.max_slots:
            job = queue[0]
            if job.arrival_s > now:
                break
            b = self.job_bytes(job)
            if b > self.budget:
                raise ValueError(f"request {job.rid} needs {b} B, more than the whole budget")
            if self.in_use + b > self.budget:
                break  # head-of-line waits for memory (FIFO, no starvation)
            queue.popleft()
            job.bytes = b
            job.admitted_s = now
            self.in_use += b
            self.slots_used += 1
            batch.append(job)
        self.max_in_use = max(self.max_in_use, self.in_use)
        self.max_slots_used = max(self.max_slots_used, self.slots_used)
        return batch

    def release(self, batch: Sequence[Job]):
        for j in batch:
            self.in_use -= j.bytes
            self.slots_used -= 1
        assert self.in_use >= 0 and self.slots_used >= 0


def serve(requests: Sequence[Job], executor, scheduler: Scheduler, clock=time.perf_counter,
          keep_results=False, sleep=time.sleep) -> ServeStats:
    """Run the request trace in real time (arrival_s relative to the start)."""
    queue = deque(sorted(requests, key=lambda j: (j.arrival_s, j.rid)))
    inflight = []  # (handle, jobs)
    t0 = clock()
    lat, pixels, batches, retries = [], 0, 0, 0
    max_jobs = 0
    results = {}
    while queue or inflight:
        now = clock() - t0
        # completions first: they free slots and memory
        still = []
        for h, jobs in inflight:
            if executor.poll(h):
                done = clock() - t0
                if executor.overflowed(h):
                    retries += 1
                    executor.resubmit(h)
                    still.append((h, jobs))
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
                still.append((h, jobs))
        inflight = still
        batch = scheduler.form_batch(queue, now, len(inflight))
        if batch:
            h = executor.submit(batch, [scheduler.est.estimate(j.scene, j.camera.width * j.camera.height,
                                                               scheduler.scene_sizes[j.scene]) for j in batch])
            inflight.append((h, batch))
            batches += 1
            max_jobs = max(max_jobs, sum(len(b) for _, b in inflight))
            continue
        if not inflight and queue:
            # idle until the next arrival
            wait = queue[0].arrival_s - (clock() - t0)
            if wait > 0:
                sleep(min(wait, 0.001))
    wall = clock() - t0
    st = ServeStats(lat, wall, len(requests), pixels, batches, max_jobs, scheduler.max_in_use, retries)
    st.results = results
    return st


# ---------------------------------------------------------------- executors
class GpuExecutor:
    """Runs a batch as one RenderPlan (one launch per stage over all jobs) on
    one of a pool of HIP streams (all at the default priority)."""

    def __init__(self, device_scenes, n_streams: int = 2):
        import torch
        self.torch = torch
        self.scenes = list(device_scenes)
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.free_streams = list(range(n_streams))
        self.live = {}
        self.next_id = 0

    def _launch(self, h):
        from .rasterize import RenderPlan
        torch = self.torch
        rec = self.live[h]
        s = self.streams[rec["stream"]]
        with torch.cuda.stream(s):
            plan = rec.get("plan")
            if plan is None:
                used = sorted(set(j.scene for j in rec["jobs"]))
                remap = {sidx: i for i, sidx in enumerate(used)}
                plan = RenderPlan([self.scenes[u] for u in used], [j.camera for j in rec["jobs"]],
                                  [remap[j.scene] for j in rec["jobs"]], pair_capacity=rec["capacity"])
                rec["plan"] = plan
            plan.preprocess(s)
            plan.bin_sort(s)
            plan.render_fwd(s)
            rec["flag_host"].copy_(plan.overflow, non_blocking=True)
            rec["pairs_host"].copy_(plan.num_pairs, non_blocking=True)
            rec["event"].record(s)

    def submit(self, jobs: Sequence[Job], pair_estimates: Sequence[int]):
        torch = self.torch
        if not self.free_streams:
            raise RuntimeError("no free stream")
        h = self.next_id
        self.next_id += 1
        self.live[h] = dict(jobs=list(jobs), stream=self.free_streams.pop(0), capacity=int(sum(pair_estimates)),
                            event=torch.cuda.Event(), flag_host=torch.zeros(1, dtype=torch.int32).pin_memory(),
                            pairs_host=torch.zeros(1, dtype=torch.int64).pin_memory())
        self._launch(h)
        return h

    def poll(self, h) -> bool:
        return self.live[h]["event"].query()

    def overflowed(self, h) -> bool:
        return bool(int(self.live[h]["flag_host"][0]))

    def resubmit(self, h):
        rec = self.live[h]
        need = int(rec["pairs_host"][0])
        rec["plan"]._alloc_pairs(int(need * 1.25) + 4096)
        self._launch(h)

    def pairs(self, h) -> List[int]:
        # pairs are counted per batch; attribute them to jobs by pixel share
        rec = self.live[h]
        tot = int(rec["pairs_host"][0])
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
    duration (fixed cost + cost per pixel), overlapped up to n_streams."""

    def __init__(self, clock, n_streams=2, fixed_s=0.002, per_mpix_s=0.001):
        self.clock = clock
        self.fixed, self.per = fixed_s, per_mpix_s
        self.live = {}
        self.next_id = 0
        self.n_streams = n_streams
        self.submitted: List[List[int]] = []

    def submit(self, jobs, pair_estimates):
        if len(self.live) >= self.n_streams:
            raise RuntimeError("too many batches in flight")
        h = self.next_id
        self.next_id += 1
        mp = sum(j.camera.width * j.camera.height for j in jobs) / 1e6
        self.live[h] = dict(jobs=list(jobs), t_done=self.clock() + self.fixed + self.per * mp)
        self.submitted.append([j.rid for j in jobs])
        return h

    def poll(self, h):
        return self.clock() >= self.live[h]["t_done"]

    def overflowed(self, h):
        return False

    def resubmit(self, h):
        pass

    def pairs(self, h):
        return [j.camera.width * j.camera.height for j in self.live[h]["jobs"]]

    def images(self, h):
        return [None for _ in self.live[h]["jobs"]]

    def release(self, h):
        self.live.pop(h)
