#!/usr/bin/env python3
"""Benchmark of the MI355X Gabor splatting rasterizer.

Default workload: forward render of 1,000,000 Gabor primitives (K = 4, SH
degree 3, 64 seeded clusters in a 20-unit box) through a 1297x840 pinhole
camera inside the scene, fp32.  One step = preprocess -> bin sort -> blend on
inputs resident in HBM.  Also reported: the training step on the same scene
(forward, L1 + 0.2 D-SSIM loss against a seeded target, backward to every
attribute), per-stage times, the roofline of the dominant kernel, and the CPU
oracle timed on a bounded sample of the same frame.

Prints one JSON line (rank 0).  Single GPU only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# fp32 VALU peak without packed-FP32 instructions (the library is compiled
# without them): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
VALU_PEAK_TFLOPS = 78.6

# Counters of one launch of each blend kernel on the default workload, from
# rocprofv3 --pmc runs of `bench.py --profile` (means over the dispatches):
#   fetch_kib / write_kib  FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each
#       scaled by what the same counter reads for the 256 MiB device copy the
#       same run makes (fetch_scale, write_scale: bytes moved / counter bytes)
#   valu_busy  SQ_ACTIVE_INST_VALU x 4 / (SIMDs x GRBM_GUI_ACTIVE / XCDs)
#       (GRBM_GUI_ACTIVE is summed over the 8 XCDs; SQ_ACTIVE_INST_VALU sums,
#       per wavefront, the quad-cycles with a VALU instruction in flight, so a
#       saturated SIMD whose transcendental instructions overlap the next
#       wavefront's issue reads above 1)
#   valu_util  SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU): active lanes
#       per issued VALU instruction
#   lds_bank_conflict  SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE: conflict
#       cycles per LDS access cycle
# Valid only for the kernel source they were taken on (hash of the kernel's
# source text); otherwise the bench reports them as null.
RENDER_FWD_COUNTERS = {
    "source_sha256": "506d5085f64925d126f209cf5bc6d837a0d12e6e52d30ba98923271a612202bc",
    "fetch_kib": 84231.7, "write_kib": 34440.4, "fetch_scale": 2.0, "write_scale": 1.0,
    "valu_busy": 0.9328, "valu_util": 0.9841, "lds_bank_conflict": 0.0043,
}
RENDER_BWD_COUNTERS = {
    "source_sha256": "725661bc35587c921f8df4c349ab0ba788771e215df09238b93172814cd618da",
    "fetch_kib": 85130.4, "write_kib": 113938.6, "fetch_scale": 2.0, "write_scale": 1.0,
    "valu_busy": 1.0492, "valu_util": 0.9779, "lds_bank_conflict": 0.0,
}

_SPLIT = "// ------------------------------------------------- wave reduce-scatter-add"


def _render_source_sha(part):
    """sha256 over the source of one blend kernel: render.hip before (forward)
    or from (backward) the backward's helpers, plus the internal headers."""
    import hashlib
    base = os.path.join(ROOT, "paper_2508_05343_amd", "csrc")
    with open(os.path.join(base, "render.hip")) as f:
        txt = f.read()
    cut = txt.index(_SPLIT)
    h = hashlib.sha256((txt[:cut] if part == "fwd" else txt[cut:]).encode())
    for hdr in ("gs_internal.h", "gs_sort.h"):
        with open(os.path.join(base, hdr)) as f:
            h.update(f.read().encode())
    return h.hexdigest()


def render_fwd_source_sha():
    return _render_source_sha("fwd")


def render_bwd_source_sha():
    return _render_source_sha("bwd")


def kernel_counters(table, sha):
    """(traffic bytes per launch or None, {valu_busy, valu_util,
    lds_bank_conflict} or Nones) for a counter table, if taken on this source."""
    keys = ("valu_busy", "valu_util", "lds_bank_conflict")
    if sha != table["source_sha256"] or table["fetch_kib"] is None:
        return None, {k: None for k in keys}
    traffic = int(1024 * (table["fetch_kib"] * table["fetch_scale"] + table["write_kib"] * table["write_scale"]))
    return traffic, {k: table[k] for k in keys}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-train", action="store_true", help="skip the training-step measurement")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-tiles", type=int, default=4346,
                    help="tiles of the frame blended by the CPU oracle (default: all 4346 of the forward "
                         "workload's frame, 10-30 s on 16 host threads)")
    ap.add_argument("--profile", action="store_true", help="few steps, no CPU baseline (for rocprofv3)")
    ap.add_argument("--no-multiview", action="store_true", help="skip the 64-view training step")
    ap.add_argument("--profile-multiview", action="store_true",
                    help="only the 64-view training step, a few steps (for rocprofv3)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-qps", type=float, default=200.0)
    ap.add_argument("--serve-sweep", type=str, default="1000,4000",
                    help="extra arrival rates (QPS) run with 600 requests each to find saturation")
    return ap.parse_args()


class StageTimer:
    """HIP events around each entry point on the stream the kernels run on."""

    def __init__(self, torch, names):
        self.torch = torch
        self.names = names
        self.ev = {n: [] for n in names}

    def pair(self, name):
        s = self.torch.cuda.Event(enable_timing=True)
        e = self.torch.cuda.Event(enable_timing=True)
        self.ev[name].append((s, e))
        return s, e

    def totals_ms(self):
        return {n: sum(s.elapsed_time(e) for s, e in v) for n, v in self.ev.items()}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the rasterizer has no multi-GPU path "
              "(one GPU renders its own views; a batch of views would shard across GPUs by view); "
              "run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.profile:
        args.steps, args.warmup, args.no_cpu_baseline = min(args.steps, 5), min(args.warmup, 2), True
        args.no_multiview, args.no_serve = True, True

    import numpy as np
    import torch

    import synth
    from paper_2508_05343_amd import _lib
    from paper_2508_05343_amd.rasterize import DeviceScene, LossBuffers, RenderPlan

    _lib.gabsplat_check_device()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.profile_multiview:
        args.steps = min(args.steps, 5)
        print(json.dumps({"multiview": multiview_step(args, torch, synth, DeviceScene, RenderPlan, LossBuffers)}),
              flush=True)
        return

    scene = synth.scene_1m_k4_sh3()
    cam = synth.camera_1297x840()
    ds = DeviceScene.from_host(scene)
    # the rendered scene stays fixed: its quaternions, frequencies and weights
    # are also packed row by row (one line per primitive) for the projection
    plan = RenderPlan([ds.with_rows()], [cam])
    # establish the pair capacity (host sync allowed outside the timed region)
    plan.forward(check_overflow=True)
    torch.cuda.synchronize()
    P = int(plan.num_pairs.item())
    vis = int((plan.tiles_touched[:plan.items] > 0).sum().item())
    pix = cam.width * cam.height

    timer = StageTimer(torch, ["preprocess", "bin_sort", "render_fwd"])

    def fwd_step(record):
        if record:
            a, b = timer.pair("preprocess"); a.record(stream)
        plan.preprocess()
        if record:
            b.record(stream); a, b = timer.pair("bin_sort"); a.record(stream)
        plan.bin_sort()
        if record:
            b.record(stream); a, b = timer.pair("render_fwd"); a.record(stream)
        plan.render_fwd()
        if record:
            b.record(stream)

    for _ in range(args.warmup):
        fwd_step(False)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(args.steps):
        fwd_step(True)
    t1.record(stream)
    torch.cuda.synchronize()
    assert int(plan.overflow.item()) == 0, "pair capacity overflow during the timed steps"
    total_ms = t0.elapsed_time(t1)
    ms_step = total_ms / args.steps
    stage = {k: v / args.steps for k, v in timer.totals_ms().items()}

    # ---- the timed region again without per-stage events (pure throughput)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(args.steps):
        fwd_step(False)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_step_clean = t0.elapsed_time(t1) / args.steps

    # ---- roofline of the blend (one kernel launch, k_render_fwd<4>).  Its work
    # is counted by the kernel itself in a separate, untimed launch: per pixel
    # the pairs walked up to the stop (each needs the envelope test) and the
    # pairs that passed it (each needs the full Gabor evaluation).
    counts = torch.zeros((pix, 2), dtype=torch.int32, device=dev)
    plan.render_fwd(eval_counts=counts)
    torch.cuda.synchronize()
    e_env = int(counts[:, 0].to(torch.int64).sum().item())
    e_full = int(counts[:, 1].to(torch.int64).sum().item())
    K = plan.k
    # per evaluation, an FMA counting 2 and a transcendental 1: the envelope test
    # (2 subtractions, 3 multiplies, 3 FMAs) and the full evaluation (exp2; per
    # component 2 FMAs for the phase, cos and an FMA; clamp, T - aT, aT, 3 colour FMAs)
    flops_env, flops_full = 10, 12 + 7 * K
    render_flops = flops_env * e_env + flops_full * e_full
    ranges = plan.ranges[:cam.num_tiles].to(torch.int64)
    bwd_walk = int(plan.n_contrib[:pix].to(torch.int64).sum().item())
    p_read = int((ranges[:, 1] - ranges[:, 0]).sum().item())
    rec_bytes = 4 * (12 + 3 * K)  # record floats the blend uses (fields + the mean's rounding residuals)
    render_bytes = p_read * (4 + rec_bytes) + pix * (12 + 4 + 4) + cam.num_tiles * 8
    stage_ms = dict(stage)
    dom = max(stage_ms, key=stage_ms.get)
    t_render = stage_ms["render_fwd"] * 1e-3
    render_tflops = render_flops / t_render / 1e12
    render_gbs = (render_bytes / 1e9) / t_render
    # pass-aware algorithmic bytes of the whole forward: preprocess (means of all,
    # parameters of the visible, records written, depth/rect/tiles of all), compaction,
    # duplication, a six-pass 8-bit sort of the pairs, ranges, and the blend
    N, V = scene.n, vis
    params_visible = 4 * (3 + 4 + 1 + 48 + 4 * K)
    b_pre = 12 * N + params_visible * V + 4 * (12 + 3 * K) * V + 4 * 4 * N
    b_scan = 8 * N
    b_dup = 16 * V + 12 * P
    b_sort = 8 * P + 24 * P * 6
    b_ranges = 8 * P + 8 * cam.num_tiles
    b_fwd = b_pre + b_scan + b_dup + b_sort + b_ranges + render_bytes
    hbm_frac_fwd = (b_fwd / 1e9) / (ms_step_clean * 1e-3) / HBM_PEAK_GBS
    fwd_traffic, fwd_ctr = kernel_counters(RENDER_FWD_COUNTERS, render_fwd_source_sha())
    out = {
        "metric": "Mpix/s fwd, fwd+bwd step ms @1M Gabor prims; serve p50/p99 latency",
        "value": round(pix / (ms_step_clean * 1e-3) / 1e6, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step_clean, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded clustered scene, random-init attributes)",
        "config": {"workload": "forward render, 1,000,000 Gabor primitives, K=4, SH degree 3, 1297x840",
                   "primitives": N, "k": K, "sh_degree": 3, "width": cam.width, "height": cam.height,
                   "visible": V, "pairs": P, "parallelism": "single GPU"},
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "fwd_pass_aware_bytes": int(b_fwd),
        "fwd_hbm_fraction": round(hbm_frac_fwd, 4),
        "roofline": {"kernel": "k_render_fwd<4>", "bound": "alu", "achieved": round(render_tflops, 3),
                     "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(render_tflops / VALU_PEAK_TFLOPS, 4),
                     "traffic": fwd_traffic, **fwd_ctr, "evaluations": e_env, "full_evaluations": e_full,
                     "flops_per_launch": int(render_flops), "kernel_ms": round(stage_ms["render_fwd"], 4),
                     "hbm_gbs": round(render_gbs, 1), "hbm_frac": round(render_gbs / HBM_PEAK_GBS, 4),
                     "dominant_stage": dom},
    }

    # ---- calibration copy of known size for the HBM counters (profile runs)
    if args.profile:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)  # 256 MiB read + 256 MiB written
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * 4
        del src, dst

    # ---- training step (forward + loss + backward).  Training changes the
    # attributes every step, so its plan reads the planes only (no rows).
    if not args.no_train:
        target = torch.from_numpy(synth.random_target(1003, (3, cam.height, cam.width))).to(dev)
        lossb = LossBuffers(3, cam.height, cam.width)
        grads = {n: torch.zeros_like(getattr(ds, n)) for n in
                 ("means", "scales", "quats", "opacities", "sh", "freqs", "weights")}
        tplan = RenderPlan([ds], [cam], pair_capacity=plan.capacity)
        img = tplan.view_image(0)

        def tfwd_step():
            tplan.preprocess()
            tplan.bin_sort()
            tplan.render_fwd()

        def train_step():
            tfwd_step()
            lossb(img, target)
            tplan.backward(lossb.grad.view(-1), [grads], accumulate=False)

        for _ in range(max(2, args.warmup // 2)):
            train_step()
        torch.cuda.synchronize()
        ts = max(5, args.steps // 2)
        t0.record(stream)
        for _ in range(ts):
            train_step()
        t1.record(stream)
        torch.cuda.synchronize()
        out["train_step_ms"] = round(t0.elapsed_time(t1) / ts, 4)
        out["train_loss"] = round(float(lossb.loss.item()), 6)

        # the same steps with HIP events between the backward's two stages
        # (the blend stage is the grad2d row clear + k_render_bwd)
        btimer = StageTimer(torch, ["loss", "render_bwd", "project_bwd"])

        def train_step_staged():
            tfwd_step()
            a, b = btimer.pair("loss"); a.record(stream)
            lossb(img, target)
            b.record(stream); a, b = btimer.pair("render_bwd"); a.record(stream)
            tplan.backward(lossb.grad.view(-1), [grads], accumulate=False, stages=_lib.BWD_BLEND)
            b.record(stream); a, b = btimer.pair("project_bwd"); a.record(stream)
            tplan.backward(lossb.grad.view(-1), [grads], accumulate=False, stages=_lib.BWD_PROJECT)
            b.record(stream)

        for _ in range(ts):
            train_step_staged()
        torch.cuda.synchronize()
        bst = {k: v / ts for k, v in btimer.totals_ms().items()}
        out["train_stages_ms"] = {k: round(v, 4) for k, v in bst.items()}
        # algorithmic work of k_render_bwd<4>: each pixel walks its list back
        # from its last contributor (n_contrib): an envelope test per pair
        # (10 flops, as the forward) and, for the pairs that pass it (the
        # forward's count up to its stop: at most the stopping pair more), the
        # alpha of the forward (12 + 7K) and its gradient (46 + 13K flops:
        # transmittance recovery, colour and opacity terms, conic, mean and
        # per-component phase terms, and the sum over pixels of the 10 + 3K
        # record gradients)
        bwd_flops = 10 * bwd_walk + (58 + 20 * K) * e_full
        t_bwd = bst["render_bwd"] * 1e-3
        bwd_tflops = bwd_flops / t_bwd / 1e12
        bwd_traffic, bwd_ctr = kernel_counters(RENDER_BWD_COUNTERS, render_bwd_source_sha())
        out["roofline_bwd"] = {"kernel": "k_render_bwd<4>", "bound": "alu", "achieved": round(bwd_tflops, 3),
                               "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": round(bwd_tflops / VALU_PEAK_TFLOPS, 4), "traffic": bwd_traffic, **bwd_ctr,
                               "walked_pairs": bwd_walk, "full_evaluations": e_full,
                               "flops_per_launch": int(bwd_flops), "kernel_ms": round(bst["render_bwd"], 4)}

    # ---- multi-view training step: 64 views of 800x800, one launch per stage
    if not args.no_multiview:
        out["multiview"] = multiview_step(args, torch, synth, DeviceScene, RenderPlan, LossBuffers)
        print(json.dumps({"progress": "multiview", **out["multiview"]}), file=sys.stderr, flush=True)

    # ---- serving: continuous batching vs one request at a time
    if not args.no_serve:
        out["serve"] = serving_run(args, torch, synth)
        print(json.dumps({"progress": "serve", **out["serve"]}), file=sys.stderr, flush=True)

    # ---- CPU oracle on a bounded sample of the same frame
    if not args.no_cpu_baseline:
        from oracle import gabor_oracle as O
        ncores = torch.get_num_threads()
        t = time.perf_counter()
        with torch.no_grad():
            pr = O.project(O.scene_tensors(scene), O.camera_tensors(cam), scene)
        t_proj = time.perf_counter() - t
        rng = np.random.Generator(np.random.PCG64(7))
        sel = rng.choice(cam.num_tiles, size=min(args.cpu_tiles, cam.num_tiles), replace=False)
        tiles = [(int(s % cam.tiles_x), int(s // cam.tiles_x)) for s in sel]
        t = time.perf_counter()
        with torch.no_grad():
            O.render(None, O.camera_tensors(cam), "binned", tiles=tiles, scene_f32=scene, pr=pr)
        t_blend = time.perf_counter() - t
        spix = sum(min(16, cam.width - 16 * tx) * min(16, cam.height - 16 * ty) for tx, ty in tiles)
        t_sample = t_blend + t_proj * spix / pix
        out["cpu_baseline"] = {"value": round(spix / t_sample / 1e6, 5), "unit": "Mpix/s", "cores": ncores,
                               "kind": "oracle",
                               "sample": f"fp64 projection of all {N} primitives ({t_proj:.1f} s, charged pro rata) "
                                         f"+ blend of {len(tiles)} seeded tiles of {cam.num_tiles} ({spix} px, "
                                         f"{t_blend:.1f} s)",
                               "host": host_cpu(), "fp32": oracle_fp32_rate(O, torch, np, scene, cam, pix, tiles)}
    print(json.dumps(out))


def host_cpu():
    """The host the CPU baseline ran on: logical CPUs the OS reports and the
    processor model (the oracle's threads are `cores`)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def oracle_fp32_rate(O, torch, np, scene, cam, pix, tiles):
    """The same oracle evaluated in float32 (its arithmetic type switched, the
    decisions it takes on float32 data unchanged) on a quarter of the sampled
    tiles: Mpix/s, projection charged pro rata as above."""
    sub = tiles[: max(1, len(tiles) // 4)]
    saved = O.DT
    O.DT = torch.float32
    try:
        t = time.perf_counter()
        with torch.no_grad():
            pr = O.project(O.scene_tensors(scene), O.camera_tensors(cam), scene)
        t_proj = time.perf_counter() - t
        t = time.perf_counter()
        with torch.no_grad():
            O.render(None, O.camera_tensors(cam), "binned", tiles=sub, scene_f32=scene, pr=pr)
        t_blend = time.perf_counter() - t
    finally:
        O.DT = saved
    spix = sum(min(16, cam.width - 16 * tx) * min(16, cam.height - 16 * ty) for tx, ty in sub)
    return {"value": round(spix / (t_blend + t_proj * spix / pix) / 1e6, 5), "unit": "Mpix/s",
            "sample": f"fp32 projection of all primitives ({t_proj:.1f} s, pro rata) + blend of {len(sub)} tiles "
                      f"({spix} px, {t_blend:.1f} s)"}


def multiview_step(args, torch, synth, DeviceScene, RenderPlan, LossBuffers):
    """300k primitives, K=4, SH3, 64 cameras on an orbit at 800x800: forward
    over all views (one launch per stage), loss over all views (one launch),
    backward over all views with the gradients summed over views in fp32."""
    scene = synth.scene_300k_k4_sh3()
    cams = synth.orbit_cameras_64x800()
    ds = DeviceScene.from_host(scene)
    plan = RenderPlan([ds], cams, [0] * len(cams), pair_capacity=12 * scene.n * len(cams))
    plan.forward(check_overflow=True)
    torch.cuda.synchronize()
    V, H, W = len(cams), cams[0].height, cams[0].width
    tgt = torch.cat([torch.from_numpy(synth.random_target(1004 + v, (3, H, W))) for v in range(V)]).cuda()
    lossb = LossBuffers(3 * V, H, W)
    grads = {n: torch.zeros_like(getattr(ds, n)) for n in
             ("means", "scales", "quats", "opacities", "sh", "freqs", "weights")}
    img = plan.image[:3 * V * H * W].view(3 * V, H, W)

    def step():
        plan.preprocess()
        plan.bin_sort()
        plan.render_fwd()
        lossb(img, tgt)
        plan.backward(lossb.grad.view(-1), [grads], accumulate=False)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    steps = max(3, args.steps // 10)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    assert int(plan.overflow.item()) == 0
    ms = e0.elapsed_time(e1) / steps
    return {"workload": "64 views x 800x800 fwd+loss+bwd, 300,000 primitives, K=4, SH3",
            "step_ms": round(ms, 3), "views_per_s": round(V / (ms * 1e-3), 1),
            "mpix_s": round(V * H * W / (ms * 1e-3) / 1e6, 1), "pairs": int(plan.num_pairs.item()),
            "loss": round(float(lossb.loss.item()), 6)}


def serving_run(args, torch, synth):
    """8 resident scenes (100k..2M primitives), Poisson requests, random
    cameras and resolutions; continuous batching vs one request at a time."""
    from paper_2508_05343_amd.rasterize import DeviceScene
    from paper_2508_05343_amd.serving import GpuExecutor, Job, Scheduler, serve
    scenes = synth.serving_scenes()
    # resident scenes stay fixed: each also carries its packed rows
    dss = [DeviceScene.from_host(s).with_rows() for s in scenes]
    reqs = synth.serving_requests(scenes, n_requests=args.serve_requests, qps=args.serve_qps)
    sizes = [s.n for s in scenes]
    budget = 6 << 30

    def jobs():
        return [Job(r.rid, r.scene, r.camera, r.arrival_s) for r in reqs]

    # warm the kernels and the allocator with a few requests of every shape
    warm = [Job(i, i % 8, r.camera, 0.0) for i, r in enumerate(reqs[:16])]
    serve(warm, GpuExecutor(dss, 2), Scheduler(sizes, budget, max_slots=16, max_batch=16, max_inflight=2))
    torch.cuda.synchronize()
    res = {}
    for mode, sch, ns in (("continuous", Scheduler(sizes, budget, max_slots=16, max_batch=16, max_inflight=2), 2),
                          ("sequential", Scheduler(sizes, budget, max_slots=1, max_batch=1, max_inflight=1), 1)):
        st = serve(jobs(), GpuExecutor(dss, ns), sch)
        sm = st.summary()
        res[mode] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in sm.items()}
    res["workload"] = (f"8 resident scenes ({sum(sizes)} primitives), {len(reqs)} Poisson requests at "
                       f"{args.serve_qps:g} QPS, resolutions 256^2..1920x1080, 6 GiB budget for job buffers "
                       "(scenes resident with packed rows)")
    sweep = []
    for q in [float(x) for x in args.serve_sweep.split(",") if x]:
        rq = synth.serving_requests(scenes, n_requests=600, qps=q, seed=1005 + int(q))
        row = {"qps": q}
        for mode, sch, ns in (("continuous", Scheduler(sizes, budget, max_slots=16, max_batch=16, max_inflight=2), 2),
                              ("sequential", Scheduler(sizes, budget, max_slots=1, max_batch=1, max_inflight=1), 1)):
            st = serve([Job(r.rid, r.scene, r.camera, r.arrival_s) for r in rq], GpuExecutor(dss, ns), sch)
            sm = st.summary()
            row[mode] = {k: round(sm[k], 3) for k in ("p50_ms", "p99_ms", "throughput_rps", "mpix_s")}
        sweep.append(row)
    res["sweep"] = sweep
    return res


if __name__ == "__main__":
    main()
