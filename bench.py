"""Benchmark of the cache's hot path on one MI355X: one step = one 1920x1080 frame with 32 lights.

A step runs every stage of the path on synthetic data resident in HBM:
  infer   hash-grid encoding + MLP for all 2,073,600 pixels   (nvc_infer, FP16 matrix cores)
  wrs     weighted reservoir light pick + neural DI per pixel   (nvc_sample_wrs)
  pixels  2^18 training pixels                                  (nvc_select_pixels)
  labels  2^18 x 32 shadow rays against 256 spheres             (nvc_shadow_labels)
  train   recomputed forward, backward, table scatter           (nvc_train_step)
  adam    Adam on 16.8M table + 12,288 MLP params, repack        (nvc_adam x2, nvc_pack_mlp)

Prints one JSON line.  `value` is visibility queries/s (one query = one pixel
against all 32 lights) over whole frames, training included.  Timed frames
run through FramePipeline: inference + WRS on one stream, the gradient pass
and Adam on a second, and the next frame's training pixels and shadow labels
on a third (they depend on the frame number and the scene only); inference
waits for the previous frame's Adam, Adam for this frame's inference.  The
per-stage times come from a separate pass that runs every stage in order on
one stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Published MI355X peaks.
PEAK_HBM_GBS = 8000.0
PEAK_F16_TFLOPS = 2500.0

STAGES = ["infer", "wrs", "pixels", "labels", "train", "adam"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100,
                    help="timed frames (the timed region ends with one frame of look-ahead work that no later frame "
                         "overlaps, so short runs overstate the per-frame time)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="train_1080p")
    ap.add_argument("--dtype", default=None, help="override the MLP dtype (f32, f16, bf16)")
    ap.add_argument("--order", default="morton", choices=["morton", "rows", "shuffled"],
                    help="pixel order of the G-buffer (morton: tiled; shuffled: the worst case for the gathers)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=131072, help="pixels of the oracle's timed sample")
    ap.add_argument("--calibrate-copy-mib", type=int, default=256,
                    help="size of a plain device copy run after timing (counter calibration); 0 = none")
    ap.add_argument("--no-rowmajor", action="store_true",
                    help="skip the extra timed frames on the row-major G-buffer (reported beside the Z-order ones)")
    ap.add_argument("--no-stages", action="store_true",
                    help="skip the serial per-stage pass (every launch of the run is then a timed-style frame)")
    ap.add_argument("--fused-labels", action="store_true",
                    help="label the training samples inside the training kernel (nvc_train_step_shadow) instead "
                         "of with the separate label kernel")
    ap.add_argument("--loop", type=int, default=0,
                    help="instead: run the frame loop for this many frames (one HIP graph per frame, light 0 "
                         "moving) and print its per-frame report")
    ap.add_argument("--loop-eval", type=int, default=65536, help="pixels of the loop's fixed evaluation subset")
    ap.add_argument("--loop-graph", choices=("pipeline", "lagged"), default="pipeline",
                    help="the loop's recorded frame: 'pipeline' (PipelineGraph); 'lagged' would run frame f's "
                         "light pick inside the replay of frame f + 1 (LaggedPickGraph, switched off: it raises)")
    ap.add_argument("--micro", action="store_true",
                    help="instead: the memory microbenchmarks (device copy, random 8-byte gathers)")
    ap.add_argument("--mlp", action="store_true",
                    help="instead: time the MLP alone (nvc_mlp_forward) on the frame's encoding and report its "
                         "matrix-core throughput")
    return ap.parse_args()


def algorithmic(wl, n_pix, batch):
    """Algorithmic bytes / operations of each stage for one frame (see the design notes)."""
    L, F, M = wl.grid.n_levels, wl.grid.n_feat, wl.mlp.n_out
    n_params = wl.grid.n_params + wl.mlp.n_params
    vis_b = 2 if wl.mlp.dtype != "f32" else 4
    # 8 corners x F x 4 B per level per query; a table that fits in the L2 (8 XCDs x 4 MiB) is read from
    # HBM once per launch instead
    table_b = wl.grid.n_params * 4
    gathers = n_pix * L * 8 * F * 4 if table_b > L2_BYTES else table_b
    return {
        # 12 B position + gathers + M visibilities out
        "infer": {"bytes": n_pix * (12 + M * vis_b) + gathers, "flops": n_pix * wl.mlp.flops_per_point},
        # visibilities + position + normal in, index/pmf/W/DI out
        "wrs": {"bytes": n_pix * (M * vis_b + 24 + 16)},
        "pixels": {"bytes": batch * 4},
        # segment-sphere tests, ~13 FP32 operations each
        "labels": {"ops": batch * M * wl.n_spheres * 13, "bytes": batch * (12 + 4 + M)},
        # forward + backward (3x the forward flops); 8 corners x F gathers and atomics per level
        "train": {"flops": batch * 3 * wl.mlp.flops_per_point,
                  "bytes": batch * (12 + 4 + M + 2 * L * 8 * F * 4)},
        # read p, g, m, v; write p, m, v, g(=0)
        "adam": {"bytes": n_params * 32},
    }


def _host_cores() -> int:
    """CPU threads this process may use (its affinity, capped by OMP_NUM_THREADS when that is set)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS", n)))
    except ValueError:
        pass
    return max(1, n)


def cpu_baseline(wl, scene, params, sample_pix: int):
    """The oracle, as it stands, on a bounded sample of the same frame, extrapolated to a frame.

    One pass: inference + light pick on `sample_pix` pixels, training pixels + labels + gradients on
    2^15 samples (2048 for the clustered cache), Adam on 2^20 parameters; each part is scaled linearly to
    the frame (all the oracle's work is per pixel, per sample or per parameter).  Timed with the BLAS
    threads limited to all host cores and to one, best of 3 after a warm-up pass each."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import clustered, hashgrid, lighting, philox, pipeline, shadow, training

    n_pix = scene["pos"].shape[0]
    sel = np.arange(sample_pix)
    batch_s = min(1 << 15, wl.train_batch)
    if wl.n_clusters:
        off, mem = clustered.kmeans(scene["lights"], wl.n_clusters)
        batch_s = min(batch_s, 2048)
    n_adam = min(1 << 20, params["table"].size)

    def one_pass():
        t0 = time.perf_counter()
        vis = pipeline.infer(scene["pos_unit"][sel], params["table"], params["weights"], wl.grid.base_res,
                             wl.grid.growth, act=wl.mlp.act, slope=wl.mlp.leaky_slope)
        if wl.n_clusters:
            clustered.sample(vis, scene["pos"][sel], scene["nrm"][sel], scene["lights"], off, mem, wl.rng_key, 0,
                             wl.n_cand, wl.vis_floor, dtype=np.float64)
        else:
            pipeline.sample(vis, scene["pos"][sel], scene["nrm"][sel], scene["lights"], wl.rng_key, 0, wl.vis_floor)
        t1 = time.perf_counter()
        pix = philox.training_pixels(wl.rng_key, 0, batch_s, n_pix)
        if wl.n_clusters:
            y = clustered.labels(scene["pos"][pix], scene["lights"], scene["spheres"],
                                 clustered.training_lights(wl.rng_key, 0, batch_s, off, mem))
        else:
            y = shadow.labels_fp32(scene["pos"][pix], scene["lights"], scene["spheres"])
        g = training.train_gradients(scene["pos_unit"][pix], params["table"], params["weights"], wl.grid.base_res,
                                     wl.grid.growth, labels=y, loss=wl.loss, act=wl.mlp.act, slope=wl.mlp.leaky_slope)
        t2 = time.perf_counter()
        z = np.zeros(n_adam)
        training.adam_step(params["table"].reshape(-1)[:n_adam], g["g_table"].reshape(-1)[:n_adam], z, z, 1,
                           training.learning_rate(1, wl.lr, wl.lr_end, wl.lr_decay_steps), wl.beta1, wl.beta2,
                           wl.adam_eps)
        t3 = time.perf_counter()
        return ((t1 - t0) * n_pix / sample_pix + (t2 - t1) * wl.train_batch / batch_s
                + (t3 - t2) * (wl.grid.n_params + wl.mlp.n_params) / n_adam), t3 - t0

    cores = _host_cores()
    runs = {}
    wall = 0.0
    for threads in (cores, 1):
        with threadpool_limits(limits=threads):
            one_pass()                                           # warm-up
            best = float("inf")
            for _ in range(3):
                frame_s, took = one_pass()
                best = min(best, frame_s)
                wall += took
        runs[threads] = best
    frame_s = runs[cores]
    return {"value": n_pix / frame_s, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "sample": (f"{sample_pix} pixels inference+WRS, {batch_s} training samples (labels+gradients), "
                       f"Adam on {n_adam} params; FP64 NumPy, best of 3 after a warm-up with {cores} BLAS "
                       f"threads, extrapolated linearly to one {n_pix}-pixel frame with a "
                       f"{wl.train_batch}-sample step"),
            "ms_per_frame": frame_s * 1e3,
            "one_thread": {"value": n_pix / runs[1], "ms_per_frame": runs[1] * 1e3},
            "seconds": round(wall, 2)}


def measured_traffic(stage, wl):
    """HBM bytes per launch of the stage's kernel from the committed counter summary, if the kernel's
    sources are still those the counters were taken on (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{stage}_1080p_traffic.txt")
    if wl.name not in ("train_1080p", "frame_1080p") or wl.mlp.dtype != "f16" or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "#")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        h = hashlib.sha256()
        for src in kv["kernel_sources"].split(","):
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != kv["kernel_sources_sha256"]:
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def unshadowed(pos, nrm, lights):
    """f[n][m] of the Lambertian point-light weight, FP32 (reporting only)."""
    import torch
    d = lights[None, :, :3] - pos[:, None, :]
    d2 = torch.clamp((d * d).sum(-1), min=1e-6)
    nd = torch.clamp((nrm[:, None, :] * d).sum(-1), min=0.0)
    return lights[None, :, 3] * nd / (d2 * torch.sqrt(d2))


def estimator_stats(f, V, v, floor):
    """Exact per-pixel moments of the one-sample light estimator sum_i f_i V_i (FP32, reporting only).

    Sampling p_i proportional to f_i (no cache) or to f_i max(v_i, floor) (cache):
    Var = sum_i (f_i V_i)^2 / p_i - mu^2, and the probability of picking an occluded light.  For the
    cache also the share of (pixel, light) pairs that are visible but predicted below 0.01 ("confident
    misses") and the share of the estimator's second moment they carry."""
    import torch
    out = {}
    mu = (f * V).sum(1)
    for name, w in (("no_cache", f), ("cache", f * torch.clamp(v, min=floor))):
        W = w.sum(1, keepdim=True)
        ok = W[:, 0] > 0
        p = torch.where(W > 0, w / torch.where(W > 0, W, torch.ones_like(W)), torch.zeros_like(w))
        term = torch.where(p > 0, (f * V) ** 2 / torch.where(p > 0, p, torch.ones_like(p)), torch.zeros_like(p))
        var = term.sum(1) - mu ** 2
        out[name] = {"var": float(var[ok].mean()), "p_occluded": float((p * (V == 0)).sum(1)[ok].mean())}
        if name == "cache":
            miss = (V > 0) & (v < 0.01) & (f > 0)
            out[name]["miss"] = float(miss.float().mean())
            out[name]["miss_share"] = float((term * miss).sum() / term.sum().clamp(min=1e-30))
    return out


L2_BYTES = 8 * 4 * 1024 * 1024

PEAK_MFMA_TFLOPS = {"f16": 2500.0, "bf16": 2500.0, "f32": 157.3}


def run_mlp(args, wl, cache, pos_unit, dev):
    """The MLP of the frame alone, on its stored encoding: matrix-core FLOP/s against the dtype's peak."""
    import numpy as np
    import torch

    from paper_2506_05930_amd import api
    n = pos_unit.shape[0]
    enc = cache.encode(pos_unit, dtype=cache.vis_dtype)
    vis = torch.empty((n, wl.mlp.n_out), dtype=cache.vis_dtype, device=dev)
    for _ in range(args.warmup):
        api.nvc_mlp_forward(cache.mlp, cache.packed, enc, vis)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    for e in evs:
        e[0].record()
        api.nvc_mlp_forward(cache.mlp, cache.packed, enc, vis)
        e[1].record()
    torch.cuda.synchronize()
    ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    flops = n * wl.mlp.flops_per_point
    io = n * (wl.mlp.n_in + wl.mlp.n_out) * vis.element_size()
    tf = flops / (ms / 1e3) / 1e12
    return {"workload": wl.name, "kernel": "infer_kernel (encoding read from memory)", "dtype": wl.mlp.dtype,
            "points": n, "flops_per_point": wl.mlp.flops_per_point, "ms": ms, "tflops": tf,
            "peak_tflops": PEAK_MFMA_TFLOPS[wl.mlp.dtype], "mfma_frac": tf / PEAK_MFMA_TFLOPS[wl.mlp.dtype],
            "io_bytes": io, "io_gbs": io / (ms / 1e3) / 1e9, "steps": args.steps}


def run_loop(args, wl, cache, scene, tens, dev):
    """The frame loop: light 0 moves on a circle; each frame is one replay of a recorded HIP graph (the
    three-stream frame, with the next frame's light, training pixels, labels and routing plan prepared
    beside this frame's work)."""
    import numpy as np
    import torch

    from paper_2506_05930_amd import api
    from paper_2506_05930_amd.cache import LaggedPickGraph, PipelineGraph
    from workloads import LightAnimation, moving_light_table

    pos_unit, pos, nrm, lights, spheres = tens
    n_frames = args.loop
    table = torch.as_tensor(moving_light_table(scene["lights"], wl.frames or 60)).to(dev)
    lagged = args.loop_graph == "lagged"
    fg = (LaggedPickGraph if lagged else PipelineGraph)(cache, pos_unit, pos, nrm, lights, spheres, wl.train_batch,
                                                        make_anim=lambda li, ctr: LightAnimation(table, li, ctr))
    fg.capture()
    n_pix = pos_unit.shape[0]
    sub = torch.as_tensor(np.random.default_rng(3).choice(n_pix, size=min(args.loop_eval, n_pix), replace=False)
                          .astype(np.int32)).to(dev)
    sub_pos_unit = pos_unit.index_select(0, sub.long()).contiguous()
    vis_sub = torch.empty((sub.shape[0], wl.mlp.n_out), dtype=cache.vis_dtype, device=dev)
    lab_sub = torch.empty((sub.shape[0], wl.mlp.n_out), dtype=torch.uint8, device=dev)
    frames = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(args.warmup):       # untimed frames to settle clocks; they also train
        fg.replay()
    torch.cuda.synchronize()
    for f in range(n_frames):
        e0.record()
        fg.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        # evaluation on the fixed subset with this frame's lights (untimed)
        lf = fg.lights_of(fg.frame - 1) if lagged else lights
        cache.infer(sub_pos_unit, vis_sub)
        api.nvc_shadow_labels(pos, sub, lf, spheres, lab_sub)
        v = vis_sub.float()
        y = lab_sub.float()
        vc = torch.clamp(v, 1e-6, 1 - 1e-6)
        rec = {"frame": int(fg.ctr[0].item()) - 1, "ms": round(ms, 4), "loss": round(float(cache.loss_buf.item()), 6),
               "vis_mae": round(float((v - y).abs().mean()), 6),
               "vis_bce": round(float(-(y * torch.log(vc) + (1 - y) * torch.log(1 - vc)).mean()), 6)}
        fsub = unshadowed(pos.index_select(0, sub.long()), nrm.index_select(0, sub.long()), lf)
        st = estimator_stats(fsub, y, v, cache.vis_floor)
        rec["var_ratio_cache_vs_none"] = round(st["cache"]["var"] / st["no_cache"]["var"], 5)
        rec["p_occluded"] = {k: round(st[k]["p_occluded"], 5) for k in st}
        rec["confident_misses"] = round(st["cache"]["miss"], 5)
        rec["confident_miss_share_of_second_moment"] = round(st["cache"]["miss_share"], 4)
        frames.append(rec)
        print(json.dumps(rec), file=sys.stderr, flush=True)
    # the same replays back to back, nothing between them (untimed above: the evaluation of each frame)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(n_frames):
        fg.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_b2b = e0.elapsed_time(e1) / n_frames
    ms = [r["ms"] for r in frames]
    return {"workload": "loop_60f", "frames": n_frames, "warmup_frames": args.warmup, "graph": True,
            "ms_per_frame_back_to_back": ms_b2b,
            "schedule": ("inference + the previous frame's WRS, gradients + Adam, next frame's light, pixels, labels "
                         "and plan on four streams" if lagged else
                         "inference + WRS, gradients + Adam, next frame's light, pixels, labels and plan on three "
                         "streams"),
            "ms_per_frame_mean": float(np.mean(ms)), "ms_per_frame_median": float(np.median(ms)),
            "per_frame": frames}


def run_micro(reps: int = 20):
    """What the memory system gives on its own: a plain device copy (HBM stream rate) and random
    8-byte gathers from tables of 64 MiB (the 1080p hash table's size, held by the 256 MiB last-level
    cache) and 4 GiB (HBM), with torch's own copy and index_select kernels (not this library's)."""
    import torch
    dev = torch.device("cuda:0")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    out = {"micro": "memory", "reps": reps}
    n = 1 << 28                                                   # 1 GiB of float32 each way
    src, dst = torch.empty(n, device=dev), torch.empty(n, device=dev)
    src.fill_(1.0)
    t = timed(lambda: dst.copy_(src))
    out["copy_GBps"] = round(2 * n * 4 / t / 1e9, 1)              # read + write
    del src, dst
    n_g = 1 << 26                                                 # 64 Mi gathers of 8 bytes per launch
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    for name, table_mib in (("gather8_64MiB", 64), ("gather8_4GiB", 4096)):
        entries = table_mib * (1 << 20) // 8
        table = torch.zeros(entries, dtype=torch.int64, device=dev)
        idx = torch.randint(0, entries, (n_g,), device=dev, generator=gen)
        res = torch.empty(n_g, dtype=torch.int64, device=dev)
        t = timed(lambda: torch.index_select(table, 0, idx, out=res))
        out[name + "_Gps"] = round(n_g / t / 1e9, 2)               # gathers per second (x 1e9)
        del table, idx, res
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.micro:
        print(json.dumps(run_micro()))
        return
    import numpy as np
    import torch

    from paper_2506_05930_amd import api
    from paper_2506_05930_amd.cache import FramePipeline, NVCache
    from workloads import box_scene, get_workload, init_params
    from workloads.scenes import SCENE_EXTENT

    over = {"mlp_dtype": args.dtype} if args.dtype else {}
    if args.loop and args.workload == "train_1080p":
        args.workload = "loop_60f"
    wl = get_workload(args.workload, **over)
    dev = torch.device("cuda:0")
    scene = box_scene(wl.scene_seed, wl.width, wl.height, wl.n_boxes, wl.n_lights, wl.n_spheres, order=args.order)
    params = init_params(wl.init_seed, wl.grid, wl.mlp, init=wl.init)
    n_pix = wl.width * wl.height
    B = wl.train_batch
    cache = NVCache(wl.grid, wl.mlp, params["table"], params["weights"], device=dev, seed=wl.rng_key, lr=wl.lr,
                    beta1=wl.beta1, beta2=wl.beta2, eps=wl.adam_eps, loss=wl.loss, vis_floor=wl.vis_floor,
                    max_batch=B, lr_end=wl.lr_end, lr_decay_steps=wl.lr_decay_steps)
    pos_unit = torch.as_tensor(scene["pos_unit"]).to(dev)
    pos = torch.as_tensor(scene["pos"]).to(dev)
    nrm = torch.as_tensor(scene["nrm"]).to(dev)
    lights = torch.as_tensor(scene["lights"]).to(dev)
    spheres = torch.as_tensor(scene["spheres"]).to(dev)
    vis = torch.empty((n_pix, wl.mlp.n_out), dtype=cache.vis_dtype, device=dev)
    clustered = wl.n_clusters > 0
    if clustered:                      # Sec. 3.6: one output per k-means cluster of the lights
        cache.set_clusters(*api.nvc_cluster_lights(scene["lights"], wl.n_clusters), n_cand=wl.n_cand)
        out = {k: torch.empty(n_pix, dtype=d, device=dev) for k, d in
               (("idx", torch.int32), ("weight", torch.float32), ("cluster", torch.int32))}
    else:
        out = {k: torch.empty(n_pix, dtype=d, device=dev) for k, d in
               (("idx", torch.int32), ("pmf", torch.float32), ("wsum", torch.float32), ("di", torch.float32))}
    pix = torch.empty(B, dtype=torch.int32, device=dev)
    labels = torch.empty((B, wl.mlp.n_out), dtype=torch.uint8, device=dev)
    pix_ws = cache.pixel_workspace(n_pix)
    stream = torch.cuda.current_stream()
    if args.loop:
        print(json.dumps(run_loop(args, wl, cache, scene, (pos_unit, pos, nrm, lights, spheres), dev)))
        return
    if args.mlp:
        print(json.dumps(run_mlp(args, wl, cache, pos_unit, dev)))
        return


    def do_sample(frame, st=None):
        if clustered:
            api.nvc_sample_clustered(vis, pos, nrm, lights, cache.cl_offsets, cache.cl_members, cache.vis_floor,
                                     cache.n_cand, cache.seed, frame, out["idx"], out["weight"], out["cluster"], st)
        else:
            api.nvc_sample_wrs(vis, pos, nrm, lights, cache.vis_floor, cache.seed, frame, out["idx"], out["pmf"],
                               out["wsum"], out["di"], st)

    nw = wl.world_batch
    if nw:
        wpos = torch.empty((nw, 3), dtype=torch.float32, device=dev)
        wunit = torch.empty_like(wpos)
        wlab = torch.empty((nw, wl.mlp.n_out), dtype=torch.uint8, device=dev)

    def do_world(frame, st=None):
        """The world-space half of the training batch: points, labels and gradients."""
        if not nw:
            return
        api.nvc_world_samples(cache.seed, frame, wl.world_box, SCENE_EXTENT, wpos, wunit, st)
        if fused:
            cache.gradients_shadow(wunit, wpos, lights, spheres, batch=nw, stream=st)
            return
        if clustered:
            api.nvc_shadow_labels_clustered(wpos, None, lights, cache.cl_offsets, cache.cl_members, spheres,
                                            cache.seed, frame, wlab, st)
        else:
            api.nvc_shadow_labels(wpos, None, lights, spheres, wlab, st)
        cache.gradients(wunit, labels=wlab, batch=nw, stream=st)

    fused = args.fused_labels and not clustered
    cache.fused_labels = fused

    def do_labels(frame, st=None):
        if fused:
            return
        if clustered:
            api.nvc_shadow_labels_clustered(pos, pix, lights, cache.cl_offsets, cache.cl_members, spheres, cache.seed,
                                            frame, labels, st)
        else:
            api.nvc_shadow_labels(pos, pix, lights, spheres, labels, st)

    def do_gradients(st=None):
        if fused:
            cache.gradients_shadow(pos_unit, pos, lights, spheres, pix=pix, batch=B, stream=st)
        else:
            cache.gradients(pos_unit, labels=labels, pix=pix, batch=B, stream=st)

    if nw:
        cache.set_world_samples(nw, wl.world_box, SCENE_EXTENT)
    pipe = FramePipeline(cache, pos_unit, pos, nrm, lights, spheres, B, main=stream)

    def step(frame, ev=None, kev=None):
        """One frame.  Timed frames go through FramePipeline: inference + WRS on `stream`, the gradient
        pass and Adam on a second stream, the next frame's training pixels and labels on a third
        (`kev`: events around the inference and WRS launches).  With `ev` every stage runs in order
        on one stream between events (the per-stage breakdown)."""
        if ev is None:
            pipe.run(frame, events=kev)
            return
        pipe.finish()
        ev[0].record(stream)
        api.nvc_infer(cache.grid, cache.mlp, cache.table, cache.packed, pos_unit, vis)
        ev[1].record(stream)
        do_sample(frame)
        ev[2].record(stream)
        api.nvc_select_pixels(cache.seed, frame, n_pix, pix, pix_ws)
        ev[3].record(stream)
        do_labels(frame)
        ev[4].record(stream)
        do_gradients()
        do_world(frame)
        ev[5].record(stream)
        cache.adam()
        ev[6].record(stream)

    for f in range(args.warmup):
        step(f)
    torch.cuda.synchronize()

    # Timed region: exactly `steps` frames between two synchronisations.
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    kevs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t_start.record(stream)
    for f in range(args.steps):
        step(args.warmup + f, kev=kevs[f])
    pipe.finish()
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_per_step = t_start.elapsed_time(t_end) / args.steps
    # Launch durations of the inference and WRS kernels inside the timed frames (they share the
    # GPU with the training half).
    timed_ms = {"infer": float(np.mean([k[0].elapsed_time(k[1]) for k in kevs])),
                "wrs": float(np.mean([k[1].elapsed_time(k[2]) for k in kevs]))}

    # Per-stage durations from HIP events on the launch stream, over a second pass of `steps` frames
    # that runs every stage in order.
    stage_ms = None
    if not args.no_stages:
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(7)] for _ in range(args.steps)]
        for f in range(args.steps):
            step(args.warmup + args.steps + f, evs[f])
        torch.cuda.synchronize()
        stage_ms = {s: float(np.mean([evs[f][i].elapsed_time(evs[f][i + 1]) for f in range(args.steps)]))
                    for i, s in enumerate(STAGES)}
    loss = float(cache.loss_buf.item())

    # The same frames on the row-major G-buffer (the pixel order of a plain scanline render): every
    # per-pixel result is the same, only the locality of the table gathers changes.
    rows_ms = None
    if args.order == "morton" and not args.no_rowmajor:
        rows = box_scene(wl.scene_seed, wl.width, wl.height, wl.n_boxes, wl.n_lights, wl.n_spheres, order="rows")
        pos_unit.copy_(torch.as_tensor(rows["pos_unit"]))
        pos.copy_(torch.as_tensor(rows["pos"]))
        nrm.copy_(torch.as_tensor(rows["nrm"]))
        f0 = args.warmup + 2 * args.steps
        for f in range(args.warmup):
            step(f0 + f)
        torch.cuda.synchronize()
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        r0.record(stream)
        for f in range(args.steps):
            step(f0 + args.warmup + f)
        pipe.finish()
        r1.record(stream)
        torch.cuda.synchronize()
        rows_ms = r0.elapsed_time(r1) / args.steps

    if args.calibrate_copy_mib:
        a = torch.empty(args.calibrate_copy_mib << 18, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()

    alg = algorithmic(wl, n_pix, B)
    rates = {}
    if stage_ms is not None:
        for s, d in alg.items():
            t = stage_ms[s] / 1e3
            rates[s] = {k: v / t for k, v in d.items()}
    # Roofline of the dominant kernel, infer_kernel (the longest single launch of the frame), from its
    # average launch duration inside the timed frames.
    t_inf = timed_ms["infer"] / 1e3
    roof = {"bound": "hbm", "achieved": alg["infer"]["bytes"] / t_inf / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = "infer_kernel"
    roof["avg_launch_ms"] = timed_ms["infer"]
    hbm = measured_traffic("infer", wl)
    roof["traffic"] = None if hbm is None else hbm / t_inf / 1e9
    roof["traffic_bytes_per_launch"] = hbm
    if stage_ms is not None:
        # the same kernel alone on the GPU (serial stage pass): inside the timed frames it shares the
        # CUs with the training half on the other stream
        roof["alone_ms"] = stage_ms["infer"]
        roof["frac_alone"] = alg["infer"]["bytes"] / (stage_ms["infer"] / 1e3) / 1e9 / PEAK_HBM_GBS

    st = stage_ms if stage_ms is not None else timed_ms
    q_infer_wrs = n_pix / ((st["infer"] + st["wrs"]) / 1e3)
    result = {
        "metric": "visibility queries/s (point x all lights) + ms/frame infer+train+WRS, 1080p x 32",
        "value": n_pix / (ms_per_step / 1e3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": wl.mlp.dtype,
        "data": "synthetic",
        "config": {"workload": wl.name, "pixels": n_pix, "lights": wl.n_lights, "spheres": wl.n_spheres,
                   "train_batch": B, **({"world_batch": wl.world_batch} if wl.world_batch else {}),
                   "grid": f"L{wl.grid.n_levels} F{wl.grid.n_feat} T2^{wl.grid.log2_T}",
                   "mlp": f"{wl.mlp.n_in}-{wl.mlp.width}x{wl.mlp.n_hidden}-{wl.mlp.n_out}",
                   "pixel_order": args.order,
                   "labels": "inside the training kernel" if fused else "label kernel"},
        "ms_per_frame": ms_per_step,
        "ms_per_frame_rowmajor": None if rows_ms is None else round(rows_ms, 4),
        "streams": "FramePipeline: inference + WRS, gradient pass + Adam, next frame's pixels + labels on three "
                   "streams; stage_ms from a serial pass",
        "timed_launch_ms": {k: round(v, 4) for k, v in timed_ms.items()},
        "ms_per_frame_serial": None if stage_ms is None else round(sum(stage_ms.values()), 4),
        "stage_ms": None if stage_ms is None else {k: round(v, 4) for k, v in stage_ms.items()},
        "queries_per_s_infer_wrs": q_infer_wrs,
        "point_lights_per_s_infer_wrs": q_infer_wrs * wl.n_lights,
        "stage_rates": {s: {k: round(v / 1e9, 2) for k, v in r.items()} for s, r in rates.items()},
        "loss": loss,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(wl, scene, params, args.cpu_sample)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
