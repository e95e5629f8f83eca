"""Benchmark: multi-view rasterizer training step (forward + loss + backward) on one MI355X.

A step is one pass of the whole hot path over one batch of views: per-view participation and
projection, the depth and tile sorts, range extraction, the blend forward, the fused loss and its
image gradient, the blend backward and the preprocessing backward with densification statistics
when the workload asks for them. Inputs are seeded synthetic scenes resident in HBM before the
timed region starts.

Prints ONE JSON line. `value` is views/s of the batched path; `one_view_loop` reports the same
views rendered one view per call; `roofline` is for the kernel that takes the most time, from HIP
events recorded on the library's stream during the timed region; `cpu_baseline` times the CPU
oracle on a bounded sample of the same workload.
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

METRIC = "fwd+bwd views/s, 1M Gaussians, 8-view batch vs 1-view loop; serve p50/p99 ms"
HBM_PEAK_GBS = 8000.0
# non-packed FP32 vector lane operations: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
ALU_PEAK_TLANEOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic lane operations per blended (pixel, Gaussian) pair. Forward: 2 subtractions and 5
# multiply/fma for the power, 1 compare, 2 for exp2, 2 for alpha and its clamp, 1 fma for T, 1
# compare, 1 weight, 3 fma for colour. Backward: the forward's 10 for power and alpha, 2 to recover
# T, 3 colour gradients, 7 for dL/dalpha, 6 for the colour-behind update, 16 for the opacity, mean
# and conic gradients, and 9 additions folding the pixel into the per-Gaussian sums.
FWD_OPS_PER_STEP = 18
BWD_OPS_PER_STEP = 57
# algorithmic lane operations per pixel-channel of the fused L1 + D-SSIM loss (separable 11-tap
# window, fused multiply-adds counted once): the five moments along x (2 multiplies and 5 fma per
# tap: 77) and along y (55), SSIM and its three derivative maps (38), the maps along x and y (66),
# and the gradient with its L1 term (8). The halo the 32x32 output tiles recompute is not counted.
SSIM_OPS_PER_PIXEL_CHANNEL = 244
STAGES = ["count", "records", "depth_sort", "emit", "tile_sort", "ranges", "blend_fwd", "loss", "blend_bwd",
          "preprocess_bwd"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uneven_1m_8view")
    ap.add_argument("--tile", default="auto", help="WxH, or auto: pick tile and pixels per lane by timing")
    ap.add_argument("--ppl", type=int, default=0, help="pixels per lane in the blend kernels (0: library default)")
    ap.add_argument("--no-loop", action="store_true", help="skip the one-view-per-call comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-views", type=int, default=2, help="views of the workload in the CPU sample")
    ap.add_argument("--serve-requests", type=int, default=2000, help="measured serving requests (0: skip)")
    ap.add_argument("--serve-warmup", type=int, default=200, help="serving requests before the measured ones")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrival rate of serving requests (1/s)")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-batch", type=int, default=8)
    ap.add_argument("--serve-budget-gib", type=float, default=16.0)
    ap.add_argument("--no-graph", action="store_true", help="time eager calls only (no HIP-graph replay)")
    ap.add_argument("--no-partial", action="store_true", help="skip the partial-rendering comparison")
    ap.add_argument("--partial-views", type=int, default=8)
    ap.add_argument("--partial-size", default="1280x720")
    ap.add_argument("--no-variance", action="store_true", help="skip the mini-batch gradient variance measurement")
    ap.add_argument("--variance-batches", type=int, default=24)
    ap.add_argument("--no-train", action="store_true", help="skip the training-iteration comparison")
    ap.add_argument("--train-steps", type=int, default=20)
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads of the benchmark set")
    ap.add_argument("--train-only", action="store_true",
                    help="run only the training-iteration comparison and print its JSON (for profiling)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a reference dispatch for the HBM byte counters)")
    return ap.parse_args()


def measure(name, args, steps, warmup, tile_arg="auto", ppl_arg=0, with_loop=True, with_graph=True, keep=False):
    """Forward + loss + backward steps of one workload: the autotuned launch shape, eager steps with
    per-stage HIP-event times recorded on the library's stream, the frame's sizes and blend work,
    the same step replayed as one HIP graph, and the one-view-per-call loop on the same GPU."""
    import ctypes as C

    import torch

    from paper_2506_12727_amd import _lib as L
    from paper_2506_12727_amd import scenes
    from paper_2506_12727_amd.raster import GaussianTensors, Rasterizer

    wl = scenes.WORKLOADS[name]
    scene = wl.scene()
    cams = wl.cameras()
    B = len(cams)
    g = GaussianTensors.from_scene(scene)
    tg = [torch.from_numpy(t).cuda() for t in scenes.make_targets(cams)]
    tuned = None
    if tile_arg == "auto":
        from paper_2506_12727_amd.tune import autotune
        tile, ppl, times = autotune(g, cams, tg, wl.w_l1, wl.w_dssim, cache=False)
        tuned = {f"{t[0]}x{t[1]}/{p}": round(1e3 * v, 3) for (t, p), v in times.items()}
    else:
        tile, ppl = tuple(int(x) for x in tile_arg.split("x")), ppl_arg
    rast = Rasterizer(tile, ppl)
    lib = L.lib()
    imgs = [torch.empty((3, c.height, c.width), device="cuda") for c in cams]
    dl = [torch.empty_like(t) for t in imgs]
    loss = torch.empty(1, device="cuda")
    grads = dict(means=torch.empty_like(g.means), scales=torch.empty_like(g.scales), quats=torch.empty_like(g.quats),
                 opacities=torch.empty_like(g.opacities), sh=torch.empty_like(g.sh))
    dz = None
    if wl.densify:
        dz = dict(e1=torch.zeros(g.P, device="cuda"), e2=torch.zeros(g.P, device="cuda"),
                  count=torch.zeros(g.P, dtype=torch.int32, device="cuda"))

    def step(idx):
        views = [cams[i] for i in idx]
        images = [imgs[i] for i in idx]
        dls = [dl[i] for i in idx]
        _, fr = rast.forward(g, views, images=images)
        rast.loss(views, images, [tg[i] for i in idx], wl.w_l1, wl.w_dssim, out=loss, grads=dls)
        rast.backward(g, fr, dls, densify=dz, grads=grads)
        return fr

    def batched():
        rast.release(step(list(range(B))))

    def loop():
        for v in range(B):
            rast.release(step([v]))

    for _ in range(warmup):
        batched()
    torch.cuda.synchronize()
    lib.mvgs_profile_reset(rast.ctx)
    lib.mvgs_profile_enable(rast.ctx, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batched()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.mvgs_profile_enable(rast.ctx, 0)
    ms = (C.c_double * L.MVGS_STAGE_COUNT)()
    calls = (C.c_int64 * L.MVGS_STAGE_COUNT)()
    L.check(lib.mvgs_profile_read(rast.ctx, ms, calls), rast.ctx)
    stage_ms = {STAGES[i]: ms[i] / max(calls[i], 1) for i in range(L.MVGS_STAGE_COUNT)}
    elapsed = t1 - t0
    ms_step = 1e3 * elapsed / steps
    views_s = B * steps / elapsed

    # frame sizes, sort passes and walk work of one batched forward (outside the timed region)
    _, fr = rast.forward(g, cams, images=imgs)
    info = fr.info()
    work = torch.zeros(2, dtype=torch.int64, device="cuda")
    L.check(lib.mvgs_frame_work(rast.ctx, C.c_void_p(torch.cuda.current_stream().cuda_stream), fr.handle,
                                work.data_ptr()), rast.ctx)
    torch.cuda.synchronize()
    steps_walk, blended = (int(x) for x in work.cpu().tolist())
    rast.release(fr)

    # the same step captured into a HIP graph (capacity mode: no host synchronization in the step)
    graph_res = None
    if with_graph:
        from paper_2506_12727_amd.graph import CapturedStep
        capacity = (int(info["records"] * 1.02) + 1024, int(info["pairs"] * 1.02) + 4096)
        gstep = CapturedStep(g, cams, tg, wl.w_l1, wl.w_dssim, tile=tile, ppl=ppl, capacity=capacity, densify=dz)
        # the first replays of a new graph leave the GPU idle between some of its kernels (seen in
        # kernel traces for about six replays): warm up past them
        for _ in range(max(warmup, 10)):
            gstep.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            gstep.replay()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gstep.check()
        graph_res = {"ms_per_step": 1e3 * (t1 - t0) / steps, "views_per_s": B * steps / (t1 - t0),
                     "capacity": {"records": capacity[0], "pairs": capacity[1]}}
        gstep.close()

    loop_res = None
    if with_loop:
        for _ in range(max(1, warmup)):
            loop()
        torch.cuda.synchronize()
        lsteps = max(3, steps // 2)
        t0 = time.perf_counter()
        for _ in range(lsteps):
            loop()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lv = B * lsteps / (t1 - t0)
        loop_res = {"value": lv, "unit": "views/s", "ms_per_step": 1e3 * (t1 - t0) / lsteps}
    rast.close()

    traffic = {k: measured_traffic(k, wl.name, tile, ppl) for k in STAGES}
    roofs = {k: roofline(k, stage_ms[k], info, blended, g, cams, wl, traffic[k]) for k in STAGES}
    dom = max(STAGES, key=lambda k: stage_ms[k])
    value, ms_value, src = views_s, ms_step, "eager calls"
    if graph_res is not None:
        value, ms_value, src = graph_res["views_per_s"], graph_res["ms_per_step"], "hip graph replay"
    if loop_res is not None:
        loop_res["batched_speedup"] = value / loop_res["value"]
    total_px = sum(c.width * c.height for c in cams)
    res = {
        "workload": wl.name, "gaussians": g.P, "sh_degree": wl.sh_degree, "views": B,
        "sizes": [[c.width, c.height] for c in cams], "tile": list(tile), "pixels_per_lane": ppl,
        "autotune_ms_per_step": tuned, "loss": {"w_l1": wl.w_l1, "w_dssim": wl.w_dssim}, "densify": wl.densify,
        "views_per_s": value, "ms_per_step": ms_value, "value_source": src,
        "gaussian_pixels_per_s": g.P * total_px / (ms_value / 1e3),
        "eager": {"ms_per_step": ms_step, "views_per_s": views_s},
        "graph": graph_res,
        "one_view_loop": loop_res,
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "frame": {"records": info["records"], "pairs": info["pairs"], "tiles": info["tiles"],
                  "depth_sort_passes": info["depth_passes"], "tile_sort_passes": info["tile_passes"],
                  "walk_steps": steps_walk, "blended_pairs": blended},
        "stage_rooflines": roofs,
        "roofline": roofs[dom],
    }
    if keep:
        res["_state"] = (wl, scene, cams, tg, g, tile, ppl)
    return res


def copy_peak_gbs(mib=2048, reps=5):
    """HBM bandwidth of a plain device-to-device copy (read + write), best of `reps`, timed with HIP
    events: the measured ceiling next to the 8 TB/s specification."""
    import torch
    src = torch.empty(mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    best = None
    for _ in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        t = a.elapsed_time(b) / 1e3
        best = t if best is None else min(best, t)
    del src, dst
    return 2.0 * (mib << 20) / best / 1e9


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the path runs on a single "
              "MI355X; across GPUs each would render its own views of a replicated scene and the "
              "per-Gaussian gradients and statistics would be all-reduced).", file=sys.stderr)
        sys.exit(2)
    import torch

    torch.cuda.set_device(0)
    if args.train_only:
        print(json.dumps({"training": train_bench(args, (32, 32), 4)}), flush=True)
        return
    if args.copy_mib:
        src = torch.empty(args.copy_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    main_res = measure(args.workload, args, args.steps, args.warmup, args.tile, args.ppl, with_loop=not args.no_loop,
                       with_graph=not args.no_graph, keep=True)
    wl, scene, cams, tg, g, tile, ppl = main_res.pop("_state")
    B = len(cams)

    # the other workloads of the benchmark set, same measurement with fewer steps
    others = {}
    if not args.no_configs:
        for name in ("small_16k_4x128", "train_300k_4x1600x1064_dssim", "large_3m_16x1280x840"):
            if name == args.workload:
                continue
            r = measure(name, args, max(5, args.steps // 2), 2, "auto", 0, with_loop=True, with_graph=True)
            others[name] = {k: r[k] for k in ("views", "gaussians", "tile", "pixels_per_lane", "views_per_s",
                                              "ms_per_step", "value_source", "gaussian_pixels_per_s", "eager",
                                              "graph", "one_view_loop", "stages_ms", "frame", "roofline",
                                              "stage_rooflines", "loss", "densify")}
            torch.cuda.empty_cache()

    partial = None
    if not args.no_partial:
        partial = partial_bench(args, g, wl, tile, ppl)

    variance = None if args.no_variance else variance_bench(args, tile, ppl)
    training = None if args.no_train else train_bench(args, tile, ppl)

    serve = None
    if args.serve_requests > 0:
        torch.cuda.synchronize()
        serve = serve_bench(args, g if (wl.P, wl.sh_degree) == (1_000_000, 3) and wl.log_scale_mean == -4.0 else None,
                            tile, ppl)
    copy_gbs = copy_peak_gbs()

    cpu = None if args.no_cpu else cpu_baseline(scene, cams, tg, wl, (16, 16), args.cpu_views)
    roof = dict(main_res["roofline"])
    out = {
        "metric": METRIC,
        "value": main_res["views_per_s"],
        "unit": "views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "gaussians": g.P, "sh_degree": wl.sh_degree, "views": B,
                   "sizes": main_res["sizes"], "tile": list(tile), "pixels_per_lane": ppl,
                   "autotune_ms_per_step": main_res["autotune_ms_per_step"],
                   "loss": {"w_l1": wl.w_l1, "w_dssim": wl.w_dssim}, "densify": wl.densify},
        "gaussian_pixels_per_s": main_res["gaussian_pixels_per_s"],
        "value_source": main_res["value_source"],
        "eager": main_res["eager"],
        "graph": main_res["graph"],
        "one_view_loop": main_res["one_view_loop"],
        "stages_ms": main_res["stages_ms"],
        "frame": main_res["frame"],
        "stage_rooflines": main_res["stage_rooflines"],
        "roofline": roof,
        "hbm_peak": {"spec_GBps": HBM_PEAK_GBS, "copy_kernel_GBps": copy_gbs,
                     "copy_over_spec": copy_gbs / HBM_PEAK_GBS},
        "configs": others,
        "partial": partial,
        "grad_variance": variance,
        "training": training,
        "serve": serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def partial_bench(args, g, wl, tile, ppl):
    """Thread-efficient partial rendering (Alg. 3) against its baselines on B views of one size
    (the scene of the main workload): every step renders the batch, takes an L1 loss and runs the
    backward. full = every pixel of every view; masked = the binary-mask baseline; compact = the
    thread-efficient scheme; single = one view, every pixel. In the partial modes each tile's pixels
    are shared out among the views (fresh random keys every step), so the batch renders one image
    plane's worth of pixels, written as one merged image. full and single use the main workload's
    launch shape; each partial mode is timed with every candidate tile and reports its fastest."""
    import ctypes as C

    import torch

    from paper_2506_12727_amd import _lib as L
    from paper_2506_12727_amd import scenes
    from paper_2506_12727_amd.raster import Rasterizer

    W, H = (int(x) for x in args.partial_size.split("x"))
    B = args.partial_views
    cams = scenes.make_cameras([(W, H)] * B, radius=wl.radius)
    tg = [torch.from_numpy(t).cuda() for t in scenes.make_targets(cams)]
    keys_tg = torch.from_numpy(scenes.make_targets(cams[:1], seed=scenes.SEED_TARGETS + 1)[0]).cuda()
    lib = L.lib()
    imgs = [torch.empty((3, H, W), device="cuda") for _ in range(B)]
    dl = [torch.empty_like(t) for t in imgs]
    merged, merged_dl = torch.empty((3, H, W), device="cuda"), torch.empty((3, H, W), device="cuda")
    loss = torch.empty(1, device="cuda")
    grads = dict(means=torch.empty_like(g.means), scales=torch.empty_like(g.scales), quats=torch.empty_like(g.quats),
                 opacities=torch.empty_like(g.opacities), sh=torch.empty_like(g.sh))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(scenes.SEED_REQUESTS)

    def full_step(rast, n):
        v = cams[:n]
        _, fr = rast.forward(g, v, images=imgs[:n])
        rast.loss(v, imgs[:n], tg[:n], 1.0, 0.0, out=loss, grads=dl[:n])
        rast.backward(g, fr, dl[:n], grads=grads)
        rast.release(fr)

    def partial_step(rast, mode):
        keys = torch.randint(-2 ** 31, 2 ** 31 - 1, (W * H,), dtype=torch.int32, device="cuda", generator=gen)
        off, pix = rast.subsample(cams, keys)
        _, fr = rast.forward_partial(g, cams, off, pix, mode, images=[merged] * B)
        rast.loss(cams[:1], [merged], [keys_tg], 1.0, 0.0, out=loss, grads=[merged_dl])
        rast.backward(g, fr, [merged_dl] * B, grads=grads)
        rast.release(fr)

    steps = max(5, args.steps // 2)
    ms = (C.c_double * L.MVGS_STAGE_COUNT)()
    calls = (C.c_int64 * L.MVGS_STAGE_COUNT)()

    def timed(rast, fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        lib.mvgs_profile_reset(rast.ctx)
        lib.mvgs_profile_enable(rast.ctx, 1)
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        lib.mvgs_profile_enable(rast.ctx, 0)
        L.check(lib.mvgs_profile_read(rast.ctx, ms, calls), rast.ctx)
        return {"ms_per_step": 1e3 * dt, "blend_fwd_ms": ms[6] / max(calls[6], 1),
                "blend_bwd_ms": ms[8] / max(calls[8], 1)}

    out = {"views": B, "size": [W, H]}
    rast = Rasterizer(tile, ppl)
    out["full"] = dict(timed(rast, lambda: full_step(rast, B)), tile=list(tile), pixels_per_lane=ppl)
    out["single"] = dict(timed(rast, lambda: full_step(rast, 1)), tile=list(tile), pixels_per_lane=ppl)
    rast.close()
    for name, mode in (("masked", L.MVGS_PARTIAL_MASKED), ("compact", L.MVGS_PARTIAL_COMPACT)):
        best = None
        for t in ((16, 16), (32, 16), (32, 32)):
            r = Rasterizer(t)
            res = dict(timed(r, lambda: partial_step(r, mode)), tile=list(t))
            r.close()
            if best is None or res["ms_per_step"] < best["ms_per_step"]:
                best = res
        out[name] = best
    out["compact_vs_full_speedup"] = out["full"]["ms_per_step"] / out["compact"]["ms_per_step"]
    out["compact_vs_masked_speedup"] = out["masked"]["ms_per_step"] / out["compact"]["ms_per_step"]
    out["compact_vs_single_view_overhead"] = out["compact"]["ms_per_step"] / out["single"]["ms_per_step"]
    return out


def variance_bench(args, tile, ppl):
    """Variance of mini-batch gradients (Sec. 3.2) on the 300k-Gaussian SH-3 scene with 16 views
    of 1600x1064: one whole view per batch, four whole views, and four views sharing one image
    plane by partial rendering (Alg. 3, as many pixels as one view). L1 loss, seeded batches."""
    import numpy as np
    import torch

    from paper_2506_12727_amd import scenes
    from paper_2506_12727_amd.raster import GaussianTensors, Rasterizer
    from paper_2506_12727_amd.train import variance_partial, variance_views

    wl = scenes.WORKLOADS["train_300k_4x1600x1064_dssim"]
    N, B, K = 16, 4, args.variance_batches
    g = GaussianTensors.from_scene(wl.scene())
    cams = scenes.make_cameras([(1600, 1064)] * N, seed=41)
    tg = [torch.from_numpy(t).cuda() for t in scenes.make_targets(cams, seed=42)]
    rng = np.random.default_rng(43)
    singles = [[int(rng.integers(N))] for _ in range(K)]
    multis = [[int(v) for v in rng.choice(N, size=B, replace=False)] for _ in range(K)]
    keys = [torch.from_numpy(rng.integers(0, 2 ** 32, size=1600 * 1064, dtype=np.uint64).astype(np.uint32)
                             .view(np.int32)).cuda() for _ in range(K)]
    r = Rasterizer(tile, ppl)
    out = {"scene": "300k Gaussians, SH 3", "views": N, "size": [1600, 1064], "batch_views": B, "batches": K,
           "loss": "L1"}
    variance_views(r, g, cams, tg, singles[:2])          # warm-up
    for name, fn in (("single_view", lambda: variance_views(r, g, cams, tg, singles)),
                     ("multi_view", lambda: variance_views(r, g, cams, tg, multis)),
                     ("partial", lambda: variance_partial(r, g, cams, tg, multis, keys))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        res["ms_per_batch"] = 1e3 * (time.perf_counter() - t0) / K
        out[name] = res
    r.close()
    v1 = out["single_view"]["variance"]
    out["ratio_multi_to_single"] = out["multi_view"]["variance"] / v1
    out["ratio_partial_to_single"] = out["partial"]["variance"] / v1
    out["sampling_law_ratio"] = (N - B) / (B * (N - 1))
    return out


def train_bench(args, tile, ppl):
    """Training iterations (forward, fused loss, backward with the densification statistics, one
    Adam step) on the 300K-Gaussian SH-3 scene with a pool of 16 views of 1600x1064, as in the
    paper's training-time comparison: one view per iteration, four whole views, and four views
    sharing one image plane by thread-efficient partial rendering, each also as one HIP-graph
    replay per iteration (Adam included). 0.8 L1 + 0.2 D-SSIM (the 3D distance-aware D-SSIM for
    the partial batches); targets are renders of a second draw."""
    import torch

    from paper_2506_12727_amd import scenes
    from paper_2506_12727_amd.raster import GaussianTensors
    from paper_2506_12727_amd.train import Trainer

    wl = scenes.WORKLOADS["train_300k_4x1600x1064_dssim"]
    cams = scenes.make_cameras([(1600, 1064)] * 16, seed=41)
    gt = GaussianTensors.from_scene(scenes.make_scene(wl.P, wl.sh_degree, seed=7))
    out = {"scene": "300K Gaussians, SH 3", "views": 16, "size": [1600, 1064], "steps": args.train_steps,
           "loss": {"w_l1": 0.8, "w_dssim": 0.2}}
    modes = (("single_view", 1, False, False), ("multi_view", 4, False, False), ("partial", 4, True, False),
             ("single_view_captured", 1, False, True), ("multi_view_captured", 4, False, True),
             ("partial_captured", 4, True, True))
    for name, B, partial, captured in modes:
        g = GaussianTensors.from_scene(wl.scene())
        t = Trainer(g, gt, cams, views_per_step=B, partial=partial, densify_every=0, tile=tile, ppl=ppl, seed=44,
                    captured=captured)
        # (eight warm-up iterations for every mode: a new graph's first replays run with idle gaps)
        for _ in range(8):
            t.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.train_steps):
            loss = t.step()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.train_steps
        out[name] = {"views_per_step": B, "ms_per_step": ms, "views_per_s": 1e3 * B / ms,
                     "last_loss": float(loss.item()), "graph": captured}
        t.close()
        del t, g
    out["partial_over_single_time"] = out["partial"]["ms_per_step"] / out["single_view"]["ms_per_step"]
    out["multi_over_single_time"] = out["multi_view"]["ms_per_step"] / out["single_view"]["ms_per_step"]
    # a small scene, where launches rather than kernels bound an eager iteration: the small
    # workload's 16,384 Gaussians (SH 0) against a second draw, a pool of 16 views of 128x128
    sm = scenes.WORKLOADS["small_16k_4x128"]
    cams_s = scenes.make_cameras([(128, 128)] * 16, seed=43)
    gt_s = GaussianTensors.from_scene(scenes.make_scene(sm.P, sm.sh_degree, seed=8))
    small = {"scene": "16K Gaussians, SH 0", "views": 16, "size": [128, 128], "views_per_step": 4}
    for name, captured in (("eager", False), ("captured", True)):
        g = GaussianTensors.from_scene(sm.scene())
        t = Trainer(g, gt_s, cams_s, views_per_step=4, densify_every=0, tile=(16, 16), seed=45, captured=captured)
        for _ in range(8):
            t.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.train_steps):
            t.step()
        torch.cuda.synchronize()
        small[name] = 1e3 * (time.perf_counter() - t0) / args.train_steps
        t.close()
        del t, g
    small["captured_speedup"] = small["eager"] / small["captured"]
    out["small_scene_ms_per_step"] = small
    return out


def serve_bench(args, g, tile, ppl):
    """Serving loop over a resident 1M-Gaussian SH-3 scene: Poisson arrivals, resolutions uniform
    over the serving set, poses on a radius-3 sphere; then the same loop with every request
    arriving at once, which measures throughput at saturation."""
    import math

    from paper_2506_12727_amd import scenes
    from paper_2506_12727_amd.raster import GaussianTensors
    from paper_2506_12727_amd.serve import Server

    if g is None:
        g = GaussianTensors.from_scene(scenes.make_scene(1_000_000, 3))
    n = args.serve_warmup + args.serve_requests
    arr, cams = scenes.make_requests(n, rate_hz=args.serve_rate)
    budget = int(args.serve_budget_gib * (1 << 30))
    # pixels per lane chosen per batch by the library: requests range from one 256x256 view to
    # batches of 1920x1080 views
    srv = Server(g, n_slots=args.serve_slots, budget_bytes=budget, max_batch=args.serve_batch, tile=tile,
                 pixels_per_lane=0)
    try:
        st = srv.run(arr, cams, measure_from=args.serve_warmup)
        n_sat = min(n, 600)
        arr2, cams2 = scenes.make_requests(n_sat, rate_hz=math.inf, seed=scenes.SEED_REQUESTS + 100)
        sat = srv.run(arr2, cams2)
    finally:
        srv.close()
    out = {"p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
           "views_per_s": st["views_per_s"], "offered_per_s": args.serve_rate, "requests": st["requests"],
           "warmup_requests": args.serve_warmup, "rejected": st["rejected"],
           "mean_batch": st["mean_batch"], "slot_overlap": st["overlap"],
           "peak_budget_gib": st["peak_budget_bytes"] / (1 << 30), "budget_gib": args.serve_budget_gib,
           "refused_batches": st["refused_batches"], "slots": args.serve_slots, "max_batch": args.serve_batch,
           "tile": list(tile), "pixels_per_lane": "per batch",
           "saturated": {"requests": sat["requests"], "views_per_s": sat["views_per_s"],
                         "pixels_per_s": sat["pixels_per_s"], "mean_batch": sat["mean_batch"],
                         "slot_overlap": sat["overlap"]},
           "resolutions": [list(r) for r in scenes.SERVE_RESOLUTIONS], "gaussians": g.P}
    return out


def measured_traffic(stage, workload, tile, ppl):
    """HBM bytes per launch of a blend kernel from the rocprofv3 counter runs recorded in
    profiles/blend_traffic.json, or None when that record is for another launch shape or workload,
    or its kernels' sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "blend_traffic.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for p in rec["sources"]:
            h.update(open(os.path.join(ROOT, p), "rb").read())
    except (OSError, ValueError, KeyError):
        return None
    if (h.hexdigest() != rec["sources_sha256"] or rec["workload"] != workload or list(rec["tile"]) != list(tile)
            or rec["pixels_per_lane"] != ppl):
        return None
    return rec["bytes_per_launch"].get(stage)


def stage_bytes(stage, info, g, cams, wl):
    """Algorithmic HBM bytes of one launch of an HBM-bound stage: what it must read and write once.
    K pairs, V records, P Gaussians with Kc = (degree + 1)^2 SH coefficients, N pixels."""
    K, V, T = info["pairs"], info["records"], info["tiles"]
    kb = 2.0 if T <= 65536 else 4.0   # bytes per pair key: 16-bit tile ids up to 65,536 tiles
    P, Kc = g.P, (g.sh_degree + 1) ** 2
    N = sum(c.width * c.height for c in cams)
    par = 44 + 12 * Kc            # mean, scale, quaternion, opacity, SH (float32)
    return {
        # geometry parameters in; records and covered tiles per Gaussian out
        "count": 44.0 * P + 8.0 * P,
        # parameters and record offsets in; 64 B record, 2 B view, 4 B depth key, 8 B tile rectangle out
        "records": (par + 4.0) * P + 78.0 * V,
        # one read and one write of the 4 B key, 4 B value and 8 B tile rectangle per record and pass
        "depth_sort": 32.0 * V * info["depth_passes"],
        # each record's tile rectangle and id in depth order read once; key and 4 B value per pair written
        "emit": 12.0 * V + (kb + 4.0) * K,
        # the passes after the one fused with emission: key and value read and written
        "tile_sort": 2.0 * (kb + 4.0) * K * max(info["tile_passes"] - 1, 0),
        # the key at each tile boundary read, 8 B per tile written
        "ranges": (kb + 8.0) * T,
        # image and target read, gradient written per pixel-channel (L1 only: with D-SSIM the
        # fused kernel is bound by its arithmetic, see roofline)
        "loss": 3.0 * N * 12.0,
        # parameters in and gradients out, record offsets, statistics read and written; per record
        # its 48 B of sums and its 2 B view
        "preprocess_bwd": 2.0 * par * P + 4.0 * P + (24.0 * P if wl.densify else 0.0) + 50.0 * V,
    }[stage]


def roofline(stage, ms, info, blended, g, cams, wl, traffic=None):
    """Achieved vs peak for one stage: lane operations per blended pair for the blend kernels
    (VALU-bound), algorithmic bytes per launch for the others; traffic is the measured HBM bytes
    per launch when known."""
    sec = ms / 1e3
    if stage in ("blend_fwd", "blend_bwd"):
        per = FWD_OPS_PER_STEP if stage == "blend_fwd" else BWD_OPS_PER_STEP
        ach = blended * per / sec / 1e12 if sec > 0 else 0.0
        return {"kernel": stage, "bound": "alu", "achieved": ach, "peak": ALU_PEAK_TLANEOPS, "unit": "Tlane-op/s",
                "frac": ach / ALU_PEAK_TLANEOPS, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE, WRITE_SIZE, calibrated)",
                "traffic_TBps": None if traffic is None or sec <= 0 else traffic / sec / 1e12,
                "units": {"blended_pairs": blended, "ops_per_pair": per}}
    if stage == "loss" and wl.w_dssim:
        n_pc = 3.0 * sum(c.width * c.height for c in cams)
        ach = n_pc * SSIM_OPS_PER_PIXEL_CHANNEL / sec / 1e12 if sec > 0 else 0.0
        return {"kernel": stage, "bound": "alu", "achieved": ach, "peak": ALU_PEAK_TLANEOPS, "unit": "Tlane-op/s",
                "frac": ach / ALU_PEAK_TLANEOPS, "traffic": traffic, "ms": ms,
                "units": {"pixel_channels": n_pc, "ops_per_pixel_channel": SSIM_OPS_PER_PIXEL_CHANNEL,
                          "hbm_bytes": stage_bytes(stage, info, g, cams, wl)}}
    byts = stage_bytes(stage, info, g, cams, wl)
    ach = byts / sec / 1e9 if sec > 0 else 0.0
    return {"kernel": stage, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "ms": ms, "units": {"bytes": byts}}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(scene, cams, tg, wl, tile, nviews):
    """The oracle (FP64, OpenMP over the host's threads) on a bounded sample: the first `nviews`
    views of the workload with the full scene, forward + loss + backward, in views/s; and the
    oracle on one thread over the smallest view of the workload."""
    import oracle
    sub = cams[:nviews]
    tgs = [t.cpu().numpy() for t in tg[:nviews]]

    def run(views, targets):
        t0 = time.perf_counter()
        f = oracle.forward(scene, views, tile)
        _, gl = oracle.loss(views, f["images"], targets, wl.w_l1, wl.w_dssim)
        oracle.backward(scene, views, gl, tile)
        return time.perf_counter() - t0

    threads = oracle.max_threads()
    dt = run(sub, tgs)
    small = min(range(len(cams)), key=lambda v: cams[v].width * cams[v].height)
    oracle.set_threads(1)
    try:
        dt1 = run([cams[small]], [tg[small].cpu().numpy()])
    finally:
        oracle.set_threads(threads)
    c1 = cams[small]
    return {"value": nviews / dt, "unit": "views/s", "cores": threads, "kind": "oracle",
            "sample": f"{nviews} view(s) {sub[0].width}x{sub[0].height} of {wl.name}, all {scene.P} Gaussians, "
                      f"forward+loss+backward, {dt:.1f} s on {threads} threads",
            "one_thread": {"value": 1.0 / dt1, "unit": "views/s", "cores": 1,
                           "sample": f"view {small} ({c1.width}x{c1.height}) of {wl.name}, all {scene.P} Gaussians, "
                                     f"forward+loss+backward, {dt1:.1f} s"},
            "host": {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": _cpu_model()}}


if __name__ == "__main__":
    main()
