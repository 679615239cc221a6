#!/usr/bin/env python3
"""Throughput of the batched CMA-ES silhouette-fitness path on one MI355X.

Workload (single-instrument tracking, 640x480): 20144-triangle procedural
closed instrument, lambda = 256 candidates of 9 parameters, loss = 1 - IoU + 0.1 x
keypoint reprojection term, 30 CMA-ES generations per frame over a seeded
100-frame trajectory with 1% pixel-flip noise in the targets and 2-degree
noise on the joint readings.  A step is one generation: sample -> FK ->
transform/project/snap -> raster -> counts -> loss -> update, all in HIP
kernels.  The frame loop re-initialises CMA-ES from the previous frame's
estimate after the constant-velocity Kalman filter (device kernels
tk_cmaes_estimate + tk_kf_step at the end of each frame); the pose errors of
the raw and filtered per-frame estimates are reported under "tracking".

Prints ONE JSON line (rank 0).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


# Counter figures of the dominant kernel from the committed rocprofv3 runs
# (profiles/raster_kernel_track640.md), with the sha256 of the kernel sources
# they were taken on; they are reported only while the sources are unchanged.
#   bytes_per_launch: HBM bytes, FETCH_SIZE and WRITE_SIZE (two passes) scaled
#     by what the same counters read for a copy of known size;
#   valu_busy: SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES x 4 waves per SIMD;
#   lds_equiv_bytes: SQ_LDS_IDX_ACTIVE per launch times the bytes the LDS
#     microbenchmark (tk_bench_lds) moves per unit of the same counter, i.e.
#     the LDS occupancy expressed as bytes at the microbenchmark's rate;
#   lds_insts, lds_bank_conflict_frac: SQ_INSTS_LDS per launch and
#     SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE.
RASTER_TRAFFIC = {"bytes_per_launch": 44476221.2, "read_bytes": 23725270.8, "write_bytes": 20750950.4,
                  "valu_busy": 0.892,
                  "lds_equiv_bytes": 600897308.7, "lds_insts": 745702.4, "lds_bank_conflict_frac": 0.236,
                  "sources": ("paper_2603_11404_amd/csrc/raster.hip",
                              "paper_2603_11404_amd/csrc/tk_internal.h",
                              "paper_2603_11404_amd/csrc/fitness_device.h",
                              "paper_2603_11404_amd/csrc/sample_device.h"),
                  "sha256": "1ce4e11ede9e5a72d1fe1ea513cc2e8b9132e4a9c4c765ebea931becb9b42699"}


def raster_profile_valid():
    import hashlib
    h = hashlib.sha256()
    for p in RASTER_TRAFFIC["sources"]:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest() == RASTER_TRAFFIC["sha256"]


def raster_traffic():
    return RASTER_TRAFFIC["bytes_per_launch"] if raster_profile_valid() else None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000, help="timed generations (default: 100 frames x 30)")
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="wall time budget of the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the graph and plain-launch comparison loops")
    ap.add_argument("--legs", default=None,
                    help="comma-separated extra legs to run (small320, bimanual960, batch64, soft640, synth700); "
                         "default: all of them unless --no-extras")
    ap.add_argument("--plain-gens", type=int, default=2)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain copy kernel over 256 MiB (reference for HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": f"bench.py measures the single-GPU path only; --gpus {args.gpus} "
                                   f"(WORLD_SIZE {world}) is not supported. Across GPUs a generation would "
                                   "shard by candidates, every GPU drawing its own slice from the counter-based "
                                   "generator, with one all-gather of the per-candidate counts before the "
                                   "identical update on every GPU."}))
        sys.exit(2)

    import torch

    import scenes
    from paper_2603_11404_amd import tk, tracker

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = scenes.workload("track640")
    mesh, cam, lam, G, F = wl["mesh"], wl["cam"], wl["lam"], wl["gens"], wl["frames"]
    chain = scenes.chain()
    scale = scenes.DEFAULT_SCALE.copy()
    log(f"workload: {mesh.n_triangles} tris, {cam.width}x{cam.height}, lambda={lam}, {G} gens x {F} frames")
    if args.copy_calibration:
        # elementwise negation: reads and writes exactly 256 MiB each, the
        # reference against which the hardware byte counters are scaled
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log("copy calibration: 3 x (read 268435456 B, write 268435456 B)")
        del src, dst

    # ---------------------------------------------------------------- inputs resident in HBM
    prob = tracker.Problem([mesh], [chain], cam, dev)
    traj = scenes.trajectory(scenes.rng_for(wl["index"], scenes.SUB_TRAJ), cam, F)
    theta_true = torch.as_tensor(traj.astype(np.float32), device=dev)
    clean = prob.render(theta_true)                                   # [F, 60, 80] int64 words
    kp_true = prob.keypoints(theta_true)                              # [F, 1, 4, 2]
    rng_f = scenes.rng_for(wl["index"], scenes.SUB_FLIPS)
    flips = np.stack([scenes.image_to_words(
        np.isin(np.arange(cam.width * cam.height), scenes.flip_indices(rng_f, cam.width, cam.height))
        .reshape(cam.height, cam.width)) for _ in range(F)])
    targets = clean ^ torch.as_tensor(flips.view(np.int64), device=dev)
    rng_q = scenes.rng_for(wl["index"], scenes.SUB_CMAES)
    # joint readings: the true joint angles (device cosine map) plus 2-degree
    # noise, back in the unconstrained coordinates
    noisy = tracker.joint_angles(prob, traj)
    noisy[:, 6:9] += rng_q.normal(size=(F, 3)) * math.radians(2.0)
    readings = tracker.joint_coordinates(prob, noisy)[:, 6:9]
    est0 = traj[0] + scale * rng_q.normal(size=9)
    torch.cuda.synchronize()

    gen = tracker.Generation(prob, lam, loss_kind=tk.LOSS_IOU, lambda_kp=0.1)
    seed0 = scenes.BASE_SEED + wl["index"] + 1000 * scenes.SUB_CMAES
    # frame loop: CMA-ES warm-started from the previous frame's filtered
    # estimate (joint means from the joint readings), temporal filter on the
    # device at the end of every frame; the next frame starts from the device
    # estimate and the per-frame results reach the host asynchronously
    trk = tracker.Tracker(gen, scale, G, seed0, filt=wl["filter"])
    state = {"frame": -1, "frame_step": 0, "log": None, "pending": [], "logged": []}

    def start_frame(f, s=0):
        if f == 0:
            trk.start(est0)                           # first frame of the trajectory: restart the filter
        trk.begin_frame(f, targets[f], kp_true[f], readings[f])
        state["frame"], state["frame_step"] = f, s

    def end_frame():
        trk.end_frame_async()                         # estimate + filter step; the 3 x 9 FP64 copy is asynchronous
        keep = state["log"] is not None and state["frame_step"] >= args.warmup
        state["pending"].append((state["frame"], keep))

    def drain():
        """Collects the ended frames (outside the timed region) and keeps those of the timed region."""
        for (f, keep), r in zip(state["pending"], trk.collect()):
            if keep:
                state["logged"].append((f, r))
        state["pending"] = []

    def ask_eval():
        tk.cmaes_ask_eval(gen.state, gen.n, gen.lam, prob.chains, prob.meshes, cam, prob.target, gen.X, gen.xf,
                          gen.counts, kp=gen.kp, ws=gen.ws)

    def tell():
        tk.cmaes_tell(gen.state, gen.n, gen.lam, gen.counts, prob.target_count, tk.LOSS_IOU, 1, kp=gen.kp,
                      kp_ref=prob.kp_ref, lambda_kp=0.1, loss=gen.loss)

    def run_step(s, events=None, between=None):
        """One generation in two launches: draw the candidates, evaluate their FK
        and raster counts (one workgroup per candidate); then compose the losses
        and update CMA-ES."""
        f, g = (s // G) % F, s % G
        if g == 0:
            if state["frame"] >= 0:
                end_frame()
            start_frame(f, s)
        if events is not None:
            events[0].record()
        ask_eval()
        if events is not None:
            events[1].record()
        if between is not None:
            between()
        tell()

    # ---------------------------------------------------------------- warm-up and timed region
    for s in range(args.warmup):
        run_step(s)
    torch.cuda.synchronize()
    drain()
    log(f"warm-up done ({args.warmup} generations)")
    t_start, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    state["log"] = True
    w0 = time.perf_counter()
    t_start.record()
    for i in range(args.steps):
        run_step(args.warmup + i)
        if (i + 1) % 500 == 0:
            log(f"timed generations queued: {i + 1}/{args.steps}")
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_ms = t_start.elapsed_time(t_end)
    ms_per_step = max(gpu_ms, wall * 1e3) / args.steps
    if (args.warmup + args.steps) % G == 0:
        end_frame()                                   # the last timed frame is complete
    state["log"] = None
    drain()
    frames_log, state["logged"] = state["logged"], []
    g0, g1 = args.warmup, args.warmup + args.steps - 1
    frames_timed = sorted({(s // G) % F for s in range(g0, g1 + 1)})
    timed_region = {"generations": [g0, g1], "frames_touched": len(frames_timed),
                    "first_frame": (g0 // G) % F, "frame_starts_timed": sum(1 for s in range(g0, g1 + 1) if s % G == 0),
                    "note": f"generations {g0}..{g1} of the {G}-generation-per-frame loop over {F} frames "
                            f"(frame index wraps); the per-frame filter step, CMA-ES restart and result copy "
                            f"run inside the timed region at every frame start it contains"}
    log(f"timed: {args.steps} generations in {wall:.3f} s wall / {gpu_ms:.1f} ms GPU events "
        f"({timed_region['frame_starts_timed']} frame starts inside)")

    # pose errors of the frames completed in the timed region (raw CMA-ES
    # estimates and temporally filtered ones) against the trajectory
    tracking = None
    if frames_log:
        fidx = np.array([f for f, _ in frames_log])
        truth = traj[fidx]
        tracking = {"frames": len(frames_log)}
        # second differences only over three consecutive frames (not across the trajectory's wrap)
        consec = (np.diff(fidx)[1:] == 1) & (np.diff(fidx)[:-1] == 1)

        def jitter_mm(x):
            d2 = np.abs(np.diff(x[:, 3:6], 2, axis=0)).sum(1)[consec]
            return float(d2.mean() * 1e3) if d2.size else None
        for key in ("z", "theta"):
            est = np.stack([r[key] for _, r in frames_log])
            e = tracker.pose_errors(prob, est, truth)
            tracking["raw" if key == "z" else "filtered"] = {
                "rot_deg_mean": float(e["rot_deg"].mean()), "trans_mm_mean": float(e["trans_m"].mean() * 1e3),
                "joint_deg_mean": float(e["joint_deg"].mean()), "trans_mm_max": float(e["trans_m"].max() * 1e3),
                # mean |second difference| of the translation over consecutive frames
                "jitter_mm": jitter_mm(est)}
        tracking["truth_jitter_mm"] = jitter_mm(truth)
        log(f"tracking over {len(frames_log)} frames: raw {tracking['raw']}, filtered {tracking['filtered']}")

    # ---------------------------------------------------------------- per-generation distribution
    # each of 300 generations (after 10 untimed ones) bracketed by its own
    # events: median, p10 and p90 of the two-launch generation
    state["frame"] = -1
    for s in range(10):
        run_step(s)
    pairs_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(300)]
    for i, (ea, eb) in enumerate(pairs_ev):
        s = 10 + i
        if s % G == 0:
            end_frame()
            start_frame((s // G) % F, s)
        ea.record()
        ask_eval()
        tell()
        eb.record()
    torch.cuda.synchronize()
    drain()
    gen_us = np.array([ea.elapsed_time(eb) * 1e3 for ea, eb in pairs_ev])
    generation_us = {"median": float(np.median(gen_us)), "p10": float(np.percentile(gen_us, 10)),
                     "p90": float(np.percentile(gen_us, 90)), "generations": len(gen_us)}
    log(f"per generation (events around each): median {generation_us['median']:.1f} us, "
        f"p10 {generation_us['p10']:.1f}, p90 {generation_us['p90']:.1f}")

    # ---------------------------------------------------------------- roofline of the ask-eval raster kernel
    # (a) KT back-to-back launches of the benchmarked ask-eval kernel on the
    # state of one generation (the launch is idempotent: it re-draws the same
    # candidates), one event pair on the launch stream around all of them;
    # (b) events around each of KS single launches, each followed by the tell
    # of its generation as in the loop (median)
    KT, KS = 200, 100
    state["frame"] = -1
    for s in range(3):
        run_step(s)
    ka, kb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(10):
        ask_eval()
    ka.record()
    for _ in range(KT):
        ask_eval()
    kb.record()
    torch.cuda.synchronize()
    kernel_us = ka.elapsed_time(kb) * 1e3 / KT
    single = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(KS)]
    for i, (ea, eb) in enumerate(single):
        run_step(3 + i, events=(ea, eb))
    torch.cuda.synchronize()
    drain()
    single_us = np.array([ea.elapsed_time(eb) * 1e3 for ea, eb in single])
    log(f"ask-eval kernel: {kernel_us:.1f} us per launch over {KT} back-to-back launches; "
        f"{np.median(single_us):.1f} us median of {KS} single event-bracketed launches")

    # work per launch from tk_raster_stats on the same inputs (the triangles the
    # kernel draws: one orientation of a closed mesh, culling applied)
    stats = torch.zeros(4, dtype=torch.int64, device=dev)
    acc = np.zeros(4)
    n_st = 0
    state["frame"] = -1
    for s in range(2 * G):
        run_step(s, between=lambda: tk.raster_stats(gen.xf, gen.lam, prob.meshes, cam, stats))
        acc += stats.cpu().numpy()
        n_st += 1
    drain()
    kept, box_px, pairs, huge = acc / n_st
    tri_all = lam * mesh.n_triangles
    vert_all = lam * mesh.n_vertices
    # per-unit costs of the method's own units (survey of the path): 25 FP32
    # operations per vertex transform and projection, 40 integer operations per
    # triangle set-up, 3 edge functions x 8 operations per pixel centre tested
    # inside a drawn triangle's clamped box
    ops = 25.0 * vert_all + 40.0 * tri_all + 24.0 * box_px
    # a finer count: 22 per vertex, 10 per triangle cull test,
    # 40 per kept triangle set-up, 5 per tested pixel centre
    ops_fine = 22.0 * vert_all + 10.0 * tri_all + 40.0 * kept + 5.0 * box_px
    peak_ops = 256 * 64 * 2.4e9
    achieved = ops / (kernel_us * 1e-6)
    log(f"per launch: kept {kept:.0f} tris, {box_px:.0f} box pixels, {pairs:.0f} block pairs, {huge:.0f} wide; "
        f"{ops:.3e} ops -> {achieved / 1e12:.2f} T ops/s ({achieved / peak_ops:.3f} of the ALU peak)")
    peaks = measure_peaks(dev)

    out = {
        "metric": "candidate pose evals/sec (FK+raster+loss) at 640x480; ms per CMA-ES generation",
        "value": lam / (ms_per_step * 1e-3),
        "unit": "candidate evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"track640: single-instrument tracking, procedural {mesh.n_triangles}-triangle "
                               "closed instrument, 640x480, lambda=256, 9-D, loss 1-IoU + 0.1 keypoints, "
                               "30 gens/frame, 100-frame trajectory",
                   "triangles": mesh.n_triangles, "width": cam.width, "height": cam.height, "lambda": lam,
                   "dims": 9, "gens_per_frame": G, "frames": F, "timed_region": timed_region},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak_ops / 1e12, "unit": "Tops/s",
                     "frac": achieved / peak_ops, "traffic": raster_traffic(),
                     "traffic_unit": "B per launch",
                     "hbm_frac": (raster_traffic() / (kernel_us * 1e-6) / (peaks["hbm_GBps"] * 1e9)
                                  if raster_traffic() is not None else None),
                     "valu_busy": RASTER_TRAFFIC["valu_busy"] if raster_profile_valid() else None,
                     "lds": raster_lds(kernel_us, peaks),
                     "constants_from_profiles": "traffic, valu_busy and lds counts are taken from the committed "
                                                "rocprofv3 counter runs (profiles/) and reported only while the "
                                                "kernel sources match the hash recorded there; null otherwise",
                     "kernel": "raster_kernel<true,false,true,1024> (tk_cmaes_ask_eval: draw, FK, raster, "
                               "counts; with workspace)",
                     "kernel_us": kernel_us,
                     "kernel_us_timing": f"mean of {KT} back-to-back launches (one event pair on the launch "
                                         f"stream); median of {KS} single event-bracketed launches: "
                                         f"{float(np.median(single_us)):.2f} us",
                     "ops_per_launch": ops,
                     "ops_formula": "25 per vertex + 40 per triangle + 24 per box pixel of a drawn triangle",
                     "ops_fine_per_launch": ops_fine,
                     "frac_fine": ops_fine / (kernel_us * 1e-6) / peak_ops,
                     "units_per_launch": {"vertices": vert_all, "triangles": tri_all, "kept": kept,
                                          "box_pixels": box_px, "block_pairs": pairs},
                     "peaks_measured": peaks},
        "fitness_evals_per_s": lam / (kernel_us * 1e-6),
        "generation_us": generation_us,
        "tracking": tracking,
    }

    # ---------------------------------------------------------------- graph replay and plain launches
    if not args.no_extras:
        state["frame"] = -1
        start_frame(0)
        graph = gen.capture()
        torch.cuda.synchronize()
        ng = 300
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for s in range(ng):
            if s % G == 0:
                start_frame((s // G) % F)
            graph.replay()
        b.record()
        torch.cuda.synchronize()
        graph_ms = a.elapsed_time(b) / ng
        log(f"graph replay: {graph_ms * 1e3:.1f} us per generation")
        start_frame(0)
        torch.cuda.synchronize()
        w = time.perf_counter()
        for _ in range(args.plain_gens):
            gen.step_plain()
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - w) * 1e3 / args.plain_gens
        log(f"plain per-candidate launches: {plain_ms:.2f} ms per generation")
        out["graph_ms_per_step"] = graph_ms
        out["plain_ms_per_step"] = plain_ms
        out["batched_vs_plain"] = plain_ms / min(graph_ms, ms_per_step)
    legs = {"small320": lambda: small_leg(dev, with_cpu=not args.no_cpu_baseline),
            "bimanual960": lambda: bimanual_leg(dev), "batch64": lambda: batch_leg(dev),
            "soft640": lambda: soft_leg(dev), "synth700": lambda: synth700_leg(dev)}
    chosen = [] if args.no_extras and args.legs is None else \
        (list(legs) if args.legs is None else [x for x in args.legs.split(",") if x])
    for name in chosen:
        if name not in legs:
            raise SystemExit(f"unknown leg {name!r}; choose from {', '.join(legs)}")
        out[name] = legs[name]()

    # ---------------------------------------------------------------- CPU baseline (oracle)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds, mesh, cam, chain, traj, flips, readings, est0, lam)

    print(json.dumps(out), flush=True)


def measure_peaks(dev):
    """Measured bandwidth roofs on this device: HBM by a streaming copy of
    1 GiB (read + write bytes over the best of 5 runs), LDS by the loop of
    conflict-free 128-bit reads and writes (2048 workgroups)."""
    import torch

    from paper_2603_11404_amd import tk

    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tk.bench_copy(src, dst, nbytes)
    best = 1e9
    for _ in range(5):
        a.record()
        tk.bench_copy(src, dst, nbytes)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    hbm = 2.0 * nbytes / (best * 1e-3)
    assert torch.equal(src, dst)
    del src, dst
    wgs, iters = 2048, 2048
    out = torch.zeros(wgs, dtype=torch.int32, device=dev)
    tk.bench_lds(wgs, 16, out)
    best = 1e9
    for _ in range(5):
        a.record()
        tk.bench_lds(wgs, iters, out)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    lds = wgs * iters * 256 * 128.0 / (best * 1e-3)
    log(f"measured peaks: HBM copy {hbm / 1e9:.0f} GB/s, LDS {lds / 1e12:.1f} TB/s")
    return {"hbm_GBps": hbm / 1e9, "hbm_spec_GBps": 8000.0, "lds_TBps": lds / 1e12,
            "lds_spec_TBps": 256 * 128 * 2.4e9 / 1e12,
            "method": "HBM: tk_bench_copy of 1 GiB (2 x bytes / time, best of 5); LDS: tk_bench_lds, "
                      "2048 workgroups x 2048 iterations of 4 + 4 conflict-free 128-bit accesses per thread"}


def raster_lds(kernel_us, peaks):
    """LDS side of the raster kernel's roofline from the committed counter run:
    the LDS occupancy per launch (SQ_LDS_IDX_ACTIVE) expressed in bytes at the
    rate of the LDS microbenchmark, over the kernel time, against the measured
    LDS roof; None while the kernel sources differ from the profiled ones."""
    if not raster_profile_valid() or RASTER_TRAFFIC.get("lds_equiv_bytes") is None:
        return None
    bps = RASTER_TRAFFIC["lds_equiv_bytes"] / (kernel_us * 1e-6)
    return {"equiv_bytes_per_launch": RASTER_TRAFFIC["lds_equiv_bytes"], "achieved_TBps": bps / 1e12,
            "peak_TBps": peaks["lds_TBps"], "frac": bps / (peaks["lds_TBps"] * 1e12),
            "lds_instructions_per_launch": RASTER_TRAFFIC["lds_insts"],
            "bank_conflict_frac": RASTER_TRAFFIC["lds_bank_conflict_frac"]}


def small_leg(dev, with_cpu=True, solves=20):
    """The small plain-method configuration: one 2044-triangle instrument,
    320x240, lambda = 16, 20-generation solves from a perturbed start, loss
    1 - IoU against the render with 1% pixel flips.  GPU: the two launches of
    each generation bracketed by events, over `solves` solves after two
    untimed ones.  CPU: the oracle runs one whole 20-generation solve on one
    host thread and on all of them."""
    import torch

    import oracle
    from oracle import cmaes
    import scenes
    from paper_2603_11404_amd import tk, tracker

    wl = scenes.workload("small")
    mesh, cam, lam, G = wl["mesh"], wl["cam"], wl["lam"], wl["gens"]
    chain = scenes.chain()
    rng = scenes.rng_for(wl["index"], scenes.SUB_POSE)
    truth = scenes.true_pose(rng, cam)
    flips = scenes.image_to_words(np.isin(np.arange(cam.width * cam.height), scenes.flip_indices(
        scenes.rng_for(wl["index"], scenes.SUB_FLIPS), cam.width, cam.height)).reshape(cam.height, cam.width))
    prob = tracker.Problem([mesh], [chain], cam, dev)
    clean = prob.render(torch.as_tensor(truth[None].astype(np.float32), device=dev))[0]
    prob.set_target(clean ^ torch.as_tensor(flips.view(np.int64), device=dev))
    gen = tracker.Generation(prob, lam, loss_kind=tk.LOSS_IOU)
    rng_m = scenes.rng_for(wl["index"], scenes.SUB_CMAES)
    starts = [truth + scenes.DEFAULT_SCALE * rng_m.normal(size=9) for _ in range(solves + 2)]
    times, err_mm = [], []
    for r, mean0 in enumerate(starts):
        gen.init(np.zeros(9), 1.0, mean0, scenes.DEFAULT_SCALE, scenes.BASE_SEED + r)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(G)]
        for ea, eb in ev:
            ea.record()
            gen.ask_eval_tell()
            eb.record()
        torch.cuda.synchronize()
        if r >= 2:
            times += [ea.elapsed_time(eb) * 1e3 for ea, eb in ev]
            est = mean0 + scenes.DEFAULT_SCALE * tk.cmaes_view(gen.state, 9, lam)["mean"]   # physical mean
            err_mm.append(float(np.linalg.norm(est[3:6] - truth[3:6]) * 1e3))
    t = np.array(times)
    out = {"workload": f"small: one {mesh.n_triangles}-triangle instrument, 320x240, lambda=16, 9-D, 20-generation solves, "
                       "loss 1-IoU, 1% pixel flips",
           "gpu_us_per_generation": {"median": float(np.median(t)), "p10": float(np.percentile(t, 10)),
                                     "p90": float(np.percentile(t, 90)), "generations": len(t)},
           "gpu_evals_per_s": lam / (float(np.median(t)) * 1e-6),
           "final_trans_err_mm_median": float(np.median(err_mm))}
    log(f"small320: {np.median(t):.1f} us per generation (p10 {np.percentile(t, 10):.1f}, "
        f"p90 {np.percentile(t, 90):.1f}) over {len(t)} generations")
    if with_cpu:
        from threadpoolctl import threadpool_limits
        _blas = threadpool_limits(1, "blas")    # the oracle's 9 x 9 numpy steps: no BLAS threads beside OpenMP
        target = oracle.render(truth, [chain], [mesh], cam) ^ flips
        m_cnt = oracle.counts(target, target, cam.width, cam.height)[2]
        cpu = {}
        for label, threads in (("one_thread", 1), ("all_threads", oracle.max_threads())):
            es = cmaes.CMAES(9, lam, np.zeros(9), 1.0, starts[2], scenes.DEFAULT_SCALE, scenes.BASE_SEED + 2)
            t0 = time.perf_counter()
            for _ in range(G):
                theta = es.sample().astype(np.float32).astype(np.float64)
                cnt = oracle.eval_batch(theta, [chain], [mesh], cam, target, n_threads=threads)
                es.update(np.array([oracle.mask_loss(cnt[k, 0], cnt[k, 1], m_cnt, 0) for k in range(lam)]))
            el = time.perf_counter() - t0
            cpu[label] = {"threads": threads, "ms_per_generation": el * 1e3 / G, "evals_per_s": G * lam / el}
        _blas.restore_original_limits()
        cpu["sample"] = f"one whole {G}-generation solve of the oracle per thread count"
        cpu["cpu"] = _cpu_model()
        out["cpu_oracle"] = cpu
        log(f"small320 oracle: {cpu['one_thread']['ms_per_generation']:.2f} ms per generation on 1 thread, "
            f"{cpu['all_threads']['ms_per_generation']:.2f} on {cpu['all_threads']['threads']}")
    return out


def bimanual_leg(dev, gens=100):
    """Bi-manual workload: two uneven instruments (20144 + 35388 triangles),
    960x540, lambda = 512, 18-D with a block-diagonal covariance, target with
    an occluding rectangle; generations of two launches (both arms in each),
    timed eagerly and as a replayed HIP graph."""
    import torch

    import scenes
    from paper_2603_11404_amd import tk, tracker

    wl = scenes.workload("bimanual960")
    cam, lam = wl["cam"], wl["lam"]
    prob = tracker.Problem(wl["meshes"], wl["chains"], cam, dev)
    rng = scenes.rng_for(wl["index"], scenes.SUB_POSE)
    truth = np.concatenate([scenes.true_pose(rng, cam), scenes.true_pose(rng, cam)]).astype(np.float32)
    words = prob.render(torch.as_tensor(truth[None], device=dev))[0].cpu().numpy().view(np.uint64)
    img = scenes.words_to_image(words, cam.width, cam.height)
    rect, _ = scenes.occluder_rect(img, scenes.rng_for(wl["index"], scenes.SUB_OCCLUDER))
    target = scenes.image_to_words(scenes.apply_occluder(img, rect))
    prob.set_target(torch.as_tensor(target.view(np.int64), device=dev))
    gen = tracker.Generation(prob, lam, loss_kind=tk.LOSS_IOU, n_blocks=wl["n_blocks"])
    scale = np.tile(scenes.DEFAULT_SCALE, 2)
    seed = scenes.BASE_SEED + wl["index"] + 1000 * scenes.SUB_CMAES
    gen.init(np.zeros(18), 1.0, truth + scale * np.random.default_rng(seed).normal(size=18), scale, seed)
    for _ in range(5):
        gen.ask_eval_tell()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(gens):
        gen.ask_eval_tell()
    b.record()
    torch.cuda.synchronize()
    eager_ms = a.elapsed_time(b) / gens
    gen.capture()
    torch.cuda.synchronize()
    a.record()
    for _ in range(gens):
        gen.replay()
    b.record()
    torch.cuda.synchronize()
    graph_ms = a.elapsed_time(b) / gens
    best = min(eager_ms, graph_ms)
    log(f"bimanual960: {eager_ms * 1e3:.1f} us per generation eager, {graph_ms * 1e3:.1f} us graph replay")
    tris = " + ".join(str(m.n_triangles) for m in wl["meshes"])
    return {"workload": f"two instruments ({tris} tris), 960x540, lambda=512, 18-D block-diagonal, occluder",
            "ms_per_generation": eager_ms, "graph_ms_per_generation": graph_ms,
            "candidate_evals_per_s": lam / (best * 1e-3), "generations": gens}


def batch_leg(dev, count=64, gens=10):
    """Batched solves: 64 independent tracking problems of mixed size
    (resolutions 320x240 .. 1280x720, lambda 64 .. 1024, meshes of 2k .. 50k
    triangles, targets with 1% pixel flips) advanced together: the ask-eval of
    all problems in one persistent launch, then the batched tell (two
    launches per generation); also with the raster launches grouped by the
    autotuned workgroup size; compared with launching each problem's
    generation separately."""
    import tempfile

    import torch

    import scenes
    from paper_2603_11404_amd import tk, tracker
    from paper_2603_11404_amd.autotune import Autotuner

    rng = scenes.rng_for(3, scenes.SUB_POSE)
    rng_f = scenes.rng_for(3, scenes.SUB_FLIPS)
    gens_ = []
    tri_total = 0
    for i, sh in enumerate(scenes.batch_problem_shapes(count)):
        cam = scenes.camera(sh["width"], sh["height"])
        mesh = scenes.instrument_mesh(sh["segments"], sh["rings"], 3, 1)
        tri_total += mesh.n_triangles * sh["lam"]
        prob = tracker.Problem([mesh], [scenes.chain()], cam, dev)
        truth = scenes.true_pose(rng, cam).astype(np.float32)
        th = torch.as_tensor(truth[None], device=dev)
        words = prob.render(th)[0].cpu().numpy().view(np.uint64)
        words = scenes.apply_flips(words, cam.width, cam.height, scenes.flip_indices(rng_f, cam.width, cam.height))
        prob.set_target(torch.as_tensor(words.view(np.int64), device=dev), prob.keypoints(th)[0])
        g = tracker.Generation(prob, sh["lam"], loss_kind=tk.LOSS_IOU, lambda_kp=0.1)
        g.init(np.zeros(9), 1.0, truth + scenes.DEFAULT_SCALE * rng.normal(size=9), scenes.DEFAULT_SCALE,
               scenes.BASE_SEED + 3 + 1000 * scenes.SUB_CMAES + i)
        gens_.append(g)
    lam_total = sum(g.lam for g in gens_)
    tuner = Autotuner(os.path.join(tempfile.gettempdir(), "tk_autotune.json"))
    threads = [tuner.choose(g) for g in gens_]
    batch = tk.Batch([g.problem_struct(t) for g, t in zip(gens_, threads)], device=dev)
    for _ in range(2):
        batch.ask_eval()
        batch.tell()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(gens):
        batch.ask_eval()
        batch.tell()
    b.record()
    torch.cuda.synchronize()
    batch_ms = a.elapsed_time(b) / gens
    # the same generations with all problems' ask-eval in one persistent launch
    for _ in range(2):
        batch.ask_eval_persistent()
        batch.tell()
    torch.cuda.synchronize()
    a.record()
    for _ in range(gens):
        batch.ask_eval_persistent()
        batch.tell()
    b.record()
    torch.cuda.synchronize()
    persist_ms = a.elapsed_time(b) / gens
    a.record()
    for _ in range(3):
        for g in gens_:
            g.ask_eval_tell()
    b.record()
    torch.cuda.synchronize()
    single_ms = a.elapsed_time(b) / 3
    # ask-eval alone per resolution class: persistent launch of the class's
    # problems against launching each of them
    shapes = scenes.batch_problem_shapes(count)
    classes = {}
    for res in scenes.BATCH_RESOLUTIONS:
        sel = [i for i, sh in enumerate(shapes) if (sh["width"], sh["height"]) == res]
        if not sel:
            continue
        sub = tk.Batch([gens_[i].problem_struct(threads[i]) for i in sel], device=dev)
        sub.ask_eval_persistent()
        torch.cuda.synchronize()
        a.record()
        for _ in range(5):
            sub.ask_eval_persistent()
        b.record()
        torch.cuda.synchronize()
        p_ms = a.elapsed_time(b) / 5
        a.record()
        for _ in range(3):
            for i in sel:
                g = gens_[i]
                tk.cmaes_ask_eval(g.state, g.n, g.lam, g.p.chains, g.p.meshes, g.p.cam, g.p.target, g.X, g.xf,
                                  g.counts, kp=g.kp, ws=g.ws)
        b.record()
        torch.cuda.synchronize()
        s_ms = a.elapsed_time(b) / 3
        classes[f"{res[0]}x{res[1]}"] = {"problems": len(sel), "persistent_ask_ms": p_ms, "per_problem_ask_ms": s_ms,
                                         "ratio": s_ms / p_ms}
    log("batch64 ask-eval per resolution (persistent vs per problem): " +
        ", ".join(f"{k} {v['persistent_ask_ms']:.2f} vs {v['per_problem_ask_ms']:.2f} ms" for k, v in classes.items()))
    log(f"batch64: {persist_ms:.2f} ms per generation with the persistent launch, {batch_ms:.2f} ms with one "
        f"launch per workgroup size, {single_ms:.2f} ms launching each problem "
        f"({lam_total} candidates, {tri_total / 1e6:.0f} M candidate-triangles)")
    return {"workload": f"{count} problems, 320x240..1280x720, lambda 64..1024, 2k..50k tris, 1% flips",
            "candidates_per_generation": lam_total, "ms_per_generation": persist_ms,
            "candidate_evals_per_s": lam_total / (persist_ms * 1e-3), "per_problem_launches_ms": single_ms,
            "batched_vs_per_problem": single_ms / persist_ms, "ask_eval_by_resolution": classes,
            "grouped_launches_ms": batch_ms, "grouped_vs_per_problem": single_ms / batch_ms,
            "workgroup_sizes": {str(t): threads.count(t) for t in sorted(set(threads))}}


def synth700_leg(dev):
    """The paper's synthetic-set protocol: one instrument at 700x493, N = 70
    candidates, 3 iterations per frame (c_mu raised x2, sigma0 0.5) over a
    1000-frame Hermite/OU trajectory whose masks are dilated / eroded and
    blobbed, the render loss (MSE + appearance, Eq. for L_render) plus 10 x
    the two-tip keypoint term of Eq. (8) in pixels with tau = 2 px, joint
    readings with 2-degree noise, Kalman-filtered estimates."""
    import torch

    import scenes
    from paper_2603_11404_amd import tk, tracker

    wl = scenes.workload("synth700")
    mesh, cam, lam, G, F = wl["mesh"], wl["cam"], wl["lam"], wl["gens"], wl["frames"]
    chain, scale = scenes.chain(), scenes.DEFAULT_SCALE.copy()
    prob = tracker.Problem([mesh], [chain], cam, dev)
    traj = scenes.hermite_trajectory(scenes.rng_for(wl["index"], scenes.SUB_TRAJ), cam, F)
    th_true = torch.as_tensor(traj.astype(np.float32), device=dev)
    clean = scenes.words_to_image(prob.render(th_true).cpu().numpy().view(np.uint64), cam.width, cam.height)
    kp_true = prob.keypoints(th_true)
    rng_m = scenes.rng_for(wl["index"], scenes.SUB_FLIPS)
    targets = torch.as_tensor(np.stack([scenes.image_to_words(scenes.perturb_mask(rng_m, im)) for im in clean])
                              .view(np.int64), device=dev)
    rng_q = scenes.rng_for(wl["index"], scenes.SUB_CMAES)
    noisy = tracker.joint_angles(prob, traj)
    noisy[:, 6:9] += rng_q.normal(size=(F, 3)) * math.radians(2.0)
    readings = tracker.joint_coordinates(prob, noisy)[:, 6:9]
    est0 = traj[0] + scale * rng_q.normal(size=9)
    gen = tracker.Generation(prob, lam, loss_kind=tk.LOSS_RENDER | tk.KP_TWO_TIPS, lambda_app=wl["lambda_app"],
                             lambda_kp=wl["lambda_kp"], tau=wl["tau"])
    trk = tracker.Tracker(gen, scale, G, scenes.BASE_SEED + wl["index"] + 1000 * scenes.SUB_CMAES,
                          filt=wl["filter"], sigma0=wl["sigma0"], c_m_scale=wl["c_m_scale"],
                          c_mu_scale=wl["c_mu_scale"])
    trk.start(est0)
    res = []
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for f in range(F):
        trk.begin_frame(f, targets[f], kp_true[f], readings[f])
        for _ in range(G):
            gen.ask_eval_tell()
        trk.end_frame_async()
    res = trk.collect()
    wall = time.perf_counter() - w0
    out = {"workload": f"{mesh.n_triangles} tris, {cam.width}x{cam.height}, lambda={lam}, {G} gens x {F} frames "
                       "(c_mu x2, sigma0 0.5), Hermite/OU trajectory, dilated/eroded/blobbed masks, "
                       "MSE + appearance + 10 x two-tip keypoints (tau 2 px)",
           "ms_per_frame": wall * 1e3 / F,
           "ms_per_generation": wall * 1e3 / (F * G), "candidate_evals_per_s": lam * F * G / wall}
    for key, name in (("z", "raw"), ("theta", "filtered")):
        e = tracker.pose_errors(prob, np.stack([r[key] for r in res]), traj)
        out[name] = {"rot_deg_mean": float(e["rot_deg"].mean()), "trans_mm_mean": float(e["trans_m"].mean() * 1e3),
                     "joint_deg_mean": float(e["joint_deg"].mean()),
                     "rot_deg_median": float(np.median(e["rot_deg"])),
                     "trans_mm_median": float(np.median(e["trans_m"]) * 1e3),
                     "rot_deg_p90": float(np.percentile(e["rot_deg"], 90)),
                     "frames_scored_on_symmetric_pose": int(np.sum(e["flipped"]))}
    log(f"synth700: {out['ms_per_generation'] * 1e3:.1f} us per generation (frame loop, results collected at the end); "
        f"raw {out['raw']}, filtered {out['filtered']}")
    return out


def soft_leg(dev, reps=10):
    """Differentiable form: soft silhouette forward + backward (FK, projection,
    binning, soft raster, loss; face-major backward, FK Jacobian) of 256
    candidates of a 49744-triangle instrument at 640x480, sigma = 1 px; and
    the refinement of one problem's CMA-ES mean by 5 Adam steps per generation."""
    import torch

    import scenes
    from paper_2603_11404_amd import tk, tracker

    wl = scenes.workload("soft640")
    mesh, cam, lam, sigma = wl["mesh"], wl["cam"], wl["lam"], wl["sigma"]
    chain = scenes.chain()
    rng = scenes.rng_for(wl["index"], scenes.SUB_POSE)
    truth = scenes.true_pose(rng, cam)
    prob = tracker.Problem([mesh], [chain], cam, dev)
    th_t = torch.as_tensor(truth[None].astype(np.float32), device=dev)
    prob.set_target(prob.render(th_t)[0])
    theta = torch.as_tensor((truth[None] + scenes.DEFAULT_SCALE[None] * rng.normal(size=(lam, 9))).astype(np.float32),
                            device=dev)
    xf = torch.empty(lam, 1, 4, 12, dtype=torch.float32, device=dev)
    ws = tk.soft_workspace(lam, prob.soft_meshes, cam, dev)
    loss = torch.empty(lam, dtype=torch.float64, device=dev)
    g = torch.empty_like(theta)

    def fwd_bwd():
        tk.fk_transform(theta, lam, 1, prob.chains, xf)
        tk.soft_forward(xf, lam, prob.soft_meshes, cam, sigma, prob.target, loss, ws)
        tk.soft_backward(theta, lam, prob.chains, prob.soft_meshes, cam, sigma, g, ws)

    fwd_bwd()
    torch.cuda.synchronize()
    a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    fwd_ms = bwd_ms = 0.0
    for _ in range(reps):
        a.record()
        tk.fk_transform(theta, lam, 1, prob.chains, xf)
        tk.soft_forward(xf, lam, prob.soft_meshes, cam, sigma, prob.target, loss, ws)
        b.record()
        tk.soft_backward(theta, lam, prob.chains, prob.soft_meshes, cam, sigma, g, ws)
        c.record()
        torch.cuda.synchronize()
        fwd_ms += a.elapsed_time(b) / reps
        bwd_ms += b.elapsed_time(c) / reps
    # refinement of one problem's mean: 5 Adam steps after each generation
    gen = tracker.Generation(prob, lam, loss_kind=tk.LOSS_IOU)
    gen.init(np.zeros(9), 1.0, truth + scenes.DEFAULT_SCALE * rng.normal(size=9), scenes.DEFAULT_SCALE, 7)
    gen.ask_eval_tell()
    gen.refine(5, 0.1, sigma)
    torch.cuda.synchronize()
    gens = 20
    a.record()
    for _ in range(gens):
        gen.ask_eval_tell()
    b.record()
    for _ in range(gens):
        gen.ask_eval_tell()
        gen.refine(5, 0.1, sigma)
    c.record()
    torch.cuda.synchronize()
    plain_gen = a.elapsed_time(b) / gens
    refined_gen = b.elapsed_time(c) / gens
    # the same generation + refinement recorded once into a HIP graph and replayed
    gen.capture(refine=(5, 0.1, sigma))
    gen.replay()
    torch.cuda.synchronize()
    a.record()
    for _ in range(gens):
        gen.replay()
    b.record()
    torch.cuda.synchronize()
    graph_gen = a.elapsed_time(b) / gens
    log(f"soft640: forward {fwd_ms:.2f} ms + backward {bwd_ms:.2f} ms for {lam} candidates; generation "
        f"{plain_gen:.3f} ms, with 5 Adam steps on the mean {refined_gen:.3f} ms ({graph_gen:.3f} ms as a graph)")
    return {"workload": f"{mesh.n_triangles} tris, {cam.width}x{cam.height}, {lam} candidates, sigma {sigma} px",
            "forward_ms": fwd_ms, "backward_ms": bwd_ms,
            "candidate_grads_per_s": lam / ((fwd_ms + bwd_ms) * 1e-3),
            "generation_ms": plain_gen, "generation_with_refine_ms": refined_gen,
            "generation_with_refine_graph_ms": graph_gen,
            "refine_ms": refined_gen - plain_gen, "refine_steps_per_generation": 5}


def cpu_baseline(seconds, mesh, cam, chain, traj, flips, readings, est0, lam):
    """The CPU oracle (C, OpenMP over candidates; numpy CMA-ES) running the same
    generations on frame 0 of the trajectory with its own rendered target."""
    import oracle
    from oracle import cmaes
    import scenes

    from threadpoolctl import threadpool_limits
    threadpool_limits(1, "blas")              # the oracle's 9 x 9 numpy steps: no BLAS threads beside OpenMP
    log("cpu baseline: oracle on the host cores")
    target = oracle.render(traj[0], [chain], [mesh], cam) ^ flips[0]
    ref_kp = oracle.keypoints(oracle.fk(traj[0], chain), chain, cam)
    m_cnt = oracle.counts(target, target, cam.width, cam.height)[2]
    mean_phys = est0.copy()
    mean_phys[6:9] = readings[0]
    es = cmaes.CMAES(9, lam, np.zeros(9), 1.0, mean_phys, scenes.DEFAULT_SCALE, 1)
    threads = oracle.max_threads()
    n_eval = 0
    gens = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        theta = es.sample().astype(np.float32).astype(np.float64)
        cnt = oracle.eval_batch(theta, [chain], [mesh], cam, target, n_threads=threads)
        loss = np.empty(lam)
        for k in range(lam):
            kp = oracle.keypoints(oracle.fk(theta[k], chain), chain, cam)
            loss[k] = oracle.mask_loss(cnt[k, 0], cnt[k, 1], m_cnt, 0) + 0.1 * oracle.kp_loss(kp, ref_kp)
        es.update(loss)
        n_eval += lam
        gens += 1
    el = time.perf_counter() - t0
    log(f"cpu baseline: {gens} generations, {n_eval / el:.0f} evals/s on {threads} threads")
    return {"value": n_eval / el, "unit": "candidate evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{gens} generations x {lam} candidates of frame 0 (same mesh/camera/loss), "
                      f"{el:.1f} s wall, ms per generation {el * 1e3 / gens:.1f}",
            "cpu": _cpu_model()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
