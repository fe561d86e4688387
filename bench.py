#!/usr/bin/env python3
"""Benchmark of the batched Gaussian-splatting RGB-D sensor renderer on one MI355X.

Workload (one step): 64 environments, each a room-sized background of 100k-1M Gaussians
(log-uniform) plus 4 posed object nodes of 20k Gaussians, SH degree 3, seen by a head and a
wrist camera at 320x240 -- 128 RGB-D frames, 9.83 Mpixels per step.  Object poses are
redrawn every step (a fresh pose set is copied into the pose buffer before the step's graph
launch).  Inputs are seeded and synthetic (the paper's scanned scenes stand in by shape).

Printed (one JSON line on stdout):
  value            batched RGB-D Mpixels/s (one hipGraph launch per step), inputs resident
  gate             sampled pixels of images of the last timed step against the FP64 oracle,
                   and the device status after every timed pose set
  persistent       the same step with the persistent compositor
  per_camera_loop  the same frames rendered by one eager call per (env, camera)
  fwd_bwd_ms_per_view   forward + L1 loss + backward, 500k Gaussians SH3, 8 views 640x480,
                   divided by 8
  configs          the plain (20k, 128x128), single-background (1M, 640x480) and composed
                   (2M + 8 x 50k, 3 x 640x480) workloads, timed the same way
  roofline         the step's dominant kernel against its bound (work model: roofline())
  cpu_baseline     the CPU oracle on the same workload (all envs within its time budget),
                   with its algorithmic Gaussian-pixel evaluation count
Progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# VALU: 256 CUs x 64 lanes x 2.4 GHz = 39,322 G lane-operations per second (no packed FP32)
PEAK_VALU_GOPS = 256 * 64 * 2.4
# VALU lane-operations any implementation needs to decide whether a Gaussian reaches a pixel:
# dx, dy (2), the quadratic form (2 multiplies, 3 fused multiply-adds) and the threshold
# compare (1).  A lower bound on the work of one Gaussian-pixel evaluation.
OPS_PER_EVAL = 8


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--envs", type=int, default=64)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--loop-steps", type=int, default=2)
    ap.add_argument("--fwdbwd-steps", type=int, default=5)
    ap.add_argument("--no-loop", action="store_true")
    ap.add_argument("--no-fwdbwd", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-gate", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--no-augment", action="store_true")
    ap.add_argument("--no-mesh", action="store_true")
    ap.add_argument("--no-lidar", action="store_true")
    ap.add_argument("--lidar-only", action="store_true", help="only the LiDAR workload (for profiling it alone)")
    ap.add_argument("--config-steps", type=int, default=10)
    ap.add_argument("--cpu-budget", type=float, default=30.0, help="seconds of oracle work at most")
    ap.add_argument("--fwdbwd-only", action="store_true",
                    help="only the differentiable workload (for profiling it alone); prints its record")
    ap.add_argument("--tile", default="auto", help="auto (autotuner) or WxH")
    ap.add_argument("--ppt", type=int, default=0, help="pixels per compositor lane with --tile (1, 2, 4)")
    ap.add_argument("--groups", type=int, default=0,
                    help="stream groups of the batched render (default: the autotuner's, 1 with --tile)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device (calibrates HBM traffic counters) and exit")
    return ap.parse_args()


def upload_nodes(nodes, dev):
    import numpy as np
    import torch
    out = []
    for nd in nodes:
        out.append({k: torch.from_numpy(np.ascontiguousarray(nd[k])).to(dev)
                    for k in ("means", "scales", "quats", "opacities", "sh")})
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: renders on one GPU; --gpus {args.gpus} is not supported "
              "(environments would shard across GPUs with no exchange between them)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * 2 ** 20 // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)
        return

    import paper_2507_21981_amd as gsr
    import synth

    if args.fwdbwd_only:
        print(json.dumps({"fwd_bwd": fwd_bwd(gsr, args)}), flush=True)
        return
    if args.lidar_only:
        print(json.dumps({"lidar": lidar_run(gsr, args)}), flush=True)
        return
    dev = "cuda"
    torch.cuda.init()
    t0 = time.time()
    wl = synth.scene_config(3, seed=args.seed, n_envs=args.envs)
    E, C, W, H = len(wl["envs"]), wl["cams_per_env"], wl["width"], wl["height"]
    n_total = sum(len(n["means"]) for e in wl["envs"] for n in e["nodes"])
    log(f"[bench] generated {E} envs, {n_total} Gaussians in {time.time() - t0:.1f}s")
    envs_t = [upload_nodes(e["nodes"], dev) for e in wl["envs"]]
    poses0 = [p for e in wl["envs"] for p in e["poses"]]
    poses = gsr.poses_tensor(poses0, dev)
    cams = gsr.cameras_tensor([c for e in wl["envs"] for c in e["cams"]], dev)
    # per-step object poses: fresh random SE(3) for every object node, background identity
    S = max(args.steps, 1) + args.warmup
    pose_np, pose_sets = [], []
    for s in range(min(S, 32)):
        ps = []
        for e in range(E):
            R, t = synth.object_poses(4, 100000 + 977 * s + e)
            ps += [poses0[e * 5]] + [(R[k], t[k]) for k in range(4)]
        pose_np.append(ps)
        pose_sets.append(gsr.poses_tensor(ps, dev))
    torch.cuda.synchronize()
    log(f"[bench] uploaded in {time.time() - t0:.1f}s")

    ctx = gsr.create(0)
    scene = gsr.compose_scene(ctx, envs_t, poses)
    if args.tile == "auto":
        (tw, th), pers = gsr.autotune(ctx, scene, cams, W, H)
    else:
        tw, th = (int(v) for v in args.tile.split("x"))
        pers = False
        ctx.set_tile(tw, th)
        if args.ppt:
            ctx.set_pixels_per_thread(args.ppt)
    if args.groups:
        ctx.set_stream_groups(args.groups)
    groups = ctx.config.stream_groups
    log(f"[bench] tile {tw}x{th} persistent={pers} stream groups {groups}")
    fl_pers = gsr.FLAG_PERSISTENT if pers else 0
    rgb, depth, alpha = gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=gsr.FLAG_CHECK | fl_pers)
    out = (rgb, depth, alpha)
    ms = timed_graph(gsr, ctx, scene, cams, W, H, C, out, poses, pose_sets, fl_pers, args)
    st = gsr.query_status(ctx)
    px_step = E * C * W * H
    value = px_step / (ms * 1e-3) / 1e6
    log(f"[bench] batched: {ms:.3f} ms/step, {value:.1f} Mpx/s, pairs {st['pairs']}")
    # correctness gate on what was timed: the device status after each timed pose set, then
    # sampled pixels of images of the last timed step against the FP64 oracle
    gate = None if args.no_gate else timed_gate(gsr, ctx, scene, cams, wl, out, poses, pose_sets, pose_np, fl_pers,
                                                (tw, th), args)
    if gate is not None:
        log(f"[bench] gate: {gate}")
    # the other compositor (persistent or one block per tile), same graph protocol
    other = {}
    if not args.no_variants:
        fl_o = 0 if pers else gsr.FLAG_PERSISTENT
        ms_o = timed_graph(gsr, ctx, scene, cams, W, H, C, out, poses, pose_sets, fl_o, args)
        other = {"persistent" if not pers else "one_block_per_tile":
                 {"ms_per_step": round(ms_o, 4), "value": round(px_step / (ms_o * 1e-3) / 1e6, 2)}}
        if groups > 1:  # the same graph protocol on one stream group
            ctx.set_stream_groups(1)
            ms_1 = timed_graph(gsr, ctx, scene, cams, W, H, C, out, poses, pose_sets, fl_pers, args)
            ctx.set_stream_groups(groups)
            other["one_stream_group"] = {"ms_per_step": round(ms_1, 4), "value": round(px_step / (ms_1 * 1e-3) / 1e6, 2)}
        log(f"[bench] variants: {other}")

    # per-stage durations (eager, HIP events between stages on the render stream; a timed render
    # keeps to one stream group) (the same kernels as the graph; evaluations are counted by a
    # checked render of each pose set)
    stage = {k: 0.0 for k in gsr.STAGES}
    n_t = max(1, min(args.steps, 5))
    evals = 0
    for s in range(n_t):
        poses.copy_(pose_sets[(args.warmup + s) % len(pose_sets)])
        gsr.render_rgbd(ctx, scene, cams, W, H, C, out=out, flags=gsr.FLAG_TIMING | fl_pers)
        for k, v in gsr.stage_times(ctx).items():
            stage[k] += v / n_t
        gsr.render_rgbd(ctx, scene, cams, W, H, C, out=out, flags=gsr.FLAG_CHECK | fl_pers)
        evals += gsr.query_status(ctx)["evals"]
    st_t = dict(gsr.query_status(ctx))
    st_t["evals"] = evals // n_t
    st_t["items"] = C * n_total
    st_t["tiles_per_image"] = ((W + tw - 1) // tw) * ((H + th - 1) // th)
    st_t["tiles"] = E * C * st_t["tiles_per_image"]
    log("[bench] stage ms: " + ", ".join(f"{k} {v:.3f}" for k, v in stage.items()))
    ppt = ctx.config.pixels_per_thread
    copy_gbs = copy_peak()
    log(f"[bench] device copy: {copy_gbs} GB/s")
    roof = roofline(stage, st_t, n_total, (tw, th, ppt, pers), copy_gbs)

    aug = None if args.no_augment else augment_run(gsr, ctx, scene, cams, wl, out, poses, pose_sets, fl_pers, args)
    if aug is not None:
        log(f"[bench] augmentation: {aug}")

    # per-camera loop on the same frames
    loop = None
    if not args.no_loop:
        loop = per_camera_loop(gsr, ctx, envs_t, wl, pose_sets, cams, args)
        log(f"[bench] per-camera loop: {loop}")
    ctx.close()

    fwdbwd = None
    if not args.no_fwdbwd:
        fwdbwd = fwd_bwd(gsr, args)
        log(f"[bench] fwd+bwd: {fwdbwd}")

    configs = None
    if not args.no_configs:
        configs = config_runs(gsr, args)
        log(f"[bench] configs: {configs}")

    lidar = None if args.no_lidar else lidar_run(gsr, args)
    if lidar is not None:
        log(f"[bench] lidar: {lidar}")

    mesh = None if args.no_mesh else mesh_run(gsr)
    if mesh is not None:
        log(f"[bench] mesh transfer: {mesh}")

    cpu = None
    algo_evals = None
    if not args.no_cpu:
        # the oracle renders the first timed pose set (poses of the graph's first timed step)
        wl_cpu = with_poses(wl, pose_np[args.warmup % len(pose_np)])
        cpu, algo_evals = cpu_baseline(wl_cpu, tw, th, args.cpu_budget)
        log(f"[bench] cpu baseline: {cpu}")

    line = {
        "metric": "RGB-D Mpixels/s batched vs per-camera at <=1e-4 err; fwd+bwd ms per 640x480 view",
        "value": round(value, 2),
        "unit": "Mpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded; stands in for the paper's scanned scenes)",
        "config": {"workload": f"batched: {E} envs x {C} cams 320x240 RGB-D, background 100k-1M Gaussians "
                               f"(log-uniform) + 4 posed objects x 20k, SH3, fresh object poses per step",
                   "gaussians": n_total, "images": E * C, "pixels_per_step": px_step, "tile": f"{tw}x{th}",
                   "pixels_per_lane": ppt, "persistent": bool(pers), "stream_groups": groups, "hipgraph": True,
                   "seed": args.seed},
        "gate": gate,
        "compositor_variant": other or None,
        "gaussian_pixel_evals_per_s": evals_rates(st_t["evals"], algo_evals, stage["composite"]),
        "evals_per_step": {"executed": st_t["evals"], "algorithmic": algo_evals},
        "pairs_per_step": st_t["pairs"],
        "stage_ms": {k: round(v, 4) for k, v in stage.items()},
        "augmentation": aug,
        "per_camera_loop": loop,
        "batched_over_loop": round(value / loop["value"], 2) if loop else None,
        "fwd_bwd_ms_per_view": fwdbwd["ms_per_view"] if fwdbwd else None,
        "fwd_bwd": fwdbwd,
        "configs": configs,
        "lidar": lidar,
        "mesh_to_gaussians": mesh,
        "parity": "pixels within 1e-4 of the FP64 oracle and keys/ranges bit-exact; gradients within 1e-5 rel-L2: "
                  "tests/test_gpu_forward.py, tests/test_gpu_fullsize.py, tests/test_gpu_backward.py; this run: gate",
        "roofline": roof,
        "cpu_baseline": cpu,
        "context": "paper: 650 FPS RGB-D 640x480 total over 5 cameras on RTX 6000 Ada (whole simulator), "
                   "i.e. ~200 Mpixels/s; not the same workload or hardware",
    }
    print(json.dumps(line), flush=True)


def with_poses(wl, pose_list):
    """The workload with its node poses replaced (env-major list of (R, t))."""
    envs = []
    k = 0
    for e in wl["envs"]:
        n = len(e["nodes"])
        envs.append(dict(e, poses=list(pose_list[k:k + n])))
        k += n
    return dict(wl, envs=envs)


def timed_graph(gsr, ctx, scene, cams, W, H, C, out, poses, pose_sets, flags, args):
    """Warm up (captures the graph), then time args.steps graph launches, each after copying
    a fresh pose set into the pose buffer; returns ms per step."""
    import torch
    for s in range(args.warmup):
        poses.copy_(pose_sets[s % len(pose_sets)])
        gsr.render_rgbd(ctx, scene, cams, W, H, C, out=out, flags=gsr.FLAG_GRAPH | flags)
    torch.cuda.synchronize()
    if gsr.query_status(ctx)["flags"]:
        # grow capacity (the pair count varies with the poses) and capture again
        for ps in pose_sets:
            poses.copy_(ps)
            gsr.render_rgbd(ctx, scene, cams, W, H, C, out=out, flags=gsr.FLAG_CHECK | flags)
        gsr.render_rgbd(ctx, scene, cams, W, H, C, out=out, flags=gsr.FLAG_GRAPH | flags)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for s in range(args.steps):
        poses.copy_(pose_sets[(args.warmup + s) % len(pose_sets)])
        gsr.render_rgbd(ctx, scene, cams, W, H, C, out=out, flags=gsr.FLAG_GRAPH | flags)
    ev1.record()
    torch.cuda.synchronize()
    st = gsr.query_status(ctx)
    if st["flags"]:
        raise SystemExit(f"bench: device status {st} after the timed region (capacity overflow)")
    return ev0.elapsed_time(ev1) / max(args.steps, 1)


def timed_gate(gsr, ctx, scene, cams, wl, out, poses, pose_sets, pose_np, flags, tile, args, sample=1500):
    """Replay the graph once per pose set the timed region used, reading the device status
    after each (an overflowed step would have been timed with dropped tiles); then compare
    sampled pixels of three images of the last timed step with the FP64 oracle (a pixel passes
    within 1e-4 of the oracle, or of its flipped branch where a blending decision lies within
    the FP32 bound of its threshold)."""
    import numpy as np
    import torch

    import oracle
    E, C, W, H = len(wl["envs"]), wl["cams_per_env"], wl["width"], wl["height"]
    used = sorted({(args.warmup + s) % len(pose_sets) for s in range(args.steps)})
    bad_status = []
    for i in used:
        poses.copy_(pose_sets[i])
        gsr.render_rgbd(ctx, scene, cams, W, H, C, out=out, flags=gsr.FLAG_GRAPH | flags)
        st = gsr.query_status(ctx)
        if st["flags"]:
            bad_status.append(i)
    last = (args.warmup + args.steps - 1) % len(pose_sets)
    poses.copy_(pose_sets[last])
    gsr.render_rgbd(ctx, scene, cams, W, H, C, out=out, flags=gsr.FLAG_GRAPH | flags)
    torch.cuda.synchronize()
    rgb, depth, alpha = (t.cpu().numpy() for t in out)
    wl_last = with_poses(wl, pose_np[last])
    tw, th = tile
    images = [(0, 0), (E // 2, C - 1), (E - 1, 0)]
    res = dict(pose_sets_checked=len(used), status_failures=len(bad_status), images=[], pixels=0, ambiguous=0,
               excluded=0, max_err=0.0, failures=0)
    gid = np.cumsum([0] + [sum(len(n["means"]) for n in e["nodes"]) for e in wl["envs"]])
    for e, c in images:
        env = wl_last["envs"][e]
        cam = env["cams"][c]
        fe = oracle.FlatEnv(env)
        rect, zb, vis = oracle.keyspec(fe, cam, W, H, tw, th)
        geo = oracle.project(fe, cam, W, H)
        _, _, lv, ranges = oracle.pairs(rect, zb, vis, W, H, tw, th, image=e * C + c, gid_base=int(gid[e]))
        pix = np.sort(np.random.default_rng(1000 + e * C + c).choice(W * H, size=sample, replace=False))
        ref = oracle.composite_sample(geo, ranges, lv, W, H, tw, th, cam["bg"], pix)
        got = np.concatenate([rgb[e, c].reshape(-1, 3)[pix], depth[e, c].reshape(-1, 1)[pix],
                              alpha[e, c].reshape(-1, 1)[pix]], axis=1).astype(np.float64)
        want = np.concatenate([ref["rgb"], ref["depth"][:, None], ref["alpha"][:, None]], axis=1)
        err = np.abs(got - want).max(axis=1)
        err_alt = np.abs(got - ref["alt"]).max(axis=1)
        amb = (ref["flags"] & 1) != 0
        exc = (ref["flags"] & 2) != 0
        ok = (err <= 1e-4) | (amb & (err_alt <= 1e-4)) | exc
        res["images"].append(e * C + c)
        res["pixels"] += int(pix.size)
        res["ambiguous"] += int(amb.sum())
        res["excluded"] += int(exc.sum())
        res["failures"] += int((~ok).sum())
        res["max_err"] = max(res["max_err"], float(err[~amb & ~exc].max()) if (~amb & ~exc).any() else 0.0)
    res["max_err"] = float(f"{res['max_err']:.3g}")
    res["pass"] = res["failures"] == 0 and res["status_failures"] == 0
    return res


def augment_run(gsr, ctx, scene, cams, wl, out, poses, pose_sets, flags, args, reps=20):
    """Image-space domain randomisation of the step's frames (overlay, HSV jitter, gamma):
    fused into the compositor's epilogue (the step's graph with the augmentation bound), and
    as a separate pass over finished frames, which is HBM-bound: 12 B of rgb and 12 B of
    overlay read and 12 B written per pixel."""
    import torch

    import synth
    E, C, W, H = len(wl["envs"]), wl["cams_per_env"], wl["width"], wl["height"]
    ov = torch.from_numpy(synth.overlay_frames(E * C, H, W, 77)).cuda().reshape(E, C, H, W, 3).contiguous()
    params = gsr.augment_tensor(synth.augment_params(E * C, 78))
    gsr.set_augment(ctx, params, ov)
    ms_fused = timed_graph(gsr, ctx, scene, cams, W, H, C, out, poses, pose_sets, flags | gsr.FLAG_AUGMENT, args)
    dst = torch.empty_like(out[0])
    gsr.augment_rgb(ctx, out[0], params, ov, out=dst)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        gsr.augment_rgb(ctx, out[0], params, ov, out=dst)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    px = E * C * W * H
    gbs = 36 * px / (ms * 1e-3) / 1e9
    return {"fused_ms_per_step": round(ms_fused, 4), "separate_pass_ms": round(ms, 4),
            "separate_pass": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                              "frac": round(gbs / PEAK_HBM_GBS, 4), "algorithmic_bytes": 36 * px}}


def lidar_run(gsr, args, reps=10):
    """LiDAR by Gaussian ray tracing on the composed workload (2M background + 8 x 50k posed
    objects, SH3), one spinning sensor of 64 beams (elevations -15..15 degrees) x 2048 azimuths
    at the head camera's position, fresh object poses per frame (written in place; the per-node
    hierarchies are not rebuilt).  Work floor: every blended hit's 64 B primitive read once."""
    import torch

    import synth
    wl = synth.scene_config(2, seed=args.seed)
    env = wl["envs"][0]
    rays = torch.from_numpy(synth.lidar_rays((0.0, 0.6, -1.0), 64, 2048, elevation=(-15, 15), tmin=0.05,
                                             tmax=50.0)).cuda()
    nodes = upload_nodes(env["nodes"], "cuda")
    poses = gsr.poses_tensor(env["poses"])
    sets = []
    for s in range(8):
        R, t = synth.object_poses(8, 300000 + 31 * s)
        sets.append(gsr.poses_tensor([env["poses"][0]] + [(R[k], t[k]) for k in range(8)]))
    small = torch.from_numpy(synth.lidar_rays((0.0, 0.6, -1.0), 32, 1024, elevation=(-15, 15), tmin=0.05,
                                              tmax=50.0)).cuda()
    ctx = gsr.create(0)
    try:
        scene = gsr.compose_scene(ctx, [nodes], poses)
        t0 = time.time()
        gsr.lidar_build(ctx, scene)
        build_s = time.time() - t0

        def timed(rr):
            out = gsr.render_lidar(ctx, scene, rr)
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            ev0.record()
            for i in range(reps):
                poses.copy_(sets[i % len(sets)])
                gsr.render_lidar(ctx, scene, rr, out=out)
            ev1.record()
            torch.cuda.synchronize()
            return ev0.elapsed_time(ev1) / reps, int(out[2].sum())

        ms, hits = timed(rays)
        ms_small, _ = timed(small)
    finally:
        ctx.close()
    n = rays.shape[0]
    b = 64 * hits
    gbs = b / (ms * 1e-3) / 1e9
    return {"workload": "2M background + 8 x 50k posed objects SH3; 64 x 2048 rays from (0, 0.6, -1), fresh poses",
            "rays": n, "ms_per_frame": round(ms, 4), "frames_per_s": round(1e3 / ms, 1),
            "Mrays_per_s": round(n / (ms * 1e-3) / 1e6, 2), "mean_hits": round(hits / n, 2),
            "hierarchy_build_s": round(build_s, 2),
            "sensor_32x1024": {"rays": int(small.shape[0]), "ms_per_frame": round(ms_small, 4),
                               "frames_per_s": round(1e3 / ms_small, 1)},
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(gbs / PEAK_HBM_GBS, 4), "algorithmic_bytes": b,
                         "note": "floor: each blended hit's primitive read once; traversal is latency-bound"}}


def mesh_run(gsr, reps=10):
    """Mesh-to-Gaussian transfer of a 2M-facet sphere mesh with vertex colours (SH degree 0
    output), bound by memory: per facet 12 B of indices read and 56 B of Gaussian written, per
    vertex 24 B (position, colour) read once."""
    import torch

    import synth
    v, f, col = synth.mesh_sphere(1000, 1000, 21, radius=0.2, degenerate=0)
    vd, fd, cd = (torch.from_numpy(x).cuda() for x in (v, f, col))
    ctx = gsr.create(0)
    try:
        gsr.mesh_to_gaussians(ctx, vd, fd, cd)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            gsr.mesh_to_gaussians(ctx, vd, fd, cd)  # synchronous: the events bracket memset, kernel, read-back
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
    finally:
        ctx.close()
    b = 68 * len(f) + 24 * len(v)
    gbs = b / (ms * 1e-3) / 1e9
    return {"faces": int(len(f)), "vertices": int(len(v)), "ms": round(ms, 4),
            "Mfaces_per_s": round(len(f) / (ms * 1e-3) / 1e6, 1),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(gbs / PEAK_HBM_GBS, 4), "algorithmic_bytes": int(b)}}


def copy_peak(mib=1024, reps=10):
    """Measured device-to-device copy rate (GB/s of read + write bytes) of a 1 GiB copy."""
    import torch
    n = mib * 2 ** 20 // 4
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del src, dst
    return round(2 * 4 * n / (ms * 1e-3) / 1e9, 1)


def evals_rates(executed, algorithmic, composite_ms):
    if not composite_ms:
        return None
    t = composite_ms * 1e-3
    return {"algorithmic": round(algorithmic / t, 1) if algorithmic else None, "executed": round(executed / t, 1)}


def config_runs(gsr, args):
    """The plain, single-background and composed workloads: one hipGraph launch per step
    (fresh object poses per step for the composed one), tile shape from the autotuner (16x16
    for the plain workload, as it specifies)."""
    import numpy as np
    import torch

    import synth
    res = {}
    for cfg in (0, 1, 2):
        wl = synth.scene_config(cfg, seed=args.seed)
        E, C, W, H = len(wl["envs"]), wl["cams_per_env"], wl["width"], wl["height"]
        envs_t = [upload_nodes(e["nodes"], "cuda") for e in wl["envs"]]
        base = [p for e in wl["envs"] for p in e["poses"]]
        poses = gsr.poses_tensor(base)
        cams = gsr.cameras_tensor([c for e in wl["envs"] for c in e["cams"]])
        sets = []
        for s in range(8):
            if cfg == 2:
                R, t = synth.object_poses(8, 200000 + 31 * s)
                sets.append(gsr.poses_tensor([base[0]] + [(R[k], t[k]) for k in range(8)]))
            else:
                sets.append(poses.clone())
        ctx = gsr.create(0)
        try:
            scene = gsr.compose_scene(ctx, envs_t, poses)
            if cfg == 0:
                tw, th, pers = 16, 16, False
            else:
                (tw, th), pers = gsr.autotune(ctx, scene, cams, W, H)
            fl = gsr.FLAG_PERSISTENT if pers else 0
            for ps in sets:  # capacity for every pose set
                poses.copy_(ps)
                out = gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=gsr.FLAG_CHECK | fl)
            a = argparse.Namespace(warmup=2, steps=max(5, args.config_steps))
            ms = timed_graph(gsr, ctx, scene, cams, W, H, C, out, poses, sets, fl, a)
            st = gsr.query_status(ctx)
            px = E * C * W * H
            res[f"workload_{cfg}"] = {"workload": synth.CONFIG_NAMES[cfg], "ms_per_step": round(ms, 4),
                                      "Mpixels_per_s": round(px / (ms * 1e-3) / 1e6, 2), "tile": f"{tw}x{th}",
                                      "persistent": bool(pers), "pairs": st["pairs"], "visible": st["visible"]}
        finally:
            ctx.close()
        del envs_t
        torch.cuda.empty_cache()
    return res


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "hbm_traffic_batched_64envs_320x240.json")


def measured_traffic():
    """Per-kernel HBM bytes per dispatch from the committed counter runs, or None when the
    kernel sources have changed since those counters were taken."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
        h = hashlib.sha256()
        root = os.path.dirname(os.path.abspath(__file__))
        for src in rec["sources"]:
            h.update(open(os.path.join(root, src), "rb").read())
    except (OSError, ValueError, KeyError):
        return None
    return rec["kernels"] if h.hexdigest() == rec["sources_sha256"] else None


def roofline(stage, st, n_total, cfg, copy_gbs):
    """Dominant kernel of the step against its bound (unit counts from device counters).

    Algorithmic bytes per unit (the job's, independent of this implementation):
      projection     12 B per Gaussian (position, for the visibility cull) + 224 B per
                     Gaussian visible from some camera (the rest of its SH3 parameters)
                     + 52 B per visible (image, Gaussian) projected record + 8 B per
                     (image, Gaussian) item (count and offset)
      whole forward before compositing (projection, sort, emission, ranges): the above
                     + 12 B per pair (emission) + 24 B per pair per sort pass + 8 B per tile,
                     with one pass (the floor) and with ceil(key bits / 8) = 6 passes
      compositor     OPS_PER_EVAL VALU lane-operations per Gaussian-pixel evaluation
    The implementation's own bytes (what its kernels must move) are reported beside them:
    projection 44 B per Gaussian + 12 K B of SH per Gaussian visible from some camera + 64 B
    written per visible (image, Gaussian) (48 B record, 16 B list entry); depth sort: the 16 B
    list entry copied into the image's segment, then four radix passes each reading the 4 B
    key (histogram) and moving the 8 B (key, source position) (the first reads the key alone;
    the last reads the pair and the 12 B id and rectangle of its source and writes those 12 B);
    emission: the 8 B rectangle read three times (chunking, counts) and the 12 B (rectangle,
    id) once, 4 B written per pair.  A stage whose counter traffic is below its bytes kept its
    working set in the 256 MB last-level cache (flagged "mall_resident").
    """
    K = 16
    visible, visible_any, pairs, evals = st["visible"], st["visible_any"], st["pairs"], st["evals"]
    items, tiles = st["items"], st["tiles"]
    alg_project = 12 * n_total + 224 * visible_any + 52 * visible + 8 * items
    own = {
        "project": ("hbm", 44 * n_total + 12 * K * visible_any + 64 * visible),
        "sort": ("hbm", (32 + (4 + 4 + 8) + 2 * (4 + 8 + 8) + (4 + 8 + 12 + 12)) * visible),
        "emit": ("hbm", 3 * 8 * visible + 12 * visible + 4 * pairs),
        "composite": ("alu", evals * OPS_PER_EVAL),
    }
    times = {"project": stage["project"], "sort": stage["gather"] + stage["depth_sort"],
             "emit": stage["chunks"] + stage["tile_counts"] + stage["tile_ranges"] + stage["emit"],
             "composite": stage["composite"]}
    tw, th, ppt, pers = cfg
    # kernel names as the profiler prints them, without the parameter list; the timed region
    # composites without evaluation counting
    kname = {"project": ["k_project<3>"],
             "emit": ["k_pair_blocks", "k_pair_scan", "k_chunk_starts", "k_tile_counts", "k_tile_seg", "k_tile_ranges",
                      f"k_emit<{16 if 12 * st['tiles_per_image'] > 8192 else 4}>"],
             "composite": [f"k_composite{'_persistent' if pers else ''}<{tw}, {th}, {ppt}, false, false>"]}
    traffic = measured_traffic()
    if traffic is not None:
        traffic = {n.split("(")[0]: v for n, v in traffic.items()}

    def kernel_traffic(k):
        if traffic is None:
            return None
        names = kname[k] if k in kname else [n for n in traffic if n.startswith(("k_radix", "k_gather", "k_seg"))]
        if not names or any(n not in traffic for n in names):
            return None
        return sum(traffic[n]["fetch_bytes"] + traffic[n]["write_bytes"] for n in names)

    units = {"gaussians": n_total, "visible_any": visible_any, "visible_records": visible, "items": items,
             "pairs": pairs, "tiles": tiles, "evals": evals}
    # the dominant single kernel (the sort and emission stages are several launches)
    dom = max(("project", "composite"), key=times.get)
    t = times[dom] * 1e-3
    if dom == "project":
        ach = alg_project / t / 1e9
        tr = kernel_traffic("project")
        r = {"kernel": kname["project"][0], "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
             "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": tr, "algorithmic_bytes": int(alg_project),
             "bytes_per_unit": {"gaussian": 12, "visible_any": 224, "visible_record": 52, "item": 8},
             "copy_peak_GBs": copy_gbs, "frac_of_copy_peak": round(ach / copy_gbs, 4) if copy_gbs else None,
             "own_model": {"algorithmic_bytes": int(own["project"][1]),
                           "GB/s": round(own["project"][1] / t / 1e9, 1),
                           "frac": round(own["project"][1] / t / 1e9 / PEAK_HBM_GBS, 4)}}
    else:
        amount = own["composite"][1]
        ach = amount / t / 1e9
        r = {"kernel": kname["composite"][0], "bound": "alu", "achieved": round(ach, 1), "peak": round(PEAK_VALU_GOPS, 1),
             "unit": "Gop/s (VALU lane-ops)", "frac": round(ach / PEAK_VALU_GOPS, 4),
             "traffic": kernel_traffic("composite"), "evals": int(evals), "ops_per_eval": OPS_PER_EVAL}
    r["kernel_ms"] = round(times[dom], 4)
    r["units"] = units
    r["others"] = {}
    for k in times:
        if k == dom or times[k] <= 0:
            continue
        tk = times[k] * 1e-3
        tr = kernel_traffic(k)
        o = {"ms": round(times[k], 4), "traffic": tr}
        if k == "project":
            o.update({"bound": "hbm", "algorithmic_bytes": int(alg_project), "GB/s": round(alg_project / tk / 1e9, 1),
                      "frac": round(alg_project / tk / 1e9 / PEAK_HBM_GBS, 4)})
        elif k == "composite":
            amt = own["composite"][1]
            o.update({"bound": "alu", "Gop/s": round(amt / tk / 1e9, 1), "frac": round(amt / tk / 1e9 / PEAK_VALU_GOPS, 4)})
        else:
            amt = own[k][1]
            o.update({"bound": "hbm", "own_bytes": int(amt), "GB/s": round(amt / tk / 1e9, 1),
                      "frac": round(amt / tk / 1e9 / PEAK_HBM_GBS, 4)})
            if tr is not None:
                o["mall_resident"] = tr < amt
        r["others"][k] = o
    tp = (times["project"] + times["emit"] + times["sort"]) * 1e-3
    fwd = {}
    for passes in (1, 6):
        b = alg_project + 12 * pairs + 24 * pairs * passes + 8 * tiles
        fwd[f"passes_{passes}"] = {"algorithmic_bytes": int(b), "GB/s": round(b / tp / 1e9, 1),
                                   "frac": round(b / tp / 1e9 / PEAK_HBM_GBS, 4)}
    fwd["ms"] = round(tp * 1e3, 4)
    r["project_sort_emit"] = fwd
    return r


def per_camera_loop(gsr, ctx, envs_t, wl, pose_sets, cams, args):
    import torch
    E, C, W, H = len(wl["envs"]), wl["cams_per_env"], wl["width"], wl["height"]
    scenes, env_poses = [], []
    for e in range(E):
        pe = pose_sets[0][e * 5:(e + 1) * 5].clone()
        env_poses.append(pe)
        scenes.append(gsr.compose_scene(ctx, [envs_t[e]], pe))
    outs = [(torch.empty((1, 1, H, W, 3), device="cuda"), torch.empty((1, 1, H, W), device="cuda"),
             torch.empty((1, 1, H, W), device="cuda")) for _ in range(E * C)]
    cam_rows = [cams[i:i + 1].clone() for i in range(E * C)]

    def step(s):
        ps = pose_sets[s % len(pose_sets)]
        for e in range(E):
            env_poses[e].copy_(ps[e * 5:(e + 1) * 5])
            for c in range(C):
                gsr.render_rgbd(ctx, scenes[e], cam_rows[e * C + c], W, H, 1, out=outs[e * C + c], flags=0)

    # warm-up with capacity check
    for e in range(E):
        for c in range(C):
            gsr.render_rgbd(ctx, scenes[e], cam_rows[e * C + c], W, H, 1, out=outs[e * C + c], flags=gsr.FLAG_CHECK)
    step(1)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    n = max(1, args.loop_steps)
    for s in range(n):
        step(2 + s)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / n
    st = gsr.query_status(ctx)
    assert st["flags"] == 0, st
    px = E * C * W * H
    return {"value": round(px / (ms * 1e-3) / 1e6, 2), "unit": "Mpixels/s", "ms_per_step": round(ms, 3),
            "calls_per_step": E * C}


def fwd_bwd(gsr, args):
    """500k Gaussians (cube geometry, SH3), 8 ring views at 640x480; L1 loss against targets
    rendered from a perturbed copy (means + N(0, 0.01^2), log-scales + N(0, 0.1^2))."""
    import numpy as np
    import torch

    import synth
    wl = synth.scene_config(4, seed=args.seed + 4)
    env = wl["envs"][0]
    nd = env["nodes"][0]
    g = synth.rng(args.seed + 44)
    pert = dict(nd)
    pert["means"] = (nd["means"] + 0.01 * g.standard_normal(nd["means"].shape, dtype=np.float32)).astype(np.float32)
    pert["scales"] = (nd["scales"] * np.exp(0.1 * g.standard_normal(nd["scales"].shape, dtype=np.float32))).astype(np.float32)
    ctx = gsr.create(0)
    try:
        poses = gsr.poses_tensor(env["poses"])
        cams = gsr.cameras_tensor(env["cams"])
        tgt_scene = gsr.compose_scene(ctx, [upload_nodes([pert], "cuda")], poses)
        target, _, _ = gsr.render_rgbd(ctx, tgt_scene, cams, 640, 480)
        target = target.clone()
        tgt_scene.close()
        node = upload_nodes([nd], "cuda")[0]
        scene = gsr.compose_scene(ctx, [[node]], poses)
        grads = [{k: torch.zeros_like(node[k]) for k in node}]
        n_el = target.numel()

        def step():
            rgb, depth, alpha = gsr.render_rgbd(ctx, scene, cams, 640, 480, flags=gsr.FLAG_SAVE)
            d_rgb = torch.sign(rgb - target) / n_el  # d mean|rgb - target| / d rgb
            for gg in grads[0].values():
                gg.zero_()
            gsr.render_backward(ctx, scene, d_rgb.contiguous(), grads=grads)
            return rgb

        gsr.render_rgbd(ctx, scene, cams, 640, 480, flags=gsr.FLAG_CHECK | gsr.FLAG_SAVE)
        step()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        n = max(1, args.fwdbwd_steps)
        for _ in range(n):
            step()
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / n
        # forward alone (same flags), for the split
        ev0.record()
        for _ in range(n):
            gsr.render_rgbd(ctx, scene, cams, 640, 480, flags=gsr.FLAG_SAVE)
        ev1.record()
        torch.cuda.synchronize()
        ms_fwd = ev0.elapsed_time(ev1) / n
        st = gsr.query_status(ctx)
        assert st["flags"] == 0, st
        gn = {k: float(v.norm()) for k, v in grads[0].items()}
        return {"ms_per_step": round(ms, 3), "views": 8, "ms_per_view": round(ms / 8, 3),
                "forward_ms_per_step": round(ms_fwd, 3), "pairs_per_step": st["pairs"],
                "workload": "500k Gaussians SH3, 8 views 640x480, L1 loss, grads for means/scales/quats/opacities/sh",
                "grad_norms": gn}
    finally:
        ctx.close()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, tw, th, budget_s=30.0):
    """The FP64 CPU oracle, timed on the host, on full frames of the workload's envs in order
    until every env is done or ``budget_s`` seconds have passed.  Also returns the oracle's
    algorithmic Gaussian-pixel evaluation count (per pixel, the entries of its tile's list up
    to and including its stopping one), for the whole step when every env was rendered."""
    import oracle
    W, H, C = wl["width"], wl["height"], wl["cams_per_env"]
    t0 = time.time()
    px = n_envs = evals = 0
    for env in wl["envs"]:
        fe = oracle.FlatEnv(env)
        for cam in env["cams"]:
            r = oracle.render(env, cam, W, H, tw, th, fe=fe)
            evals += int(r["evals"].sum())
            px += W * H
        n_envs += 1
        if time.time() - t0 >= budget_s:
            break
    dt = time.time() - t0
    complete = n_envs == len(wl["envs"])
    return ({"value": round(px / dt / 1e6, 4), "unit": "Mpixels/s", "cores": oracle.num_threads(), "kind": "oracle",
             "cpu_model": cpu_model(), "evals_per_s": round(evals / dt, 1),
             "sample": f"{'all' if complete else 'first'} {n_envs} of {len(wl['envs'])} envs x {C} cams, full "
                       f"{W}x{H} frames ({px} pixels) of the first timed step's poses, projection + key sort + FP64 "
                       f"compositing, {dt:.1f} s"},
            evals if complete else None)


if __name__ == "__main__":
    main()
