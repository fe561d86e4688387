"""Helpers for the GPU parity tests: upload seeded scenes, run the oracle per image, compare.

The oracle is the CPU reference; the GPU path is the library under test.  Both read the same
seeded inputs from synth/; no expected value comes from the GPU.
"""
import sys

import numpy as np

import oracle

# pixel tolerance (max-abs per channel, FP32 GPU vs FP64 oracle)
TOL = 1e-4
# Caps on the pixels the near-threshold rule touches, as fractions of the compared pixels: a
# pixel is ambiguous when one of its blending decisions lies within the oracle's derived FP32
# error bound of its threshold (either branch is then correct), excluded when two do.  With
# the bound, the workloads give 0.5-2.7 % ambiguous and at most 0.05 % excluded pixels.
MAX_AMBIGUOUS = 0.05
MAX_EXCLUDED = 0.002


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def upload(workload, device="cuda"):
    import torch
    import paper_2507_21981_amd as gsr  # noqa: F401
    envs_t, poses = [], []
    for env in workload["envs"]:
        nodes = []
        for nd in env["nodes"]:
            n = len(nd["means"])
            K = nd["sh"].shape[1]
            nodes.append(dict(
                means=torch.from_numpy(np.ascontiguousarray(nd["means"], np.float32)).to(device),
                scales=torch.from_numpy(np.ascontiguousarray(nd["scales"], np.float32)).to(device),
                quats=torch.from_numpy(np.ascontiguousarray(nd["quats"], np.float32)).to(device),
                opacities=torch.from_numpy(np.ascontiguousarray(nd["opacities"], np.float32)).to(device),
                sh=torch.from_numpy(np.ascontiguousarray(nd["sh"], np.float32).reshape(n, K, 3)).to(device)))
        envs_t.append(nodes)
        poses += list(env["poses"])
    cams = [c for env in workload["envs"] for c in env["cams"]]
    return envs_t, gsr.poses_tensor(poses, device), gsr.cameras_tensor(cams, device)


def render_gpu(ctx, workload, flags=None, device="cuda"):
    import paper_2507_21981_amd as gsr
    envs_t, poses, cams = upload(workload, device)
    scene = gsr.compose_scene(ctx, envs_t, poses)
    fl = gsr.FLAG_CHECK if flags is None else flags
    rgb, depth, alpha = gsr.render_rgbd(ctx, scene, cams, workload["width"], workload["height"],
                                        cams_per_env=workload["cams_per_env"], flags=fl)
    import torch
    torch.cuda.synchronize()
    return scene, cams, rgb, depth, alpha


def oracle_images(workload, tw, th, full=True, sample=None, seed=0):
    """Per image (env-major, camera-minor): oracle keys/values/ranges and pixels.

    full=True composites every pixel; else ``sample`` pixels per image (seeded)."""
    W, H = workload["width"], workload["height"]
    out = []
    gid_base = 0
    image = 0
    for env in workload["envs"]:
        fe = oracle.FlatEnv(env)
        for cam in env["cams"]:
            rect, zb, vis = oracle.keyspec(fe, cam, W, H, tw, th)
            geo = oracle.project(fe, cam, W, H)
            keys, vals, lv, ranges = oracle.pairs(rect, zb, vis, W, H, tw, th, image=image, gid_base=gid_base)
            rec = dict(keys=keys, vals=vals, ranges=ranges, vis=vis)
            if full:
                rec.update(oracle.composite(geo, ranges, lv, W, H, tw, th, cam["bg"]))
                rec["pix"] = None
            else:
                g = np.random.default_rng(seed + image)
                pix = np.sort(g.choice(W * H, size=min(sample, W * H), replace=False))
                r = oracle.composite_sample(geo, ranges, lv, W, H, tw, th, cam["bg"], pix)
                r["pix"] = pix
                rec.update(r)
            out.append(rec)
            image += 1
        gid_base += fe.n
    return out


def compare_image(ref, rgb, depth, alpha, tol=TOL, depth_tol=None):
    """Check one GPU image (numpy [H,W,3], [H,W], [H,W]) against the oracle record.

    A pixel passes if rgb, depth and alpha are all within tol of the oracle, or -- when the
    oracle flags a decision within its margin of a threshold -- within tol of the oracle's
    flipped-branch result.  Pixels with two or more near-threshold decisions are excluded and
    counted.  Returns a stats dict; raises AssertionError on failure.
    """
    dt = tol if depth_tol is None else depth_tol
    if ref["pix"] is not None:
        rgb = rgb.reshape(-1, 3)[ref["pix"]]
        depth = depth.reshape(-1)[ref["pix"]]
        alpha = alpha.reshape(-1)[ref["pix"]]
        ref_rgb, ref_d, ref_a, flags, alt = ref["rgb"], ref["depth"], ref["alpha"], ref["flags"], ref["alt"]
    else:
        ref_rgb = ref["rgb"].reshape(-1, 3)
        ref_d, ref_a = ref["depth"].reshape(-1), ref["alpha"].reshape(-1)
        flags, alt = ref["flags"].reshape(-1), ref["alt"].reshape(-1, 5)
        rgb, depth, alpha = rgb.reshape(-1, 3), depth.reshape(-1), alpha.reshape(-1)
    e_main = np.maximum(np.abs(rgb - ref_rgb).max(axis=1), np.maximum(np.abs(alpha - ref_a), np.abs(depth - ref_d) * tol / dt))
    e_alt = np.maximum(np.abs(rgb - alt[:, :3]).max(axis=1),
                       np.maximum(np.abs(alpha - alt[:, 4]), np.abs(depth - alt[:, 3]) * tol / dt))
    excluded = (flags & 2) != 0
    ok = (e_main <= tol) | (((flags & 1) != 0) & (e_alt <= tol)) | excluded
    stats = dict(pixels=int(e_main.size), max_err=float(e_main[~excluded].max()) if (~excluded).any() else 0.0,
                 ambiguous=int(((flags & 1) != 0).sum()), used_alt=int((((flags & 1) != 0) & (e_main > tol)).sum()),
                 excluded=int(excluded.sum()), bad=int((~ok).sum()))
    assert stats["ambiguous"] <= MAX_AMBIGUOUS * stats["pixels"] + 2, f"too many ambiguous pixels: {stats}"
    assert stats["excluded"] <= MAX_EXCLUDED * stats["pixels"] + 1, f"too many excluded pixels: {stats}"
    if stats["bad"]:
        i = np.argmax(np.where(ok, 0, e_main))
        raise AssertionError(f"{stats}; worst pixel {i}: gpu rgb {rgb[i]} d {depth[i]} a {alpha[i]} / oracle rgb "
                             f"{ref_rgb[i]} d {ref_d[i]} a {ref_a[i]} flags {flags[i]}")
    return stats


def check_keys(refs, keys, vals, ranges, tiles_per_image):
    """Bit-exact: sorted keys, values and per-tile ranges of every image."""
    keys = keys.astype(np.uint64)
    vals = vals.astype(np.uint32)
    ranges = ranges.astype(np.int64)
    base = 0
    for i, r in enumerate(refs):
        n = len(r["keys"])
        assert np.array_equal(keys[base:base + n], r["keys"]), f"image {i}: keys differ"
        assert np.array_equal(vals[base:base + n], r["vals"]), f"image {i}: values differ"
        rr = ranges[i * tiles_per_image:(i + 1) * tiles_per_image] - base
        assert np.array_equal(rr, r["ranges"]), f"image {i}: ranges differ"
        base += n
    assert base == len(keys), "pair count differs"
