"""GPU parity at the workloads' full sizes, in the launch configuration the benchmark times.

Keys (tile, z bits), values (ids) and per-tile ranges are compared bit for bit for selected
images; pixels are compared on a seeded sample (the FP64 oracle composites those pixels one
by one) under the near-threshold rule.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import compare_image, log, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gsr():
    import paper_2507_21981_amd as g
    g.lib()
    return g


def _oracle_image(env, cam, W, H, tw, th, image, gid_base, sample, seed):
    fe = oracle.FlatEnv(env)
    rect, zb, vis = oracle.keyspec(fe, cam, W, H, tw, th)
    geo = oracle.project(fe, cam, W, H)
    keys, vals, lv, ranges = oracle.pairs(rect, zb, vis, W, H, tw, th, image=image, gid_base=gid_base)
    pix = np.sort(np.random.default_rng(seed).choice(W * H, size=sample, replace=False))
    r = oracle.composite_sample(geo, ranges, lv, W, H, tw, th, cam["bg"], pix)
    r.update(keys=keys, vals=vals, ranges=ranges, pix=pix)
    return r


def _check(gsr, ctx, wl, images, tw, th, out, sample=3000):
    """Compare the listed (env, cam) images of a rendered workload with the oracle."""
    rgb, depth, alpha = (t.cpu().numpy() for t in out)
    W, H, C = wl["width"], wl["height"], wl["cams_per_env"]
    tpi = ((W + tw - 1) // tw) * ((H + th - 1) // th)
    E = len(wl["envs"])
    keys, vals, ranges = gsr.copy_pairs(ctx, E * C * tpi)
    ranges = ranges.cpu().numpy().view(np.uint32).astype(np.int64)
    gid_base = np.cumsum([0] + [sum(len(n["means"]) for n in e["nodes"]) for e in wl["envs"]])
    for e, c in images:
        img = e * C + c
        log(f"oracle env {e} cam {c}")
        ref = _oracle_image(wl["envs"][e], wl["envs"][e]["cams"][c], W, H, tw, th, img, int(gid_base[e]), sample,
                            seed=img)
        r0, r1 = ranges[img * tpi, 0], ranges[(img + 1) * tpi - 1, 1]
        gk = keys[r0:r1].cpu().numpy().view(np.uint64)
        gv = vals[r0:r1].cpu().numpy().view(np.uint32)
        assert np.array_equal(gk, ref["keys"]) and np.array_equal(gv, ref["vals"]), f"image {img}: keys differ"
        assert np.array_equal(ranges[img * tpi:(img + 1) * tpi] - r0, ref["ranges"]), f"image {img}: ranges differ"
        st = compare_image(ref, rgb[e, c], depth[e, c], alpha[e, c])
        log(f"image {img}: pairs {len(gk)}, {st}")


def test_single_background_1m_sh3_640x480(gsr):
    ctx = gsr.create(0)
    try:
        wl = synth.scene_config(1, seed=0)
        envs_t, poses, cams = upload(wl)
        scene = gsr.compose_scene(ctx, envs_t, poses)
        out = gsr.render_rgbd(ctx, scene, cams, 640, 480, 1, flags=gsr.FLAG_CHECK)
        _check(gsr, ctx, wl, [(0, 0)], 16, 16, out)
    finally:
        ctx.close()


def test_composed_step_2m_plus_8_objects_3_cams(gsr):
    ctx = gsr.create(0, tile=(16, 8))
    try:
        wl = synth.scene_config(2, seed=0)
        envs_t, poses, cams = upload(wl)
        scene = gsr.compose_scene(ctx, envs_t, poses)
        out = gsr.render_rgbd(ctx, scene, cams, 640, 480, 3, flags=gsr.FLAG_CHECK)
        _check(gsr, ctx, wl, [(0, 0), (0, 1), (0, 2)], 16, 8, out)
    finally:
        ctx.close()


@pytest.mark.parametrize("ppt", [1, 2])
@pytest.mark.parametrize("persistent", [False, True])
def test_batched_64_envs_in_the_benchmark_configuration(gsr, persistent, ppt):
    """64 envs x 2 cams, one hipGraph launch, 16x16 tiles, one or two pixels per lane (the
    autotuner's choices for this workload), persistent or one block per tile."""
    import torch
    ctx = gsr.create(0, tile=(16, 16))
    try:
        ctx.set_pixels_per_thread(ppt)
        wl = synth.scene_config(3, seed=0)
        envs_t, poses, cams = upload(wl)
        scene = gsr.compose_scene(ctx, envs_t, poses)
        fl = gsr.FLAG_PERSISTENT if persistent else 0
        out = gsr.render_rgbd(ctx, scene, cams, 320, 240, 2, flags=gsr.FLAG_CHECK | fl)
        out = tuple(torch.full_like(t, -1.0) for t in out)
        for _ in range(2):
            gsr.render_rgbd(ctx, scene, cams, 320, 240, 2, out=out, flags=gsr.FLAG_GRAPH | fl)
        torch.cuda.synchronize()
        assert gsr.query_status(ctx)["flags"] == 0
        _check(gsr, ctx, wl, [(0, 0), (0, 1), (37, 0), (63, 1)], 16, 16, out, sample=2000)
    finally:
        ctx.close()


def test_differentiable_500k_one_view(gsr):
    ctx = gsr.create(0)
    try:
        wl = synth.scene_config(4, seed=0)
        env = wl["envs"][0]
        env["cams"] = env["cams"][:2]
        wl["cams_per_env"] = 2
        envs_t, poses, cams = upload(wl)
        scene = gsr.compose_scene(ctx, envs_t, poses)
        out = gsr.render_rgbd(ctx, scene, cams, 640, 480, 2, flags=gsr.FLAG_CHECK | gsr.FLAG_SAVE)
        _check(gsr, ctx, wl, [(0, 1)], 16, 16, out)
    finally:
        ctx.close()
