"""The no-allocation backward entry point (gsr_render_backward_noalloc) against the
allocating one (gsr_render_backward), through the C ABI: two calls in a row on one context,
the second with a smaller saved render, so that what the first left in the shared static
scratch cannot leak into the second; and a render too large for the scratch is refused
before any launch."""
import math

import numpy as np
import pytest

import synth
from gpu_util import log, upload
from test_gpu_backward import GROUPS, _compare

pytestmark = pytest.mark.gpu


def _workload(n_bg, n_obj, n_cams, W, H, seed):
    bg = synth.gaussians_uniform_cube(n_bg, seed, sh_degree=3)
    ob = synth.gaussians_object(n_obj, seed + 1, sh_degree=3, radius=0.3, log_scale=(-3.5, 0.3))
    R = synth.random_rotation(synth.rng(seed + 2)).astype(np.float32)
    cams = []
    for k in range(n_cams):
        a = 2 * math.pi * k / n_cams
        cams.append(synth.camera((3 * math.sin(a), 0.2, -3 * math.cos(a)), (0, 0, 0), W, H))
    env = dict(nodes=[bg, ob], poses=[(np.eye(3, dtype=np.float32), np.zeros(3, np.float32)),
                                      (R, np.array([0.2, -0.1, 0.1], np.float32))], cams=cams)
    return dict(envs=[env], cams_per_env=n_cams, width=W, height=H)


def _both(gsr, ctx, wl, seed):
    import torch
    envs_t, poses, cams = upload(wl)
    scene = gsr.compose_scene(ctx, envs_t, poses)
    E, C, W, H = 1, wl["cams_per_env"], wl["width"], wl["height"]
    gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=gsr.FLAG_CHECK | gsr.FLAG_SAVE)
    g = np.random.default_rng(seed)
    d_rgb = torch.tensor(g.standard_normal((E, C, H, W, 3)), dtype=torch.float32, device="cuda")
    d_depth = torch.tensor(g.standard_normal((E, C, H, W)), dtype=torch.float32, device="cuda")
    d_alpha = torch.tensor(g.standard_normal((E, C, H, W)), dtype=torch.float32, device="cuda")
    zeros = lambda: [{k: torch.zeros_like(n[k]) for k in GROUPS} for n in scene.nodes]
    ref, got = zeros(), zeros()
    p_ref = torch.zeros((len(scene.nodes), 6), device="cuda")
    p_got = torch.zeros_like(p_ref)
    gsr.render_backward(ctx, scene, d_rgb, d_depth, d_alpha, grads=ref, d_poses=p_ref)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    gsr.render_backward(ctx, scene, d_rgb, d_depth, d_alpha, grads=got, d_poses=p_got, noalloc=True)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, f"device memory changed by {free0 - free1} bytes"
    for a, b, pa, pb in zip(ref, got, p_ref, p_got):
        a["pose"], b["pose"] = pa, pb
    return _compare(got, ref, groups=GROUPS + ("pose",))


def test_noalloc_backward_matches_the_allocating_one_twice():
    import paper_2507_21981_amd as gsr
    ctx = gsr.create(0)
    try:
        ctx.set_tile(16, 16)
        log("large", _both(gsr, ctx, _workload(30000, 3000, 4, 160, 120, 91), 1))
        log("smaller", _both(gsr, ctx, _workload(6000, 800, 2, 96, 64, 93), 2))
    finally:
        ctx.close()


def test_noalloc_backward_refuses_a_render_beyond_its_scratch():
    import torch
    import paper_2507_21981_amd as gsr
    ctx = gsr.create(0)
    try:
        wl = _workload(800000, 10, 8, 64, 48, 95)  # 8 x 800k records x 48 B > 256 MiB
        envs_t, poses, cams = upload(wl)
        scene = gsr.compose_scene(ctx, envs_t, poses)
        gsr.render_rgbd(ctx, scene, cams, 64, 48, 8, flags=gsr.FLAG_CHECK | gsr.FLAG_SAVE)
        d_rgb = torch.ones((1, 8, 48, 64, 3), device="cuda")
        grads = [{k: torch.zeros_like(n[k]) for k in GROUPS} for n in scene.nodes]
        with pytest.raises(gsr.GsrError) as e:
            gsr.render_backward(ctx, scene, d_rgb, grads=grads, noalloc=True)
        assert e.value.code == -4 and "scratch" in str(e.value)
        torch.cuda.synchronize()
        assert all(float(g[k].abs().sum()) == 0.0 for g in grads for k in GROUPS)
    finally:
        ctx.close()
