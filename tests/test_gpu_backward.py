"""GPU backward parity: FP32 gradients against the FP64 oracle's analytic gradient.

The oracle's analytic gradient is itself pinned to FP64 central finite differences
(tests/test_oracle_pins.py).  Tolerances, per parameter group (means, scales, quaternions,
opacities, SH, node poses): relative L2 error <= 1e-5 and max-abs error <= 3e-5 * max|g|.
The paper states none; the worst measured values over these tests (every tile shape, up to
the full 500k-Gaussian 8-view workload) are 4.2e-6 and 1.5e-5.  The record gradients are summed
by float atomics in no fixed order, so the worst single element moves from run to run; the
bounds sit about 2x above the worst seen (and far below the 1e-4 / 1e-3 first proposed for
this comparison).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import log, upload

pytestmark = pytest.mark.gpu

REL_L2 = 1e-5
MAX_ABS = 3e-5
GROUPS = ("means", "scales", "quats", "opacities", "sh")


@pytest.fixture(scope="module")
def gsr():
    import paper_2507_21981_amd as g
    g.lib()
    return g


@pytest.fixture(scope="module")
def ctx(gsr):
    c = gsr.create(0)
    yield c
    c.close()


def _oracle_grads(wl, weights, tw, th):
    """Sum over every image of the oracle's analytic gradient of sum(w . outputs), per node,
    with the node-pose gradient (omega, rho) under "pose"."""
    W, H = wl["width"], wl["height"]
    out = []
    image = 0
    for env in wl["envs"]:
        fe = oracle.FlatEnv(env)
        acc = None
        for cam in env["cams"]:
            ref = oracle.render(env, cam, W, H, tw, th, fe=fe)
            wr, wd, wa = weights[image]
            g = oracle.backward(ref, cam, W, H, wr, wd, wa, tw, th)
            if acc is None:
                acc = {k: g[k].copy() for k in GROUPS + ("pose",)}
            else:
                for k in acc:
                    acc[k] += g[k]
            image += 1
        # split the env's concatenation back into nodes
        off = 0
        for j, n in enumerate(env["nodes"]):
            m = len(n["means"])
            d = {k: acc[k][off:off + m] for k in GROUPS}
            d["pose"] = acc["pose"][j]
            out.append(d)
            off += m
    return out


def _np(x):
    """float64 numpy copy of a tensor (any device) or array, flattened"""
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    return np.asarray(x, np.float64).reshape(-1)


def _compare(gpu_grads, ref_grads, rel_l2=REL_L2, max_abs=MAX_ABS, groups=GROUPS):
    """Per parameter group: relative L2 error and max-abs error over max |g| (both asserted)."""
    worst = {}
    for k in groups:
        g = np.concatenate([_np(gg[k]) for gg in gpu_grads])
        r = np.concatenate([_np(rr[k]) for rr in ref_grads])
        nr = np.linalg.norm(r)
        rel = np.linalg.norm(g - r) / max(nr, 1e-30)
        mx = np.abs(g - r).max() / max(np.abs(r).max(), 1e-30)
        worst[k] = (float(f"{rel:.3g}"), float(f"{mx:.3g}"))
        assert rel <= rel_l2 and mx <= max_abs, f"{k}: rel L2 {rel:.3g}, max-abs/max {mx:.3g}"
    return worst


def _weights(wl, seed):
    g = np.random.default_rng(seed)
    W, H = wl["width"], wl["height"]
    n = len(wl["envs"]) * wl["cams_per_env"]
    return [(g.standard_normal((H, W, 3)), g.standard_normal((H, W)), g.standard_normal((H, W))) for _ in range(n)]


def _gpu_grads(gsr, ctx, wl, weights, tile):
    import torch
    ctx.set_tile(*tile)
    envs_t, poses, cams = upload(wl)
    scene = gsr.compose_scene(ctx, envs_t, poses)
    E, C, W, H = len(wl["envs"]), wl["cams_per_env"], wl["width"], wl["height"]
    gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=gsr.FLAG_CHECK | gsr.FLAG_SAVE)
    wr = torch.tensor(np.stack([w[0] for w in weights]).reshape(E, C, H, W, 3), dtype=torch.float32, device="cuda")
    wd = torch.tensor(np.stack([w[1] for w in weights]).reshape(E, C, H, W), dtype=torch.float32, device="cuda")
    wa = torch.tensor(np.stack([w[2] for w in weights]).reshape(E, C, H, W), dtype=torch.float32, device="cuda")
    d_poses = torch.zeros((len(scene.nodes), 6), dtype=torch.float32, device="cuda")
    grads = gsr.render_backward(ctx, scene, wr, wd, wa, d_poses=d_poses)
    torch.cuda.synchronize()
    for g, p in zip(grads, d_poses.cpu().numpy().astype(np.float64)):
        g["pose"] = p
    return grads


def test_gradients_small_posed_scene(gsr, ctx):
    # background + posed SH3 object, two cameras
    bg = synth.gaussians_uniform_cube(300, 41, sh_degree=3, half=0.6, log_scale=(-2.6, 0.3), hi_sigma=0.1)
    ob = synth.gaussians_object(80, 42, sh_degree=3, radius=0.3, log_scale=(-2.8, 0.3), hi_sigma=0.1)
    R = synth.random_rotation(synth.rng(43)).astype(np.float32)
    env = dict(nodes=[bg, ob], poses=[(np.eye(3, dtype=np.float32), np.zeros(3, np.float32)),
                                      (R, np.array([0.1, 0.05, -0.2], np.float32))],
               cams=[synth.camera((0.2, 0.3, -2.2), (0, 0, 0), 48, 40, bg=(0.2, 0.1, 0.3)),
                     synth.camera((-0.4, 0.1, -2.0), (0, 0, 0), 48, 40, bg=(0.0, 0.3, 0.1))])
    wl = dict(envs=[env], cams_per_env=2, width=48, height=40)
    w = _weights(wl, 1)
    ref = _oracle_grads(wl, w, 16, 16)
    got = _gpu_grads(gsr, ctx, wl, w, (16, 16))
    log("worst", _compare(got, ref, groups=GROUPS + ("pose",)))


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 8), (32, 8)])
def test_gradients_differentiable_subset(gsr, ctx, tile):
    # the differentiable workload's finite-difference subset: 2,000 Gaussians (cube geometry,
    # SH3) seen from two ring views at 64x64 (fx = 55.43)
    nd = synth.gaussians_uniform_cube(2000, 51, sh_degree=3)
    cams = []
    for k in (0, 4):
        a = 2 * math.pi * k / 8
        cams.append(synth.camera((3 * math.sin(a), 0.0, -3 * math.cos(a)), (0, 0, 0), 64, 64))
    env = dict(nodes=[nd], poses=[(np.eye(3, dtype=np.float32), np.zeros(3, np.float32))], cams=cams)
    wl = dict(envs=[env], cams_per_env=2, width=64, height=64)
    w = _weights(wl, 2)
    ref = _oracle_grads(wl, w, *tile)
    got = _gpu_grads(gsr, ctx, wl, w, tile)
    log("worst", _compare(got, ref))


def test_gradients_with_partial_saturation(gsr, ctx):
    """Three near splats of opacity 0.99 saturate part of the image in front of 3000 splats:
    the pixels' contributor counts differ widely within a tile, so the backward culls each
    batch against the box of the pixels whose counts reach into it."""
    from helpers import cam_identity, env_of, node
    wall = node([[-0.35, 0.0, 1.0], [-0.35, 0.0, 1.05], [-0.35, 0.0, 1.1]], 0.25, opac=0.99,
                colours=[(0.9, 0.1, 0.1), (0.1, 0.9, 0.1), (0.1, 0.1, 0.9)])
    back = synth.gaussians_uniform_cube(3000, 5)
    back["sh"] = back["sh"][:, :1]
    eye = np.eye(3, dtype=np.float32)
    env = env_of([wall, back], poses=[(eye, np.zeros(3, np.float32)), (eye, np.array([0, 0, 4], np.float32))])
    env["cams"] = [cam_identity(64, 64, 64.0)]
    wl = dict(envs=[env], cams_per_env=1, width=64, height=64)
    w = _weights(wl, 3)
    ref = _oracle_grads(wl, w, 16, 16)
    got = _gpu_grads(gsr, ctx, wl, w, (16, 16))
    log("worst", _compare(got, ref))


def test_gradients_batched_envs(gsr, ctx):
    wl = synth.scene_config(3, seed=61, scale=0.004, n_envs=3)
    for env in wl["envs"]:
        for c in env["cams"]:
            c["fx"] = c["fy"] = np.float32(c["fx"] * 0.25)
            c["cx"], c["cy"] = np.float32(40), np.float32(30)
    wl["width"], wl["height"] = 80, 60
    w = _weights(wl, 3)
    ref = _oracle_grads(wl, w, 16, 8)
    got = _gpu_grads(gsr, ctx, wl, w, (16, 8))
    log("worst", _compare(got, ref, groups=GROUPS + ("pose",)))


def test_autograd_function_l1_loss(gsr, ctx):
    import torch
    nd = synth.gaussians_uniform_cube(1500, 71, sh_degree=1)
    cam = synth.camera((0.3, 0.2, -3.0), (0, 0, 0), 48, 48)
    R = synth.random_rotation(synth.rng(72)).astype(np.float32)
    env = dict(nodes=[nd], poses=[(R, np.array([0.05, -0.1, 0.2], np.float32))], cams=[cam])
    wl = dict(envs=[env], cams_per_env=1, width=48, height=48)
    envs_t, poses, cams = upload(wl)
    ctx.set_tile(16, 16)
    params = [envs_t[0][0][k].clone().requires_grad_(True) for k in ("means", "scales", "quats", "opacities", "sh")]
    node = dict(zip(("means", "scales", "quats", "opacities", "sh"), params))
    scene = gsr.compose_scene(ctx, [[node]], poses)
    target = torch.rand((1, 1, 48, 48, 3), device="cuda")
    tangent = torch.zeros((1, 6), device="cuda", requires_grad=True)
    rgb, depth, alpha = gsr.RenderRGBD.apply(ctx, scene, cams, 48, 48, tangent, *params)
    loss = (rgb - target).abs().mean() + 0.1 * depth.mean()
    loss.backward()
    # oracle: d loss / d rgb = sign(rgb - target) / n, d loss / d depth = 0.1 / n
    ref = oracle.render(env, cam, 48, 48)
    gr = np.sign(ref["rgb"] - target[0, 0].cpu().numpy().astype(np.float64)) / (48 * 48 * 3)
    gd = np.full((48, 48), 0.1 / (48 * 48))
    og = oracle.backward(ref, cam, 48, 48, gr, gd, None)
    got = [dict(means=params[0].grad, scales=params[1].grad, quats=params[2].grad, opacities=params[3].grad,
                sh=params[4].grad, pose=tangent.grad[0])]
    want = [{k: og[k] for k in ("means", "scales", "quats", "opacities", "sh")}]
    want[0]["pose"] = og["pose"][0]
    log("worst", _compare(got, want, groups=GROUPS + ("pose",)))


def test_backward_of_a_replaced_render_is_refused(gsr, ctx):
    """Two differentiable renders on one context, then the earlier one's backward: its saved
    state is gone, so the call fails before any launch instead of pairing its upstream
    gradients with the later render's pairs; upstream gradients of the wrong shape are
    refused too."""
    import torch
    nd = synth.gaussians_uniform_cube(400, 81)
    cam = synth.camera((0.0, 0.0, -3.0), (0, 0, 0), 32, 32)
    env = dict(nodes=[nd], poses=[(np.eye(3, dtype=np.float32), np.zeros(3, np.float32))], cams=[cam])
    wl = dict(envs=[env], cams_per_env=1, width=32, height=32)
    envs_t, poses, cams = upload(wl)
    ctx.set_tile(16, 16)
    params = [envs_t[0][0][k].clone().requires_grad_(True) for k in ("means", "scales", "quats", "opacities", "sh")]
    scene = gsr.compose_scene(ctx, [[dict(zip(("means", "scales", "quats", "opacities", "sh"), params))]], poses)
    rgb1, _, _ = gsr.RenderRGBD.apply(ctx, scene, cams, 32, 32, None, *params)
    rgb2, _, _ = gsr.RenderRGBD.apply(ctx, scene, cams, 32, 32, None, *params)
    rgb2.sum().backward()  # the saved render: fine
    g_ok = params[0].grad.clone()
    with pytest.raises(gsr.GsrError) as e:
        rgb1.sum().backward()
    assert e.value.code == -6
    torch.cuda.synchronize()
    assert torch.equal(params[0].grad, g_ok)  # nothing was accumulated by the refused call
    gsr.render_rgbd(ctx, scene, cams, 32, 32, flags=gsr.FLAG_CHECK | gsr.FLAG_SAVE)
    with pytest.raises(ValueError):
        gsr.render_backward(ctx, scene, torch.zeros((1, 1, 16, 16, 3), device="cuda"))


def test_gradients_differentiable_500k_8views_sampled_pixels(gsr):
    """The differentiable workload at full size, in the benchmark's launch configuration
    (500k Gaussians SH3, 8 ring views 640x480, 16x16 tiles, two pixels per lane): upstream
    gradients on 2,000 seeded pixels per view (N(0, 1) for rgb, depth and alpha), zero at
    pixels where the oracle finds a blending decision within the FP32 bound of its threshold
    (there two results are correct).  The oracle differentiates those pixels one by one."""
    import torch
    wl = synth.scene_config(4, seed=4)
    env = wl["envs"][0]
    W, H, tw, th = 640, 480, 16, 16
    fe = oracle.FlatEnv(env)
    g = np.random.default_rng(11)
    C = len(env["cams"])
    d_rgb = np.zeros((1, C, H, W, 3), np.float32)
    d_depth = np.zeros((1, C, H, W), np.float32)
    d_alpha = np.zeros((1, C, H, W), np.float32)
    acc = None
    for v, cam in enumerate(env["cams"]):
        log(f"oracle view {v}")
        rect, zb, vis = oracle.keyspec(fe, cam, W, H, tw, th)
        geo = oracle.project(fe, cam, W, H)
        _, _, lv, ranges = oracle.pairs(rect, zb, vis, W, H, tw, th)
        pix = np.sort(g.choice(W * H, size=2000, replace=False))
        fwd = oracle.composite_sample(geo, ranges, lv, W, H, tw, th, cam["bg"], pix)
        clean = (fwd["flags"] == 0).astype(np.float64)
        gr = g.standard_normal((pix.size, 3)).astype(np.float32).astype(np.float64) * clean[:, None]
        gd = g.standard_normal(pix.size).astype(np.float32).astype(np.float64) * clean
        ga = g.standard_normal(pix.size).astype(np.float32).astype(np.float64) * clean
        d_rgb[0, v].reshape(-1, 3)[pix] = gr
        d_depth[0, v].reshape(-1)[pix] = gd
        d_alpha[0, v].reshape(-1)[pix] = ga
        ref = dict(fe=fe, ranges=ranges, lvals=lv, geo=geo)
        og = oracle.backward_sample(ref, cam, W, H, pix, gr, gd, ga, tw, th)
        log(f"  pairs {len(lv)}, ambiguous sampled pixels {int(pix.size - clean.sum())}")
        if acc is None:
            acc = {k: og[k].copy() for k in GROUPS + ("pose",)}
        else:
            for k in acc:
                acc[k] += og[k]
    ctx = gsr.create(0, tile=(tw, th))
    try:
        ctx.set_pixels_per_thread(2)
        envs_t, poses, cams = upload(wl)
        scene = gsr.compose_scene(ctx, envs_t, poses)
        gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=gsr.FLAG_CHECK | gsr.FLAG_SAVE)
        d_poses = torch.zeros((1, 6), device="cuda")
        grads = gsr.render_backward(ctx, scene, torch.from_numpy(d_rgb).cuda(), torch.from_numpy(d_depth).cuda(),
                                    torch.from_numpy(d_alpha).cuda(), d_poses=d_poses)
        torch.cuda.synchronize()
        grads[0]["pose"] = d_poses[0]
        ref = {k: acc[k] for k in GROUPS}
        ref["pose"] = acc["pose"][0]
        log("worst", _compare(grads, [ref], groups=GROUPS + ("pose",)))
    finally:
        ctx.close()
