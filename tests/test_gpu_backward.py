"""GPU backward parity: FP32 gradients against the FP64 oracle's analytic gradient.

The oracle's analytic gradient is itself pinned to FP64 central finite differences
(tests/test_oracle_pins.py).  Tolerances (no value is stated by the paper): per parameter
group, relative L2 error <= 2e-3 and max-abs error <= 2e-3 * max|g|; FP32 compositing
recomputes transmittance by division back to front, which costs a few digits.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import log, upload

pytestmark = pytest.mark.gpu

REL_L2 = 2e-3
MAX_ABS = 2e-3


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
    """Sum over every image of the oracle's analytic gradient of sum(w . outputs)."""
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
                acc = {k: g[k].copy() for k in ("means", "scales", "quats", "opacities", "sh")}
            else:
                for k in acc:
                    acc[k] += g[k]
            image += 1
        # split the env's concatenation back into nodes
        off = 0
        for n in env["nodes"]:
            m = len(n["means"])
            out.append({k: v[off:off + m] for k, v in acc.items()})
            off += m
    return out


def _compare(gpu_grads, ref_grads):
    worst = {}
    for k in ("means", "scales", "quats", "opacities", "sh"):
        g = np.concatenate([gg[k].detach().cpu().numpy().reshape(-1) for gg in gpu_grads])
        r = np.concatenate([rr[k].reshape(-1) for rr in ref_grads])
        nr = np.linalg.norm(r)
        rel = np.linalg.norm(g - r) / max(nr, 1e-30)
        mx = np.abs(g - r).max() / max(np.abs(r).max(), 1e-30)
        worst[k] = (rel, mx)
        assert rel <= REL_L2 and mx <= MAX_ABS, f"{k}: rel L2 {rel:.3g}, max-abs/max {mx:.3g}"
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
    grads = gsr.render_backward(ctx, scene, wr, wd, wa)
    torch.cuda.synchronize()
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
    log("worst", _compare(got, ref))


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
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
    log("worst", _compare(got, ref))


def test_autograd_function_l1_loss(gsr, ctx):
    import torch
    nd = synth.gaussians_uniform_cube(1500, 71, sh_degree=1)
    cam = synth.camera((0.3, 0.2, -3.0), (0, 0, 0), 48, 48)
    env = dict(nodes=[nd], poses=[(np.eye(3, dtype=np.float32), np.zeros(3, np.float32))], cams=[cam])
    wl = dict(envs=[env], cams_per_env=1, width=48, height=48)
    envs_t, poses, cams = upload(wl)
    ctx.set_tile(16, 16)
    params = [envs_t[0][0][k].clone().requires_grad_(True) for k in ("means", "scales", "quats", "opacities", "sh")]
    node = dict(zip(("means", "scales", "quats", "opacities", "sh"), params))
    scene = gsr.compose_scene(ctx, [[node]], poses)
    target = torch.rand((1, 1, 48, 48, 3), device="cuda")
    rgb, depth, alpha = gsr.RenderRGBD.apply(ctx, scene, cams, 48, 48, *params)
    loss = (rgb - target).abs().mean() + 0.1 * depth.mean()
    loss.backward()
    # oracle: d loss / d rgb = sign(rgb - target) / n, d loss / d depth = 0.1 / n
    ref = oracle.render(env, cam, 48, 48)
    gr = np.sign(ref["rgb"] - target[0, 0].cpu().numpy().astype(np.float64)) / (48 * 48 * 3)
    gd = np.full((48, 48), 0.1 / (48 * 48))
    og = oracle.backward(ref, cam, 48, 48, gr, gd, None)
    got = [dict(means=params[0].grad, scales=params[1].grad, quats=params[2].grad, opacities=params[3].grad,
                sh=params[4].grad)]
    want = [{k: og[k] for k in ("means", "scales", "quats", "opacities", "sh")}]
    log("worst", _compare(got, want))
