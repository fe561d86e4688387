"""GPU parity of the LiDAR ray tracer (paper Sec. III-C) against the brute-force FP64 oracle.

Per ray: alpha within 1e-4 and range within 1e-4 (1 + range) of the oracle (the range is a
sum of alpha T t over hits metres away, so its FP32 error scales with it); where the oracle
finds a decision within its FP32 bound of a threshold, either branch passes (two such
decisions: excluded and counted); blended-hit counts must match wherever no decision is
ambiguous."""
import math

import numpy as np
import pytest

import synth
from gpu_util import log, upload
from oracle import lidar as L

pytestmark = pytest.mark.gpu
TOL = 1e-4


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


def _compare(ref, rng, alpha, hits):
    rng, alpha = rng.astype(np.float64), alpha.astype(np.float64)
    e_main = np.maximum(np.abs(alpha - ref["alpha"]), np.abs(rng - ref["range"]) / (1 + np.abs(ref["range"])))
    e_alt = np.maximum(np.abs(alpha - ref["alt"][:, 1]), np.abs(rng - ref["alt"][:, 0]) / (1 + np.abs(ref["alt"][:, 0])))
    amb = (ref["flags"] & 1) != 0
    exc = (ref["flags"] & 2) != 0
    ok = (e_main <= TOL) | (amb & (e_alt <= TOL)) | exc
    clean = ~amb & ~exc
    hit_ok = (hits == ref["hits"]) | ~clean
    st = dict(rays=len(rng), with_hits=int((ref["hits"] > 0).sum()), max_err=float(e_main[clean].max()) if clean.any()
              else 0.0, ambiguous=int(amb.sum()), excluded=int(exc.sum()), bad=int((~ok).sum()),
              hit_count_mismatch=int((~hit_ok).sum()))
    assert st["bad"] == 0 and st["hit_count_mismatch"] == 0, st
    assert st["excluded"] <= 0.002 * len(rng) + 1, st
    return st


def _aim(rays, forward, weight):
    rays = rays.copy()
    d = rays[:, 3:6].astype(np.float64) + weight * np.asarray(forward, np.float64)
    rays[:, 3:6] = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    return rays


def _run(gsr, ctx, wl, rays_per_env):
    import torch
    envs_t, poses, _ = upload(wl)
    scene = gsr.compose_scene(ctx, envs_t, poses)
    gsr.lidar_build(ctx, scene)
    rays = np.concatenate(rays_per_env, axis=0)
    out = gsr.render_lidar(ctx, scene, torch.from_numpy(rays).cuda(), rays_per_env=len(rays_per_env[0]))
    torch.cuda.synchronize()
    return scene, [t.cpu().numpy().reshape(-1) for t in out]


def test_small_posed_scene(gsr, ctx):
    bg = synth.gaussians_uniform_cube(3000, 51, sh_degree=1, half=1.0, log_scale=(-2.8, 0.5))
    ob = synth.gaussians_object(600, 52, sh_degree=1, radius=0.25, log_scale=(-3.5, 0.4))
    R = synth.random_rotation(synth.rng(53)).astype(np.float32)
    env = dict(nodes=[bg, ob], poses=[(np.eye(3, dtype=np.float32), np.zeros(3, np.float32)),
                                      (R, np.array([0.1, -0.2, -0.3], np.float32))], cams=[])
    wl = dict(envs=[env], cams_per_env=1, width=8, height=8)
    rays = _aim(synth.lidar_rays((0.0, 0.2, -2.6), 24, 96, elevation=(-25, 25), tmin=0.05, tmax=8.0), (0, 0, 1), 1.5)
    _, (rng, alpha, hits) = _run(gsr, ctx, wl, [rays])
    ref = L.trace(L.WorldEnv(env), rays)
    st = _compare(ref, rng, alpha, hits)
    log("small posed scene", st, "max hits", int(ref["hits"].max()), "max candidates", int(ref["cand"].max()))
    assert st["with_hits"] > 1000


def test_batched_envs_and_pose_updates_without_rebuild(gsr, ctx):
    import torch
    wl = synth.scene_config(3, seed=57, scale=0.01, n_envs=3)
    rays = [_aim(synth.lidar_rays((0.0, 0.4, -1.0), 16, 64, elevation=(-30, 10), tmin=0.05, tmax=12.0), (0, -0.3, 1), 1.0)
            for _ in wl["envs"]]
    envs_t, poses, _ = upload(wl)
    scene = gsr.compose_scene(ctx, envs_t, poses)
    gsr.lidar_build(ctx, scene)
    rt = torch.from_numpy(np.concatenate(rays)).cuda()
    for step in range(2):
        if step == 1:  # new object poses written in place: no rebuild
            for e, env in enumerate(wl["envs"]):
                Rs, ts = synth.object_poses(4, 700 + e)
                env["poses"] = [env["poses"][0]] + [(Rs[k], ts[k]) for k in range(4)]
            poses.copy_(gsr.poses_tensor([p for env in wl["envs"] for p in env["poses"]]))
        rng, alpha, hits = (t.cpu().numpy() for t in gsr.render_lidar(ctx, scene, rt, rays_per_env=len(rays[0])))
        for e, env in enumerate(wl["envs"]):
            ref = L.trace(L.WorldEnv(env), rays[e])
            st = _compare(ref, rng[e], alpha[e], hits[e])
            log(f"step {step} env {e}", st)


def test_wavefronts_spanning_several_envs(gsr, ctx):
    """25 rays per env (an odd count, so with packets of two rays, the size this ray count gets,
    packets at the env boundaries hold rays of two envs, which walk different hierarchies in
    the same wavefront)."""
    import torch
    wl = synth.scene_config(3, seed=59, scale=0.005, n_envs=5)
    rays = [_aim(synth.lidar_rays((0.0, 0.4, -1.0), 5, 5, elevation=(-30, 10), tmin=0.05, tmax=12.0), (0, -0.3, 1),
                 1.0) for _ in wl["envs"]]
    n = len(rays[0])
    _, (rng, alpha, hits) = _run(gsr, ctx, wl, rays)
    for e, env in enumerate(wl["envs"]):
        ref = L.trace(L.WorldEnv(env), rays[e])
        st = _compare(ref, rng[e * n:(e + 1) * n], alpha[e * n:(e + 1) * n], hits[e * n:(e + 1) * n])
        log(f"env {e}", st)


def test_build_required_and_empty_rays(gsr, ctx):
    import torch
    bg = synth.gaussians_uniform_cube(500, 61)
    env = dict(nodes=[bg], poses=[(np.eye(3, dtype=np.float32), np.zeros(3, np.float32))], cams=[])
    envs_t, poses, _ = upload(dict(envs=[env], cams_per_env=1, width=8, height=8))
    scene = gsr.compose_scene(ctx, envs_t, poses)
    rays = torch.from_numpy(synth.lidar_rays((0.0, 0.0, -3.0), 4, 8)).cuda()
    with pytest.raises(gsr.GsrError) as e:
        gsr.render_lidar(ctx, scene, rays)
    assert e.value.code == -6
    gsr.lidar_build(ctx, scene)
    # rays pointing away from the cube, and a window that holds no centre
    away = synth.lidar_rays((0.0, 0.0, -3.0), 4, 8)
    away[:, 3:6] = [0, 0, -1]
    nothing = synth.lidar_rays((0.0, 0.0, -3.0), 4, 8, tmin=0.05, tmax=0.1)
    for r in (away, nothing):
        rng, alpha, hits = gsr.render_lidar(ctx, scene, torch.from_numpy(r).cuda())
        torch.cuda.synchronize()
        assert float(rng.abs().max()) == 0.0 and float(alpha.abs().max()) == 0.0 and int(hits.max()) == 0
    # recomposing invalidates the hierarchy
    scene = gsr.compose_scene(ctx, envs_t, poses, scene=scene)
    with pytest.raises(gsr.GsrError):
        gsr.render_lidar(ctx, scene, rays)


def test_composed_step_full_size_sampled_rays(gsr):
    """The composed workload at full size (2M background + 8 x 50k posed objects, SH3) and the
    benchmark's sensor (64 beams x 2048 azimuths at the head camera's position); the oracle
    traces 300 seeded rays by brute force over all 2.4M Gaussians."""
    import torch
    wl = synth.scene_config(2, seed=0)
    env = wl["envs"][0]
    rays = synth.lidar_rays((0.0, 0.6, -1.0), 64, 2048, elevation=(-15, 15), tmin=0.05, tmax=50.0)
    ctx = gsr.create(0)
    try:
        envs_t, poses, _ = upload(wl)
        scene = gsr.compose_scene(ctx, envs_t, poses)
        gsr.lidar_build(ctx, scene)
        rng, alpha, hits = (t.cpu().numpy().reshape(-1) for t in
                            gsr.render_lidar(ctx, scene, torch.from_numpy(rays).cuda()))
    finally:
        ctx.close()
    pick = np.sort(np.random.default_rng(3).choice(len(rays), 300, replace=False))
    ref = L.trace(L.WorldEnv(env), rays[pick])
    st = _compare(ref, rng[pick], alpha[pick], hits[pick])
    log("full size", st, "mean hits", float(ref["hits"].mean()))


@pytest.mark.parametrize("beams,azimuths", [(35, 2000), (100, 3000), (150, 4000), (270, 4100)])
def test_packet_sizes(gsr, ctx, beams, azimuths):
    """Frames of 70k, 300k, 600k and 1.1M rays, which the tracer packs 4, 16, 32 and 64 rays to
    a wavefront (16, 4, 2 and 1 lanes per ray sharing a leaf's primitive tests), on a small
    posed scene; the oracle traces 150 seeded rays of each frame."""
    import torch
    bg = synth.gaussians_uniform_cube(3000, 71, sh_degree=1, half=1.0, log_scale=(-2.8, 0.5))
    ob = synth.gaussians_object(600, 72, sh_degree=1, radius=0.25, log_scale=(-3.5, 0.4))
    R = synth.random_rotation(synth.rng(73)).astype(np.float32)
    env = dict(nodes=[bg, ob], poses=[(np.eye(3, dtype=np.float32), np.zeros(3, np.float32)),
                                      (R, np.array([0.1, -0.2, -0.3], np.float32))], cams=[])
    wl = dict(envs=[env], cams_per_env=1, width=8, height=8)
    rays = _aim(synth.lidar_rays((0.0, 0.2, -2.6), beams, azimuths, elevation=(-25, 25), tmin=0.05, tmax=8.0),
                (0, 0, 1), 1.5)
    _, (rng, alpha, hits) = _run(gsr, ctx, wl, [rays])
    pick = np.sort(np.random.default_rng(beams).choice(len(rays), 150, replace=False))
    ref = L.trace(L.WorldEnv(env), rays[pick])
    st = _compare(ref, rng[pick], alpha[pick], hits[pick])
    log(f"{len(rays)} rays", st)
    assert st["with_hits"] > 50
