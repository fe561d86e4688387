"""GPU parity of the forward path (keys, ranges, pixels) against the CPU oracle.

Sort keys (tile, z bits) with Gaussian-id values and per-tile ranges must match the
oracle's FP32 key specification bit for bit; pixels (rgb, depth, alpha) must be within 1e-4
of the FP64 oracle, where a pixel whose blending decision sits within the oracle's margin of
a threshold may instead match the oracle's flipped branch (paper Sec. III-A renderer,
Sec. III-C RGB-D sensor).
"""
import numpy as np
import pytest

import synth
from gpu_util import TOL, check_keys, compare_image, log, oracle_images, render_gpu, upload

pytestmark = pytest.mark.gpu


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


def _run(gsr, ctx, wl, tile=(16, 16), full=True, sample=2000, depth_tol=None, flags=None):
    import torch
    ctx.set_tile(*tile)
    log(f"render {wl.get('name', '')} tile {tile}")
    scene, cams, rgb, depth, alpha = render_gpu(ctx, wl, flags=flags)
    st = gsr.query_status(ctx)
    assert st["flags"] == 0, st
    W, H = wl["width"], wl["height"]
    tw, th = tile
    tpi = ((W + tw - 1) // tw) * ((H + th - 1) // th)
    images = len(wl["envs"]) * wl["cams_per_env"]
    keys, vals, ranges = gsr.copy_pairs(ctx, images * tpi)
    log("oracle")
    refs = oracle_images(wl, tw, th, full=full, sample=sample)
    check_keys(refs, keys.cpu().numpy().view(np.uint64), vals.cpu().numpy().view(np.uint32),
               ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), tpi)
    rgb_n, d_n, a_n = rgb.cpu().numpy(), depth.cpu().numpy(), alpha.cpu().numpy()
    C = wl["cams_per_env"]
    allst = []
    for i, ref in enumerate(refs):
        e, c = divmod(i, C)
        allst.append(compare_image(ref, rgb_n[e, c], d_n[e, c], a_n[e, c], depth_tol=depth_tol))
    log("stats", allst[0], "... images", len(allst), "pairs", st["pairs"])
    torch.cuda.synchronize()
    return scene, cams, rgb, depth, alpha, refs, allst


@pytest.mark.parametrize("tile", [(16, 16), (16, 8), (8, 8), (32, 8)])
def test_plain_forward_20k_sh0_128(gsr, ctx, tile):
    wl = synth.scene_config(0)
    wl["name"] = "20k SH0 128x128"
    _run(gsr, ctx, wl, tile)


@pytest.mark.parametrize("tile,ppt", [((16, 16), 4), ((32, 8), 4), ((16, 16), 1), ((16, 8), 1)])
def test_pixels_per_lane_variants(gsr, ctx, tile, ppt):
    wl = synth.scene_config(0, seed=19)
    wl["name"] = f"20k SH0 128x128, {ppt} pixels per lane"
    ctx.set_pixels_per_thread(ppt)
    try:
        _run(gsr, ctx, wl, tile)
    finally:
        ctx.set_pixels_per_thread(2)


def test_composed_scene_three_cameras(gsr, ctx):
    # background + 8 posed object nodes, SH degree 3, head + two wrist cameras
    wl = synth.scene_config(2, seed=3, scale=0.03)
    wl["name"] = "composed 60k+8x1.5k SH3 3 cams 640x480"
    _run(gsr, ctx, wl, (16, 16))


def test_batched_uneven_envs(gsr, ctx):
    wl = synth.scene_config(3, seed=5, scale=0.04, n_envs=5)
    wl["name"] = "batched 5 envs uneven"
    _run(gsr, ctx, wl, (16, 8))


def test_image_without_visible_gaussians_between_others(gsr, ctx):
    """Three envs of two cameras; the middle env's second camera looks away from its scene, so
    its image has an empty segment between non-empty ones in the depth-sort buffers."""
    wl = synth.scene_config(3, seed=11, scale=0.02, n_envs=3)
    env = wl["envs"][1]
    env["cams"][1] = synth.camera((0.0, 0.6, -7.0), (0.0, 0.6, -20.0), wl["width"], wl["height"])
    wl["name"] = "3 envs, one image empty"
    _, _, _, _, _, refs, _ = _run(gsr, ctx, wl, (16, 16))
    assert len(refs[3]["keys"]) == 0 and all(len(refs[i]["keys"]) > 0 for i in (0, 1, 2, 4, 5))


def test_ragged_image_partial_tiles(gsr, ctx):
    wl = synth.scene_config(0, seed=7, scale=0.5)
    cam = synth.camera((0.2, -0.1, -3.0), (0, 0, 0), 100, 75)
    wl["envs"][0]["cams"] = [cam]
    wl["width"], wl["height"] = 100, 75
    wl["name"] = "ragged 100x75"
    for tile in [(16, 16), (32, 8)]:
        _run(gsr, ctx, wl, tile)


def test_full_hd_image_beyond_64_kib_of_tile_state(gsr, ctx):
    """1920x1080 with 16x16 tiles: 8160 tiles per image, so the emission's per-tile state
    (12 B per tile in LDS) and the tile-count grid of a block exceed 64 KiB."""
    wl = synth.scene_config(0, seed=23)
    cam = synth.camera((0.1, 0.05, -2.6), (0, 0, 0), 1920, 1080)
    wl["envs"][0]["cams"] = [cam]
    wl["width"], wl["height"] = 1920, 1080
    wl["name"] = "20k SH0 1920x1080"
    _run(gsr, ctx, wl, (16, 16), full=False, sample=4000)


def test_too_many_tiles_per_image_is_refused(gsr, ctx):
    """2048x1024 with 8x8 tiles is 32768 tiles per image: beyond the emission's LDS state, the
    render fails with GSR_E_UNSUPPORTED before touching the device."""
    wl = synth.scene_config(0, seed=2, scale=0.05)
    cam = synth.camera((0, 0, -3), (0, 0, 0), 2048, 1024)
    wl["envs"][0]["cams"] = [cam]
    wl["width"], wl["height"] = 2048, 1024
    ctx.set_tile(8, 8)
    with pytest.raises(gsr.GsrError) as err:
        render_gpu(ctx, wl)
    assert err.value.code == -5


def test_empty_zero_opacity_and_behind_camera_give_background(gsr, ctx):
    import torch
    bg = (0.25, 0.5, 0.75)
    cam = synth.camera((0, 0, -3), (0, 0, 0), 64, 48, bg=bg)
    empty = synth.gaussians_uniform_cube(0, 1)
    zero = synth.gaussians_uniform_cube(300, 2)
    zero["opacities"][:] = 0
    behind = synth.gaussians_uniform_cube(300, 3)
    behind["means"][:, 2] = -3.5  # behind the camera at z = -3 looking +z
    eye = np.eye(3, dtype=np.float32)
    z3 = np.zeros(3, np.float32)
    for nd in (empty, zero, behind):
        wl = dict(envs=[dict(nodes=[nd], poses=[(eye, z3)], cams=[cam])], cams_per_env=1, width=64, height=48)
        ctx.set_tile(16, 16)
        _, _, rgb, depth, alpha = render_gpu(ctx, wl)
        bgv = torch.tensor(bg, dtype=torch.float32, device=rgb.device)
        assert torch.equal(rgb, bgv.expand_as(rgb)) and torch.all(depth == 0) and torch.all(alpha == 0)
        assert gsr.query_status(ctx)["pairs"] == 0


def test_nonfinite_parameters_are_culled_and_counted(gsr, ctx):
    wl = synth.scene_config(0, seed=9, scale=0.1)
    nd = wl["envs"][0]["nodes"][0]
    nd["means"][5, 1] = np.nan
    nd["scales"][17, 0] = np.inf
    nd["quats"][33, 2] = -np.inf
    nd["opacities"][40] = np.nan
    _run(gsr, ctx, wl, (16, 16))
    assert gsr.query_status(ctx)["nonfinite"] == 4


def test_one_gaussian_covering_every_tile(gsr, ctx):
    from helpers import node
    cam = synth.camera((0, 0, -3), (0, 0, 0), 96, 64)
    big = node([[0.0, 0.0, 0.0]], 2.0, opac=0.9, colours=(0.2, 0.7, 0.4))
    small = synth.gaussians_uniform_cube(200, 4)
    eye = np.eye(3, dtype=np.float32)
    z3 = np.zeros(3, np.float32)
    small["sh"] = small["sh"][:, :1]
    wl = dict(envs=[dict(nodes=[big, small], poses=[(eye, z3), (eye, z3)], cams=[cam])], cams_per_env=1,
              width=96, height=64, name="one Gaussian covers all tiles")
    _, _, _, _, _, refs, _ = _run(gsr, ctx, wl, (16, 16))
    assert refs[0]["vis"][0] == 0 and all((refs[0]["ranges"][:, 1] - refs[0]["ranges"][:, 0]) >= 1)


def test_partial_saturation_shrinks_the_live_pixel_cull(gsr, ctx):
    """Three near splats of opacity 0.99 saturate a region whose edge crosses many wavefront
    sub-tiles, with 3000 splats behind it (tile lists of 52 to 1155 entries): the compositor
    culls each later batch against the box of the pixels still live, which must leave every
    pixel as the oracle composites it."""
    from helpers import cam_identity, env_of, node
    wall = node([[-0.35, 0.0, 1.0], [-0.35, 0.0, 1.05], [-0.35, 0.0, 1.1]], 0.25, opac=0.99,
                colours=[(0.9, 0.1, 0.1), (0.1, 0.9, 0.1), (0.1, 0.1, 0.9)])
    back = synth.gaussians_uniform_cube(3000, 5)
    back["sh"] = back["sh"][:, :1]
    eye = np.eye(3, dtype=np.float32)
    env = env_of([wall, back], poses=[(eye, np.zeros(3, np.float32)), (eye, np.array([0, 0, 4], np.float32))])
    env["cams"] = [cam_identity(64, 64, 64.0)]
    wl = dict(envs=[env], cams_per_env=1, width=64, height=64, name="partial saturation")
    _, _, _, _, _, refs, _ = _run(gsr, ctx, wl, (16, 16))
    a = refs[0]["alpha"].reshape(64, 64)
    assert (a > 0.99).sum() > 200 and (a < 0.9).sum() > 200  # both saturated and live regions


def test_pair_capacity_overflow_is_reported_then_grown(gsr):
    import torch
    wl = synth.scene_config(0, seed=11, scale=0.25)
    c = gsr.create(0, pair_capacity=1000)
    try:
        scene, cams, rgb, depth, alpha = render_gpu(c, wl, flags=0)
        st = gsr.query_status(c)
        assert st["flags"] & gsr.STATUS_OVERFLOW and st["pairs"] > 1000 and st["pair_capacity"] == 1000
        scene, cams, rgb, depth, alpha = render_gpu(c, wl, flags=gsr.FLAG_CHECK)
        st = gsr.query_status(c)
        assert st["flags"] == 0 and st["pair_capacity"] >= st["pairs"]
        refs = oracle_images(wl, 16, 16)
        compare_image(refs[0], rgb[0, 0].cpu().numpy(), depth[0, 0].cpu().numpy(), alpha[0, 0].cpu().numpy())
        torch.cuda.synchronize()
    finally:
        c.close()


def test_long_tile_lists(gsr, ctx):
    # dense cube, small image: per-tile lists above 32768 entries, written by many emission
    # chunks of the depth-sorted Gaussians
    wl = synth.scene_config(0, seed=13, scale=3.0)
    cam = synth.camera((0, 0, -3), (0, 0, 0), 48, 48)
    cam["fx"] = cam["fy"] = np.float32(41.57)
    wl["envs"][0]["cams"] = [cam]
    wl["width"], wl["height"] = 48, 48
    wl["name"] = "dense 60k, 48x48"
    _, _, _, _, _, refs, _ = _run(gsr, ctx, wl, (16, 16))
    lens = refs[0]["ranges"][:, 1] - refs[0]["ranges"][:, 0]
    log("max tile list", lens.max())
    assert lens.max() > 16384 * 2


@pytest.mark.parametrize("spread_ulps,outlier", [(6, True), (0, True), (0, False)])
def test_clustered_depths_sort_exactly(gsr, ctx, spread_ulps, outlier):
    """Thousands of entries per tile within a few ulps of one depth (or at exactly one depth,
    ordered by id), with or without a far entry in the same tiles: the depth sort and the
    emission must still give the oracle's (z bits, id) order bit for bit."""
    from helpers import cam_identity, env_of, node
    rng = np.random.default_rng(41)
    n = 3000
    zb = np.float32(3.0).view(np.uint32) + rng.integers(0, spread_ulps + 1, n).astype(np.uint32)
    means = np.c_[rng.uniform(-0.02, 0.02, (n, 2)).astype(np.float32), zb.view(np.float32)]
    if outlier:
        means = np.r_[means, [[0.0, 0.0, 30.0]]].astype(np.float32)
    g = node(means, 0.005, opac=0.05, colours=rng.uniform(0, 1, (len(means), 3)))
    env = env_of([g])
    env["cams"] = [cam_identity(32, 32, 40.0)]
    wl = dict(envs=[env], cams_per_env=1, width=32, height=32,
              name=f"{n} entries within {spread_ulps} ulps, outlier {outlier}")
    _, _, _, _, _, refs, _ = _run(gsr, ctx, wl, (16, 16))
    lens = refs[0]["ranges"][:, 1] - refs[0]["ranges"][:, 0]
    assert lens.max() > 2000


@pytest.mark.parametrize("n", [1025, 8193, 8256, 16385])
def test_depth_sort_chunk_boundaries(gsr, ctx, n):
    """One 16x16 image, every Gaussian inside it: the tile's list holds exactly n entries, so
    the image's depth-sorted Gaussians fill radix chunks of 2048 and emission chunks of 1024
    pairs with a short last chunk (1 or 64 entries)."""
    from helpers import cam_identity, env_of, node
    rng = np.random.default_rng(n)
    means = np.c_[rng.uniform(-0.02, 0.02, (n, 2)), rng.uniform(2.0, 6.0, n)].astype(np.float32)
    g = node(means, 0.002, opac=0.02, colours=rng.uniform(0, 1, (n, 3)))
    env = env_of([g])
    env["cams"] = [cam_identity(16, 16, 20.0)]
    wl = dict(envs=[env], cams_per_env=1, width=16, height=16, name=f"one tile, {n} entries")
    _, _, _, _, _, refs, _ = _run(gsr, ctx, wl, (16, 16))
    assert refs[0]["ranges"][0, 1] - refs[0]["ranges"][0, 0] == n


def test_graph_replay_matches_eager_bitwise(gsr, ctx):
    import torch
    wl = synth.scene_config(3, seed=17, scale=0.02, n_envs=3)
    envs_t, poses, cams = upload(wl)
    ctx.set_tile(16, 16)
    scene = gsr.compose_scene(ctx, envs_t, poses)
    W, H, C = wl["width"], wl["height"], wl["cams_per_env"]
    ref = [t.clone() for t in gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=gsr.FLAG_CHECK)]
    out = gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=0)
    out = tuple(torch.empty_like(t) for t in out)
    for rep in range(4):
        for t in out:
            t.fill_(-1.0)
        gsr.render_rgbd(ctx, scene, cams, W, H, C, out=out, flags=gsr.FLAG_GRAPH)
        torch.cuda.synchronize()
        for a, b in zip(out, ref):
            assert torch.equal(a, b), f"replay {rep} differs"
        # eager work between replays
        gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=0)
        torch.cuda.synchronize()
    assert gsr.query_status(ctx)["flags"] == 0


def test_repeat_renders_bitwise_identical(gsr, ctx):
    import torch
    wl = synth.scene_config(2, seed=19, scale=0.01)
    envs_t, poses, cams = upload(wl)
    ctx.set_tile(16, 16)
    scene = gsr.compose_scene(ctx, envs_t, poses)
    ref = [t.clone() for t in gsr.render_rgbd(ctx, scene, cams, 640, 480, 3)]
    for _ in range(5):
        out = gsr.render_rgbd(ctx, scene, cams, 640, 480, 3, flags=0)
        for a, b in zip(out, ref):
            assert torch.equal(a, b)


def test_permutation_of_gaussians_is_bitwise_invariant(gsr, ctx):
    import torch
    # the first seed whose keys (tile, z bits) are all distinct: equal keys are ordered by id,
    # which a permutation changes
    for seed in range(23, 60):
        wl = synth.scene_config(0, seed=seed, scale=0.3)
        ref = oracle_images(wl, 16, 16)[0]
        if len(np.unique(ref["keys"])) == len(ref["keys"]):
            break
    else:
        pytest.fail("no tie-free seed")
    _, _, rgb, depth, alpha = render_gpu(ctx, wl)
    rgb, depth = rgb.clone(), depth.clone()
    perm = np.random.default_rng(1).permutation(len(wl["envs"][0]["nodes"][0]["means"]))
    nd = wl["envs"][0]["nodes"][0]
    wl["envs"][0]["nodes"][0] = {k: (v[perm] if isinstance(v, np.ndarray) else v) for k, v in nd.items()}
    _, _, rgb2, depth2, _ = render_gpu(ctx, wl)
    assert torch.equal(rgb, rgb2) and torch.equal(depth, depth2)


@pytest.mark.parametrize("axis", ["y", "x"])
def test_joint_rigid_motion_of_scene_and_camera(gsr, ctx, axis):
    """A rotation of scene and cameras together leaves every pixel unchanged.  The rotation is
    a signed permutation (90 degrees about y, 180 about x), so the moved poses and cameras are
    exactly representable in FP32 and the renderer's FP64 camera-node maps see the same
    products summed in another order: every pixel must agree within 1e-4 (a general rotation
    also rounds its inputs; the oracle's pins cover that case)."""
    import torch
    wl = synth.scene_config(2, seed=29, scale=0.01)
    _, _, rgb, depth, alpha = render_gpu(ctx, wl)
    rgb, depth, alpha = rgb.clone(), depth.clone(), alpha.clone()
    R0 = np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]], np.float64) if axis == "y" else np.diag([1.0, -1.0, -1.0])
    env = wl["envs"][0]
    env["poses"] = [((R0 @ R.astype(np.float64)).astype(np.float32), (R0 @ t.astype(np.float64)).astype(np.float32))
                    for R, t in env["poses"]]
    for c in env["cams"]:
        c["R"] = (c["R"].astype(np.float64) @ R0.T).astype(np.float32)
    _, _, rgb2, depth2, alpha2 = render_gpu(ctx, wl)
    d = max((rgb - rgb2).abs().max().item(), (depth - depth2).abs().max().item(), (alpha - alpha2).abs().max().item())
    log(f"rigid motion about {axis}: max difference {d:.3g}, bitwise {torch.equal(rgb, rgb2)}")
    assert d <= TOL


def test_batched_equals_per_camera_loop_bitwise(gsr, ctx):
    """Every image of one batched render (5 envs of uneven size x 2 cameras, one key space)
    is bitwise equal to the eager render of that env and camera alone, at the same tile
    shape: batching changes the launch structure, never the arithmetic."""
    import torch
    wl = synth.scene_config(3, seed=37, scale=0.03, n_envs=5)
    envs_t, poses, cams = upload(wl)
    W, H, C = wl["width"], wl["height"], wl["cams_per_env"]
    for tile in [(16, 16), (8, 8)]:
        ctx.set_tile(*tile)
        scene = gsr.compose_scene(ctx, envs_t, poses)
        batched = [t.clone() for t in gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=gsr.FLAG_CHECK)]
        for e in range(len(wl["envs"])):
            pe = poses[e * 5:(e + 1) * 5].clone()
            one = gsr.compose_scene(ctx, [envs_t[e]], pe)
            for c in range(C):
                out = gsr.render_rgbd(ctx, one, cams[e * C + c:e * C + c + 1].clone(), W, H, 1, flags=gsr.FLAG_CHECK)
                for b, o in zip(batched, out):
                    assert torch.equal(b[e, c], o[0, 0]), f"env {e} cam {c} tile {tile}"
            one.close()
        log(f"tile {tile}: {len(wl['envs']) * C} images bitwise equal")


def test_stream_groups_render_exactly_as_one_group(gsr, ctx):
    """Environments split into 2, 3 or 4 stream groups (sub-contexts with their own workspace
    on their own streams, forked from and joined back to the caller's stream) give every image
    bit for bit as one group does: checked, eager and replayed graphs (the outputs cleared by
    the caller's own work between replays).  The status sums the groups; the per-context
    state of a grouped render is refused; a saved render keeps to one group."""
    import torch
    wl = synth.scene_config(3, seed=43, scale=0.03, n_envs=5)
    envs_t, poses, cams = upload(wl)
    W, H, C = wl["width"], wl["height"], wl["cams_per_env"]
    E = len(wl["envs"])
    ctx.set_tile(16, 16)
    scene = gsr.compose_scene(ctx, envs_t, poses)
    ref = [t.clone() for t in gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=gsr.FLAG_CHECK)]
    st_ref = gsr.query_status(ctx)
    tiles = E * C * ((W + 15) // 16) * ((H + 15) // 16)
    try:
        for G in (2, 3, 4):
            ctx.set_stream_groups(G)
            out = gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=gsr.FLAG_CHECK)
            for a, b in zip(out, ref):
                assert torch.equal(a, b), f"{G} groups, checked"
            st = gsr.query_status(ctx)
            for k in ("flags", "pairs", "visible", "visible_any", "evals", "nonfinite", "max_tile_pairs"):
                assert st[k] == st_ref[k], (G, k, st[k], st_ref[k])
            eager = gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=0)
            for a, b in zip(eager, ref):
                assert torch.equal(a, b), f"{G} groups, eager"
            outg = tuple(torch.empty_like(t) for t in ref)
            for rep in range(3):
                for t in outg:
                    t.fill_(-1.0)
                gsr.render_rgbd(ctx, scene, cams, W, H, C, out=outg, flags=gsr.FLAG_GRAPH)
                for a, b in zip(outg, ref):
                    assert torch.equal(a, b), f"{G} groups, graph replay {rep}"
            with pytest.raises(gsr.GsrError):
                gsr.copy_pairs(ctx, tiles)
            log(f"{G} stream groups: {E * C} images bitwise equal to one group (checked, eager, graph)")
        # saved for backward: one group, the context's own state
        gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=gsr.FLAG_SAVE | gsr.FLAG_CHECK)
        keys, _, _ = gsr.copy_pairs(ctx, tiles)
        assert keys.numel() == st_ref["pairs"]
    finally:
        ctx.set_stream_groups(1)
    scene.close()


def test_scene_outliving_its_context(gsr):
    """A scene (and its stream groups' scenes on the sub-contexts) destroyed after its context:
    the context detaches its scenes, so the late destroy frees only the scene's own tables."""
    wl = synth.scene_config(3, seed=47, scale=0.01, n_envs=3)
    envs_t, poses, cams = upload(wl)
    W, H, C = wl["width"], wl["height"], wl["cams_per_env"]
    c = gsr.create(0)
    c.set_stream_groups(2)
    scene = gsr.compose_scene(c, envs_t, poses)
    gsr.render_rgbd(c, scene, cams, W, H, C, flags=gsr.FLAG_CHECK)
    c.close()
    scene.close()
    # and a context that renders again after one of its scenes was destroyed
    c = gsr.create(0)
    c.set_stream_groups(2)
    s1 = gsr.compose_scene(c, envs_t, poses)
    ref = [t.clone() for t in gsr.render_rgbd(c, s1, cams, W, H, C, flags=gsr.FLAG_CHECK)]
    s1.close()
    s2 = gsr.compose_scene(c, envs_t, poses)
    out = gsr.render_rgbd(c, s2, cams, W, H, C, flags=gsr.FLAG_CHECK)
    import torch
    for a, b in zip(out, ref):
        assert torch.equal(a, b)
    s2.close()
    c.close()


def test_persistent_composite_matches_one_block_per_tile(gsr, ctx):
    import torch
    wl = synth.scene_config(3, seed=31, scale=0.03, n_envs=4)
    envs_t, poses, cams = upload(wl)
    W, H, C = wl["width"], wl["height"], wl["cams_per_env"]
    for tile in [(16, 16), (8, 8)]:
        ctx.set_tile(*tile)
        scene = gsr.compose_scene(ctx, envs_t, poses)
        ref = [t.clone() for t in gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=gsr.FLAG_CHECK)]
        ev_ref = gsr.query_status(ctx)["evals"]
        assert ev_ref > 0
        out = gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=gsr.FLAG_CHECK | gsr.FLAG_PERSISTENT)
        for a, b in zip(out, ref):
            assert torch.equal(a, b)
        assert gsr.query_status(ctx)["evals"] == ev_ref
        # and inside a graph
        out2 = gsr.render_rgbd(ctx, scene, cams, W, H, C, flags=gsr.FLAG_GRAPH | gsr.FLAG_PERSISTENT)
        out2 = gsr.render_rgbd(ctx, scene, cams, W, H, C, out=out2, flags=gsr.FLAG_GRAPH | gsr.FLAG_PERSISTENT)
        torch.cuda.synchronize()
        for a, b in zip(out2, ref):
            assert torch.equal(a, b)
