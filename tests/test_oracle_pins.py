"""Pins of the CPU oracle against mathematics (no GPU).

The paper (DISCOVERSE, arXiv 2507.21981) prints no pixel, key or gradient
values for its renderer (Sec. III-A names the stages; Sec. III-C defines RGB
and depth as alpha-composited colour and camera-space z), so every pin here
comes from closed forms, textbook identities, brute force and invariants,
chosen so that a dropped term, wrong sign, transposed operand or wrong index
in the oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import synth
from helpers import cam_identity, env_of, node, rot_axis

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- SH basis
def test_sh_matches_textbook_closed_forms(orc):
    rows = np.loadtxt(os.path.join(GOLDEN, "sh_closed_forms.txt"))
    for r in rows:
        Y = orc.sh_eval(3, r[:3])
        np.testing.assert_allclose(Y, r[3:], rtol=0, atol=1e-14)
        # also through a non-unit vector (the basis is evaluated at v/|v|)
        np.testing.assert_allclose(orc.sh_eval(3, 2.5 * r[:3]), r[3:], rtol=0, atol=1e-14)


def test_sh_addition_theorem(orc):
    g = np.random.default_rng(1)
    for _ in range(50):
        d = g.standard_normal(3)
        Y = orc.sh_eval(3, d)
        for l in range(4):
            s = np.sum(Y[l * l:(l + 1) * (l + 1)] ** 2)
            assert abs(s - (2 * l + 1) / (4 * math.pi)) < 1e-13


def test_sh_orthonormal_by_quadrature(orc):
    # Gauss-Legendre in z times uniform in phi: exact for the degree <= 6 products
    zs, wz = np.polynomial.legendre.leggauss(8)
    nphi = 16
    G = np.zeros((16, 16))
    for z, w in zip(zs, wz):
        r = math.sqrt(1 - z * z)
        for k in range(nphi):
            ph = 2 * math.pi * k / nphi
            Y = orc.sh_eval(3, np.array([r * math.cos(ph), r * math.sin(ph), z]))
            G += w * (2 * math.pi / nphi) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-13)


def test_sh_gradient_matches_finite_differences(orc):
    g = np.random.default_rng(2)
    for _ in range(10):
        v = g.standard_normal(3) * 1.7
        Y, dY = orc.sh_eval(3, v, grad=True)
        h = 1e-6
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            fd = (orc.sh_eval(3, v + e) - orc.sh_eval(3, v - e)) / (2 * h)
            np.testing.assert_allclose(dY[:, j], fd, atol=1e-8)


# ---------------------------------------------------------- SH rotation
def _rand_rot(seed):
    return synth.random_rotation(synth.rng(seed))


def test_wigner_blocks_orthogonal_and_compose(orc):
    R1, R2 = _rand_rot(3), _rand_rot(4)
    D1, D2, D12 = orc.wigner(3, R1), orc.wigner(3, R2), orc.wigner(3, R1 @ R2)
    np.testing.assert_allclose(D1 @ D1.T, np.eye(16), atol=1e-12)
    # Y((R1 R2)^T d) = D(R2) Y(R1^T d) = D(R2) D(R1) Y(d)
    np.testing.assert_allclose(D12, D2 @ D1, atol=1e-12)
    # degree 0 untouched, block structure kept
    assert abs(D1[0, 0] - 1) < 1e-13
    assert np.abs(D1[0, 1:]).max() < 1e-13 and np.abs(D1[1:4, 4:]).max() < 1e-13


def test_wigner_rotates_evaluation(orc):
    R = _rand_rot(5)
    D = orc.wigner(3, R)
    g = np.random.default_rng(6)
    k = g.standard_normal(16)
    for _ in range(20):
        d = g.standard_normal(3)
        # sum_k k Y(R^T d) == (D^T k) . Y(d)
        np.testing.assert_allclose(k @ orc.sh_eval(3, R.T @ d), (D.T @ k) @ orc.sh_eval(3, d), atol=1e-12)


# ------------------------------------------------- closed-form footprints
def _render(orc, nodes, cam, poses=None, tw=16, th=16):
    env = env_of(nodes, poses)
    return orc.render(env, cam, cam["width"], cam["height"], tw, th)


def _alpha_closed(Sigma2, u, v, o, W, H):
    py, px = np.mgrid[0:H, 0:W]
    dx = px + 0.5 - u
    dy = py + 0.5 - v
    Q = np.linalg.inv(Sigma2)
    power = -0.5 * (Q[0, 0] * dx * dx + Q[1, 1] * dy * dy) - Q[0, 1] * dx * dy
    a = np.minimum(0.99, o * np.exp(power))
    return np.where(a < 1 / 255, 0.0, a)


def f32(x):
    """The FP32 rounding of an input value, as the oracle receives it."""
    return np.asarray(x, np.float32).astype(np.float64)


@pytest.mark.parametrize("W,sig,o", [(64, 0.05, 0.7), (63, 0.2, 1.0)])
def test_isotropic_gaussian_on_axis_closed_form(orc, W, sig, o):
    H = W
    f, z0, c = 50.0, 2.0, (0.9, 0.4, 0.2)
    cam = cam_identity(W, H, f)
    r = _render(orc, [node([[0, 0, z0]], sig, opac=o, colours=c)], cam)
    sig, o = f32(sig), f32(o)
    s2 = (f * sig / z0) ** 2 + 0.3
    a = _alpha_closed(np.eye(2) * s2, W / 2, H / 2, o, W, H)
    np.testing.assert_allclose(r["alpha"], a, atol=1e-12)
    np.testing.assert_allclose(r["rgb"], a[..., None] * np.array(c), atol=1e-7)  # colour in FP32 input
    np.testing.assert_allclose(r["depth"], a * z0, atol=1e-12)
    # the 1/255 edge sits at r* = s sqrt(2 ln(255 o))
    rstar = math.sqrt(s2) * math.sqrt(2 * math.log(255 * o))
    py, px = np.mgrid[0:H, 0:W]
    rr = np.hypot(px + 0.5 - W / 2, py + 0.5 - H / 2)
    assert np.all(r["alpha"][rr < rstar - 1e-9] > 0) and np.all(r["alpha"][rr > rstar + 1e-9] == 0)
    if o == 1.0:
        assert np.sum(r["alpha"] == 0.99) >= 1  # the 0.99 clamp is reached at the centre


def test_anisotropic_gaussian_off_axis_closed_form(orc):
    W, H = 96, 64
    f = 60.0
    x0, y0, z0 = 0.3, -0.2, 2.5
    s = np.array([0.08, 0.02, 0.05])
    R = rot_axis([1, 2, 3], 0.7)
    # quaternion (w, x, y, z) of R, written from its axis-angle form
    ax = np.array([1, 2, 3]) / np.linalg.norm([1, 2, 3])
    q = np.array([math.cos(0.35), *(math.sin(0.35) * ax)])
    cam = cam_identity(W, H, f)
    o = 0.6
    r = _render(orc, [node([[x0, y0, z0]], s, quats=q, opac=o)], cam)
    o = f32(o)
    Rf = R.astype(np.float32).astype(np.float64)  # close to R; exact R used by the oracle from q
    Sig = R @ np.diag(s.astype(np.float32).astype(np.float64) ** 2) @ R.T
    x0f, y0f, z0f = (np.float32(v) for v in (x0, y0, z0))
    J = np.array([[f / z0f, 0, -f * x0f / z0f ** 2], [0, f / z0f, -f * y0f / z0f ** 2]])
    S2 = J @ Sig @ J.T + 0.3 * np.eye(2)
    u, v = f * x0f / z0f + W / 2, f * y0f / z0f + H / 2
    a = _alpha_closed(S2, u, v, o, W, H)
    # quaternion -> float32 -> normalised rotation differs from R by ~1e-8
    np.testing.assert_allclose(r["alpha"], a, atol=2e-6)
    assert np.abs(Rf - R).max() < 1e-7


def test_two_layer_compositing_closed_form(orc):
    W = H = 48
    f = 40.0
    cam = cam_identity(W, H, f, bg=(0.1, 0.2, 0.3))
    n1 = node([[0, 0, 2.0], [0.05, 0.02, 3.0]], [[0.06] * 3, [0.09] * 3], opac=[0.8, 0.5],
              colours=[[1.0, 0.0, 0.25], [0.0, 1.0, 0.75]])
    r = _render(orc, [n1], cam)
    a1 = _alpha_closed(np.eye(2) * ((f * f32(0.06) / 2.0) ** 2 + 0.3), W / 2, H / 2, f32(0.8), W, H)
    x2, y2, z2 = f32(0.05), f32(0.02), 3.0
    u2 = f * x2 / z2 + W / 2
    v2 = f * y2 / z2 + H / 2
    J = np.array([[f / z2, 0, -f * x2 / z2 ** 2], [0, f / z2, -f * y2 / z2 ** 2]])
    a2 = _alpha_closed(f32(0.09) ** 2 * J @ J.T + 0.3 * np.eye(2), u2, v2, 0.5, W, H)
    c1 = np.array([1.0, 0.0, 0.25])
    c2 = np.array([0.0, 1.0, 0.75])
    bg = np.array([0.1, 0.2, 0.3], np.float32).astype(np.float64)
    T = (1 - a1) * (1 - a2)
    exp_rgb = a1[..., None] * c1 + ((1 - a1) * a2)[..., None] * c2 + T[..., None] * bg
    np.testing.assert_allclose(r["rgb"], exp_rgb, atol=1e-7)
    np.testing.assert_allclose(r["depth"], a1 * 2.0 + (1 - a1) * a2 * 3.0, atol=1e-12)
    np.testing.assert_allclose(r["alpha"], 1 - T, atol=1e-12)


def test_termination_thirteen_layers(orc):
    # 20 co-located identical Gaussians, alpha exactly 1/2 at the pixel centre:
    # (1/2)^14 < 1e-4 <= (1/2)^13, so exactly 13 layers blend.
    cam = cam_identity(1, 1, 10.0)
    n = node(np.tile([[0, 0, 1.0]], (20, 1)), 0.05, opac=0.5, colours=[0.75, 0.5, 0.25])
    r = _render(orc, [n], cam)
    assert r["alpha"][0, 0] == 1 - 2.0 ** -13
    c = np.array([0.75, 0.5, 0.25])
    assert np.all(np.abs(r["rgb"][0, 0] - (1 - 2.0 ** -13) * c) < 1e-7)
    assert r["last"][0, 0] == 13 and r["evals"][0, 0] == 14


# --------------------------------------------------- brute force, invariants
def _small_scene(seed, n_bg=2000, n_obj=300, sh=3):
    bg = synth.gaussians_uniform_cube(n_bg, seed, sh_degree=sh)
    ob = synth.gaussians_object(n_obj, seed + 1, sh_degree=sh, radius=0.3, log_scale=(-4.0, 0.4))
    R = _rand_rot(seed + 2).astype(np.float32)
    t = np.array([0.2, -0.1, -0.3], np.float32)
    eye = np.eye(3, dtype=np.float32)
    z3 = np.zeros(3, np.float32)
    return dict(nodes=[bg, ob], poses=[(eye, z3), (R, t)], cams=[])


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 8), (32, 8)])
def test_brute_force_equals_tiled(orc, tile):
    env = _small_scene(10)
    cam = synth.camera((0.4, 0.3, -3.0), (0, 0, 0), 64, 64)
    r = orc.render(env, cam, 64, 64, *tile)
    b = orc.render_brute(env, cam, 64, 64)
    assert np.array_equal(r["rgb"], b["rgb"]) and np.array_equal(r["depth"], b["depth"])
    assert np.array_equal(r["alpha"], b["alpha"])
    assert r["alpha"].max() > 0.5  # the scene is actually in view


def test_brute_force_equals_tiled_near_camera(orc):
    # Gaussians close to the camera have large footprints and clamp in J
    env = _small_scene(11)
    cam = synth.camera((0.0, 0.0, -1.2), (0, 0, 0), 48, 40, znear=0.05)
    r = orc.render(env, cam, 48, 40, 16, 8)
    b = orc.render_brute(env, cam, 48, 40)
    assert np.array_equal(r["rgb"], b["rgb"]) and np.array_equal(r["depth"], b["depth"])


def test_empty_and_zero_opacity_give_background(orc):
    cam = synth.camera((0, 0, -3), (0, 0, 0), 32, 32, bg=(0.25, 0.5, 0.75))
    bgv = np.array([0.25, 0.5, 0.75], np.float32).astype(np.float64)
    r = _render(orc, [node(np.zeros((0, 3)), 0.1)], cam)
    assert np.all(r["rgb"] == bgv) and np.all(r["depth"] == 0) and np.all(r["alpha"] == 0)
    g = synth.gaussians_uniform_cube(500, 3)
    g["opacities"][:] = 0
    r = _render(orc, [g], cam)
    assert np.all(r["rgb"] == bgv) and np.all(r["depth"] == 0) and np.all(r["alpha"] == 0)
    assert len(r["keys"]) == 0 and np.all(r["vis"] == 2)


def test_permutation_invariance(orc):
    env = _small_scene(12, n_bg=1500, n_obj=0)
    env["nodes"], env["poses"] = env["nodes"][:1], env["poses"][:1]
    cam = synth.camera((0.1, 0.2, -3.0), (0, 0, 0), 64, 48)
    r = orc.render(env, cam, 64, 48)
    zb = r["zbits"][r["vis"] == 0]
    assert len(np.unique(zb)) == len(zb), "z ties: pick another seed"
    perm = np.random.default_rng(0).permutation(1500)
    g = {k: (v[perm] if isinstance(v, np.ndarray) else v) for k, v in env["nodes"][0].items()}
    r2 = orc.render(dict(nodes=[g], poses=env["poses"], cams=[]), cam, 64, 48)
    assert np.array_equal(r["rgb"], r2["rgb"]) and np.array_equal(r["depth"], r2["depth"])


def _move(env, cam, R0, t0):
    R0 = np.asarray(R0, np.float64)
    t0 = np.asarray(t0, np.float64)
    poses = [((R0 @ R.astype(np.float64)).astype(np.float32), (R0 @ t.astype(np.float64) + t0).astype(np.float32))
             for R, t in env["poses"]]
    Rc = cam["R"].astype(np.float64) @ R0.T
    tc = cam["t"].astype(np.float64) - Rc @ t0
    c2 = dict(cam, R=Rc.astype(np.float32), t=tc.astype(np.float32))
    return dict(env, poses=poses), c2


def test_joint_rigid_motion_exact(orc):
    # a 90 degree turn and dyadic shift are exact in FP32: only FP64 rounding remains
    env = _small_scene(13, n_bg=800, n_obj=200)
    env["poses"][1] = (np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]], np.float32), np.array([0.25, -0.125, 0.5], np.float32))
    cam = synth.camera((0, 0, -3), (0, 0, 0), 48, 48)
    r = orc.render(env, cam, 48, 48)
    R0 = np.array([[0, 1, 0], [0, 0, -1], [-1, 0, 0]], np.float64)
    env2, cam2 = _move(env, cam, R0, [0.5, -0.25, 1.0])
    r2 = orc.render(env2, cam2, 48, 48)
    assert np.array_equal(r["vals"], r2["vals"])
    np.testing.assert_allclose(r2["rgb"], r["rgb"], atol=1e-12)
    np.testing.assert_allclose(r2["depth"], r["depth"], atol=1e-12)


def test_joint_rigid_motion_general(orc):
    env = _small_scene(14, n_bg=800, n_obj=200)
    cam = synth.camera((0.3, -0.2, -3), (0, 0, 0), 48, 48)
    r = orc.render(env, cam, 48, 48)
    env2, cam2 = _move(env, cam, _rand_rot(99), [0.3, 0.7, -0.2])
    r2 = orc.render(env2, cam2, 48, 48)
    # FP32 rounding of the moved poses and camera perturbs inputs by ~1e-7
    np.testing.assert_allclose(r2["rgb"], r["rgb"], atol=5e-5)
    np.testing.assert_allclose(r2["depth"], r["depth"], atol=5e-5)


# ------------------------------------------------------- keys and ranges
def test_pairs_sorted_and_ranges_by_definition(orc):
    env = _small_scene(15, n_bg=300, n_obj=50)
    cam = synth.camera((0, 0, -3), (0, 0, 0), 40, 24)
    fe = orc.FlatEnv(env)
    rect, zb, vis = orc.keyspec(fe, cam, 40, 24, 8, 8)
    keys, vals, lv, ranges = orc.pairs(rect, zb, vis, 40, 24, 8, 8, image=3, gid_base=1000)
    tiles_x, T = 5, 15
    ref = []
    for i in range(fe.n):
        if vis[i] != 0:
            continue
        x0, y0, x1, y1 = rect[i]
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                ref.append((((3 * T + ty * tiles_x + tx) << 32) | int(zb[i]), 1000 + i))
    ref.sort()
    assert [int(k) for k in keys] == [k for k, _ in ref] and [int(v) for v in vals] == [v for _, v in ref]
    for t in range(T):
        s, e = ranges[t]
        tl = [(k >> 32) - 3 * T for k, _ in ref]
        assert s == sum(1 for x in tl if x < t) and e == sum(1 for x in tl if x <= t)


def test_keyspec_z_and_centre_agree_with_fp64(orc):
    env = _small_scene(16)
    cam = synth.camera((0.4, 0.3, -3.0), (0, 0, 0), 64, 64)
    fe = orc.FlatEnv(env)
    rect, zb, vis = orc.keyspec(fe, cam, 64, 64, 16, 16)
    geo = orc.project(fe, cam, 64, 64)
    m = vis == 0
    z32 = zb[m].view(np.float32).astype(np.float64)
    assert np.abs(z32 - geo[m, 9]).max() < 1e-6 * np.abs(geo[m, 9]).max()


# ------------------------------------------------------------- gradients
def _fd_scene():
    g = np.random.default_rng(21)
    n_bg, n_ob = 10, 6
    bg = synth.gaussians_uniform_cube(n_bg, 21, sh_degree=3, half=0.6, log_scale=(-2.3, 0.3), hi_sigma=0.1)
    ob = synth.gaussians_object(n_ob, 22, sh_degree=3, radius=0.3, log_scale=(-2.5, 0.3), hi_sigma=0.1)
    for n in (bg, ob):
        # keep colours off the 0 clamp and opacity off the 0.99 clamp
        n["sh"][:, 0, :] = (g.uniform(0.3, 0.7, size=n["sh"][:, 0, :].shape) - 0.5) / (0.5 / math.sqrt(math.pi))
        n["opacities"][:] = g.uniform(0.3, 0.9, size=n["opacities"].shape)
        n["quats"] *= g.uniform(0.5, 2.0, size=(len(n["quats"]), 1)).astype(np.float32)  # unnormalised
    R = _rand_rot(23).astype(np.float32)
    env = dict(nodes=[bg, ob], poses=[(np.eye(3, dtype=np.float32), np.zeros(3, np.float32)),
                                      (R, np.array([0.1, 0.05, -0.2], np.float32))], cams=[])
    cam = synth.camera((0.2, 0.3, -2.2), (0, 0, 0), 32, 32, bg=(0.2, 0.1, 0.3))
    return env, cam


def test_analytic_gradient_matches_fp64_finite_differences(orc):
    env, cam = _fd_scene()
    W = H = 32
    g = np.random.default_rng(5)
    wr, wd, wa = g.standard_normal((H, W, 3)), g.standard_normal((H, W)), g.standard_normal((H, W))
    fe = orc.FlatEnv(env)
    rect, zb, vis = orc.keyspec(fe, cam, W, H, 16, 16)
    keys, vals, lv, ranges = orc.pairs(rect, zb, vis, W, H, 16, 16)

    def fwd():
        geo = orc.project(fe, cam, W, H)
        out = orc.composite(geo, ranges, lv, W, H, 16, 16, cam["bg"])
        return float(np.sum(wr * out["rgb"]) + np.sum(wd * out["depth"]) + np.sum(wa * out["alpha"])), out["trace"]

    base_L, base_tr = fwd()
    ref = dict(fe=fe, ranges=ranges, lvals=lv, geo=orc.project(fe, cam, W, H))
    grads = orc.backward(ref, cam, W, H, wr, wd, wa)
    gmap = dict(means=grads["means"], scales=grads["scales"], quats=grads["quats"], opac=grads["opacities"],
                sh=grads["sh"].reshape(-1))
    checked = skipped = 0
    worst = 0.0
    for name in ("means", "scales", "quats", "opac", "sh"):
        arr = fe.p64[name].reshape(-1)
        ga = gmap[name].reshape(-1)
        scale = np.abs(ga).max() + 1e-30
        for j in range(arr.size):
            x = arr[j]
            h = 1e-6 * max(1.0, abs(x))
            arr[j] = x + h
            Lp, tp = fwd()
            arr[j] = x - h
            Lm, tm = fwd()
            arr[j] = x
            if not (np.array_equal(tp, base_tr) and np.array_equal(tm, base_tr)):
                skipped += 1
                continue
            fd = (Lp - Lm) / (2 * h)
            err = abs(fd - ga[j]) / max(abs(fd), 1e-3 * scale)
            worst = max(worst, err)
            checked += 1
            assert err < 1e-5, (name, j, fd, ga[j])
    assert checked > 0.8 * (checked + skipped) and checked > 500, (checked, skipped)


def test_fd_gradients_dense_scene_with_termination(orc):
    # many overlapping, fairly opaque Gaussians: most pixels stop on the 1e-4 rule
    g = np.random.default_rng(31)
    n = 40
    nd = synth.gaussians_uniform_cube(n, 31, sh_degree=1, half=0.15, log_scale=(-2.0, 0.2), hi_sigma=0.1)
    nd["sh"][:, 0, :] = (g.uniform(0.3, 0.7, size=(n, 3)) - 0.5) / (0.5 / math.sqrt(math.pi))
    nd["opacities"][:] = g.uniform(0.6, 0.95, size=n)
    env = dict(nodes=[nd], poses=[(np.eye(3, dtype=np.float32), np.zeros(3, np.float32))], cams=[])
    cam = synth.camera((0.0, 0.0, -2.0), (0, 0, 0), 16, 16)
    W = H = 16
    fe = orc.FlatEnv(env)
    rect, zb, vis = orc.keyspec(fe, cam, W, H, 16, 16)
    keys, vals, lv, ranges = orc.pairs(rect, zb, vis, W, H, 16, 16)
    wr, wd, wa = g.standard_normal((H, W, 3)), g.standard_normal((H, W)), g.standard_normal((H, W))

    def fwd():
        geo = orc.project(fe, cam, W, H)
        out = orc.composite(geo, ranges, lv, W, H, 16, 16, cam["bg"])
        return float(np.sum(wr * out["rgb"]) + np.sum(wd * out["depth"]) + np.sum(wa * out["alpha"])), out

    L0, out0 = fwd()
    assert np.sum(out0["evals"] > out0["last"]) > 0.5 * W * H and np.all(out0["T"] < 1.1e-4) is not None
    ref = dict(fe=fe, ranges=ranges, lvals=lv, geo=orc.project(fe, cam, W, H))
    gr = orc.backward(ref, cam, W, H, wr, wd, wa)
    checked = 0
    for name, ga in (("means", gr["means"]), ("opac", gr["opacities"]), ("scales", gr["scales"])):
        arr = fe.p64[name].reshape(-1)
        ga = ga.reshape(-1)
        scale = np.abs(ga).max()
        for j in range(arr.size):
            x = arr[j]
            h = 1e-6 * max(1.0, abs(x))
            arr[j] = x + h
            Lp, op = fwd()
            arr[j] = x - h
            Lm, om = fwd()
            arr[j] = x
            if not (np.array_equal(op["trace"], out0["trace"]) and np.array_equal(om["trace"], out0["trace"])):
                continue
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - ga[j]) <= 1e-5 * max(abs(fd), 1e-3 * scale), (name, j, fd, ga[j])
            checked += 1
    assert checked > 200


def test_clamped_alpha_has_zero_opacity_gradient(orc):
    # centre pixel of an odd image sits exactly on the mean: o G = 1 >= 0.99, clamped
    cam = cam_identity(15, 15, 20.0)
    env = env_of([node([[0, 0, 2.0]], 0.3, opac=1.0, colours=(0.6, 0.6, 0.6))])
    r = orc.render(env, cam, 15, 15)
    assert r["alpha"][7, 7] == 0.99
    wr = np.zeros((15, 15, 3))
    wr[7, 7, :] = 1.0
    gr = orc.backward(r, cam, 15, 15, wr)
    assert gr["opacities"][0] == 0.0 and np.all(gr["means"][0] == 0.0)
    assert gr["sh"][0, 0, 0] != 0.0  # colour still receives alpha * T


def test_closed_form_opacity_and_colour_derivative(orc):
    # one Gaussian on axis: d rgb / d o = G c and d rgb / d c = alpha (unclamped)
    W = H = 16
    f, z0, sig, o = 20.0, 2.0, 0.1, 0.6
    cam = cam_identity(W, H, f)
    env = env_of([node([[0, 0, z0]], sig, opac=o, colours=(0.9, 0.5, 0.3))])
    r = orc.render(env, cam, W, H)
    sig, o = f32(sig), f32(o)
    wr = np.zeros((H, W, 3))
    wr[5, 7, 1] = 1.0
    gr = orc.backward(r, cam, W, H, wr)
    s2 = (f * sig / z0) ** 2 + 0.3
    dx, dy = 7.5 - W / 2, 5.5 - H / 2
    G = math.exp(-(dx * dx + dy * dy) / (2 * s2))
    assert abs(gr["opacities"][0] - G * 0.5) < 1e-12
    C0 = 0.5 / math.sqrt(math.pi)
    assert abs(gr["sh"][0, 0, 1] - o * G * C0) < 1e-12
    assert gr["sh"][0, 0, 0] == 0.0 and gr["sh"][0, 0, 2] == 0.0


# ------------------------------------------------------------- colour clamp
C1 = math.sqrt(3 / (4 * math.pi))


def test_colour_clamp_closed_form_and_zero_gradient(orc):
    """One SH-degree-1 Gaussian on the optical axis (view direction (0, 0, 1), so only the
    m = 0 coefficient of degree 1 contributes, with Y = C1): channel 0 has a coefficient that
    drives its colour below zero, so colour = max(0, 0.5 - 2 C1) = 0; channel 1 stays at
    0.5 + C1.  Gradients of an upstream gradient on channel 0 alone vanish for every
    parameter (the clamp cuts the colour path, and with a black background alpha has no
    effect on that channel); on channel 1 the SH gradient of the m = 0 coefficient is
    alpha C1."""
    W = H = 15
    f, z0, sig, o = 20.0, 2.0, 0.15, 0.7
    cam = cam_identity(W, H, f)
    sh = np.zeros((1, 4, 3), np.float32)
    sh[0, 2, 0], sh[0, 2, 1] = -2.0, 1.0
    env = env_of([node([[0, 0, z0]], sig, opac=o, sh_degree=1, sh=sh)])
    r = orc.render(env, cam, W, H)
    s2 = (f * f32(sig) / z0) ** 2 + 0.3
    a = _alpha_closed(np.eye(2) * s2, W / 2, H / 2, f32(o), W, H)
    assert 0.5 - 2 * C1 < 0
    np.testing.assert_array_equal(r["rgb"][..., 0], 0.0)
    np.testing.assert_allclose(r["rgb"][..., 1], a * (0.5 + C1), atol=1e-12)
    np.testing.assert_allclose(r["rgb"][..., 2], a * 0.5, atol=1e-12)
    wr = np.zeros((H, W, 3))
    wr[:, :, 0] = np.random.default_rng(0).standard_normal((H, W))
    gr = orc.backward(r, cam, W, H, wr)
    for k in ("means", "scales", "quats", "opacities", "sh"):
        assert np.all(gr[k] == 0.0), k
    wr = np.zeros((H, W, 3))
    wr[7, 7, 1] = 1.0
    gr = orc.backward(r, cam, W, H, wr)
    assert abs(gr["sh"][0, 2, 1] - a[7, 7] * C1) < 1e-12 and gr["sh"][0, 2, 0] == 0.0


def test_view_direction_sign_off_axis(orc):
    """Off-axis Gaussian at (x0, 0, z0): the view direction is (x0, 0, z0) / |.|, and the m = 1
    coefficient of degree 1 (basis -C1 x) moves the colour by -C1 k x0 / |.|."""
    W = H = 31
    f, x0, z0, k = 30.0, 0.4, 2.0, 0.6
    cam = cam_identity(W, H, f)
    sh = np.zeros((1, 4, 3), np.float32)
    sh[0, 3, :] = [k, -k, 0.0]
    env = env_of([node([[x0, 0, z0]], 0.1, opac=0.9, sh_degree=1, sh=sh)])
    r = orc.render(env, cam, W, H)
    xf, zf = float(np.float32(x0)), float(np.float32(z0))
    dxn = xf / math.hypot(xf, zf)
    col = np.array([0.5 - C1 * f32(k) * dxn, 0.5 + C1 * f32(k) * dxn, 0.5])
    m = r["alpha"] > 0
    np.testing.assert_allclose(r["rgb"][m], r["alpha"][m][:, None] * col[None, :], atol=1e-12)


# ------------------------------------------------- ambiguous decisions
def _edge_sigma(o, k, target, z0, f):
    """World sigma of an on-axis isotropic Gaussian whose alpha at a pixel k px from its
    centre (one axis) is target: o exp(-k^2 / (2 s^2)) = target, s^2 = (f sigma / z0)^2 + 0.3."""
    s2 = -k * k / (2 * math.log(target / o))
    return z0 / f * math.sqrt(s2 - 0.3)


@pytest.mark.parametrize("side", [+1, -1])
def test_alpha_decision_at_the_threshold_is_ambiguous(orc, side):
    """alpha = (1/255)(1 + side 3e-6) at one pixel: within the FP32 error of alpha (a few 1e-6
    there), so the oracle flags the decision and returns the other branch as the alternative:
    the Gaussian blended (rgb = alpha c) on one branch, skipped (rgb = background) on the
    other.  A pixel at (1/255)(1 + 1e-3) is not flagged."""
    W = H = 15
    f, z0, o, k = 20.0, 2.0, 0.8, 3
    cam = cam_identity(W, H, f, bg=(0.1, 0.2, 0.3))
    thr = 1 / 255
    c = np.array([0.9, 0.4, 0.2])
    sig = np.float32(_edge_sigma(o, k, thr * (1 + side * 3e-6), z0, f))
    env = env_of([node([[0, 0, z0]], sig, opac=o, colours=c)])
    r = orc.render(env, cam, W, H)
    s2 = (f * float(sig) / z0) ** 2 + 0.3
    al = f32(o) * math.exp(-k * k / (2 * s2))
    assert abs(al / thr - 1) < 4e-6 and np.sign(al - thr) == side
    py, px = 7, 7 + k
    bg = f32([0.1, 0.2, 0.3])
    blended, skipped = al * c + (1 - al) * bg, bg
    assert r["flags"][py, px] == 1  # one ambiguous decision, an alpha one
    main, alt = (blended, skipped) if side > 0 else (skipped, blended)
    np.testing.assert_allclose(r["rgb"][py, px], main, atol=1e-7)
    np.testing.assert_allclose(r["alt"][py, px, :3], alt, atol=1e-7)
    np.testing.assert_allclose(r["alt"][py, px, 4], al if side < 0 else 0.0, atol=1e-12)
    # clear of the threshold: no flag
    sig2 = np.float32(_edge_sigma(o, k, thr * (1 + 1e-3), z0, f))
    r2 = orc.render(env_of([node([[0, 0, z0]], sig2, opac=o, colours=c)]), cam, W, H)
    assert r2["flags"][py, px] == 0


@pytest.mark.parametrize("side", [+1, -1])
def test_stop_decision_at_the_threshold_is_ambiguous(orc, side):
    """n = 10 co-located identical Gaussians of alpha = o at the centre pixel, with
    (1 - o)^n = 1e-4 (1 + side 5e-6): the n-th transmittance test sits within the FP32 error
    of T (about 1e-5 after ten blends) of its threshold.  One branch blends n layers (alpha =
    1 - (1 - o)^n), the other n - 1; the oracle's main result and alternative are the two.
    With (1 - o)^n = 1e-4 (1 + 1e-2) the decision is not flagged."""
    n = 10
    cam = cam_identity(15, 15, 20.0)
    c = np.array([0.75, 0.5, 0.25])

    def run(rel):
        o = np.float32(1 - (1e-4 * (1 + rel)) ** (1 / n))
        nd = node(np.tile([[0, 0, 1.5]], (n + 3, 1)), 0.05, opac=o, colours=c)
        return o, orc.render(env_of([nd]), cam, 15, 15)

    o, r = run(side * 5e-6)
    q = 1 - float(o)
    assert abs(q ** n / 1e-4 - 1 - side * 5e-6) < 2e-6
    a_n, a_m = 1 - q ** n, 1 - q ** (n - 1)  # n and n - 1 layers
    main, alt = (a_n, a_m) if side > 0 else (a_m, a_n)
    assert r["flags"][7, 7] == 1 | 4  # one ambiguous decision, a stopping one
    assert abs(r["alpha"][7, 7] - main) < 1e-12 and abs(r["alt"][7, 7, 4] - alt) < 1e-12
    np.testing.assert_allclose(r["rgb"][7, 7], main * c, atol=1e-7)
    np.testing.assert_allclose(r["alt"][7, 7, :3], alt * c, atol=1e-7)
    np.testing.assert_allclose(r["alt"][7, 7, 3], alt * 1.5, atol=1e-12)
    _, r2 = run(1e-2)
    assert r2["flags"][7, 7] == 0


# ------------------------------------------------------------- node poses
def _so3_exp(w):
    th = np.linalg.norm(w)
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-300:
        return np.eye(3)
    return np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * (K @ K)


def test_pose_gradient_matches_fp64_finite_differences(orc):
    """dL/d(pose) of both nodes (background and a posed SH3 object) along the world-frame left
    perturbation R' = exp([omega]x) R, t' = exp([omega]x) t + rho, against FP64 central
    differences of the FP64 forward taken with the exact exponential map (h = 1e-6)."""
    env, cam = _fd_scene()
    W = H = 32
    g = np.random.default_rng(7)
    wr, wd, wa = g.standard_normal((H, W, 3)), g.standard_normal((H, W)), g.standard_normal((H, W))
    fe = orc.FlatEnv(env)
    rect, zb, vis = orc.keyspec(fe, cam, W, H, 16, 16)
    keys, vals, lv, ranges = orc.pairs(rect, zb, vis, W, H, 16, 16)
    R0 = fe.p64["pose_R"].copy().reshape(-1, 3, 3)
    t0 = fe.p64["pose_t"].copy().reshape(-1, 3)

    def fwd():
        geo = orc.project(fe, cam, W, H)
        out = orc.composite(geo, ranges, lv, W, H, 16, 16, cam["bg"])
        return float(np.sum(wr * out["rgb"]) + np.sum(wd * out["depth"]) + np.sum(wa * out["alpha"])), out["trace"]

    L0, tr0 = fwd()
    ref = dict(fe=fe, ranges=ranges, lvals=lv, geo=orc.project(fe, cam, W, H))
    gp = orc.backward(ref, cam, W, H, wr, wd, wa)["pose"]
    h = 1e-6
    checked = 0
    for k in range(fe.n_nodes):
        for j in range(6):
            vals_ = []
            for sgn in (1, -1):
                e = np.zeros(6)
                e[j] = sgn * h
                Rw = _so3_exp(e[:3])
                Rk, tk = fe.p64["pose_R"].reshape(-1, 3, 3), fe.p64["pose_t"].reshape(-1, 3)
                Rk[k] = Rw @ R0[k]
                tk[k] = Rw @ t0[k] + e[3:]
                vals_.append(fwd())
                Rk[k], tk[k] = R0[k], t0[k]
            (Lp, tp), (Lm, tm) = vals_
            if not (np.array_equal(tp, tr0) and np.array_equal(tm, tr0)):
                continue
            fd = (Lp - Lm) / (2 * h)
            scale = np.abs(gp[k]).max()
            assert abs(fd - gp[k, j]) <= 1e-5 * max(abs(fd), 1e-3 * scale), (k, j, fd, gp[k, j])
            checked += 1
    assert checked >= 10, checked
    assert np.abs(gp).min() > 0  # every component is exercised
