"""Pins of the LiDAR ray-tracing oracle (paper Sec. III-C) against closed forms, brute-force
minimisation, invariants, and an independent FP32 evaluation for its error bound (no GPU)."""
import math

import numpy as np

import synth
from helpers import env_of, node, rot_axis
from oracle import lidar as L


def f32(x):
    """the value a float32 input array holds"""
    return float(np.float32(x))


def _ray(o, d, tmin=0.05, tmax=100.0):
    d = np.asarray(d, np.float64)
    d = d / np.linalg.norm(d)
    return np.array([*o, *d, tmin, tmax])


def test_single_gaussian_on_and_off_axis():
    sig, dist, o = f32(0.1), 2.0, f32(0.8)
    we = L.WorldEnv(env_of([node([[0, 0, dist]], sig, opac=o)]))
    on = L.trace(we, [_ray([0, 0, 0], [0, 0, 1])])
    assert abs(on["alpha"][0] - o) < 1e-14 and abs(on["range"][0] - o * dist) < 1e-14 and on["hits"][0] == 1
    h = 0.15  # perpendicular offset of the ray
    off = L.trace(we, [_ray([h, 0, 0], [0, 0, 1])])
    a = o * math.exp(-h * h / (2 * sig * sig))
    assert abs(off["alpha"][0] - a) < 1e-14 and abs(off["range"][0] - a * dist) < 1e-14
    # the 0.99 clamp
    we2 = L.WorldEnv(env_of([node([[0, 0, dist]], sig, opac=1.0)]))
    assert abs(L.trace(we2, [_ray([0, 0, 0], [0, 0, 1])])["alpha"][0] - 0.99) < 1e-14


def test_mahalanobis_minimum_by_brute_force_along_the_ray():
    from scipy.optimize import minimize_scalar
    g = np.random.default_rng(1)
    for k in range(20):
        s = np.exp(g.normal(-2.5, 0.7, 3)).astype(np.float32).astype(np.float64)
        q = g.standard_normal(4).astype(np.float32).astype(np.float64)
        mu = (g.uniform(-1, 1, 3) + [0, 0, 3]).astype(np.float32).astype(np.float64)
        env = env_of([node([mu], s, quats=[q], opac=0.99)])
        o = g.uniform(-0.2, 0.2, 3)
        d = mu - o + g.normal(0, 0.05, 3)
        d /= np.linalg.norm(d)
        r = L.trace(L.WorldEnv(env), [_ray(o, d)])
        # brute force: the smallest Mahalanobis distance over t on a grid, then a bounded
        # scalar minimisation around the best grid point
        R = L.quat_matrix(q)
        Minv = R @ np.diag(1 / s ** 2) @ R.T
        m = lambda t: float((o + t * d - mu) @ Minv @ (o + t * d - mu))
        ts = np.linspace(0, 6, 60001)
        P = o + ts[:, None] * d - mu
        i = int(np.argmin(np.einsum("ni,ij,nj->n", P, Minv, P)))
        D2 = minimize_scalar(m, bounds=(ts[max(i - 1, 0)], ts[min(i + 1, len(ts) - 1)]), method="bounded",
                             options=dict(xatol=1e-12)).fun
        want = f32(0.99) * math.exp(-0.5 * D2)
        if want >= 1 / 255 * 1.01:
            assert abs(r["alpha"][0] - min(0.99, want)) < 1e-9, (k, r["alpha"][0], want)
        elif want < 1 / 255 * 0.99:
            assert r["alpha"][0] == 0.0


def test_two_gaussians_in_order_of_their_centres_along_the_ray():
    n = node([[0.03, 0, 3.0], [0, 0.02, 1.5]], 0.1, opac=[0.6, 0.5])  # listed far first
    we = L.WorldEnv(env_of([n]))
    r = L.trace(we, [_ray([0, 0, 0], [0, 0, 1])])
    s2 = 2 * f32(0.1) ** 2
    a1 = f32(0.5) * math.exp(-f32(0.02) ** 2 / s2)
    a2 = f32(0.6) * math.exp(-f32(0.03) ** 2 / s2)
    assert abs(r["alpha"][0] - (1 - (1 - a1) * (1 - a2))) < 1e-14
    assert abs(r["range"][0] - (a1 * 1.5 + (1 - a1) * a2 * 3.0)) < 1e-13
    # the window (tmin, tmax) keeps only the nearer centre
    r2 = L.trace(we, [_ray([0, 0, 0], [0, 0, 1], tmax=2.0)])
    assert abs(r2["alpha"][0] - a1) < 1e-14


def test_thirteen_layers_of_one_half():
    zs = (2.0 + 0.01 * np.arange(20)).astype(np.float32).astype(np.float64)
    n = node([[0, 0, z] for z in zs], 0.05, opac=0.5)
    r = L.trace(L.WorldEnv(env_of([n])), [_ray([0, 0, 0], [0, 0, 1])])
    assert r["hits"][0] == 13
    assert abs(r["alpha"][0] - (1 - 2.0 ** -13)) < 1e-15
    assert abs(r["range"][0] - sum(0.5 ** (k + 1) * zs[k] for k in range(13))) < 1e-14


def test_permutation_and_joint_rigid_motion_invariance():
    bg = synth.gaussians_uniform_cube(400, 3, half=0.8, log_scale=(-2.5, 0.4))
    ob = synth.gaussians_object(100, 4, radius=0.3, log_scale=(-3.0, 0.3))
    Rk = synth.random_rotation(synth.rng(5))
    env = dict(nodes=[bg, ob], poses=[(np.eye(3), np.zeros(3)), (Rk, np.array([0.2, 0.1, -0.3]))])
    rays = synth.lidar_rays((0.0, 0.1, -2.5), 8, 32, elevation=(-20, 20), tmin=0.05, tmax=10).astype(np.float64)
    rays[:, 3:6] = np.tile([0, 0, 1], (len(rays), 1)) * 2.0 + rays[:, 3:6]  # aim forward, into the scene
    rays[:, 3:6] /= np.linalg.norm(rays[:, 3:6], axis=1, keepdims=True)
    ref = L.trace(L.WorldEnv(env), rays)
    assert (ref["hits"] > 0).sum() > 100
    # permute the background's Gaussians
    p = np.random.default_rng(6).permutation(400)
    bgp = {k: (v[p] if isinstance(v, np.ndarray) and len(v) == 400 else v) for k, v in bg.items()}
    perm = L.trace(L.WorldEnv(dict(nodes=[bgp, ob], poses=env["poses"])), rays)
    for k in ("range", "alpha", "hits"):
        np.testing.assert_allclose(perm[k], ref[k], atol=1e-12)
    # move scene and sensor together
    R0 = rot_axis([0.2, 1.0, -0.4], 1.1)
    t0 = np.array([1.0, -2.0, 0.5])
    env2 = dict(nodes=[bg, ob], poses=[(R0, t0), (R0 @ Rk, R0 @ np.array([0.2, 0.1, -0.3]) + t0)])
    rays2 = rays.copy()
    rays2[:, 0:3] = rays[:, 0:3] @ R0.T + t0
    rays2[:, 3:6] = rays[:, 3:6] @ R0.T
    mov = L.trace(L.WorldEnv(env2), rays2)
    for k in ("range", "alpha", "hits"):
        np.testing.assert_allclose(mov[k], ref[k], atol=1e-10)


def test_posed_node_equals_pretransformed_gaussians():
    ob = synth.gaussians_object(200, 7, radius=0.3, log_scale=(-3.0, 0.3))
    Rk = synth.random_rotation(synth.rng(8))
    tk = np.array([0.1, -0.05, 1.5])
    posed = L.WorldEnv(dict(nodes=[ob], poses=[(Rk, tk)]))
    moved = dict(ob)
    moved["means"] = ob["means"].astype(np.float64) @ Rk.T + tk
    Rq = L.quat_matrix(ob["quats"])
    W = Rk @ Rq
    # quaternion of W: through the matrix (the oracle normalises quaternions itself)
    from scipy.spatial.transform import Rotation
    xyzw = Rotation.from_matrix(W).as_quat()
    moved["quats"] = np.concatenate([xyzw[:, 3:4], xyzw[:, 0:3]], axis=1)
    pre = L.WorldEnv(dict(nodes=[moved], poses=[(np.eye(3), np.zeros(3))]))
    rays = synth.lidar_rays((0.0, 0.0, 0.0), 16, 16, elevation=(-10, 10), tmax=5).astype(np.float64)
    rays[:, 3:6] = np.array([0, 0, 1.0]) + 0.15 * rays[:, 3:6]
    rays[:, 3:6] /= np.linalg.norm(rays[:, 3:6], axis=1, keepdims=True)
    a, b = L.trace(posed, rays), L.trace(pre, rays)
    assert (a["hits"] > 0).sum() > 50
    for k in ("range", "alpha", "hits"):
        np.testing.assert_allclose(a[k], b[k], atol=1e-10)


def test_flipped_branches():
    sig, dist = 0.1, 2.0
    # skip decision: alpha at (1/255)(1 + 1e-7) on the axis
    o = f32((1 / 255) * (1 + 2e-7))
    assert o > 1 / 255
    r = L.trace(L.WorldEnv(env_of([node([[0, 0, dist]], sig, opac=o)])), [_ray([0, 0, 0], [0, 0, 1])])
    assert r["flags"][0] & 1 and r["hits"][0] == 1
    assert r["alt"][0, 1] == 0.0 and r["alt"][0, 0] == 0.0  # the other branch skips it
    # stop decision: ten layers with (1 - o)^10 = 1e-4 (1 + 1e-7), then more
    a = f32(1 - (1e-4 * (1 + 2e-7)) ** 0.1)
    assert (1 - a) ** 10 > 1e-4
    zs = (2.0 + 0.01 * np.arange(14)).astype(np.float32).astype(np.float64)
    r = L.trace(L.WorldEnv(env_of([node([[0, 0, z] for z in zs], 0.05, opac=a)])), [_ray([0, 0, 0], [0, 0, 1])])
    assert r["flags"][0] & 1
    # main: the tenth is blended (T(1-a) just above 1e-4), the other branch stops before it
    assert r["hits"][0] == 10
    T9 = (1 - a) ** 9
    assert abs(r["alt"][0, 1] - (1 - T9)) < 1e-12
    assert abs(r["alt"][0, 0] - sum(a * (1 - a) ** k * zs[k] for k in range(9))) < 1e-12


def test_fp32_bound_covers_an_independent_fp32_tracer():
    """An FP32 evaluation written here, in the node frame as a GPU would do it (ray moved by
    the FP32 pose, local mean, A = S^-1 R^T rounded to FP32), never exceeds the oracle's bound
    on D^2 / 2 over many (ray, Gaussian) pairs, including far and thin Gaussians."""
    f32 = np.float32
    g = np.random.default_rng(9)
    worst = 0.0
    for trial in range(6):
        n = 3000
        nd = synth.gaussians_object(n, 10 + trial, radius=0.4 + 3 * trial, log_scale=(-4.0 - 0.3 * trial, 0.6))
        Rk = synth.random_rotation(synth.rng(20 + trial)).astype(np.float32)
        tk = (g.uniform(-5, 5, 3) * trial).astype(np.float32)
        we = L.WorldEnv(dict(nodes=[nd], poses=[(Rk, tk)]))
        o = (tk + g.uniform(-1, 1, 3)).astype(np.float32)
        # rays aimed at random Gaussians with small offsets
        tgt = we.mu[g.integers(0, n, 64)] + g.normal(0, 0.02, (64, 3))
        d = (tgt - o).astype(np.float32)
        d /= np.linalg.norm(d, axis=1, keepdims=True).astype(np.float32)
        Rq = L.quat_matrix(nd["quats"])
        A32 = (np.transpose(Rq, (0, 2, 1)) / nd["scales"].astype(np.float64)[:, :, None]).astype(f32)
        mu32 = nd["means"].astype(f32)
        for r in range(64):
            ol = (Rk.T.astype(f32) @ (o - tk).astype(f32)).astype(f32)
            dl = (Rk.T.astype(f32) @ d[r]).astype(f32)
            q = (mu32 - ol).astype(f32)
            tc = (q @ dl).astype(f32)
            delta = (tc[:, None] * dl - q).astype(f32)
            Ad = np.einsum("nij,j->ni", A32, dl).astype(f32)
            Adel = np.einsum("nij,nj->ni", A32, delta).astype(f32)
            dd = np.sum(Adel * Adel, axis=1, dtype=f32)
            x = np.sum(Adel * Ad, axis=1, dtype=f32)
            aa = np.sum(Ad * Ad, axis=1, dtype=f32)
            D2_32 = np.maximum(dd - x * x / aa, f32(0)).astype(np.float64)
            # FP64 reference and bound
            q64 = we.mu - o.astype(np.float64)
            d64 = d[r].astype(np.float64)
            tc64 = q64 @ d64
            de = tc64[:, None] * d64 - q64
            Md = we.M @ d64
            Mde = np.einsum("nij,nj->ni", we.M, de)
            dd64 = np.einsum("ni,ni->n", de, Mde)
            D2 = np.maximum(dd64 - np.einsum("ni,ni->n", de, Md) ** 2 / (Md @ d64), 0.0)
            b = L._fp32_bound(D2, np.sqrt(dd64), np.linalg.norm(q64, axis=1), we.inv_smin, we.far,
                              np.linalg.norm(o.astype(np.float64)))
            near = D2 < 12.0  # pairs whose alpha can reach 1/255
            ratio = np.abs(0.5 * D2_32 - 0.5 * D2)[near] / b[near]
            if ratio.size:
                worst = max(worst, ratio.max())
    print("worst error / bound", worst)
    assert 0.02 < worst < 1.0, worst  # covers, and is within 50x of the worst error
