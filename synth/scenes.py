"""Seeded scene, pose and camera generators (float32 numpy arrays).

Conventions of the produced data (they are inputs, not renderer logic):

* A Gaussian set is a dict with ``means [n,3]``, ``scales [n,3]`` (activated,
  > 0), ``quats [n,4]`` (w, x, y, z; unit length up to rounding),
  ``opacities [n]`` (activated, in (0, 1)) and ``sh [n, K, 3]`` with
  K = (degree + 1)^2.
* The degree-0 colour v ~ U(0, 1) is stored as the DC coefficient
  (v - 0.5) / C0 with C0 = 1 / (2 sqrt(pi)) so that a renderer adding 0.5
  after SH evaluation reproduces v.  Higher orders are raw N(0, sigma^2).
* Cameras are world-to-camera rigid maps with OpenCV axes (x right, y down,
  z forward), world y up, built by look-at; intrinsics from a horizontal
  field of view with the principal point at the image centre.
* Node poses map node-local coordinates to world coordinates.
"""
import math
import os

import numpy as np

__all__ = [
    "rng", "gaussians_uniform_cube", "gaussians_room", "gaussians_object",
    "random_rotation", "object_poses", "look_at", "camera", "ring_cameras",
    "scene_config", "CONFIG_NAMES", "augment_params", "overlay_frames", "mesh_sphere", "lidar_rays",
]

C0 = 0.5 / math.sqrt(math.pi)


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _finish(g, n, means, log_scale_mu, log_scale_sigma, sh_degree, hi_sigma):
    """Draw everything after the means, in the fixed order (float32 draws)."""
    K = (sh_degree + 1) ** 2
    f32 = np.float32
    scales = np.exp(f32(log_scale_mu) + f32(log_scale_sigma) * g.standard_normal((n, 3), dtype=f32))
    q = g.standard_normal((n, 4), dtype=f32)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logits = g.standard_normal(n, dtype=f32)
    opac = (1.0 / (1.0 + np.exp(-logits))).astype(f32)
    dc = g.random((n, 3), dtype=f32)
    sh = np.empty((n, K, 3), dtype=f32)
    sh[:, 0, :] = (dc - f32(0.5)) * f32(1.0 / C0)
    if K > 1:
        hi = g.standard_normal((n, K - 1, 3), dtype=f32)
        hi *= f32(hi_sigma)
        sh[:, 1:, :] = hi
    return dict(means=np.ascontiguousarray(means, dtype=f32), scales=scales.astype(f32),
                quats=q, opacities=opac, sh=sh, sh_degree=sh_degree)


def gaussians_uniform_cube(n, seed, sh_degree=0, half=1.0, log_scale=(-3.0, 0.5), hi_sigma=0.05):
    """Means uniform in [-half, half]^3, log-scales N(mu, sigma^2) per axis."""
    g = rng(seed)
    means = (g.random((n, 3), dtype=np.float32) * np.float32(2 * half) - np.float32(half))
    return _finish(g, n, means, log_scale[0], log_scale[1], sh_degree, hi_sigma)


def gaussians_room(n, seed, sh_degree=3, clusters=64, half=5.0, spread=0.5,
                   log_scale=(-3.0, 0.5), hi_sigma=0.05):
    """A room-sized background: a mixture of ``clusters`` isotropic blobs.

    Cluster centres are uniform in the 10 m cube [-half, half]^3, each
    Gaussian picks a cluster uniformly and is offset by N(0, spread^2 I),
    clipped to the cube.
    """
    g = rng(seed)
    centres = g.uniform(-half, half, size=(clusters, 3))
    which = g.integers(0, clusters, size=n)
    off = g.standard_normal((n, 3), dtype=np.float32)
    off *= np.float32(spread)
    off += centres[which].astype(np.float32)
    means = np.clip(off, -half, half)
    return _finish(g, n, means, log_scale[0], log_scale[1], sh_degree, hi_sigma)


def gaussians_object(n, seed, sh_degree=3, radius=0.1, log_scale=(-5.5, 0.5), hi_sigma=0.05):
    """A small object node: means uniform in a ball of ``radius`` metres."""
    g = rng(seed)
    d = g.standard_normal((n, 3), dtype=np.float32)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = np.float32(radius) * g.random((n, 1), dtype=np.float32) ** np.float32(1.0 / 3.0)
    return _finish(g, n, d * r, log_scale[0], log_scale[1], sh_degree, hi_sigma)


def random_rotation(g):
    """Haar-uniform rotation: QR of a Gaussian matrix with the sign fixed."""
    A = g.standard_normal((3, 3))
    Q, Rq = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(Rq))[None, :]
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


OBJECT_ANCHORS = np.array([[x, 0.0, z] for z in (-0.15, 0.15) for x in (-0.45, -0.15, 0.15, 0.45)])


def object_poses(count, seed, jitter=0.5):
    """Per-step object poses: anchor + U[-jitter, jitter]^3, rotation uniform.

    Returns R [count, 3, 3] and t [count, 3] (float32), node-local -> world.
    """
    g = rng(seed)
    R = np.zeros((count, 3, 3))
    t = np.zeros((count, 3))
    for i in range(count):
        R[i] = random_rotation(g)
        t[i] = OBJECT_ANCHORS[i % len(OBJECT_ANCHORS)] + g.uniform(-jitter, jitter, size=3)
    return R.astype(np.float32), t.astype(np.float32)


def look_at(eye, target, up=(0.0, 1.0, 0.0)):
    """World-to-camera (R, t), OpenCV axes, for a camera at ``eye``."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ eye
    return R.astype(np.float32), t.astype(np.float32)


def camera(eye, target, width, height, hfov_deg=60.0, znear=0.2, bg=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)):
    R, t = look_at(eye, target, up)
    fx = (0.5 * width) / math.tan(math.radians(hfov_deg) * 0.5)
    return dict(R=R, t=t, fx=np.float32(fx), fy=np.float32(fx), cx=np.float32(0.5 * width),
                cy=np.float32(0.5 * height), znear=np.float32(znear),
                bg=np.asarray(bg, dtype=np.float32), width=int(width), height=int(height))


def ring_cameras(count, radius, width, height, hfov_deg=60.0, znear=0.2):
    cams = []
    for k in range(count):
        a = 2.0 * math.pi * k / count
        eye = (radius * math.sin(a), 0.0, -radius * math.cos(a))
        cams.append(camera(eye, (0.0, 0.0, 0.0), width, height, hfov_deg, znear))
    return cams


CONFIG_NAMES = {
    0: "plain forward: 20k Gaussians SH0, one 128x128 camera, 16x16 tiles",
    1: "single background: 1M Gaussians SH3 room, one 640x480 camera",
    2: "composed sim step: 2M background + 8x50k posed objects SH3, 3 cameras 640x480",
    3: "batched: 64 envs (100k-1M background + 4x20k posed objects each, SH3), 2 cameras 320x240 per env",
    4: "differentiable: 500k Gaussians SH3, 8 ring views 640x480",
}


def scene_config(cfg, seed=0, scale=1.0, n_envs=None):
    """Build a workload as ``dict(envs=[...], cams_per_env=C, width, height)``.

    Each env is ``dict(nodes=[gaussian dicts], poses=[(R, t)], cams=[camera dicts])``
    with node 0 the background (identity pose).  ``scale`` shrinks Gaussian
    counts (for tests); ``n_envs`` overrides the env count of the batched
    workload.
    """
    def cnt(n):
        return max(1, int(round(n * scale)))

    eye3 = np.eye(3, dtype=np.float32)
    z3 = np.zeros(3, dtype=np.float32)
    if cfg == 0:
        bg = gaussians_uniform_cube(cnt(20000), seed, sh_degree=0)
        cams = [camera((0, 0, -3), (0, 0, 0), 128, 128)]
        return dict(envs=[dict(nodes=[bg], poses=[(eye3, z3)], cams=cams)], cams_per_env=1,
                    width=128, height=128)
    if cfg == 1:
        bg = gaussians_room(cnt(1_000_000), seed)
        cams = [camera((0, 0, -4.5), (0, 0, 0), 640, 480)]
        return dict(envs=[dict(nodes=[bg], poses=[(eye3, z3)], cams=cams)], cams_per_env=1,
                    width=640, height=480)
    if cfg == 2:
        bg = gaussians_room(cnt(2_000_000), seed)
        nodes = [bg] + [gaussians_object(cnt(50_000), seed + 1 + k) for k in range(8)]
        R, t = object_poses(8, seed + 100)
        poses = [(eye3, z3)] + [(R[k], t[k]) for k in range(8)]
        cams = [camera((0, 0.6, -1.0), (0, 0, 0), 640, 480, znear=0.05),
                camera((0.3, 0.3, -0.4), (0.1, 0, 0), 640, 480, znear=0.05),
                camera((-0.3, 0.3, -0.4), (-0.1, 0, 0), 640, 480, znear=0.05)]
        return dict(envs=[dict(nodes=nodes, poses=poses, cams=cams)], cams_per_env=3,
                    width=640, height=480)
    if cfg == 3:
        E = 64 if n_envs is None else n_envs
        g = rng(seed)
        sizes = np.round(np.exp(g.uniform(math.log(1e5), math.log(1e6), size=E))).astype(np.int64)

        def make_env(e):
            bg = gaussians_room(cnt(int(sizes[e])), seed + 1000 + e)
            objs = [gaussians_object(cnt(20_000), seed + 5000 + 4 * e + k) for k in range(4)]
            R, t = object_poses(4, seed + 9000 + e)
            poses = [(eye3, z3)] + [(R[k], t[k]) for k in range(4)]
            cams = [camera((0, 0.6, -1.0), (0, 0, 0), 320, 240, znear=0.05),
                    camera((0.3, 0.3, -0.4), (0.1, 0, 0), 320, 240, znear=0.05)]
            return dict(nodes=[bg] + objs, poses=poses, cams=cams)

        # every env has its own seeds, so the result does not depend on the thread count
        from concurrent.futures import ThreadPoolExecutor
        workers = min(16, os.cpu_count() or 1)
        with ThreadPoolExecutor(workers) as ex:
            envs = list(ex.map(make_env, range(E)))
        return dict(envs=envs, cams_per_env=2, width=320, height=240)
    if cfg == 4:
        bg = gaussians_uniform_cube(cnt(500_000), seed, sh_degree=3)
        cams = ring_cameras(8, 3.0, 640, 480)
        return dict(envs=[dict(nodes=[bg], poses=[(eye3, z3)], cams=cams)], cams_per_env=8,
                    width=640, height=480)
    raise ValueError(f"unknown workload {cfg}")


def augment_params(n_images, seed, overlay_max=0.5, hue=0.05, sat=(0.7, 1.3), val=(0.7, 1.3), gamma=(0.7, 1.4)):
    """Per-image draws of the image-space augmentation, [n, 5] float32:
    overlay weight U(0, overlay_max), hue shift U(-hue, hue) turns, saturation and value scales
    uniform in their ranges, gamma log-uniform in its range."""
    g = rng(seed)
    p = np.empty((n_images, 5), np.float32)
    p[:, 0] = g.uniform(0.0, overlay_max, n_images)
    p[:, 1] = g.uniform(-hue, hue, n_images)
    p[:, 2] = g.uniform(sat[0], sat[1], n_images)
    p[:, 3] = g.uniform(val[0], val[1], n_images)
    p[:, 4] = np.exp(g.uniform(math.log(gamma[0]), math.log(gamma[1]), n_images))
    return p


def overlay_frames(n_images, height, width, seed):
    """Stand-ins for video crops: per image a few random low-frequency colour waves plus pixel
    noise, in [0, 1], [n, H, W, 3] float32."""
    g = rng(seed)
    yy, xx = np.meshgrid(np.arange(height, dtype=np.float32) / height, np.arange(width, dtype=np.float32) / width,
                         indexing="ij")
    out = np.empty((n_images, height, width, 3), np.float32)
    for i in range(n_images):
        img = np.full((height, width, 3), 0.5, np.float32)
        for _ in range(3):
            f = g.uniform(0.5, 4.0, 2).astype(np.float32)
            ph = g.uniform(0, 2 * math.pi, 3).astype(np.float32)
            amp = g.uniform(0.05, 0.25, 3).astype(np.float32)
            w = np.sin(2 * np.float32(math.pi) * (f[0] * xx + f[1] * yy))
            img += amp * np.stack([np.sin(w + ph[k]) for k in range(3)], axis=-1)
        img += np.float32(0.05) * g.standard_normal((height, width, 3), dtype=np.float32)
        out[i] = np.clip(img, 0.0, 1.0)
    return out


def mesh_sphere(n_lat, n_lon, seed, radius=0.1, noise=0.05, degenerate=4):
    """A closed latitude-longitude sphere mesh with radial noise (vertices [nv, 3] float32,
    faces [nf, 3] int32, outward winding), per-vertex colours U(0, 1), and ``degenerate``
    extra faces that repeat a vertex (zero area)."""
    g = rng(seed)
    verts = [[0.0, 0.0, radius], [0.0, 0.0, -radius]]
    for i in range(1, n_lat):
        th = math.pi * i / n_lat
        for j in range(n_lon):
            ph = 2 * math.pi * j / n_lon
            verts.append([radius * math.sin(th) * math.cos(ph), radius * math.sin(th) * math.sin(ph),
                          radius * math.cos(th)])
    v = np.asarray(verts, np.float64)
    v *= (1.0 + noise * g.standard_normal((len(v), 1)))
    ring = lambda i, j: 2 + (i - 1) * n_lon + (j % n_lon)
    faces = []
    for j in range(n_lon):
        faces.append([0, ring(1, j), ring(1, j + 1)])
        faces.append([1, ring(n_lat - 1, j + 1), ring(n_lat - 1, j)])
    for i in range(1, n_lat - 1):
        for j in range(n_lon):
            faces.append([ring(i, j), ring(i + 1, j), ring(i + 1, j + 1)])
            faces.append([ring(i, j), ring(i + 1, j + 1), ring(i, j + 1)])
    for k in range(degenerate):
        i = int(g.integers(0, len(v)))
        faces.append([i, i, int(g.integers(0, len(v)))])
    colours = g.random((len(v), 3), dtype=np.float32)
    return v.astype(np.float32), np.asarray(faces, np.int32), colours


def lidar_rays(origin, n_beams, n_azimuth, elevation=(-15.0, 15.0), tmin=0.05, tmax=50.0, R=None):
    """A spinning LiDAR's rays, [n_beams * n_azimuth, 8] float32 rows (origin[3], unit
    direction[3], tmin, tmax): beams at elevations uniform in ``elevation`` degrees (y up),
    azimuths uniform over the full turn, beam-major; ``R`` rotates the sensor frame to the
    world."""
    el = np.radians(np.linspace(elevation[0], elevation[1], n_beams))
    az = 2 * math.pi * np.arange(n_azimuth) / n_azimuth
    E, A = np.meshgrid(el, az, indexing="ij")
    d = np.stack([np.cos(E) * np.sin(A), np.sin(E), np.cos(E) * np.cos(A)], axis=-1).reshape(-1, 3)
    if R is not None:
        d = d @ np.asarray(R, np.float64).T
    d = d.astype(np.float32)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    out = np.empty((len(d), 8), np.float32)
    out[:, 0:3] = np.asarray(origin, np.float32)
    out[:, 3:6] = d
    out[:, 6] = tmin
    out[:, 7] = tmax
    return out
