"""Small scene builders shared by the tests (inputs only, no renderer arithmetic)."""
import math

import numpy as np

C0 = 0.5 / math.sqrt(math.pi)


def node(means, scales, quats=None, opac=None, colours=None, sh_degree=0, sh=None):
    means = np.asarray(means, np.float32).reshape(-1, 3)
    n = len(means)
    K = (sh_degree + 1) ** 2
    scales = np.broadcast_to(np.asarray(scales, np.float32), (n, 3)).copy()
    if quats is None:
        quats = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1))
    quats = np.broadcast_to(np.asarray(quats, np.float32), (n, 4)).copy()
    opac = np.broadcast_to(np.asarray(0.8 if opac is None else opac, np.float32), (n,)).copy()
    if sh is None:
        sh = np.zeros((n, K, 3), np.float32)
        cols = np.broadcast_to(np.asarray(0.5 if colours is None else colours, np.float64), (n, 3))
        sh[:, 0, :] = (cols - 0.5) / C0
    return dict(means=means, scales=scales, quats=quats, opacities=opac,
                sh=np.asarray(sh, np.float32).reshape(n, K, 3), sh_degree=sh_degree)


def cam_identity(width, height, f, znear=0.2, bg=(0.0, 0.0, 0.0)):
    """Camera at the world origin looking along +z (world == camera axes)."""
    return dict(R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32), fx=np.float32(f),
                fy=np.float32(f), cx=np.float32(width / 2), cy=np.float32(height / 2),
                znear=np.float32(znear), bg=np.asarray(bg, np.float32), width=width, height=height)


def env_of(nodes, poses=None):
    eye = np.eye(3, dtype=np.float32)
    z3 = np.zeros(3, np.float32)
    if poses is None:
        poses = [(eye, z3)] * len(nodes)
    return dict(nodes=list(nodes), poses=list(poses), cams=[])


def rot_axis(axis, angle):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)
