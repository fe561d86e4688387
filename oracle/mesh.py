"""Oracle of the mesh-to-Gaussian transfer (paper Sec. IV-B, "Mesh-Gaussian Transfer").

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark, never by the renderer
package.  Plain numpy in FP64, one face at a time in vectorised form, in the order the paper
states the construction:

  * one Gaussian per mesh facet, its centre at the facet's barycentre;
  * the ellipsoid flattened to a planar primitive whose local frame is aligned with the face
    normal: the frame's third axis is the unit normal n = (b - a) x (c - a) / |...|, the first
    the unit direction of the edge a -> b, the second n x t1 (a reading: the paper fixes only
    the normal; the two tangent scales are equal, so the covariance does not depend on the
    in-plane axes);
  * both tangent scales equal the mean distance from the barycentre to the three vertices;
    the normal scale is ``flatten`` times that (a reading of "flatten ... to 2D");
  * opacity ``opacity`` and colour the mean of the vertex colours (grey 0.5 without them),
    stored as the degree-0 SH coefficient (colour - 0.5) / C0 with C0 = 1 / (2 sqrt(pi)); the
    higher SH orders are zero (readings: the paper initialises only geometry).
  * a degenerate facet (zero area) keeps its centre and scales, gets opacity 0 and the
    identity rotation.
"""
import math

import numpy as np

C0 = 0.5 / math.sqrt(math.pi)


def mesh_to_gaussians(vertices, faces, colours=None, flatten=0.01, opacity=0.9, sh_degree=0):
    v = np.asarray(vertices, np.float64).reshape(-1, 3)
    f = np.asarray(faces, np.int64).reshape(-1, 3)
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    g = (a + b + c) / 3.0
    st = (np.linalg.norm(a - g, axis=1) + np.linalg.norm(b - g, axis=1) + np.linalg.norm(c - g, axis=1)) / 3.0
    cr = np.cross(b - a, c - a)
    area2 = np.linalg.norm(cr, axis=1)
    e1 = np.linalg.norm(b - a, axis=1)
    ok = (area2 > 0) & (e1 > 0)
    n = cr / np.where(ok, area2, 1.0)[:, None]
    t1 = (b - a) / np.where(ok, e1, 1.0)[:, None]
    t2 = np.cross(n, t1)
    R = np.stack([t1, t2, n], axis=2)  # columns: t1, t2, n
    R[~ok] = np.eye(3)
    scales = np.stack([st, st, flatten * st], axis=1)
    K = (sh_degree + 1) ** 2
    sh = np.zeros((len(f), K, 3))
    col = np.full((len(f), 3), 0.5) if colours is None else (
        np.asarray(colours, np.float64).reshape(-1, 3)[f].sum(axis=1) / 3.0)
    sh[:, 0, :] = (col - 0.5) / C0
    op = np.where(ok, opacity, 0.0)
    return dict(means=g, scales=scales, R=R, opacities=op, sh=sh, normal=np.where(ok[:, None], n, 0.0))


def quat_to_matrix(q):
    """Rotation matrix of quaternions (w, x, y, z) of any non-zero length, [n, 3, 3]."""
    q = np.asarray(q, np.float64).reshape(-1, 4)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], axis=1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], axis=1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], axis=1)], axis=1)


def covariance(R, scales):
    """R diag(s)^2 R^T per Gaussian."""
    M = np.asarray(R, np.float64) * np.asarray(scales, np.float64)[:, None, :]
    return M @ np.transpose(M, (0, 2, 1))
