"""Pins of the mesh-to-Gaussian transfer oracle (paper Sec. IV-B) against closed forms and
invariants (no GPU)."""
import math

import numpy as np

import synth
from helpers import rot_axis
from oracle import mesh as M


def test_equilateral_triangle_closed_form():
    r = 0.3
    tri = np.array([[r * math.cos(2 * math.pi * k / 3), r * math.sin(2 * math.pi * k / 3), 0.0] for k in range(3)])
    out = M.mesh_to_gaussians(tri, [[0, 1, 2]], flatten=0.05, opacity=0.7)
    np.testing.assert_allclose(out["means"][0], 0.0, atol=1e-15)
    np.testing.assert_allclose(out["scales"][0], [r, r, 0.05 * r], atol=1e-15)  # circumradius
    np.testing.assert_allclose(out["normal"][0], [0, 0, 1], atol=1e-15)  # counter-clockwise seen from +z
    np.testing.assert_allclose(M.covariance(out["R"], out["scales"])[0], np.diag([r * r, r * r, (0.05 * r) ** 2]),
                               atol=1e-15)
    assert out["opacities"][0] == 0.7
    # the other winding flips the normal, not the covariance
    o2 = M.mesh_to_gaussians(tri, [[0, 2, 1]], flatten=0.05)
    np.testing.assert_allclose(o2["normal"][0], [0, 0, -1], atol=1e-15)
    np.testing.assert_allclose(M.covariance(o2["R"], o2["scales"]), M.covariance(out["R"], out["scales"]), atol=1e-15)


def test_right_triangle_closed_form():
    tri = np.array([[0.0, 0, 0], [3, 0, 0], [0, 3, 0]])
    out = M.mesh_to_gaussians(tri, [[0, 1, 2]], flatten=0.0)
    np.testing.assert_allclose(out["means"][0], [1, 1, 0], atol=1e-15)
    st = (math.sqrt(2) + 2 * math.sqrt(5)) / 3
    np.testing.assert_allclose(out["scales"][0], [st, st, 0], atol=1e-14)
    # frame: first axis along the edge a -> b, normal +z, second = n x t1 = +y
    np.testing.assert_allclose(out["R"][0], np.eye(3), atol=1e-15)


def test_frame_is_a_rotation_with_the_normal_third():
    v, f, _ = synth.mesh_sphere(12, 20, 1, degenerate=0)
    out = M.mesh_to_gaussians(v, f)
    R = out["R"]
    np.testing.assert_allclose(R @ np.transpose(R, (0, 2, 1)), np.broadcast_to(np.eye(3), R.shape), atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-12)
    np.testing.assert_allclose(R[:, :, 2], out["normal"], atol=1e-15)
    # the normal of an outward-wound closed sphere points away from the centre
    assert (np.sum(out["normal"] * out["means"], axis=1) > 0).all()


def test_rigid_motion_moves_means_and_rotates_covariances():
    v, f, col = synth.mesh_sphere(8, 12, 2, degenerate=0)
    Rm = rot_axis([0.3, -1.0, 0.5], 0.9)
    t = np.array([0.5, -0.2, 1.0])
    a = M.mesh_to_gaussians(v, f, col, flatten=0.02)
    b = M.mesh_to_gaussians(v.astype(np.float64) @ Rm.T + t, f, col, flatten=0.02)
    np.testing.assert_allclose(b["means"], a["means"] @ Rm.T + t, atol=1e-12)
    np.testing.assert_allclose(b["scales"], a["scales"], atol=1e-12)
    Sa, Sb = M.covariance(a["R"], a["scales"]), M.covariance(b["R"], b["scales"])
    np.testing.assert_allclose(Sb, Rm @ Sa @ Rm.T, atol=1e-12)
    np.testing.assert_allclose(b["sh"], a["sh"], atol=0)


def test_colour_is_the_mean_vertex_colour_through_the_dc_coefficient():
    v, f, col = synth.mesh_sphere(6, 8, 3, degenerate=0)
    out = M.mesh_to_gaussians(v, f, col, sh_degree=2)
    want = col.astype(np.float64)[f].mean(axis=1)
    np.testing.assert_allclose(out["sh"][:, 0, :] * M.C0 + 0.5, want, atol=1e-12)
    assert out["sh"].shape == (len(f), 9, 3) and not out["sh"][:, 1:].any()


def test_degenerate_faces_are_transparent():
    v, f, _ = synth.mesh_sphere(6, 8, 4, degenerate=5)
    out = M.mesh_to_gaussians(v, f)
    deg = f[:, 0] == f[:, 1]
    assert deg.sum() == 5
    assert (out["opacities"][deg] == 0).all() and (out["opacities"][~deg] > 0).all()
    np.testing.assert_allclose(out["R"][deg], np.broadcast_to(np.eye(3), (5, 3, 3)))


def test_quaternion_matrix_is_the_textbook_rotation():
    # 90 degrees about z: (w, x, y, z) = (cos 45, 0, 0, sin 45); also any positive multiple
    q = np.array([[math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)], [2 * math.cos(math.pi / 4), 0, 0,
                                                                           2 * math.sin(math.pi / 4)]])
    R = M.quat_to_matrix(q)
    np.testing.assert_allclose(R[0], [[0, -1, 0], [1, 0, 0], [0, 0, 1]], atol=1e-15)
    np.testing.assert_allclose(R[1], R[0], atol=1e-15)
    np.testing.assert_allclose(M.quat_to_matrix([[0.3, -0.2, 0.9, 0.1]])[0], rot_axis(
        [-0.2, 0.9, 0.1], 2 * math.acos(0.3 / math.sqrt(0.3 ** 2 + 0.2 ** 2 + 0.9 ** 2 + 0.1 ** 2))), atol=1e-12)
