"""GPU parity of the mesh-to-Gaussian transfer (paper Sec. IV-B) against the FP64 oracle.

Compared: centres, scales, opacities and SH directly; the rotation through what is unique --
the covariance R diag(s)^2 R^T (the two tangent scales are equal, so it does not depend on the
in-plane axes) and the normal (the rotation's third column).  Tolerances from FP32 rounding
of a few operations on coordinates of size |x|: centres and scales within 1e-6 (|x| + d),
covariances within 1e-5 max|S|, normals within 1e-5 (the cross product loses digits on thin
facets; the meshes here have none thinner than about 1:20)."""
import numpy as np
import pytest

import synth
from gpu_util import log
from oracle import mesh as M

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


@pytest.mark.parametrize("sh_degree,with_colours", [(0, True), (3, True), (1, False)])
def test_mesh_transfer_matches_oracle(gsr, ctx, sh_degree, with_colours):
    import torch
    v, f, col = synth.mesh_sphere(150, 200, 11, radius=0.2, degenerate=7)
    ref = M.mesh_to_gaussians(v, f, col if with_colours else None, flatten=0.02, opacity=0.85, sh_degree=sh_degree)
    node = gsr.mesh_to_gaussians(ctx, torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda(),
                                 torch.from_numpy(col).cuda() if with_colours else None, flatten=0.02, opacity=0.85,
                                 sh_degree=sh_degree)
    torch.cuda.synchronize()
    got = {k: t.cpu().numpy().astype(np.float64) for k, t in node.items()}
    scale = np.abs(v).max() + ref["scales"].max()
    assert np.abs(got["means"] - ref["means"]).max() <= 1e-6 * scale
    assert np.abs(got["scales"] - ref["scales"]).max() <= 1e-6 * scale
    assert np.array_equal(got["opacities"] == 0, ref["opacities"] == 0)
    np.testing.assert_allclose(got["opacities"], ref["opacities"], atol=1e-7)
    np.testing.assert_allclose(got["sh"], ref["sh"], atol=1e-5)
    np.testing.assert_allclose(np.linalg.norm(got["quats"], axis=1), 1.0, atol=1e-6)
    Rg = M.quat_to_matrix(got["quats"])
    ok = ref["opacities"] > 0
    nerr = np.abs(Rg[ok][:, :, 2] - ref["normal"][ok]).max()
    Sg, Sr = M.covariance(Rg, got["scales"]), M.covariance(ref["R"], ref["scales"])
    serr = np.abs(Sg - Sr).max() / np.abs(Sr).max()
    log(f"{len(f)} faces: max normal error {nerr:.3g}, covariance {serr:.3g}")
    assert nerr <= 1e-5 and serr <= 1e-5


def test_mesh_transfer_refuses_out_of_range_faces(gsr, ctx):
    import torch
    v, f, col = synth.mesh_sphere(10, 12, 12, degenerate=0)
    f = f.copy()
    f[5, 1] = len(v)  # one past the last vertex
    with pytest.raises(gsr.GsrError) as e:
        gsr.mesh_to_gaussians(ctx, torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda())
    assert e.value.code == -1 and "1 faces" in str(e.value)


def test_transferred_mesh_composes_and_renders(gsr, ctx):
    """The output is a node: a posed sphere mesh composed beside a background renders, and
    its pixels cover the sphere's silhouette (the facets tile the surface)."""
    import torch
    v, f, col = synth.mesh_sphere(40, 60, 13, radius=0.3, noise=0.0, degenerate=0)
    node = gsr.mesh_to_gaussians(ctx, torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda(),
                                 torch.from_numpy(col).cuda(), flatten=0.01, opacity=0.99, sh_degree=0)
    cam = synth.camera((0, 0, -2.0), (0, 0, 0), 64, 64)
    scene = gsr.compose_scene(ctx, [[node]], gsr.poses_tensor([(np.eye(3), np.zeros(3))]))
    ctx.set_tile(16, 16)
    rgb, depth, alpha = gsr.render_rgbd(ctx, scene, gsr.cameras_tensor([cam]), 64, 64)
    torch.cuda.synchronize()
    a = alpha[0, 0].cpu().numpy()
    # silhouette radius: f r / sqrt(d^2 - r^2) pixels around the centre
    rpx = float(cam["fx"]) * 0.3 / np.sqrt(4.0 - 0.09)
    yy, xx = np.mgrid[0:64, 0:64] + 0.5
    rr = np.hypot(xx - 32, yy - 32)
    assert a[rr < rpx - 2].min() > 0.99 and a[rr > rpx + 3].max() < 0.05
