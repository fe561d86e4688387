"""Pins of the oracle's FP32 error bound (which blending decisions are ambiguous) against an
independent FP32 renderer written here with numpy float32 arithmetic (no GPU).

The oracle flags a decision as ambiguous when its distance to the threshold is below a
first-order bound of the error an FP32 renderer makes in the compared quantity
(oracle/gsr_oracle.c: fp32_bounds, decision_bound).  Two checks pin that bound to something
other than itself:

* every (Gaussian, pixel) pair: the FP32 alpha of this emulation lies within the bound of
  the FP64 alpha (the bound is not too small), while the bound stays within a modest factor
  of the error actually seen (it is not vacuous);
* every pixel: the emulation's RGB-D result equals the oracle's, or, for a pixel with one
  ambiguous decision, the oracle's flipped-branch result (the rule the GPU tests apply).

The emulation follows the FP32 operation sequence of the key specification for the camera
map, the projection and the 2D covariance (fma written as an exactly rounded product plus a
sum rounded twice, within one ulp of a fused one), divides for the conic and evaluates the
exponent with fma chains; it shares nothing with the HIP kernels.  Scenes are chosen to
stress each term of the bound: room-scale coordinates seen from a close camera (cancellation
in the camera map), elongated splats (ill-conditioned 2D covariance), splats beyond the
J clamp, and dense stacks that stop on the transmittance test.
"""
import math

import numpy as np
import pytest

import synth
from helpers import cam_identity

F = np.float32


def fma(a, b, c):
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(F)


def emulate_projection(fe, cam, W, H):
    """FP32 u, v, conic (A, B, C), log2 o, colour (SH degree 0) and z of every Gaussian;
    valid marks the Gaussians an FP32 renderer keeps (z > znear, det > 0)."""
    n = fe.n
    Rc = np.asarray(cam["R"], F).astype(np.float64).reshape(3, 3)
    tc = np.asarray(cam["t"], F).astype(np.float64)
    node = fe.node
    Wn = np.zeros((fe.n_nodes, 3, 3), F)
    wn = np.zeros((fe.n_nodes, 3), F)
    for k in range(fe.n_nodes):
        Rk = fe.pose_R[k].reshape(3, 3).astype(np.float64)
        tk = fe.pose_t[k].astype(np.float64)
        Wn[k] = (Rc @ Rk).astype(F)
        wn[k] = (Rc @ tk + tc).astype(F)
    Wg, wg = Wn[node], wn[node]
    mu = fe.means
    p = [fma(Wg[:, r, 0], mu[:, 0], fma(Wg[:, r, 1], mu[:, 1], fma(Wg[:, r, 2], mu[:, 2], wg[:, r]))) for r in range(3)]
    z = p[2]
    fx, fy, cx, cy, zn = (F(cam[k]) for k in ("fx", "fy", "cx", "cy", "znear"))
    with np.errstate(all="ignore"):
        iz = F(1) / z
        xz, yz = p[0] * iz, p[1] * iz
        u, v = fma(fx, xz, cx), fma(fy, yz, cy)
        q = fe.quats
        n2 = fma(q[:, 0], q[:, 0], fma(q[:, 1], q[:, 1], fma(q[:, 2], q[:, 2], q[:, 3] * q[:, 3])))
        rn = F(1) / np.sqrt(n2)
        qw, qx, qy, qz = q[:, 0] * rn, q[:, 1] * rn, q[:, 2] * rn, q[:, 3] * rn
        xx, yy, zz = qx * qx, qy * qy, qz * qz
        xy, xzq, yzq, wx, wy, wz = qx * qy, qx * qz, qy * qz, qw * qx, qw * qy, qw * qz
        R = [[fma(F(-2), yy + zz, F(1)), F(2) * (xy - wz), F(2) * (xzq + wy)],
             [F(2) * (xy + wz), fma(F(-2), xx + zz, F(1)), F(2) * (yzq - wx)],
             [F(2) * (xzq - wy), F(2) * (yzq + wx), fma(F(-2), xx + yy, F(1))]]
        s = fe.scales
        M = [[fma(Wg[:, r, 0], R[0][c], fma(Wg[:, r, 1], R[1][c], Wg[:, r, 2] * R[2][c])) * s[:, c] for c in range(3)]
             for r in range(3)]
        S = [[fma(M[a][0], M[b][0], fma(M[a][1], M[b][1], M[a][2] * M[b][2])) for b in range(3)] for a in range(3)]
        limx = F(1.3) * ((F(0.5) * F(W)) / fx)
        limy = F(1.3) * ((F(0.5) * F(H)) / fy)
        xc, yc = np.clip(xz, -limx, limx), np.clip(yz, -limy, limy)
        j00, j11 = fx * iz, fy * iz
        j02, j12 = -(j00 * xc), -(j11 * yc)
        T0 = [fma(j00, S[0][k], j02 * S[2][k]) for k in range(3)]
        T1 = [fma(j11, S[1][k], j12 * S[2][k]) for k in range(3)]
        a = fma(T0[0], j00, T0[2] * j02) + F(0.3)
        b = fma(T0[1], j11, T0[2] * j12)
        c = fma(T1[1], j11, T1[2] * j12) + F(0.3)
        det = fma(a, c, -(b * b))
        A, B, C = c / det, -b / det, a / det
        lo = np.log2(fe.opac)
        col = np.maximum(fma(F(0.5 / math.sqrt(math.pi)), fe.sh[:, 0:3], F(0.5)), F(0))
    valid = (z > zn) & (det > 0) & (fe.opac >= F(1 / 255))
    return dict(u=u, v=v, A=A, B=B, C=C, lo=lo, col=col, z=z, valid=valid)


def emulate_alpha(pr, i, px, py):
    """FP32 o G (before the 0.99 clamp) of Gaussian i at pixel (px, py)."""
    dx = (px.astype(F) + F(0.5)) - pr["u"][i]
    dy = (py.astype(F) + F(0.5)) - pr["v"][i]
    Ap = F(-0.7213475204444817) * pr["A"][i]
    Bp = F(-1.4426950408889634) * pr["B"][i]
    Cp = F(-0.7213475204444817) * pr["C"][i]
    qv = fma(Bp * dx, dy, fma(Cp * dy, dy, fma(Ap * dx, dx, pr["lo"][i])))
    with np.errstate(all="ignore"):
        return np.exp2(qv)


def emulate_composite(pr, ranges, lvals, W, H, tw, th, bg):
    """FP32 front-to-back compositing of every pixel (the rule of the oracle, in float32)."""
    rgb = np.zeros((H, W, 3), F)
    depth = np.zeros((H, W), F)
    alpha = np.zeros((H, W), F)
    tiles_x = (W + tw - 1) // tw
    thr = F(1 / 255)
    for t in range(len(ranges)):
        ty, tx = divmod(t, tiles_x)
        ys, xs = np.mgrid[ty * th:min(H, ty * th + th), tx * tw:min(W, tx * tw + tw)]
        px, py = xs.reshape(-1), ys.reshape(-1)
        T = np.ones(px.size, F)
        live = np.ones(px.size, bool)
        Cc = np.zeros((px.size, 3), F)
        D = np.zeros(px.size, F)
        for j in range(ranges[t, 0], ranges[t, 1]):
            i = lvals[j]
            al = np.minimum(F(0.99), emulate_alpha(pr, i, px, py))
            blend = live & (al >= thr)
            w = al * T
            Tn = T - w
            stop = blend & (Tn < F(1e-4))
            live &= ~stop
            blend &= ~stop
            wb = np.where(blend, w, F(0))
            Cc = fma(wb[:, None], pr["col"][i][None, :], Cc)
            D = fma(wb, pr["z"][i], D)
            T = np.where(blend, Tn, T)
            if not live.any():
                break
        bgv = np.asarray(bg, F)
        rgb[py, px] = fma(T[:, None], bgv[None, :], Cc)
        depth[py, px] = D
        alpha[py, px] = F(1) - T
    return rgb, depth, alpha


def _pairs_in_rects(rect, vis, W, H, tw, th):
    gi, pxs, pys = [], [], []
    for i in np.nonzero(vis == 0)[0]:
        x0, y0, x1, y1 = rect[i]
        ys, xs = np.mgrid[y0 * th:min(H, y1 * th), x0 * tw:min(W, x1 * tw)]
        gi.append(np.full(xs.size, i, np.int32))
        pxs.append(xs.reshape(-1))
        pys.append(ys.reshape(-1))
    return np.concatenate(gi), np.concatenate(pxs).astype(np.int32), np.concatenate(pys).astype(np.int32)


def _sh0(g):
    g = dict(g)
    g["sh"] = np.ascontiguousarray(g["sh"][:, :1])
    g["sh_degree"] = 0
    return g


def _scenes():
    eye, z3 = np.eye(3, dtype=np.float32), np.zeros(3, np.float32)
    out = {}
    # room-scale coordinates seen from a camera 1 m from the origin (cancellation in W mu + w)
    room = _sh0(synth.gaussians_room(4000, 3, clusters=8, half=5.0, spread=0.6, log_scale=(-3.3, 0.5)))
    out["room, close camera"] = (dict(nodes=[room], poses=[(eye, z3)], cams=[]),
                                 synth.camera((0.0, 0.6, -1.0), (0, 0, 0), 96, 72, znear=0.05), (16, 16), 0.01)
    # elongated splats (axis ratios up to ~50): ill-conditioned 2D covariances
    el = _sh0(synth.gaussians_uniform_cube(1500, 4, half=0.8, log_scale=(-3.5, 0.9)))
    obj = _sh0(synth.gaussians_object(300, 5, radius=0.4, log_scale=(-4.0, 1.0)))
    R = synth.random_rotation(synth.rng(6)).astype(np.float32)
    out["elongated, posed node"] = (dict(nodes=[el, obj], poses=[(eye, z3), (R, np.array([0.3, -0.2, 0.1], np.float32))],
                                         cams=[]), synth.camera((0.4, 0.3, -2.5), (0, 0, 0), 80, 64), (16, 8), 0.05)
    # splats close to the camera and beyond the J clamp
    near = _sh0(synth.gaussians_uniform_cube(1200, 7, half=1.5, log_scale=(-2.8, 0.5)))
    out["near camera, J clamp"] = (dict(nodes=[near], poses=[(eye, z3)], cams=[]),
                                   synth.camera((0.0, 0.0, -1.6), (0, 0, 0), 64, 48, znear=0.05), (8, 8), 0.01)
    # a background whose means lie 300 m from the world origin, seen from 1.5 m: the camera map
    # cancels terms of 300 m in FP32 (a posed node's offset would cancel in the FP64 composition)
    far = _sh0(synth.gaussians_uniform_cube(1500, 9, half=0.5, log_scale=(-4.0, 0.4)))
    off = np.array([300.0, -40.0, 250.0], np.float32)
    far["means"] = (far["means"] + off).astype(np.float32)
    cam = synth.camera(off + np.array([0.2, 0.3, -1.5]), off, 64, 64, znear=0.05)
    out["means 300 m from the origin"] = (dict(nodes=[far], poses=[(eye, z3)], cams=[]), cam, (16, 16), None)
    # a dense stack of opaque splats: most pixels stop on the transmittance test
    g = np.random.default_rng(8)
    dense = _sh0(synth.gaussians_uniform_cube(900, 8, half=0.25, log_scale=(-2.3, 0.3)))
    dense["opacities"] = g.uniform(0.3, 0.995, size=900).astype(np.float32)
    out["dense stack"] = (dict(nodes=[dense], poses=[(eye, z3)], cams=[]), cam_identity(48, 48, 60.0), (16, 16), 0.01)
    return out


SCENES = _scenes()


@pytest.mark.parametrize("name", list(SCENES))
def test_fp32_alpha_within_the_oracle_bound(orc, name):
    env, cam, (tw, th), _ = SCENES[name]
    W, H = cam["width"], cam["height"]
    fe = orc.FlatEnv(env)
    rect, zb, vis = orc.keyspec(fe, cam, W, H, tw, th)
    geo = orc.project(fe, cam, W, H)
    pr = emulate_projection(fe, cam, W, H)
    assert np.array_equal(pr["valid"] & (vis == 0), vis == 0)
    gi, px, py = _pairs_in_rects(rect, vis, W, H, tw, th)
    a64, bound = orc.alpha_bounds(geo, gi, px, py)
    a32 = emulate_alpha(pr, gi, px, py).astype(np.float64)
    m = a64 > 1e-6  # FP32 exp2 underflows far below the 1/255 threshold
    err = np.abs(a32[m] - a64[m]) / a64[m]
    ratio = err / bound[m]
    print(f"{name}: {m.sum()} pairs, FP32 alpha rel. error median {np.median(err):.2e} max {err.max():.2e}; "
          f"bound median {np.median(bound[m]):.2e}; error / bound median {np.median(ratio):.3f} max {ratio.max():.3f}")
    assert m.sum() > 5000
    assert ratio.max() <= 1.0, "an FP32 alpha left the oracle's bound"
    # not vacuous: the largest error seen comes within 20x of its bound (a bound inflated by a
    # stray factor, or a term of the wrong order, would not)
    assert ratio.max() >= 0.05, ratio.max()


@pytest.mark.parametrize("name", list(SCENES))
def test_fp32_renderer_matches_oracle_under_the_ambiguity_rule(orc, name):
    env, cam, (tw, th), cap = SCENES[name]
    if cap is None:
        pytest.skip("FP32 pixel values of this scene carry errors beyond 1e-4 (300 m coordinates): bound pin only")
    W, H = cam["width"], cam["height"]
    r = orc.render(env, cam, W, H, tw, th)
    pr = emulate_projection(r["fe"], cam, W, H)
    rgb, depth, alpha = emulate_composite(pr, r["ranges"], r["lvals"], W, H, tw, th, cam["bg"])
    rgb, depth, alpha = rgb.reshape(-1, 3), depth.reshape(-1), alpha.reshape(-1)
    e_main = np.maximum(np.abs(rgb - r["rgb"].reshape(-1, 3)).max(1),
                        np.maximum(np.abs(depth - r["depth"].reshape(-1)), np.abs(alpha - r["alpha"].reshape(-1))))
    alt = r["alt"].reshape(-1, 5)
    e_alt = np.maximum(np.abs(rgb - alt[:, :3]).max(1),
                       np.maximum(np.abs(depth - alt[:, 3]), np.abs(alpha - alt[:, 4])))
    flags = r["flags"].reshape(-1)
    amb, excl = (flags & 1) != 0, (flags & 2) != 0
    tol = 1e-4
    ok = (e_main <= tol) | (amb & (e_alt <= tol)) | excl
    flipped = int((amb & (e_main > tol)).sum())
    print(f"{name}: {W * H} px, ambiguous {int(amb.sum())}, excluded {int(excl.sum())}, FP32 took the other branch "
          f"at {flipped}, max err outside ambiguous {e_main[~amb].max():.2e}, alpha max {r['alpha'].max():.3f}")
    assert ok.all(), f"{int((~ok).sum())} pixels differ beyond both branches"
    # few ambiguous pixels (the stress scene of very elongated splats has more), fewer excluded
    assert amb.sum() <= max(3, cap * W * H) and excl.sum() <= max(1, 0.1 * cap * W * H)
