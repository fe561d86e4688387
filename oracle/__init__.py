"""CPU oracle for the tiled Gaussian-splatting RGB-D renderer.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark, never by the renderer package.  The
arithmetic lives in ``gsr_oracle.c`` (FP64 pixels, projection and gradients;
an FP32 key-specification path for tile rectangles and depth keys).  This
module only marshals numpy arrays and does the key sort and range search with
numpy library primitives (``lexsort``, ``searchsorted``).

Key layout (batched key space): for image ``i`` (env-major, camera-minor),
global tile = i * tiles_per_image + ty * tiles_x + tx; key = (global tile << 32)
| FP32 bit pattern of z; value = scene-global Gaussian id (env-major
concatenation of node sets).  Pairs are ordered by (key, value).
"""
import ctypes
import os

import numpy as np

from .build import LIB, build as _build

_lib = None
_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_c_int = ctypes.c_int
_c_dbl = ctypes.c_double

GEO = 28
G2D = 10
# Ambiguous decisions: a blending decision is ambiguous when its relative distance to the
# threshold (alpha vs 1/255, T (1 - alpha) vs 1e-4) is below ERR_SAFETY times the oracle's
# first-order bound of an FP32 renderer's relative error of that quantity, plus ERR_FLOOR
# (which covers the FP32 roundings of the three threshold constants).  The bound is derived
# per decision from the magnitudes of the Gaussian's projection (gsr_oracle.c, fp32_bounds
# and decision_bound); the factor 2 covers the second-order terms the bound drops.
ERR_SAFETY = 2.0
ERR_FLOOR = 2e-7


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            _build()
        L = ctypes.CDLL(LIB)
        scene32 = [_c_int, _c_int, _f32p, _f32p, _f32p, _f32p, _i32p, _c_int, _f32p, _f32p]
        scene = [_c_int, _c_int, _f64p, _f64p, _f64p, _f64p, _f64p, _i32p, _c_int, _f64p, _f64p]
        L.or_keyspec_flat.argtypes = scene32 + [_f32p, _c_int, _c_int, _c_int, _c_int, _i32p, _u32p, _i32p]
        L.or_keyspec_flat.restype = None
        L.or_project_flat.argtypes = scene + [_f64p, _c_int, _c_int, _f64p]
        L.or_project_flat.restype = None
        L.or_backward_project_flat.argtypes = scene + [_f64p, _c_int, _c_int, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p,
                                                       _f64p]
        L.or_backward_project_flat.restype = None
        L.or_composite.argtypes = [_c_int, _c_int, _c_int, _c_int, _i64p, _i32p, _f64p, _f32p, _c_dbl, _c_dbl,
                                   _f64p, _f64p, _f64p, _f64p, _i32p, _i32p, _f64p, _i32p, _f64p, _i64p]
        L.or_composite.restype = None
        L.or_composite_sample.argtypes = [_c_int, _c_int, _c_int, _c_int, _i64p, _i32p, _f64p, _f32p, _c_dbl, _c_dbl,
                                          _i64p, ctypes.c_int64, _f64p, _i32p, _f64p]
        L.or_composite_sample.restype = None
        L.or_backward_2d.argtypes = [_c_int, _c_int, _c_int, _c_int, _i64p, _i32p, _f64p, _f32p, _f64p,
                                     ctypes.c_void_p, ctypes.c_void_p, _c_int, _f64p]
        L.or_backward_2d.restype = None
        L.or_backward_2d_sample.argtypes = [_c_int, _c_int, _c_int, _c_int, _i64p, _i32p, _f64p, _f32p, _i64p,
                                            ctypes.c_int64, _f64p, ctypes.c_void_p, ctypes.c_void_p, _c_int, _f64p]
        L.or_backward_2d_sample.restype = None
        L.or_sh_eval.argtypes = [_c_int, _f64p, _f64p, ctypes.c_void_p]
        L.or_sh_eval.restype = None
        L.or_wigner.argtypes = [_c_int, _f64p, _f64p]
        L.or_wigner.restype = _c_int
        L.or_compose_view.argtypes = [_f32p, _f32p, _f32p, _f32p, _f32p]
        L.or_compose_view.restype = None
        L.or_alpha_bounds.argtypes = [_f64p, ctypes.c_int64, _i32p, _i32p, _i32p, _f64p, _f64p]
        L.or_alpha_bounds.restype = None
        L.or_num_threads.argtypes = []
        L.or_num_threads.restype = _c_int
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# marshalling helpers
# --------------------------------------------------------------------------
def cam_array(cam):
    """camera dict -> float32[20] (R, t, fx, fy, cx, cy, znear, bg)."""
    a = np.zeros(20, dtype=np.float32)
    a[0:9] = np.asarray(cam["R"], dtype=np.float32).reshape(9)
    a[9:12] = np.asarray(cam["t"], dtype=np.float32)
    a[12], a[13], a[14], a[15], a[16] = cam["fx"], cam["fy"], cam["cx"], cam["cy"], cam["znear"]
    a[17:20] = np.asarray(cam["bg"], dtype=np.float32)
    return a


class FlatEnv:
    """One environment's node sets concatenated (node order, local index)."""

    def __init__(self, env):
        nodes = env["nodes"]
        degs = {n["sh_degree"] for n in nodes}
        if len(degs) != 1:
            raise ValueError("all nodes of a scene share one SH degree")
        self.sh_degree = degs.pop()
        self.K = (self.sh_degree + 1) ** 2
        cat = lambda k: np.ascontiguousarray(np.concatenate([n[k] for n in nodes], axis=0), dtype=np.float32)
        self.means, self.scales, self.quats = cat("means"), cat("scales"), cat("quats")
        self.opac, self.sh = cat("opacities"), cat("sh").reshape(-1, self.K * 3)
        self.sizes = [len(n["means"]) for n in nodes]
        self.n = int(sum(self.sizes))
        self.node = np.ascontiguousarray(np.repeat(np.arange(len(nodes), dtype=np.int32), self.sizes))
        self.n_nodes = len(nodes)
        self.pose_R = np.ascontiguousarray(np.stack([np.asarray(R, np.float32).reshape(9) for R, _ in env["poses"]]))
        self.pose_t = np.ascontiguousarray(np.stack([np.asarray(t, np.float32).reshape(3) for _, t in env["poses"]]))
        # FP64 copies used by the FP64 path (exact conversions; finite-difference
        # tests perturb these while the FP32 key specification keeps the originals)
        self.p64 = dict(means=self.means.astype(np.float64), scales=self.scales.astype(np.float64),
                        quats=self.quats.astype(np.float64), opac=self.opac.astype(np.float64),
                        sh=self.sh.astype(np.float64).reshape(-1),
                        pose_R=self.pose_R.astype(np.float64).reshape(-1), pose_t=self.pose_t.astype(np.float64).reshape(-1))

    def args32(self):
        return (self.n, self.sh_degree, self.means, self.scales, self.quats, self.opac, self.node, self.n_nodes,
                np.ascontiguousarray(self.pose_R.reshape(-1)), np.ascontiguousarray(self.pose_t.reshape(-1)))

    def args(self):
        p = self.p64
        c = np.ascontiguousarray
        return (self.n, self.sh_degree, c(p["means"]).reshape(-1), c(p["scales"]).reshape(-1),
                c(p["quats"]).reshape(-1), c(p["opac"]).reshape(-1), c(p["sh"]).reshape(-1), self.node,
                self.n_nodes, c(p["pose_R"]), c(p["pose_t"]))


def keyspec(fe, cam, width, height, tw, th):
    n = fe.n
    rect = np.zeros((n, 4), dtype=np.int32)
    zbits = np.zeros(n, dtype=np.uint32)
    vis = np.zeros(n, dtype=np.int32)
    lib().or_keyspec_flat(*fe.args32(), cam_array(cam), width, height, tw, th,
                          rect.reshape(-1), zbits, vis)
    return rect, zbits, vis


def project(fe, cam, width, height):
    geo = np.zeros((fe.n, GEO), dtype=np.float64)
    lib().or_project_flat(*fe.args(), cam_array(cam).astype(np.float64), width, height, geo.reshape(-1))
    return geo


def pairs(rect, zbits, vis, width, height, tw, th, image=0, gid_base=0):
    """Sorted (key, value) pairs and per-tile [start, end) ranges for one image.

    Returns keys (uint64, global tile << 32 | zbits), values (uint32 global id),
    local value indices (int32), ranges (int64 [tiles, 2], local to this image).
    """
    tiles_x = (width + tw - 1) // tw
    tiles_y = (height + th - 1) // th
    T = tiles_x * tiles_y
    vis_idx = np.nonzero(vis == 0)[0]
    r = rect[vis_idx].astype(np.int64)
    w = r[:, 2] - r[:, 0]
    cnt = w * (r[:, 3] - r[:, 1])
    ids = np.repeat(vis_idx.astype(np.int64), cnt)
    first = np.repeat(np.cumsum(cnt) - cnt, cnt)
    k = np.arange(ids.size, dtype=np.int64) - first
    wr = np.repeat(w, cnt)
    tx = np.repeat(r[:, 0], cnt) + k % np.maximum(wr, 1)
    ty = np.repeat(r[:, 1], cnt) + k // np.maximum(wr, 1)
    tiles = (ty * tiles_x + tx).astype(np.uint64)
    gtile = tiles + np.uint64(image * T)
    keys = (gtile << np.uint64(32)) | zbits[ids].astype(np.uint64)
    vals = (ids + gid_base).astype(np.uint32)
    order = np.lexsort((vals, keys))
    keys, vals, ids = keys[order], vals[order], ids[order]
    ltile = (keys >> np.uint64(32)) - np.uint64(image * T)
    starts = np.searchsorted(ltile, np.arange(T, dtype=np.uint64), side="left")
    ends = np.searchsorted(ltile, np.arange(T, dtype=np.uint64), side="right")
    ranges = np.ascontiguousarray(np.stack([starts, ends], axis=1).astype(np.int64))
    return keys, vals, np.ascontiguousarray(ids.astype(np.int32)), ranges


def composite(geo, ranges, local_vals, width, height, tw, th, bg, safety=ERR_SAFETY, floor=ERR_FLOOR):
    P = width * height
    out = dict(rgb=np.zeros((height, width, 3)), depth=np.zeros((height, width)),
               alpha=np.zeros((height, width)), T=np.zeros((height, width)),
               last=np.zeros((height, width), np.int32), evals=np.zeros((height, width), np.int32),
               margin=np.zeros((height, width)), flags=np.zeros((height, width), np.int32),
               alt=np.zeros((height, width, 5)), trace=np.zeros((height, width), np.int64))
    lib().or_composite(width, height, tw, th, np.ascontiguousarray(ranges, dtype=np.int64),
                       np.ascontiguousarray(local_vals, dtype=np.int32), np.ascontiguousarray(geo),
                       np.asarray(bg, np.float32), safety, floor,
                       out["rgb"].reshape(-1), out["depth"].reshape(-1), out["alpha"].reshape(-1),
                       out["T"].reshape(-1), out["last"].reshape(-1), out["evals"].reshape(-1),
                       out["margin"].reshape(-1), out["flags"].reshape(-1), out["alt"].reshape(-1),
                       out["trace"].reshape(-1))
    assert P == out["depth"].size
    return out


def composite_sample(geo, ranges, local_vals, width, height, tw, th, bg, pix, safety=ERR_SAFETY, floor=ERR_FLOOR):
    """Oracle pixels at flat indices ``pix`` (py * width + px)."""
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    out = np.zeros((pix.size, 8))
    flags = np.zeros(pix.size, np.int32)
    alt = np.zeros((pix.size, 5))
    lib().or_composite_sample(width, height, tw, th, np.ascontiguousarray(ranges, dtype=np.int64),
                              np.ascontiguousarray(local_vals, dtype=np.int32), np.ascontiguousarray(geo),
                              np.asarray(bg, np.float32), safety, floor, pix, pix.size, out.reshape(-1), flags,
                              alt.reshape(-1))
    return dict(rgb=out[:, 0:3], depth=out[:, 3], alpha=out[:, 4], T=out[:, 5], last=out[:, 6].astype(np.int64),
                evals=out[:, 7].astype(np.int64), flags=flags, alt=alt)


def render(env, cam, width, height, tw=16, th=16, fe=None, image=0, gid_base=0, safety=ERR_SAFETY,
           floor=ERR_FLOOR):
    """Full oracle frame for one camera of one environment."""
    fe = fe or FlatEnv(env)
    rect, zbits, vis = keyspec(fe, cam, width, height, tw, th)
    geo = project(fe, cam, width, height)
    keys, vals, lvals, ranges = pairs(rect, zbits, vis, width, height, tw, th, image, gid_base)
    out = composite(geo, ranges, lvals, width, height, tw, th, cam["bg"], safety, floor)
    out.update(rect=rect, zbits=zbits, vis=vis, geo=geo, keys=keys, vals=vals, lvals=lvals, ranges=ranges, fe=fe)
    return out


def render_brute(env, cam, width, height, fe=None, safety=ERR_SAFETY, floor=ERR_FLOOR):
    """Every Gaussian in front of the camera, for every pixel, no tile rectangles.

    The candidate list is all Gaussians that pass the non-geometric culls
    (finite, opacity >= 1/255, z > znear, det > 0), ordered by (z bits, id).
    """
    fe = fe or FlatEnv(env)
    rect, zbits, vis = keyspec(fe, cam, width, height, 16, 16)
    geo = project(fe, cam, width, height)
    cand = np.nonzero((vis == 0) | (vis == 6))[0]
    z32 = zbits
    order = np.lexsort((cand, z32[cand]))
    lst = np.ascontiguousarray(cand[order].astype(np.int32))
    ranges = np.array([[0, len(lst)]], dtype=np.int64)
    return composite(geo, ranges, lst, width, height, width, height, cam["bg"], safety, floor)


def backward(ref, cam, width, height, g_rgb, g_depth=None, g_alpha=None, tw=16, th=16):
    """FP64 analytic gradients (means, scales, quats, opacities, sh) for one camera."""
    fe = ref["fe"]
    g2d = np.zeros((fe.n, G2D), dtype=np.float64)
    gr = np.ascontiguousarray(g_rgb, dtype=np.float64).reshape(-1)
    gd = None if g_depth is None else np.ascontiguousarray(g_depth, dtype=np.float64).reshape(-1)
    ga = None if g_alpha is None else np.ascontiguousarray(g_alpha, dtype=np.float64).reshape(-1)
    lib().or_backward_2d(width, height, tw, th, ref["ranges"], ref["lvals"], ref["geo"],
                         np.asarray(cam["bg"], np.float32), gr,
                         None if gd is None else gd.ctypes.data_as(ctypes.c_void_p),
                         None if ga is None else ga.ctypes.data_as(ctypes.c_void_p),
                         fe.n, g2d.reshape(-1))
    return _project_grads(fe, cam, width, height, g2d)


def backward_sample(ref, cam, width, height, pix, g_rgb, g_depth=None, g_alpha=None, tw=16, th=16):
    """FP64 analytic gradients for one camera when only the pixels ``pix`` (flat indices
    py * width + px) carry upstream gradients: g_rgb [len(pix), 3], g_depth and g_alpha
    [len(pix)] or None.  Same result as ``backward`` with those gradients scattered into
    otherwise zero frames."""
    fe = ref["fe"]
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    g2d = np.zeros((fe.n, G2D), dtype=np.float64)
    gr = np.ascontiguousarray(g_rgb, dtype=np.float64).reshape(-1)
    gd = None if g_depth is None else np.ascontiguousarray(g_depth, dtype=np.float64).reshape(-1)
    ga = None if g_alpha is None else np.ascontiguousarray(g_alpha, dtype=np.float64).reshape(-1)
    lib().or_backward_2d_sample(width, height, tw, th, ref["ranges"], ref["lvals"], ref["geo"],
                                np.asarray(cam["bg"], np.float32), pix, pix.size, gr,
                                None if gd is None else gd.ctypes.data_as(ctypes.c_void_p),
                                None if ga is None else ga.ctypes.data_as(ctypes.c_void_p),
                                fe.n, g2d.reshape(-1))
    return _project_grads(fe, cam, width, height, g2d)


def _project_grads(fe, cam, width, height, g2d):
    grads = dict(means=np.zeros((fe.n, 3)), scales=np.zeros((fe.n, 3)), quats=np.zeros((fe.n, 4)),
                 opacities=np.zeros(fe.n), sh=np.zeros((fe.n, fe.K * 3)), pose=np.zeros((fe.n_nodes, 6)))
    lib().or_backward_project_flat(*fe.args(), cam_array(cam).astype(np.float64), width, height, g2d.reshape(-1),
                                   grads["means"].reshape(-1), grads["scales"].reshape(-1),
                                   grads["quats"].reshape(-1), grads["opacities"], grads["sh"].reshape(-1),
                                   grads["pose"].reshape(-1))
    grads["sh"] = grads["sh"].reshape(fe.n, fe.K, 3)
    grads["g2d"] = g2d
    return grads


def alpha_bounds(geo, gidx, px, py):
    """FP64 o exp(power) of Gaussian gidx[i] at pixel (px[i], py[i]) and the bound of an FP32
    renderer's relative error of it."""
    gidx = np.ascontiguousarray(gidx, np.int32)
    px = np.ascontiguousarray(px, np.int32)
    py = np.ascontiguousarray(py, np.int32)
    a = np.zeros(gidx.size)
    b = np.zeros(gidx.size)
    lib().or_alpha_bounds(np.ascontiguousarray(geo), gidx.size, gidx, px, py, a, b)
    return a, b


def num_threads():
    return int(lib().or_num_threads())


def sh_eval(L, v, grad=False):
    v = np.ascontiguousarray(v, dtype=np.float64)
    K = (L + 1) ** 2
    Y = np.zeros(K)
    if grad:
        dY = np.zeros(K * 3)
        lib().or_sh_eval(L, v, Y, dY.ctypes.data_as(ctypes.c_void_p))
        return Y, dY.reshape(K, 3)
    lib().or_sh_eval(L, v, Y, None)
    return Y


def wigner(L, R):
    K = (L + 1) ** 2
    D = np.zeros(K * K)
    rc = lib().or_wigner(L, np.ascontiguousarray(R, dtype=np.float64).reshape(9), D)
    if rc != 0:
        raise RuntimeError("singular least-squares system")
    return D.reshape(K, K)


def compose_view(cam, R, t):
    W = np.zeros(9, np.float32)
    w = np.zeros(3, np.float32)
    lib().or_compose_view(cam_array(cam), np.ascontiguousarray(R, np.float32).reshape(9),
                          np.ascontiguousarray(t, np.float32).reshape(3), W, w)
    return W.reshape(3, 3), w
