"""Python binding of libgsr.so, the gfx950 Gaussian-splatting RGB-D sensor renderer.

Argument marshalling only: every stage of rendering runs in the library's HIP
kernels.  PyTorch supplies device memory (``data_ptr``) and the stream
(``torch.cuda.current_stream().cuda_stream``).  The library must be built
(``python paper_2507_21981_amd/build.py``); importing the renderer without it
raises ``ImportError`` -- there is no CPU fallback.

Names follow the C ABI in include/gsr.h: ``create``, ``compose_scene``,
``render_rgbd``, ``saved_render``, ``render_backward``, ``query_status``, ``copy_pairs``,
``copy_pixel_state``, ``autotune``.  ``RenderRGBD`` is the autograd Function.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsr.so")

GSR_OK = 0
FLAG_CHECK = 1
FLAG_SAVE = 2
FLAG_GRAPH = 4
FLAG_PERSISTENT = 8
FLAG_TIMING = 16
FLAG_AUGMENT = 32
STATUS_OVERFLOW = 1
STAGES = ("views", "project", "gather", "depth_sort", "chunks", "tile_counts", "tile_ranges", "emit", "composite")

_ERRORS = {-1: "GSR_E_INVALID", -2: "GSR_E_NOMEM", -3: "GSR_E_HIP", -4: "GSR_E_CAPACITY",
           -5: "GSR_E_UNSUPPORTED", -6: "GSR_E_STATE"}


class GsrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class Gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacities", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class GaussianGrads(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacities", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class Config(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("pair_capacity", ctypes.c_int64),
                ("persistent_grid", ctypes.c_int32), ("pixels_per_thread", ctypes.c_int32),
                ("stream_groups", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


class StatusInfo(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("nonfinite", ctypes.c_uint32), ("pairs", ctypes.c_uint64),
                ("pair_capacity", ctypes.c_uint64), ("max_tile_pairs", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("visible", ctypes.c_uint64), ("visible_any", ctypes.c_uint64),
                ("evals", ctypes.c_uint64)]


_lib = None


def lib():
    """Load libgsr.so (raises ImportError if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python paper_2507_21981_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        L.gsr_create.argtypes = [ctypes.c_int, ctypes.POINTER(Config), ctypes.POINTER(vp)]
        L.gsr_destroy.argtypes = [vp]
        L.gsr_destroy.restype = None
        L.gsr_last_error.argtypes = [vp]
        L.gsr_last_error.restype = ctypes.c_char_p
        L.gsr_get_config.argtypes = [vp, ctypes.POINTER(Config)]
        L.gsr_set_tile.argtypes = [vp, i32, i32]
        L.gsr_set_pixels_per_thread.argtypes = [vp, i32]
        L.gsr_set_stream_groups.argtypes = [vp, i32]
        L.gsr_compose_scene.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(Gaussians), i32, vp,
                                        ctypes.POINTER(vp)]
        L.gsr_scene_destroy.argtypes = [vp]
        L.gsr_scene_destroy.restype = None
        L.gsr_scene_gaussians.argtypes = [vp, i32]
        L.gsr_scene_gaussians.restype = i64
        L.gsr_render_rgbd.argtypes = [vp, vp, i32, vp, i32, i32, vp, vp, vp, u32, vp]
        L.gsr_saved_render.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(i32),
                                       ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.gsr_render_backward.argtypes = [vp, vp, ctypes.c_uint64, vp, vp, vp, ctypes.POINTER(GaussianGrads), vp,
                                          vp]
        L.gsr_render_backward_noalloc.argtypes = L.gsr_render_backward.argtypes
        L.gsr_augment_rgb.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp]
        L.gsr_set_augment.argtypes = [vp, vp, vp]
        L.gsr_lidar_build.argtypes = [vp, vp]
        L.gsr_render_lidar.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp]
        L.gsr_mesh_to_gaussians.argtypes = [vp, i64, vp, vp, i64, vp, ctypes.c_float, ctypes.c_float, i32,
                                            ctypes.POINTER(GaussianGrads), vp]
        L.gsr_query_status.argtypes = [vp, ctypes.POINTER(StatusInfo)]
        L.gsr_copy_pairs.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(i64)]
        L.gsr_copy_pixel_state.argtypes = [vp, vp, vp]
        L.gsr_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
        L.gsr_autotune.argtypes = [vp, vp, i32, vp, i32, i32, vp, vp, vp, ctypes.POINTER(i32),
                                   ctypes.POINTER(i32), ctypes.POINTER(i32), vp]
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != GSR_OK:
        msg = lib().gsr_last_error(ctx.handle if ctx is not None else None)
        raise GsrError(rc, msg.decode() if msg else "")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f32(x, shape_tail, name):
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    if tuple(x.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} has shape {tuple(x.shape)}, expected [n, {', '.join(map(str, shape_tail))}]")
    return x


# --------------------------------------------------------------------------- context
class Context:
    """A renderer context on one device (workspace, configuration, saved state)."""

    def __init__(self, device=0, tile=(16, 16), pair_capacity=0, persistent_grid=0):
        lib()
        cfg = Config()
        cfg.tile_w, cfg.tile_h = tile
        cfg.pair_capacity = pair_capacity
        cfg.persistent_grid = persistent_grid
        h = ctypes.c_void_p()
        _check(lib().gsr_create(device, ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            lib().gsr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def config(self):
        c = Config()
        _check(lib().gsr_get_config(self.handle, ctypes.byref(c)), self)
        return c

    def set_tile(self, tw, th):
        _check(lib().gsr_set_tile(self.handle, tw, th), self)

    def set_pixels_per_thread(self, ppt):
        _check(lib().gsr_set_pixels_per_thread(self.handle, ppt), self)

    def set_stream_groups(self, groups):
        """Render environments as `groups` concurrent groups on the library's streams."""
        _check(lib().gsr_set_stream_groups(self.handle, groups), self)


def create(device=0, tile=(16, 16), pair_capacity=0, persistent_grid=0):
    return Context(device, tile, pair_capacity, persistent_grid)


# --------------------------------------------------------------------------- scene
class Scene:
    """A composed scene: per env a background node plus posed nodes (device tensors)."""

    def __init__(self, ctx):
        self.ctx = ctx
        self.handle = ctypes.c_void_p()
        self.nodes = []
        self.poses = None
        self.env_offsets = []

    def close(self):
        if self.handle:
            lib().gsr_scene_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_envs(self):
        return len(self.env_offsets) - 1

    def gaussians(self, env=-1):
        return int(lib().gsr_scene_gaussians(self.handle, env))


def compose_scene(ctx, envs, poses, scene=None):
    """Compose environments.

    envs: list (per env) of lists of node dicts with CUDA float32 tensors
    ``means [n,3], scales [n,3], quats [n,4], opacities [n], sh [n,K,3]``
    (activated values); node 0 of each env is its background.
    poses: CUDA float32 tensor [n_nodes, 12] (R row-major then t), node-local
    -> world, read at every render (update it in place between steps).
    """
    sc = scene if scene is not None else Scene(ctx)
    nodes = [n for e in envs for n in e]
    offs = [0]
    for e in envs:
        offs.append(offs[-1] + len(e))
    arr = (Gaussians * len(nodes))()
    for i, n in enumerate(nodes):
        m = _dev_f32(n["means"], (3,), "means")
        K = n["sh"].shape[1]
        deg = {1: 0, 4: 1, 9: 2, 16: 3}.get(K)
        if deg is None:
            raise ValueError(f"sh has {K} coefficients per channel; expected 1, 4, 9 or 16")
        arr[i].n = m.shape[0]
        arr[i].sh_degree = deg
        arr[i].means = m.data_ptr()
        arr[i].scales = _dev_f32(n["scales"], (3,), "scales").data_ptr()
        arr[i].quats = _dev_f32(n["quats"], (4,), "quats").data_ptr()
        op = n["opacities"]
        if not (op.is_cuda and op.dtype == torch.float32 and op.is_contiguous() and op.dim() == 1):
            raise TypeError("opacities must be a contiguous float32 CUDA tensor [n]")
        arr[i].opacities = op.data_ptr()
        arr[i].sh = _dev_f32(n["sh"], (K, 3), "sh").data_ptr()
    _dev_f32(poses, (12,), "poses")
    if poses.shape[0] != len(nodes):
        raise ValueError("poses must have one row per node")
    offs_c = (ctypes.c_int32 * len(offs))(*offs)
    _check(lib().gsr_compose_scene(ctx.handle, len(envs), offs_c, arr, len(nodes), _ptr(poses),
                                   ctypes.byref(sc.handle)), ctx)
    sc.nodes = nodes  # keep the borrowed tensors alive
    sc.poses = poses
    sc.env_offsets = offs
    return sc


def cameras_tensor(cams, device="cuda"):
    """Pack camera dicts (R, t, fx, fy, cx, cy, znear, bg) into a [n, 20] float32 tensor."""
    import numpy as np
    a = np.zeros((len(cams), 20), np.float32)
    for i, c in enumerate(cams):
        a[i, 0:9] = np.asarray(c["R"], np.float32).reshape(9)
        a[i, 9:12] = np.asarray(c["t"], np.float32)
        a[i, 12:17] = [c["fx"], c["fy"], c["cx"], c["cy"], c["znear"]]
        a[i, 17:20] = np.asarray(c["bg"], np.float32)
    return torch.from_numpy(a).to(device)


def poses_tensor(poses, device="cuda"):
    """Pack (R, t) pairs into a [n, 12] float32 tensor."""
    import numpy as np
    a = np.zeros((len(poses), 12), np.float32)
    for i, (R, t) in enumerate(poses):
        a[i, 0:9] = np.asarray(R, np.float32).reshape(9)
        a[i, 9:12] = np.asarray(t, np.float32)
    return torch.from_numpy(a).to(device)


# --------------------------------------------------------------------------- render
def render_rgbd(ctx, scene, cams, width, height, cams_per_env=None, out=None, flags=FLAG_CHECK,
                want_alpha=True, stream=None):
    """Render every env from its cameras.  cams: CUDA float32 [n_envs * C, 20].

    Returns (rgb [E, C, H, W, 3], depth [E, C, H, W], alpha [E, C, H, W] or None).
    """
    E = scene.n_envs
    _dev_f32(cams, (20,), "cams")
    C = cams_per_env if cams_per_env is not None else cams.shape[0] // E
    if C * E != cams.shape[0]:
        raise ValueError("cams must hold n_envs * cams_per_env rows")
    if out is None:
        dev = cams.device
        rgb = torch.empty((E, C, height, width, 3), device=dev, dtype=torch.float32)
        depth = torch.empty((E, C, height, width), device=dev, dtype=torch.float32)
        alpha = torch.empty((E, C, height, width), device=dev, dtype=torch.float32) if want_alpha else None
    else:
        rgb, depth, alpha = out
    _check(lib().gsr_render_rgbd(ctx.handle, scene.handle, C, _ptr(cams), width, height, _ptr(rgb), _ptr(depth),
                                 _ptr(alpha), flags, _stream(stream)), ctx)
    return rgb, depth, alpha


def saved_render(ctx):
    """(render_id, images, width, height) of the render a backward would use (id 0: none)."""
    rid = ctypes.c_uint64()
    n, w, h = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().gsr_saved_render(ctx.handle, ctypes.byref(rid), ctypes.byref(n), ctypes.byref(w), ctypes.byref(h)),
           ctx)
    return rid.value, n.value, w.value, h.value


def render_backward(ctx, scene, d_rgb, d_depth=None, d_alpha=None, grads=None, d_poses=None, render_id=None,
                    stream=None, noalloc=False):
    """Accumulate gradients of a saved render into ``grads`` (list of per-node dicts of CUDA
    float32 tensors shaped like the parameters; missing keys are skipped) and, if ``d_poses``
    (CUDA float32 [n_nodes, 6]) is given, the node-pose gradients (omega, rho) into it.  If
    grads is None, zero-initialised ones are allocated and returned.  ``render_id`` names the
    forward render (``saved_render`` right after it); None means the last saved render.  The
    upstream gradients must have the saved render's shape [E, C, H, W(, 3)].  ``noalloc``
    calls gsr_render_backward_noalloc (scratch in the library's static device array; pass
    ``grads``, so that nothing is allocated here either)."""
    rid, images, W, H = saved_render(ctx)
    if render_id is None:
        render_id = rid
    E = scene.n_envs
    C = images // E if E else 0
    for t, tail, name in ((d_rgb, (H, W, 3), "d_rgb"), (d_depth, (H, W), "d_depth"), (d_alpha, (H, W), "d_alpha")):
        if t is None:
            continue
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise TypeError("upstream gradients must be contiguous float32 CUDA tensors")
        if rid != 0 and tuple(t.shape) != (E, C, *tail):
            raise ValueError(f"{name} has shape {tuple(t.shape)}; the saved render is {(E, C, *tail)}")
    if grads is None:
        grads = [{k: torch.zeros_like(n[k]) for k in ("means", "scales", "quats", "opacities", "sh")}
                 for n in scene.nodes]
    arr = (GaussianGrads * len(scene.nodes))()
    for i, g in enumerate(grads):
        for k in ("means", "scales", "quats", "opacities", "sh"):
            t = g.get(k)
            setattr(arr[i], k, None if t is None else t.data_ptr())
    if d_poses is not None:
        _dev_f32(d_poses, (6,), "d_poses")
        if d_poses.shape[0] != len(scene.nodes):
            raise ValueError("d_poses must have one row per node")
    fn = lib().gsr_render_backward_noalloc if noalloc else lib().gsr_render_backward
    _check(fn(ctx.handle, scene.handle, render_id, _ptr(d_rgb), _ptr(d_depth), _ptr(d_alpha), arr, _ptr(d_poses),
              _stream(stream)), ctx)
    return grads


def augment_tensor(params, device="cuda"):
    """Per-image augmentation draws [n, 5] (overlay weight, hue shift in turns, saturation
    scale, value scale, gamma) -> the [n, 8] float32 rows of gsr_augment."""
    import numpy as np
    p = np.zeros((len(params), 8), np.float32)
    p[:, :5] = np.asarray(params, np.float32).reshape(-1, 5)
    return torch.from_numpy(p).to(device)


def augment_rgb(ctx, rgb, params, overlay=None, out=None, stream=None):
    """Image-space domain randomisation of rendered frames rgb [..., H, W, 3] (CUDA float32):
    params [images, 8] (``augment_tensor``), overlay like rgb or None.  Returns ``out``."""
    if not (rgb.is_cuda and rgb.dtype == torch.float32 and rgb.is_contiguous() and rgb.shape[-1] == 3):
        raise TypeError("rgb must be a contiguous float32 CUDA tensor [..., H, W, 3]")
    H, W = rgb.shape[-3], rgb.shape[-2]
    images = rgb.numel() // (H * W * 3)
    _dev_f32(params, (8,), "params")
    if params.shape[0] != images:
        raise ValueError(f"params has {params.shape[0]} rows for {images} images")
    if overlay is not None and (tuple(overlay.shape) != tuple(rgb.shape) or not overlay.is_contiguous()
                                or overlay.dtype != torch.float32):
        raise ValueError("overlay must be a contiguous float32 tensor shaped like rgb")
    out = torch.empty_like(rgb) if out is None else out
    _check(lib().gsr_augment_rgb(ctx.handle, images, W, H, _ptr(rgb), _ptr(overlay), _ptr(params), _ptr(out),
                                 _stream(stream)), ctx)
    return out


def set_augment(ctx, params, overlay=None):
    """Bind the augmentation that renders with FLAG_AUGMENT apply in the compositor (the
    tensors must stay alive and may be rewritten in place between renders)."""
    _dev_f32(params, (8,), "params")
    _check(lib().gsr_set_augment(ctx.handle, _ptr(params), _ptr(overlay)), ctx)
    ctx._augment = (params, overlay)


def lidar_build(ctx, scene):
    """Build the per-node hierarchies the LiDAR tracer needs (again after recomposing)."""
    _check(lib().gsr_lidar_build(ctx.handle, scene.handle), ctx)


def render_lidar(ctx, scene, rays, rays_per_env=None, out=None, want_hits=True, stream=None):
    """Trace rays (CUDA float32 [n_envs * rays_per_env, 8] rows: origin, unit direction,
    tmin, tmax).  Returns (range, alpha, hits or None), each [n_envs, rays_per_env]."""
    _dev_f32(rays, (8,), "rays")
    E = scene.n_envs
    n = rays.shape[0]
    R = rays_per_env if rays_per_env is not None else n // E
    if R * E != n:
        raise ValueError("rays must hold n_envs * rays_per_env rows")
    if out is None:
        rng = torch.empty((E, R), device=rays.device)
        alpha = torch.empty((E, R), device=rays.device)
        hits = torch.empty((E, R), dtype=torch.int32, device=rays.device) if want_hits else None
    else:
        rng, alpha, hits = out
    _check(lib().gsr_render_lidar(ctx.handle, scene.handle, R, _ptr(rays), _ptr(rng), _ptr(alpha), _ptr(hits),
                                  _stream(stream)), ctx)
    return rng, alpha, hits


def mesh_to_gaussians(ctx, vertices, faces, colours=None, flatten=0.01, opacity=0.9, sh_degree=0, stream=None):
    """One Gaussian per facet of a triangle mesh (CUDA tensors: vertices float32 [nv, 3], faces
    int32 [nf, 3], colours float32 [nv, 3] or None).  Returns a node dict (means, scales,
    quats, opacities, sh) ready for compose_scene."""
    _dev_f32(vertices, (3,), "vertices")
    if colours is not None:
        _dev_f32(colours, (3,), "colours")
    if not (faces.is_cuda and faces.dtype == torch.int32 and faces.is_contiguous() and faces.dim() == 2
            and faces.shape[1] == 3):
        raise TypeError("faces must be a contiguous int32 CUDA tensor [nf, 3]")
    nf, K, dev = faces.shape[0], (sh_degree + 1) ** 2, vertices.device
    node = dict(means=torch.empty((nf, 3), device=dev), scales=torch.empty((nf, 3), device=dev),
                quats=torch.empty((nf, 4), device=dev), opacities=torch.empty(nf, device=dev),
                sh=torch.empty((nf, K, 3), device=dev))
    o = GaussianGrads(node["means"].data_ptr(), node["scales"].data_ptr(), node["quats"].data_ptr(),
                      node["opacities"].data_ptr(), node["sh"].data_ptr())
    _check(lib().gsr_mesh_to_gaussians(ctx.handle, vertices.shape[0], _ptr(vertices), _ptr(colours), nf, _ptr(faces),
                                       flatten, opacity, sh_degree, ctypes.byref(o), _stream(stream)), ctx)
    return node


def query_status(ctx):
    s = StatusInfo()
    _check(lib().gsr_query_status(ctx.handle, ctypes.byref(s)), ctx)
    return dict(flags=s.flags, nonfinite=s.nonfinite, pairs=s.pairs, pair_capacity=s.pair_capacity,
                max_tile_pairs=s.max_tile_pairs, visible=s.visible, visible_any=s.visible_any, evals=s.evals)


def stage_times(ctx):
    """{stage: ms} of the last render made with FLAG_TIMING."""
    ms = (ctypes.c_float * len(STAGES))()
    _check(lib().gsr_stage_times(ctx.handle, ms), ctx)
    return dict(zip(STAGES, list(ms)))


def copy_pairs(ctx, tiles, device="cuda"):
    """Sorted keys (int64 holding the uint64 (tile << 32 | z bits)), values (int32 holding the
    uint32 Gaussian ids) and per-tile [start, end) ranges of the last render."""
    st = query_status(ctx)
    n = int(st["pairs"])
    keys = torch.empty(max(n, 1), dtype=torch.int64, device=device)
    vals = torch.empty(max(n, 1), dtype=torch.int32, device=device)
    ranges = torch.empty(2 * tiles, dtype=torch.int32, device=device)
    got = ctypes.c_int64()
    _check(lib().gsr_copy_pairs(ctx.handle, _ptr(keys), _ptr(vals), _ptr(ranges), keys.numel(), ctypes.byref(got)),
           ctx)
    return keys[:n], vals[:n], ranges.view(tiles, 2)


def copy_pixel_state(ctx, n_pixels, device="cuda"):
    T = torch.empty(n_pixels, dtype=torch.float32, device=device)
    nc = torch.empty(n_pixels, dtype=torch.int32, device=device)
    _check(lib().gsr_copy_pixel_state(ctx.handle, _ptr(T), _ptr(nc)), ctx)
    return T, nc


def autotune(ctx, scene, cams, width, height, cams_per_env=None, stream=None):
    """Pick tile shape, pixels per thread and persistent compositing for this workload.
    Returns ((tile_w, tile_h), persistent); the context keeps the choice."""
    E = scene.n_envs
    C = cams_per_env if cams_per_env is not None else cams.shape[0] // E
    rgb = torch.empty((E, C, height, width, 3), device=cams.device)
    depth = torch.empty((E, C, height, width), device=cams.device)
    tw, th, pers = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().gsr_autotune(ctx.handle, scene.handle, C, _ptr(cams), width, height, _ptr(rgb), _ptr(depth), None,
                              ctypes.byref(tw), ctypes.byref(th), ctypes.byref(pers), _stream(stream)), ctx)
    return (tw.value, th.value), bool(pers.value)


# --------------------------------------------------------------------------- autograd
class RenderRGBD(torch.autograd.Function):
    """rgb, depth, alpha = RenderRGBD.apply(ctx, scene, cams, W, H, pose_tangent, *params).

    params: for every node of the scene, in order, (means, scales, quats, opacities, sh)
    -- the same tensors the scene was composed from.  pose_tangent: None, or a float32 CUDA
    tensor [n_nodes, 6] standing for a perturbation (omega, rho) of the node poses at zero
    (its value is not read; the scene's poses are used as they are): its gradient is the
    derivative along R' = exp([omega]x) R, t' = exp([omega]x) t + rho.  The cameras are
    constants.  Each forward keeps the id of its render; a backward after another saved render
    on the same context raises instead of mixing the two.
    """

    @staticmethod
    def forward(fctx, rctx, scene, cams, width, height, pose_tangent, *params):
        rgb, depth, alpha = render_rgbd(rctx, scene, cams, width, height, flags=FLAG_CHECK | FLAG_SAVE)
        fctx.rctx, fctx.scene, fctx.nparams = rctx, scene, len(params)
        fctx.render_id = saved_render(rctx)[0]
        fctx.want_pose = pose_tangent is not None
        return rgb, depth, alpha

    @staticmethod
    def backward(fctx, g_rgb, g_depth, g_alpha):
        scene = fctx.scene
        d_poses = torch.zeros((len(scene.nodes), 6), dtype=torch.float32, device=g_rgb.device) \
            if fctx.want_pose else None
        grads = render_backward(fctx.rctx, scene, g_rgb.contiguous(),
                                None if g_depth is None else g_depth.contiguous(),
                                None if g_alpha is None else g_alpha.contiguous(),
                                d_poses=d_poses, render_id=fctx.render_id)
        flat = []
        for g in grads:
            flat += [g["means"], g["scales"], g["quats"], g["opacities"], g["sh"]]
        return (None, None, None, None, None, d_poses, *flat)


def node_params(scene):
    out = []
    for n in scene.nodes:
        out += [n["means"], n["scales"], n["quats"], n["opacities"], n["sh"]]
    return out
