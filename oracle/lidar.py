"""Oracle of the LiDAR sensor: Gaussian ray tracing (paper Sec. III-C, "Sensor": LiDAR by a
BVH-accelerated native Gaussian ray tracer).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark, never by the renderer
package.  Plain numpy in FP64 and brute force: every Gaussian of the environment is tested
against every ray (no acceleration structure), in the order of the definition.  The paper
states only that LiDAR returns come from ray tracing the Gaussians; the readings:

  * node poses as for the cameras: world mean mu' = R_k mu + t_k, world frame R_k R(q/|q|);
  * a Gaussian meets the ray o + t d (|d| = 1) where its density along the ray peaks; its
    response there is G = exp(-D^2 / 2) with D^2 = min_t (o + t d - mu')^T Sigma^-1 (...), and
    alpha = min(0.99, opacity G) as in the camera (skip below 1/255);
  * hits are ordered by t_c = (mu' - o) . d, the distance along the ray of the centre's
    projection (the camera orders by the centre's z), ties by Gaussian id, and only centres
    with tmin < t_c < tmax count;
  * front-to-back compositing with the camera's rules (stop before blending when
    T (1 - alpha) < 1e-4): range = sum alpha T t_c (unnormalised, as the camera's depth;
    range / alpha is the expected distance), alpha = 1 - T, hits = blended count.

D^2 is evaluated from the closest-approach offset delta = t_c d - (mu' - o) (the point of the
ray nearest the centre, minus the centre), which stays of the Gaussian's size: with
M = Sigma^-1, D^2 = delta^T M delta - (delta^T M d)^2 / (d^T M d).

Near-threshold decisions: an FP32 ray tracer computes D^2 with an error the oracle bounds per
(ray, Gaussian) (``_fp32_bound``); a decision whose distance to its threshold is below that
bound is ambiguous, flagged, and its other branch provided, as for the camera.
"""
import numpy as np

U = 2.0 ** -24
ALPHA_MIN = 1.0 / 255.0
T_MIN = 1e-4


def quat_matrix(q):
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


class WorldEnv:
    """One environment's Gaussians in world coordinates (FP64), env-local ids in node order."""

    def __init__(self, env):
        mus, Ms, ops, sizes, snorm, far = [], [], [], [], [], []
        for nd, (R, t) in zip(env["nodes"], env["poses"]):
            R = np.asarray(R, np.float64)
            t = np.asarray(t, np.float64)
            mu = np.asarray(nd["means"], np.float64) @ R.T + t
            Rg = R @ quat_matrix(nd["quats"])
            s = np.asarray(nd["scales"], np.float64)
            A = np.transpose(Rg, (0, 2, 1)) / s[:, :, None]  # S^-1 Rg^T: rows scaled by 1/s
            Ms.append(np.transpose(A, (0, 2, 1)) @ A)        # Sigma^-1 = A^T A
            mus.append(mu)
            ops.append(np.asarray(nd["opacities"], np.float64))
            snorm.append(1.0 / s.min(axis=1))
            # magnitudes an FP32 tracer works with in the node frame (local mean, pose translation)
            far.append(np.linalg.norm(np.asarray(nd["means"], np.float64), axis=1) + np.linalg.norm(t))
            sizes.append(len(mu))
        self.mu = np.concatenate(mus)
        self.M = np.concatenate(Ms)
        self.o = np.concatenate(ops)
        self.inv_smin = np.concatenate(snorm)
        self.far = np.concatenate(far)
        self.n = len(self.mu)
        self.sizes = sizes


def _fp32_bound(D2, ad, q_norm, inv_smin, far, o_norm):
    """First-order bound of an FP32 tracer's error in D^2 / 2 for one ray and the Gaussians:
    the closest-approach offset is formed from the ray moved into the node frame and the local
    mean, each coordinate rounded relative to its magnitude (about 8 U (|o| + far + |q|)
    absolute), which moves the Mahalanobis offset by inv_smin times that; the matrix A =
    S^-1 R^T, its products and the final difference add about 24 U of D^2 and of |A delta|^2.
    A factor 2 covers the second-order terms."""
    e_delta = 8.0 * U * (o_norm + far + q_norm) * inv_smin
    e = ad * e_delta + 0.5 * e_delta ** 2 + 24.0 * U * (D2 + ad ** 2) + 4.0 * U
    return 2.0 * e


def trace(we, rays, tmin=None, tmax=None):
    """rays [n, 8] = (o[3], d[3], tmin, tmax) with |d| = 1.  Returns dict of range, alpha,
    hits, flags (bit 0: one ambiguous decision, alternative in alt; bit 1: two or more) and
    alt [n, 2] (range, alpha of the flipped branch)."""
    rays = np.asarray(rays, np.float64).reshape(-1, 8)
    n = len(rays)
    out = dict(range=np.zeros(n), alpha=np.zeros(n), hits=np.zeros(n, np.int64), flags=np.zeros(n, np.int32),
               alt=np.zeros((n, 2)), cand=np.zeros(n, np.int64))
    ok_o = we.o >= ALPHA_MIN
    for r in range(n):
        o, d = rays[r, 0:3], rays[r, 3:6]
        lo, hi = rays[r, 6], rays[r, 7]
        q = we.mu - o
        tc = q @ d
        delta = tc[:, None] * d - q
        Md = we.M @ d
        dMd = Md @ d
        dMdelta = np.einsum("ni,ni->n", delta, Md)
        Mdelta = np.einsum("nij,nj->ni", we.M, delta)
        dd = np.einsum("ni,ni->n", delta, Mdelta)
        D2 = np.maximum(dd - dMdelta ** 2 / dMd, 0.0)
        G = np.exp(-0.5 * D2)
        a_raw = we.o * G
        sel = ok_o & (tc > lo) & (tc < hi)
        bound = _fp32_bound(D2, np.sqrt(np.maximum(dd, 0.0)), np.linalg.norm(q, axis=1), we.inv_smin, we.far,
                            np.linalg.norm(o))
        # candidates: alpha >= 1/255, or within the bound of it (the flipped branch)
        la = np.log(np.maximum(a_raw, 1e-300)) - np.log(ALPHA_MIN)
        cand = np.nonzero(sel & (la > -bound))[0]
        order = cand[np.lexsort((cand, tc[cand]))]
        out["cand"][r] = len(order)
        res = _composite(tc[order], np.minimum(0.99, a_raw[order]), la[order], bound[order])
        out["range"][r], out["alpha"][r], out["hits"][r], out["flags"][r] = res[0], res[1], res[2], res[3]
        out["alt"][r] = res[4]
    return out


def _composite(t, alpha, la, bound, flip=-1):
    """Front to back; decision k (0, 1, ... in order of evaluation) is flipped when k == flip.
    Returns range, alpha, hits, flags, alt (range, alpha of the first ambiguous decision's
    flipped branch)."""
    T, R, hits = 1.0, 0.0, 0
    lnT_err2 = 0.0
    k = 0
    amb = []
    for i in range(len(t)):
        # skip decision: alpha >= 1/255 (la >= 0)
        take = la[i] >= 0.0
        if abs(la[i]) < bound[i]:
            amb.append(k)
            if k == flip:
                take = not take
        k += 1
        if not take:
            continue
        a = alpha[i]
        # stop decision: T (1 - a) < 1e-4
        stop = T * (1.0 - a) < T_MIN
        e = np.sqrt(lnT_err2 + (bound[i] * a / (1.0 - a)) ** 2) + 1e-6
        if abs(np.log(T * (1.0 - a)) - np.log(T_MIN)) < e:
            amb.append(k)
            if k == flip:
                stop = not stop
        k += 1
        if stop:
            break
        R += a * T * t[i]
        T *= 1.0 - a
        hits += 1
        lnT_err2 += (bound[i] * a / (1.0 - a)) ** 2
    flags = 0
    alt = np.zeros(2)
    if flip < 0 and amb:
        flags = 1 if len(amb) == 1 else 3
        r2 = _composite(t, alpha, la, bound, flip=amb[0])
        alt = np.array([r2[0], r2[1]])
    return R, 1.0 - T, hits, flags, alt
