"""Oracle of the image-space domain randomisation (paper Sec. IV-C, "Domain Randomization";
the footnotes of Tables II and III list the same three augmentations).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's CPU leg, never by the
renderer package.  Plain numpy in FP64, one formula per step, in the order the paper names
them.  The paper gives no formulas, so each step is a reading:

  1. the rendered colour is taken into display range: x = clamp(rgb, 0, 1);
  2. random video overlay ("Internet video crops ... linearly blended into the simulation
     stream"): x = (1 - lam) x + lam clamp(overlay, 0, 1), with the crop already cut to the
     image size by the caller;
  3. HSV-space augmentation in the hexcone model (value = max channel, saturation = chroma /
     value, hue in turns): hue shifted by dh modulo 1, saturation and value scaled and clamped
     to [0, 1];
  4. random gamma correction: y = x ** gamma per channel.

The random draws (lam, dh, saturation scale, value scale, gamma per image) are inputs.
"""
import numpy as np


def rgb_to_hsv(x):
    """Hexcone HSV of colours x [..., 3] in [0, 1]: hue in turns [0, 1), saturation, value."""
    r, g, b = x[..., 0], x[..., 1], x[..., 2]
    v = np.max(x, axis=-1)
    m = np.min(x, axis=-1)
    c = v - m
    s = np.where(v > 0, c / np.where(v > 0, v, 1.0), 0.0)
    safe = np.where(c > 0, c, 1.0)
    # hue sector by the largest channel (red first on ties, then green), in sixths of a turn
    h6 = np.where(v == r, np.mod((g - b) / safe, 6.0), np.where(v == g, (b - r) / safe + 2.0, (r - g) / safe + 4.0))
    h = np.where(c > 0, h6 / 6.0, 0.0)
    return np.stack([h, s, v], axis=-1)


def hsv_to_rgb(hsv):
    """Inverse hexcone map: chroma c = v s, the second-largest channel c (1 - |h6 mod 2 - 1|),
    the smallest v - c, placed by the hue's sector."""
    h, s, v = hsv[..., 0], hsv[..., 1], hsv[..., 2]
    h6 = np.mod(h, 1.0) * 6.0
    c = v * s
    xx = c * (1.0 - np.abs(np.mod(h6, 2.0) - 1.0))
    m = v - c
    sector = np.minimum(np.floor(h6), 5).astype(np.int64)
    z = np.zeros_like(c)
    table = [(c, xx, z), (xx, c, z), (z, c, xx), (z, xx, c), (xx, z, c), (c, z, xx)]
    out = np.zeros(h.shape + (3,))
    for k, (r1, g1, b1) in enumerate(table):
        sel = sector == k
        out[..., 0] = np.where(sel, r1 + m, out[..., 0])
        out[..., 1] = np.where(sel, g1 + m, out[..., 1])
        out[..., 2] = np.where(sel, b1 + m, out[..., 2])
    return out


def augment(rgb, params, overlay=None):
    """rgb [I, H, W, 3] (any float), params [I, 5] = (lam, dh, sat_scale, val_scale, gamma),
    overlay [I, H, W, 3] or None; returns the augmented images in FP64."""
    x = np.clip(np.asarray(rgb, np.float64), 0.0, 1.0)
    p = np.asarray(params, np.float64).reshape(-1, 5)
    shape = (-1,) + (1,) * (x.ndim - 1)
    lam, dh, ss, vs, gam = (p[:, k].reshape(shape) for k in range(5))
    if overlay is not None:
        ov = np.clip(np.asarray(overlay, np.float64), 0.0, 1.0)
        x = (1.0 - lam) * x + lam * ov
    hsv = rgb_to_hsv(x)
    hsv[..., 0] = np.mod(hsv[..., 0] + dh[..., 0], 1.0)
    hsv[..., 1] = np.clip(hsv[..., 1] * ss[..., 0], 0.0, 1.0)
    hsv[..., 2] = np.clip(hsv[..., 2] * vs[..., 0], 0.0, 1.0)
    y = hsv_to_rgb(hsv)
    return np.power(y, gam)
