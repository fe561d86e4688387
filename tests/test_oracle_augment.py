"""Pins of the domain-randomisation oracle (paper Sec. IV-C: video overlays, HSV-space
augmentation, random gamma) against mathematics and a library routine (no GPU).

The hexcone HSV map is checked against Python's ``colorsys`` (the textbook routine); hue
rotation by a third of a turn is a cyclic permutation of the channels; the other steps
reduce to closed forms with the remaining parameters at identity.
"""
import colorsys

import numpy as np

from oracle import augment as A

IDENT = (0.0, 0.0, 1.0, 1.0, 1.0)


def _colours(n, seed):
    g = np.random.default_rng(seed)
    x = g.random((n, 3))
    # include greys, pure and saturated colours, black and white
    x[:20] = [[0, 0, 0], [1, 1, 1], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [0, 1, 1], [1, 0, 1], [0.5, 0.5, 0.5],
              [0.2, 0.2, 0.2], [1, 0.5, 0], [0.3, 0.3, 0.9], [0.9, 0.9, 0.1], [0.25, 0.75, 0.75], [0.6, 0.2, 0.2],
              [0.0, 0.4, 0.4], [0.7, 0.7, 0.0], [1e-9, 0, 0], [1, 1, 1 - 1e-9], [0.5, 0.25, 0.5]]
    return x


def test_hsv_matches_colorsys():
    x = _colours(5000, 1)
    hsv = A.rgb_to_hsv(x)
    ref = np.array([colorsys.rgb_to_hsv(*c) for c in x])
    np.testing.assert_allclose(hsv[:, 1:], ref[:, 1:], atol=1e-12)
    # hue: equal modulo 1 where the chroma is positive (colorsys also uses 0 for greys)
    dh = np.abs(np.mod(hsv[:, 0] - ref[:, 0] + 0.5, 1.0) - 0.5)
    assert dh.max() < 1e-9
    back = A.hsv_to_rgb(hsv)
    ref_back = np.array([colorsys.hsv_to_rgb(*h) for h in hsv])
    np.testing.assert_allclose(back, ref_back, atol=1e-12)
    np.testing.assert_allclose(back, x, atol=1e-12)


def test_identity_parameters_only_clamp():
    g = np.random.default_rng(2)
    rgb = g.uniform(-0.3, 1.4, (2, 8, 9, 3))
    out = A.augment(rgb, np.array([IDENT, IDENT]))
    np.testing.assert_allclose(out, np.clip(rgb, 0, 1), atol=1e-12)


def test_hue_third_of_a_turn_permutes_channels():
    x = _colours(2000, 3).reshape(1, 40, 50, 3)
    out = A.augment(x, np.array([[0.0, 1.0 / 3.0, 1.0, 1.0, 1.0]]))
    # a hue rotation by 120 degrees sends red to green: (r, g, b) -> (b, r, g)
    np.testing.assert_allclose(out, x[..., [2, 0, 1]], atol=1e-12)
    out = A.augment(x, np.array([[0.0, -1.0 / 3.0, 1.0, 1.0, 1.0]]))
    np.testing.assert_allclose(out, x[..., [1, 2, 0]], atol=1e-12)
    red = A.augment(np.array([[[[1.0, 0.0, 0.0]]]]), np.array([[0.0, 1.0 / 6.0, 1.0, 1.0, 1.0]]))
    np.testing.assert_allclose(red[0, 0, 0], [1.0, 1.0, 0.0], atol=1e-12)  # red + 60 degrees = yellow


def test_saturation_value_and_gamma_closed_forms():
    x = _colours(2000, 4).reshape(1, 40, 50, 3)
    v = x.max(axis=-1, keepdims=True)
    # zero saturation: the grey of the value
    out = A.augment(x, np.array([[0.0, 0.0, 0.0, 1.0, 1.0]]))
    np.testing.assert_allclose(out, np.broadcast_to(v, x.shape), atol=1e-12)
    # value scale 0.5 halves every channel (the hexcone map is homogeneous in v)
    out = A.augment(x, np.array([[0.0, 0.0, 1.0, 0.5, 1.0]]))
    np.testing.assert_allclose(out, 0.5 * x, atol=1e-12)
    # value scale 2 clamps the value at 1: the colour scales by 1 / v
    out = A.augment(x, np.array([[0.0, 0.0, 1.0, 2.0, 1.0]]))
    want = np.where(v > 0, x * np.minimum(2.0, 1.0 / np.maximum(v, 1e-300)), 0.0)
    np.testing.assert_allclose(out, want, atol=1e-12)
    # saturation scale 2 on a colour of saturation s: s' = min(1, 2 s), chroma and minimum follow
    s = (v[..., 0] - x.min(axis=-1))
    s = np.where(v[..., 0] > 0, s / np.where(v[..., 0] > 0, v[..., 0], 1), 0)
    out = A.augment(x, np.array([[0.0, 0.0, 2.0, 1.0, 1.0]]))
    np.testing.assert_allclose(out.min(axis=-1), v[..., 0] * (1 - np.minimum(1, 2 * s)), atol=1e-12)
    np.testing.assert_allclose(out.max(axis=-1), v[..., 0], atol=1e-12)
    # gamma alone
    out = A.augment(x, np.array([[0.0, 0.0, 1.0, 1.0, 0.7]]))
    np.testing.assert_allclose(out, x ** 0.7, atol=1e-12)


def test_overlay_blend():
    g = np.random.default_rng(5)
    x = g.random((3, 6, 7, 3))
    ov = g.uniform(-0.2, 1.2, (3, 6, 7, 3))
    p = np.array([[0.0, 0, 1, 1, 1], [0.3, 0, 1, 1, 1], [1.0, 0, 1, 1, 1]])
    out = A.augment(x, p, ov)
    np.testing.assert_allclose(out[0], x[0], atol=1e-12)
    np.testing.assert_allclose(out[1], 0.7 * x[1] + 0.3 * np.clip(ov[1], 0, 1), atol=1e-12)
    np.testing.assert_allclose(out[2], np.clip(ov[2], 0, 1), atol=1e-12)


def test_steps_compose_in_the_stated_order():
    """overlay, then HSV, then gamma: with all three active the result equals the three
    closed forms applied in that order (hue by a third of a turn, value halved, gamma 2)."""
    g = np.random.default_rng(6)
    x = g.random((1, 5, 5, 3))
    ov = g.random((1, 5, 5, 3))
    out = A.augment(x, np.array([[0.25, 1.0 / 3.0, 1.0, 0.5, 2.0]]), ov)
    blend = 0.75 * x + 0.25 * ov
    np.testing.assert_allclose(out, (0.5 * blend[..., [2, 0, 1]]) ** 2.0, atol=1e-12)
