"""Closed-form microphone energies of plane reflectors (image sources), shared by the
oracle pins and the GPU tests.

Everything here is written from the geometry alone: a plane reflector seen from a
point source acts as a mirror-image source of strength (1 - alpha) (paper Section 2:
reflections lose energy; image sources are the method's stated background), two
perpendicular planes add a second-order image of strength (1 - alpha_1)(1 - alpha_2),
and the direct path spreads as W / (4 pi d^2).  Nothing here calls the oracle or the
GPU library; the functions return reference energies and the microphones where the
closed form applies.
"""
from __future__ import annotations

import math

import numpy as np

FOUR_PI = 4.0 * math.pi


def f32(x) -> float:
    """A scene value as both tracers see it (inputs are rounded to float32 once)."""
    return float(np.float32(x))


def _spread(m, s):
    return 1.0 / (FOUR_PI * ((m - s) ** 2).sum(1))


def _grazing_ok(m, img, normal, min_deg):
    """The path from an image to each microphone crosses the reflector at more than
    min_deg degrees (beams near the reflector's horizon straddle it)."""
    d = m - img
    s = np.abs(d @ np.asarray(normal, np.float64)) / np.linalg.norm(d, axis=1)
    return np.degrees(np.arcsin(np.minimum(s, 1.0))) > min_deg


def ground_offset(scene, ground_z, alpha, min_deg=15.0):
    """Ground plane z = h, source above it: direct path plus the image at (x, y, 2h - z_s)
    weighted 1 - alpha.  Returns (reference energies, microphones the form covers)."""
    m = scene.mic_positions()
    s = scene.sources[0].astype(np.float64)
    h = f32(ground_z)
    img = s.copy()
    img[2] = 2.0 * h - s[2]
    ref = _spread(m, s) + (1.0 - f32(alpha)) * _spread(m, img)
    return ref, _grazing_ok(m, img, (0.0, 0.0, 1.0), min_deg)


def wall_offset(scene, wall_x, alpha, min_deg=15.0):
    """Vertical wall x = c, source and microphones in front of it: direct path plus the
    image at (2c - x_s, y_s, z_s) weighted 1 - alpha."""
    m = scene.mic_positions()
    s = scene.sources[0].astype(np.float64)
    c = f32(wall_x)
    img = s.copy()
    img[0] = 2.0 * c - s[0]
    ref = _spread(m, s) + (1.0 - f32(alpha)) * _spread(m, img)
    return ref, _grazing_ok(m, img, (1.0, 0.0, 0.0), min_deg)


def _cross(a, b, axis, value):
    t = (value - a[..., axis]) / (b[..., axis] - a[..., axis])
    return a + t[..., None] * (b - a)


def corner(scene, wall_x, alpha_ground, alpha_wall, min_margin=0.03):
    """Ground z = 0 (x <= c) and wall x = c (z >= 0), source and microphones inside the
    corner.  A right-angle corner shows every point inside it all three images: the ground
    image (x, y, -z) weighted 1 - a_g, the wall image (2c - x, y, z) weighted 1 - a_w, and
    the second-order image (2c - x, y, -z) weighted (1 - a_g)(1 - a_w), reached through
    the ground then the wall or the wall then the ground, whichever the microphone sees.

    Returns (reference, ok, last_on_wall): ok keeps the microphones whose every reflection
    point lies farther from the corner line than min_margin radians as seen from the
    apex it is reached from (a beam there straddles both planes); last_on_wall tells
    which of the two second-order paths reaches each microphone."""
    m = scene.mic_positions()
    n = m.shape[0]
    s = scene.sources[0].astype(np.float64)
    c = f32(wall_x)
    s_g = s * np.array([1.0, 1.0, -1.0])
    s_w = s.copy()
    s_w[0] = 2.0 * c - s[0]
    s_gw = s_w * np.array([1.0, 1.0, -1.0])
    ag, aw = f32(alpha_ground), f32(alpha_wall)
    ref = _spread(m, s) + (1 - ag) * _spread(m, s_g) + (1 - aw) * _spread(m, s_w) \
        + (1 - ag) * (1 - aw) * _spread(m, s_gw)

    def line_dist(p):   # distance to the corner line x = c, z = 0
        return np.hypot(p[:, 0] - c, p[:, 2])

    margins = []
    p = _cross(np.broadcast_to(s_g, (n, 3)), m, 2, 0.0)
    margins.append(line_dist(p) / np.linalg.norm(p - s, axis=1))
    p = _cross(np.broadcast_to(s_w, (n, 3)), m, 0, c)
    margins.append(line_dist(p) / np.linalg.norm(p - s, axis=1))
    # second order, unfolded from the microphone: the plane its line to s_gw meets first
    # is the last reflector
    t_w = (c - m[:, 0]) / (s_gw[0] - m[:, 0])
    t_g = (0.0 - m[:, 2]) / (s_gw[2] - m[:, 2])
    last_on_wall = t_w < t_g
    p2 = m + np.where(last_on_wall, t_w, t_g)[:, None] * (s_gw - m)
    first_img = np.where(last_on_wall[:, None], s_g[None, :], s_w[None, :])
    p1 = np.where(last_on_wall[:, None], _cross(np.broadcast_to(s_g, (n, 3)), p2, 2, 0.0),
                  _cross(np.broadcast_to(s_w, (n, 3)), p2, 0, c))
    margins.append(line_dist(p1) / np.linalg.norm(p1 - s, axis=1))
    margins.append(line_dist(p2) / np.linalg.norm(p2 - first_img, axis=1))
    ok = np.min(np.stack(margins), axis=0) > min_margin
    return ref, ok, last_on_wall


def sealed_box_threshold(alpha, generation, eps):
    """Energy threshold that stops a level-0 sealed box at a chosen generation.  The 20
    level-0 beams are congruent, so every beam of generation g carries W (1 - alpha)^g / 20
    (W = 1).  A child is kept when its power after absorption exceeds e_min; with
    e_min = (1 - alpha)^G / 20 (1 + eps), eps > 0 ends the run before generation G, eps < 0
    after it.  Returns (e_min, expected beams per generation for generations 0..)."""
    a = f32(alpha)
    e_min = (1.0 - a) ** generation / 20.0 * (1.0 + eps)
    alive = generation if eps > 0 else generation + 1
    return e_min, alive
