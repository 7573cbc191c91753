"""Pinhole cameras around the scene cube (input generation only).

Cameras sit on a sphere around the scene and look at its centre, like the
hemisphere camera placements of the RTMV environments (section 3).  Images are
square with the same full field of view on both axes; pixel centres are at
+1/2; row 0 is the top row.  Directions are normalised in FP64, then rounded
to FP32, so depth along a ray is measured in units of |d| ~= 1.
"""

from __future__ import annotations

import numpy as np


class Camera:
    def __init__(self, position, width, height, fov_deg, target=(0.0, 0.0, 0.0)):
        self.pos = np.asarray(position, np.float64)
        self.W, self.H = int(width), int(height)
        self.fov = float(fov_deg)
        f = np.asarray(target, np.float64) - self.pos
        f /= np.linalg.norm(f)
        up = np.array([0.0, 0.0, 1.0])
        if abs(f @ up) > 0.999:
            up = np.array([0.0, 1.0, 0.0])
        r = np.cross(f, up)
        r /= np.linalg.norm(r)
        u = np.cross(r, f)
        self.f, self.r, self.u = f, r, u

    def rays(self, pixel_index=None):
        """FP32 (o, d) for flat pixel indices (row-major), default all."""
        if pixel_index is None:
            pixel_index = np.arange(self.W * self.H, dtype=np.int64)
        py = pixel_index // self.W
        px = pixel_index % self.W
        t = np.tan(np.deg2rad(self.fov) * 0.5)
        x = (2.0 * (px + 0.5) / self.W - 1.0) * t
        y = (1.0 - 2.0 * (py + 0.5) / self.H) * t
        d = self.f[None, :] + x[:, None] * self.r[None, :] + y[:, None] * self.u[None, :]
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        o = np.broadcast_to(self.pos, d.shape)
        return (np.ascontiguousarray(o, dtype=np.float32),
                np.ascontiguousarray(d, dtype=np.float32))


def sphere_camera(rng, radius, width, height, fov_deg=50.0):
    v = rng.standard_normal(3)
    v /= np.linalg.norm(v)
    return Camera(v * radius, width, height, fov_deg)
