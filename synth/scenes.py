"""Analytic scenes, cameras and exact first-hit depths (FP64, emitted as FP32).

A scene is a union of solid primitives (spheres, axis-aligned boxes) plus an
optional hollow room (the camera lives inside it and sees its walls).  The
depth of a ray is its along-ray distance ``D`` to the first surface, so that
``p* = o + D v`` with unit ``v``; a ray that hits nothing gets ``+inf``.

Rays are produced in FP64, rounded to FP32, and depths are computed from the
rounded FP32 rays promoted back to FP64, so the stored depth is consistent
with the stored ray.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


@dataclass
class Sphere:
    center: tuple
    radius: float
    albedo: tuple = (0.8, 0.8, 0.8)

    def hit(self, o, v):
        c = np.asarray(self.center, dtype=np.float64)
        oc = o - c
        b = np.einsum("ij,ij->i", v, oc)
        cc = np.einsum("ij,ij->i", oc, oc) - self.radius ** 2
        vv = np.einsum("ij,ij->i", v, v)
        disc = b * b - vv * cc
        t = np.full(o.shape[0], np.inf)
        ok = disc >= 0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        t0 = (-b - sq) / vv
        t1 = (-b + sq) / vv
        first = np.where(t0 > 0, t0, np.where(t1 > 0, t1, np.inf))
        t[ok] = first[ok]
        return t

    def sdf(self, p):
        return np.linalg.norm(p - np.asarray(self.center), axis=-1) - self.radius


@dataclass
class Box:
    lo: tuple
    hi: tuple
    albedo: tuple = (0.8, 0.8, 0.8)

    def _slabs(self, o, v):
        lo = np.asarray(self.lo, dtype=np.float64)
        hi = np.asarray(self.hi, dtype=np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / v
            t1 = (lo - o) * inv
            t2 = (hi - o) * inv
        # axis with v == 0: inside the slab -> (-inf, inf), outside -> empty
        zero = v == 0
        inside = (o >= lo) & (o <= hi)
        tn = np.minimum(t1, t2)
        tf = np.maximum(t1, t2)
        tn = np.where(zero, np.where(inside, -np.inf, np.inf), tn)
        tf = np.where(zero, np.where(inside, np.inf, -np.inf), tf)
        return tn.max(axis=1), tf.min(axis=1)

    def hit(self, o, v):
        tmin, tmax = self._slabs(o, v)
        ok = (tmax >= tmin) & (tmin > 0)
        return np.where(ok, tmin, np.inf)

    def sdf(self, p):
        lo = np.asarray(self.lo)
        hi = np.asarray(self.hi)
        c = 0.5 * (lo + hi)
        e = 0.5 * (hi - lo)
        q = np.abs(p - c) - e
        return np.linalg.norm(np.maximum(q, 0.0), axis=-1) + np.minimum(q.max(axis=-1), 0.0)


@dataclass
class Room:
    """Hollow box: free space inside, walls at its faces."""
    lo: tuple
    hi: tuple
    albedo: tuple = (0.7, 0.7, 0.7)

    def hit(self, o, v):
        tmin, tmax = Box(self.lo, self.hi)._slabs(o, v)
        ok = (tmax > 0) & (tmax >= tmin)
        return np.where(ok, tmax, np.inf)

    def sdf(self, p):
        # distance to the nearest wall, positive inside the room
        return -Box(self.lo, self.hi).sdf(p)


@dataclass
class Scene:
    prims: list = field(default_factory=list)

    def depth(self, o, v):
        """First-hit along-ray distance for FP64 rays [R,3]; +inf on a miss."""
        return self.hit_prim(o, v)[1]

    def hit_prim(self, o, v, chunk=16384):
        """Index of the primitive hit first (-1 on a miss) and its depth.

        Solid boxes are tested together (slab test broadcast over boxes),
        the other primitives one by one.
        """
        o = np.asarray(o, dtype=np.float64)
        v = np.asarray(v, dtype=np.float64)
        best = np.full(o.shape[0], np.inf)
        idx = np.full(o.shape[0], -1, dtype=np.int64)
        box_ids = [k for k, p in enumerate(self.prims) if type(p) is Box]
        for k, p in enumerate(self.prims):
            if k in box_ids:
                continue
            t = p.hit(o, v)
            better = t < best
            best = np.where(better, t, best)
            idx = np.where(better, k, idx)
        if box_ids:
            lo = np.array([self.prims[k].lo for k in box_ids], dtype=np.float64)
            hi = np.array([self.prims[k].hi for k in box_ids], dtype=np.float64)
            ids = np.array(box_ids)
            for s in range(0, o.shape[0], chunk):
                oo = o[s:s + chunk, None, :]
                vv = v[s:s + chunk]
                inv = 1.0 / np.where(vv == 0, 1e-300, vv)
                t1 = (lo[None] - oo) * inv[:, None, :]
                t2 = (hi[None] - oo) * inv[:, None, :]
                tn = np.minimum(t1, t2).max(axis=2)
                tf = np.maximum(t1, t2).min(axis=2)
                t = np.where((tf >= tn) & (tn > 0), tn, np.inf)
                j = t.argmin(axis=1)
                tb = t[np.arange(t.shape[0]), j]
                better = tb < best[s:s + chunk]
                best[s:s + chunk] = np.where(better, tb, best[s:s + chunk])
                idx[s:s + chunk] = np.where(better, ids[j], idx[s:s + chunk])
        return idx, best

    def clearance(self, p):
        """Distance from points [N,3] to the nearest surface (free space > 0)."""
        p = np.atleast_2d(np.asarray(p, dtype=np.float64))
        d = np.full(p.shape[0], np.inf)
        for prim in self.prims:
            d = np.minimum(d, prim.sdf(p))
        return d


def _look_frame(forward, up=(0.0, 0.0, 1.0)):
    f = np.asarray(forward, dtype=np.float64)
    f = f / np.linalg.norm(f)
    up = np.asarray(up, dtype=np.float64)
    if abs(np.dot(f, up)) > 0.999:
        up = np.array([0.0, 1.0, 0.0])
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)  # image "down"
    return r, d, f


def pinhole_rays(center, forward, width, height, fov_y_deg=None, fov_x_deg=None,
                 up=(0.0, 0.0, 1.0)):
    """Per-pixel rays of a pinhole camera, pixel centres at +1/2, row-major.

    Returns FP32 ``o [H*W,3]`` and unit ``v [H*W,3]``.
    """
    r, d, f = _look_frame(forward, up)
    if fov_x_deg is not None:
        fx = 0.5 * width / np.tan(np.radians(fov_x_deg) / 2)
        fy = fx
    else:
        fy = 0.5 * height / np.tan(np.radians(fov_y_deg) / 2)
        fx = fy
    jj, ii = np.meshgrid(np.arange(height, dtype=np.float64),
                         np.arange(width, dtype=np.float64), indexing="ij")
    x = (ii.ravel() + 0.5 - width / 2) / fx
    y = (jj.ravel() + 0.5 - height / 2) / fy
    dirs = x[:, None] * r[None] + y[:, None] * d[None] + f[None]
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    v = dirs.astype(np.float32)
    o = np.broadcast_to(np.asarray(center, dtype=np.float32), v.shape).copy()
    return o, v


def equirect_rays(center, width, height, yaw0=0.0):
    """Equirectangular panorama rays (longitude across, latitude down)."""
    jj, ii = np.meshgrid(np.arange(height, dtype=np.float64),
                         np.arange(width, dtype=np.float64), indexing="ij")
    lon = yaw0 + 2 * np.pi * (ii.ravel() + 0.5) / width
    lat = np.pi / 2 - np.pi * (jj.ravel() + 0.5) / height
    dirs = np.stack([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)], 1)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    v = dirs.astype(np.float32)
    o = np.broadcast_to(np.asarray(center, dtype=np.float32), v.shape).copy()
    return o, v


def ray_depth(scene, o32, v32):
    """FP32 depth of FP32 rays, computed in FP64 from the FP32 values."""
    d = scene.depth(o32.astype(np.float64), v32.astype(np.float64))
    return d.astype(np.float32)


def sensor_depth(scene, o32, v32):
    """Depth reading of rays whose origins may lie anywhere, e.g. rays cast
    from voxel centres to fill unseen space: a sensor whose origin is inside
    a solid (clearance < 0) is blocked at once and reports the shortest valid
    depth, 2^-16 m (a zero or missing reading would mean free space)."""
    d = ray_depth(scene, o32, v32)
    inside = scene.clearance(o32.astype(np.float64)) < 0
    return np.where(inside, np.float32(2.0 ** -16), d).astype(np.float32)


def surface_normal(prim, p):
    """Outward (towards free space) unit normal of `prim` at surface points p."""
    p = np.atleast_2d(np.asarray(p, np.float64))
    if isinstance(prim, Sphere):
        n = p - np.asarray(prim.center)
        return n / np.linalg.norm(n, axis=1, keepdims=True)
    lo = np.asarray(prim.lo)
    hi = np.asarray(prim.hi)
    c = 0.5 * (lo + hi)
    e = 0.5 * (hi - lo)
    q = (p - c) / e
    a = np.abs(q).argmax(axis=1)
    n = np.zeros_like(p)
    n[np.arange(p.shape[0]), a] = np.sign(q[np.arange(p.shape[0]), a])
    return -n if isinstance(prim, Room) else n


LIGHT_DIR = np.array([0.3, 0.5, 0.81]) / np.linalg.norm([0.3, 0.5, 0.81])


def shade(scene, o32, v32):
    """Analytic target colour: albedo * (0.25 + 0.75 max(0, n . l)); black on a miss."""
    o = o32.astype(np.float64)
    v = v32.astype(np.float64)
    idx, d = scene.hit_prim(o, v)
    rgb = np.zeros((o.shape[0], 3))
    for k, prim in enumerate(scene.prims):
        sel = idx == k
        if not sel.any():
            continue
        p = o[sel] + d[sel, None] * v[sel]
        n = surface_normal(prim, p)
        lam = 0.25 + 0.75 * np.clip(n @ LIGHT_DIR, 0.0, None)
        rgb[sel] = lam[:, None] * np.asarray(prim.albedo)[None]
    return rgb.astype(np.float32)
