"""The five synthetic workloads (C1..C5) and their seeded inputs.

Every generator is deterministic given its seed (NumPy PCG64).  The scenes
stand in for the paper's datasets (which are not used): C2 mirrors Replica
room 0's view count and image size with an indoor box room, C5 mirrors the
scale and thin partitions of the large panoramic Lobby scene.

Grid constants (origin, voxel size, truncation) are multiples of 2^-20 m so
that ray snapping onto the 2^-20 m lattice keeps voxel traversal exact.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field, replace
import os

import numpy as np

from .scenes import Scene, Sphere, Box, Room, pinhole_rays, equirect_rays, ray_depth, shade
from .weights import SdfNet, ColorNet, sdf_params, color_params

CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5", "c1n", "c2n")


@dataclass(frozen=True)
class Grid:
    n: tuple            # voxels per axis (x, y, z)
    lo: tuple           # min corner [m]
    h: float            # voxel edge [m]
    d_t: float          # truncation distance D_T [m]
    d_s: float          # surface criterion D_s [m]
    nb_radius: int = 2  # neighbourhood (2r+1)^3 for the inside test
    m_consec: int = 15  # M: consecutive inside voxels that fix t_f

    @property
    def hi(self):
        return tuple(self.lo[a] + self.n[a] * self.h for a in range(3))

    @property
    def n_vox(self):
        return self.n[0] * self.n[1] * self.n[2]


@dataclass(frozen=True)
class Sampling:
    rho_num: int = 1     # samples per traversed voxel = rho_num / rho_den
    rho_den: int = 1
    n_min: int = 1
    n_max: int = 16
    t_far: float = float("inf")


@dataclass
class Config:
    name: str
    grid: Grid
    sdf: SdfNet
    color: ColorNet
    in_center: tuple
    in_scale: float
    sampling: Sampling
    neus_s: float = 64.0
    precision: str = "fp32"
    build_scene: object = None
    integ_views: object = None      # callable(scene) -> list of (o, v) per view
    render_view: object = None      # callable(scene) -> (o, v)
    notes: str = ""
    # depth of a density field (NeRF-like) instead of the exact surface
    # distance: per view, seeded Gaussian error of sigma_vox voxels on every
    # ray and, on a fraction `floaters` of the rays, a spurious hit uniformly
    # between 30% and 100% of the true depth (None: exact depths)
    depth_noise: tuple = None       # (sigma_vox, floaters)

    # -- cached products -------------------------------------------------
    _scene: object = field(default=None, repr=False)

    def scene(self):
        if self._scene is None:
            self._scene = self.build_scene()
        return self._scene

    def integration_rays(self, views=None, progress=None, tile=0):
        """FP32 (o, v, depth) of the training views (all, or a subset);
        progress(done, total), if given, is called every 25 depth maps.
        tile > 0 lists each square view's rays by tile x tile pixel blocks
        (blocks row by row, pixels row by row inside a block) instead of
        row by row: the same rays in another order."""
        sc = self.scene()
        vs = self.integ_views(sc)
        if views is not None:
            vs = [vs[i] for i in views]
        workers = max(1, min(16, os.cpu_count() or 1, len(vs)))
        ds_ = []
        with ThreadPoolExecutor(workers) as ex:
            for k, dk in enumerate(ex.map(lambda ov: ray_depth(sc, ov[0], ov[1]), vs)):
                ds_.append(dk)
                if progress is not None and (k + 1) % 25 == 0:
                    progress(k + 1, len(vs))
        if self.depth_noise is not None:
            ids = range(len(vs)) if views is None else views
            ds_ = [self._noisy(d, i) for d, i in zip(ds_, ids)]
        if tile > 0:
            perms = [tile_order(o.shape[0], tile) for o, _ in vs]
            vs = [(o[p], v[p]) for (o, v), p in zip(vs, perms)]
            ds_ = [d[p] for d, p in zip(ds_, perms)]
        return (np.concatenate([o for o, _ in vs]), np.concatenate([v for _, v in vs]),
                np.concatenate(ds_))

    def _noisy(self, d, view):
        sigma_vox, floaters = self.depth_noise
        rng = np.random.Generator(np.random.PCG64(1000 + view))
        d64 = d.astype(np.float64)
        e = rng.normal(0.0, sigma_vox * self.grid.h, d.shape)
        fl = rng.uniform(size=d.shape) < floaters
        spur = rng.uniform(0.3, 1.0, d.shape) * d64
        out = np.where(fl, spur, d64 + e)
        out = np.where(np.isfinite(d64), np.maximum(out, 1e-3), d64)
        return out.astype(np.float32)

    def render_rays(self):
        o, v = self.render_view(self.scene())
        return o, v

    def training_batch(self, n_rays, seed=0):
        """Random pixels of the training views, with analytic target colours."""
        rng = np.random.Generator(np.random.PCG64(seed))
        vs = self.integ_views(self.scene())
        pix = vs[0][0].shape[0]
        view = rng.integers(0, len(vs), n_rays)
        px = rng.integers(0, pix, n_rays)
        o = np.stack([vs[a][0][b] for a, b in zip(view, px)])
        v = np.stack([vs[a][1][b] for a, b in zip(view, px)])
        return o, v, shade(self.scene(), o, v)

    def eikonal_points(self, n, seed=0):
        """Uniform points in the grid cube (FP32)."""
        rng = np.random.Generator(np.random.PCG64(seed))
        lo = np.asarray(self.grid.lo)
        hi = np.asarray(self.grid.hi)
        return rng.uniform(lo, hi, (n, 3)).astype(np.float32)

    def sdf_params(self):
        return sdf_params(self.sdf)

    def color_params(self):
        return color_params(self.color)


# ---------------------------------------------------------------- scenes ----

def _scene_c1():
    return Scene([Sphere((0.0, 0.0, 0.0), 0.5, (0.9, 0.3, 0.2)),
                  Box((0.3, -0.3, -0.3), (0.9, 0.3, 0.3), (0.2, 0.5, 0.9))])


def _random_albedo(rng):
    return tuple(float(x) for x in rng.uniform(0.2, 0.95, 3))


def _scene_room(seed, size, n_boxes, n_slabs, slab_thick, walls=()):
    rng = np.random.Generator(np.random.PCG64(seed))
    sx, sy, sz = size
    prims = [Room((0.0, 0.0, 0.0), (sx, sy, sz), (0.7, 0.7, 0.65))]
    prims += list(walls)
    for _ in range(n_boxes):
        he = rng.uniform(0.1, 0.5, 3)
        cx = rng.uniform(he[0], sx - he[0])
        cy = rng.uniform(he[1], sy - he[1])
        prims.append(Box((cx - he[0], cy - he[1], 0.0), (cx + he[0], cy + he[1], 2 * he[2]),
                         _random_albedo(rng)))
    for _ in range(n_slabs):
        length = rng.uniform(1.5, 2.5)
        height = rng.uniform(1.0, sz)
        normal_x = rng.uniform() < 0.5
        if normal_x:
            cx = rng.uniform(0.5, sx - 0.5)
            cy = rng.uniform(length / 2, sy - length / 2)
            lo = (cx - slab_thick / 2, cy - length / 2, 0.0)
            hi = (cx + slab_thick / 2, cy + length / 2, height)
        else:
            cx = rng.uniform(length / 2, sx - length / 2)
            cy = rng.uniform(0.5, sy - 0.5)
            lo = (cx - length / 2, cy - slab_thick / 2, 0.0)
            hi = (cx + length / 2, cy + slab_thick / 2, height)
        prims.append(Box(lo, hi, _random_albedo(rng)))
    return Scene(prims)


def _scene_c2():
    return _scene_room(0, (6.0, 6.0, 3.0), 20, 4, 0.02)


def _c5_walls():
    t = 0.05  # half thickness: 10 cm partition walls
    ws = []
    # wall x = 6 with doorways at y in [1.5,2.5] and [5.5,6.5]
    for y0, y1 in ((0.0, 1.5), (2.5, 5.5), (6.5, 8.0)):
        ws.append(Box((6.0 - t, y0, 0.0), (6.0 + t, y1, 3.0)))
    # wall y = 4 with doorways at x in [2.5,3.5] and [8.5,9.5]
    for x0, x1 in ((0.0, 2.5), (3.5, 6.0 - t), (6.0 + t, 8.5), (9.5, 12.0)):
        ws.append(Box((x0, 4.0 - t, 0.0), (x1, 4.0 + t, 3.0)))
    return ws


def _scene_c5():
    return _scene_room(0, (12.0, 8.0, 3.0), 60, 10, 0.01, walls=_c5_walls())


# --------------------------------------------------------------- cameras ----

def _orbit_views(seed, n, radius, width, height, fov_y):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        c = radius * d
        out.append(pinhole_rays(c, -c, width, height, fov_y_deg=fov_y))
    return out


def _free_pose(rng, scene, size, clearance=0.3, z_range=(0.8, 2.2)):
    sx, sy, _ = size
    while True:
        c = np.array([rng.uniform(clearance, sx - clearance),
                      rng.uniform(clearance, sy - clearance),
                      rng.uniform(*z_range)])
        if scene.clearance(c)[0] >= clearance:
            yaw = rng.uniform(0, 2 * np.pi)
            pitch = np.radians(rng.uniform(-30, 30))
            fwd = np.array([np.cos(pitch) * np.cos(yaw), np.cos(pitch) * np.sin(yaw), np.sin(pitch)])
            return c, fwd


def _room_views(seed, n, size, width, height, fov_x):
    def make(scene):
        rng = np.random.Generator(np.random.PCG64(seed))
        out = []
        for _ in range(n):
            c, fwd = _free_pose(rng, scene, size)
            out.append(pinhole_rays(c, fwd, width, height, fov_x_deg=fov_x))
        return out
    return make


def tile_order(n, tile):
    """Pixel order of a square n-pixel image by tile x tile blocks (blocks
    row by row, pixels row by row inside a block); identity when the image
    is not square or its side is not a multiple of tile."""
    side = int(round(n ** 0.5))
    if side * side != n or side % tile:
        return np.arange(n)
    y, x = np.divmod(np.arange(n), side)
    key = ((y // tile) * (side // tile) + x // tile) * tile * tile + (y % tile) * tile + x % tile
    return np.argsort(key, kind="stable")


# --------------------------------------------------------------- configs ----

def _c1():
    h = 1.0 / 32
    return Config(
        name="c1",
        grid=Grid((64, 64, 64), (-1.0, -1.0, -1.0), h, 3 * h, h),
        sdf=SdfNet(width=64, n_hidden=4, pe_freqs=0, skip_at=-1, n_feat=64),
        color=ColorNet(width=64, n_hidden=2, n_feat=64),
        in_center=(0.0, 0.0, 0.0), in_scale=1.0,
        sampling=Sampling(1, 1, 1, 16),
        build_scene=_scene_c1,
        integ_views=lambda sc: _orbit_views(0, 8, 2.5, 64, 64, 45.0),
        render_view=lambda sc: _orbit_views(1, 1, 2.5, 64, 64, 45.0)[0],
        notes="sphere r=0.5 + box half 0.3 at (0.6,0,0); 8 orbit views 64x64",
    )


def _c2():
    h = 7.0 / 256
    size = (6.0, 6.0, 3.0)

    def render(scene):
        rng = np.random.Generator(np.random.PCG64(1))
        c, fwd = _free_pose(rng, scene, size)
        return pinhole_rays(c, fwd, 640, 480, fov_x_deg=90.0)

    return Config(
        name="c2",
        grid=Grid((256, 256, 256), (-0.5, -0.5, -0.5), h, 5 * h, h),
        sdf=SdfNet(inside_out=True), color=ColorNet(),
        # inside-out geometric-init sphere of radius 1 m centred at the render
        # camera, so that the untrained network's zero level set crosses most
        # TSDF bounds of the view (about 2/3 of them contain t = 1 m)
        in_center=(4.77, 2.51, 1.57), in_scale=2.0,
        sampling=Sampling(1, 2, 1, 64),
        build_scene=_scene_c2,
        integ_views=_room_views(0, 100, size, 384, 384, 90.0),
        render_view=render,
        notes="6x6x3 m room, 20 boxes, 4 slabs of 2 cm; 100 views 384^2; render 640x480",
    )


def _c5():
    h = 13.0 / 512
    size = (12.0, 8.0, 3.0)

    def render(scene):
        rng = np.random.Generator(np.random.PCG64(1))
        c, _ = _free_pose(rng, scene, size)
        return equirect_rays(c, 2048, 1024)

    return Config(
        name="c5",
        grid=Grid((512, 512, 512), (-0.5, -0.5, -0.5), h, 5 * h, h),
        # inside-out geometric-init sphere of radius 1.5 m centred at the
        # panorama's viewpoint (median hit distance 1.47 m)
        sdf=SdfNet(inside_out=True), color=ColorNet(),
        in_center=(11.11, 2.61, 1.39), in_scale=3.0,
        sampling=Sampling(1, 2, 1, 64),
        precision="bf16",
        build_scene=_scene_c5,
        integ_views=_room_views(0, 300, size, 512, 512, 90.0),
        render_view=render,
        notes="12x8x3 m, 2x2 rooms, 60 boxes, 10 slabs of 1 cm; 300 views 512^2; equirect 2048x1024",
    )


def _nerf_mode(cfg, name):
    """The same scene and views fused from density-field-like depths with
    the bound parameters used for NeRF: D_T = 39h, D_s = 27h, 7^3
    neighbourhood, M = 15."""
    g = cfg.grid
    return replace(cfg, name=name, grid=replace(g, d_t=39 * g.h, d_s=27 * g.h, nb_radius=3),
                   depth_noise=(2.0, 0.01),
                   notes=cfg.notes + "; NeRF-mode bounds on noisy depths (sigma 2h, 1% floaters)")


def get_config(name: str) -> Config:
    name = name.lower()
    if name == "c1n":
        return _nerf_mode(_c1(), "c1n")
    if name == "c2n":
        return _nerf_mode(_c2(), "c2n")
    if name == "c1":
        return _c1()
    if name == "c2":
        return _c2()
    if name == "c3":
        return replace(_c2(), name="c3", precision="bf16")
    if name == "c4":
        return replace(_c2(), name="c4")
    if name == "c5":
        return _c5()
    raise KeyError(name)
