"""Oracle: TSDF integration, finalize, voxel flags, Alg. 1 bounds, placement.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper passages followed:
  * Sec. 3.2 "TSDF Integration" and the supplementary Alg. "TSDF integration":
    clamped projective distance, running weighted average, initial values
    (V = "unseen", W = 0), break at the first voxel with s <= -D_T.
  * Sec. 3.3 "Sample Boundary Detection" and Alg. 1: phase 1 (V <= D_s) sets
    t_n, phase 2 (M consecutive voxels whose neighbourhood is all negative)
    sets t_f; Sec. 4.2 fixes D_T = 5h, D_s = 1h, a 5x5x5 neighbourhood, M = 15.
  * Sec. 3.4 "Adaptive Sampling": equal intervals inside the bound, count
    proportional to the bound's length.
  * Sec. 4.3: voxels no ray has updated can be filled by casting more rays
    (frontier: where they border observed free space).
Readings where the paper is silent are listed in the design notes and in
``tsdf_oracle.c``: unit integration weight, "unseen" stored as -D_T, voxel
traversal on the 2^-20 m lattice, length measured in traversed voxels.
"""
from __future__ import annotations

import ctypes
import numpy as np

from . import _native

ST_HIT, ST_NO_FAR, ST_MISS, ST_INVALID = 0, 1, 2, 3


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _gargs(grid):
    n = np.ascontiguousarray(grid.n, dtype=np.int32)
    lo = np.ascontiguousarray([float(np.float32(x)) for x in grid.lo], dtype=np.float64)
    return n, lo, float(np.float32(grid.h))


def walk(grid, o, v, cap=1 << 16):
    """Voxels visited by one ray: (linear index, FP32 entry, FP32 exit)."""
    n, lo, h = _gargs(grid)
    o = np.ascontiguousarray(o, dtype=np.float32)
    v = np.ascontiguousarray(v, dtype=np.float32)
    vox = np.zeros(cap, np.int64)
    te = np.zeros(cap, np.float32)
    tx = np.zeros(cap, np.float32)
    cnt = ctypes.c_int64(0)
    rc = _native.lib().oracle_walk(_ptr(n), _ptr(lo), h, _ptr(o), _ptr(v), cap, _ptr(vox),
                                   _ptr(te), _ptr(tx), ctypes.byref(cnt))
    if rc < 0:
        raise ValueError("grid not on the 2^-20 lattice")
    if rc == 1:
        return None
    k = min(cnt.value, cap)
    return vox[:k], te[:k], tx[:k]


def ray_range(grid, o, v):
    """FP32 parameter range [t_in, t_out] of each ray inside the grid (0,0 on a miss)."""
    n, lo, h = _gargs(grid)
    o = np.ascontiguousarray(o, dtype=np.float32)
    v = np.ascontiguousarray(v, dtype=np.float32)
    R = o.shape[0]
    t_in = np.zeros(R, np.float32)
    t_out = np.zeros(R, np.float32)
    _native.lib().oracle_ray_range(_ptr(n), _ptr(lo), h, _ptr(o), _ptr(v), R, _ptr(t_in), _ptr(t_out))
    return t_in, t_out


class Integration:
    """Accumulated integration state: sum of s and update count per voxel."""

    def __init__(self, grid):
        self.grid = grid
        N = grid.n_vox
        self.sum_s = np.zeros(N, np.float64)
        self.cnt = np.zeros(N, np.int64)
        self.ties = 0
        self.updates = 0
        self.invalid = 0

    def add(self, o, v, depth, tie_eps=1e-9):
        g = self.grid
        n, lo, h = _gargs(g)
        o = np.ascontiguousarray(o, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        depth = np.ascontiguousarray(depth, dtype=np.float32)
        ties = ctypes.c_int64(0)
        upd = ctypes.c_int64(0)
        inv = ctypes.c_int64(0)
        rc = _native.lib().oracle_integrate(
            _ptr(n), _ptr(lo), h, float(np.float32(g.d_t)), _ptr(o), _ptr(v), _ptr(depth),
            o.shape[0], _ptr(self.sum_s), _ptr(self.cnt), tie_eps, ctypes.byref(ties),
            ctypes.byref(upd), ctypes.byref(inv))
        if rc < 0:
            raise ValueError("grid not on the 2^-20 lattice")
        self.ties += ties.value
        self.updates += upd.value
        self.invalid += inv.value
        return self


def integrate(grid, o, v, depth, tie_eps=1e-9):
    return Integration(grid).add(o, v, depth, tie_eps)


def finalize(grid, state: Integration):
    """V = weighted mean of s (unit weights); unseen voxels (W = 0) hold -D_T.

    Returned as FP64, shape [nz, ny, nx] (x fastest in memory).
    """
    d_t = float(np.float32(grid.d_t))
    V = np.full(grid.n_vox, -d_t, np.float64)
    seen = state.cnt > 0
    V[seen] = state.sum_s[seen] / state.cnt[seen]
    nx, ny, nz = grid.n
    return V.reshape(nz, ny, nx)


def flags(grid, V):
    """Voxel flags used by Alg. 1.

    bit0: V(X) <= D_s (the "surface" group of phase 1).
    bit1: every voxel Y in the (2r+1)^3 cube centred on X has V(Y) < 0
          (phase 2's inside test); neighbours outside the grid are unseen,
          i.e. negative.
    """
    d_s = float(np.float32(grid.d_s))
    r = grid.nb_radius
    V = np.asarray(V, dtype=np.float64)
    neg = V < 0
    padded = np.pad(neg, r, mode="constant", constant_values=True)
    nz, ny, nx = V.shape
    inside = np.ones_like(neg)
    for dz in range(2 * r + 1):
        for dy in range(2 * r + 1):
            for dx in range(2 * r + 1):
                inside &= padded[dz:dz + nz, dy:dy + ny, dx:dx + nx]
    out = (V <= d_s).astype(np.uint8) | (inside.astype(np.uint8) << 1)
    return out


def bounds(grid, flag_vol, o, v, t_far=np.inf):
    """Alg. 1 per ray on the flag volume; returns a dict of per-ray arrays."""
    n, lo, h = _gargs(grid)
    o = np.ascontiguousarray(o, dtype=np.float32)
    v = np.ascontiguousarray(v, dtype=np.float32)
    fl = np.ascontiguousarray(flag_vol, dtype=np.uint8).ravel()
    assert fl.size == grid.n_vox
    R = o.shape[0]
    out = dict(t_n=np.zeros(R, np.float32), t_f=np.zeros(R, np.float32),
               first_hit=np.zeros(R, np.int32), n_vox=np.zeros(R, np.int32),
               status=np.zeros(R, np.uint8), n_steps=np.zeros(R, np.int32))
    rc = _native.lib().oracle_bounds(_ptr(n), _ptr(lo), h, int(grid.m_consec), _ptr(fl), _ptr(o),
                                     _ptr(v), R, float(np.float32(t_far)), _ptr(out["t_n"]),
                                     _ptr(out["t_f"]), _ptr(out["first_hit"]), _ptr(out["n_vox"]),
                                     _ptr(out["status"]), _ptr(out["n_steps"]))
    if rc < 0:
        raise ValueError("grid not on the 2^-20 lattice")
    return out


def sample_counts(n_vox, status, rho_num, rho_den, n_min, n_max):
    """Adaptive count: proportional to the bound length in traversed voxels."""
    n_vox = np.asarray(n_vox, dtype=np.int64)
    n = -((-n_vox * rho_num) // rho_den)            # ceil(n_vox * rho)
    n = np.clip(n, n_min, n_max)
    ok = (status == ST_HIT) | (status == ST_NO_FAR)
    return np.where(ok, n, 0).astype(np.int64)


def place(t_n, t_f, n_vox, status, rho_num, rho_den, n_min, n_max):
    """Samples at the midpoints of n equal sections of [t_n, t_f] (FP64)."""
    counts = sample_counts(n_vox, status, rho_num, rho_den, n_min, n_max)
    offsets = np.zeros(counts.size + 1, np.int64)
    offsets[1:] = np.cumsum(counts)
    S = int(offsets[-1])
    ray_id = np.repeat(np.arange(counts.size), counts)
    k = np.arange(S) - offsets[:-1][ray_id]
    tn = np.asarray(t_n, np.float64)[ray_id]
    tf = np.asarray(t_f, np.float64)[ray_id]
    dt = (tf - tn) / counts[ray_id]
    t = tn + (k + 0.5) * dt
    return dict(counts=counts, offsets=offsets, t=t, dt=dt, ray_id=ray_id)


LEN_Q = float(1 << 24)   # fixed-point unit of the summed lengths: 2^-24 m


def containment(t_in, t_out, b, depth):
    """The counting of Table 1 (Sec. 4.3) over the rays that carry an
    integration depth: how many, how many fail (status not HIT / NO_FAR, or
    the depth outside [t_n, t_f]), and the summed original range t_out - t_in
    (the ray's span of the grid) and reduced range t_f - t_n (zero for rays
    without a bound).  Lengths are the FP32 differences, summed exactly in
    units of 2^-24 m (round half to even), so that any summation order gives
    the same integers.
    """
    depth = np.asarray(depth, np.float32)
    hit = np.isfinite(depth)
    st = b["status"]
    ok = (st == ST_HIT) | (st == ST_NO_FAR)
    t_n, t_f = np.float32(b["t_n"]), np.float32(b["t_f"])
    inside = ok & (t_n <= depth) & (depth <= t_f)
    orig = np.float32(t_out) - np.float32(t_in)
    red = np.where(ok, t_f - t_n, np.float32(0.0)).astype(np.float32)
    q = lambda x: int(np.rint(x[hit].astype(np.float64) * LEN_Q).astype(np.int64).sum())
    return dict(rays=int(hit.sum()), failed=int((hit & ~inside).sum()),
                original_q=q(orig), reduced_q=q(red))


# neighbour order of the frontier rays: -x, +x, -y, +y, -z, +z
_NB = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))


def frontier(grid, cnt, flag_vol):
    """Voxels no integration ray has updated (count 0) that border observed
    free space (a 6-neighbour with count > 0 and flag bit0 clear, i.e.
    V > D_s), in ascending linear order, each with a ray into it: from the
    centre of its first such neighbour (order -x, +x, -y, +y, -z, +z) along
    the axis towards it.  Centres are lo + (i + 1/2) h evaluated in FP32 as a
    product then a sum (two roundings).  Returns idx [n], o [n,3], v [n,3]."""
    nx, ny, nz = grid.n
    cnt = np.asarray(cnt).reshape(nz, ny, nx)
    fl = np.asarray(flag_vol).reshape(nz, ny, nx)
    free = (cnt > 0) & ((fl & 1) == 0)
    unseen = cnt == 0
    choice = np.full((nz, ny, nx), -1, np.int64)
    for k in range(5, -1, -1):                 # the first direction in order wins
        dx, dy, dz = _NB[k]
        nb = np.zeros_like(free)
        zs = slice(max(0, -dz), nz - max(0, dz))
        ys = slice(max(0, -dy), ny - max(0, dy))
        xs = slice(max(0, -dx), nx - max(0, dx))
        zs2 = slice(max(0, dz), nz + min(0, dz))
        ys2 = slice(max(0, dy), ny + min(0, dy))
        xs2 = slice(max(0, dx), nx + min(0, dx))
        nb[zs, ys, xs] = free[zs2, ys2, xs2]
        choice[unseen & nb] = k
    idx = np.flatnonzero(choice.ravel() >= 0)
    ks = choice.ravel()[idx]
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    d = np.array(_NB)[ks]                      # neighbour offset
    Y = np.stack([x, y, z], 1) + d
    h = np.float32(grid.h)
    lo = np.float32(grid.lo)
    o = (Y.astype(np.float32) + np.float32(0.5)) * h + lo
    v = (-d).astype(np.float32)
    return idx, o.astype(np.float32), v



def bricks(grid, state, B=8):
    """Two-level layout of an integration state (the multi-resolution
    direction of Sec. 5, limitations and future work): bricks of B^3 voxels,
    ceil(n/B) per axis, x fastest.  A band brick holds a seen voxel whose mean
    V is below D_T, i.e. one that received an update inside the truncation
    band (no update exceeds D_T).  Returns band [nbz, nby, nbx] (bool) and
    seen [N] (bool, count > 0)."""
    d_t = float(np.float32(grid.d_t))
    V = finalize(grid, state).ravel()
    seen = state.cnt > 0
    nx, ny, nz = grid.n
    nb = [(x + B - 1) // B for x in grid.n]
    i = np.flatnonzero(seen & (V < d_t))
    band = np.zeros((nb[2], nb[1], nb[0]), bool)
    band[(i // (nx * ny)) // B, ((i // nx) % ny) // B, (i % nx) // B] = True
    return band, seen


def bricks_expand(grid, state, band, B=8):
    """V of the two-level volume, [nz, ny, nx]: the voxel's own mean in a band
    brick; elsewhere D_T where seen and -D_T where unseen."""
    d_t = float(np.float32(grid.d_t))
    V = finalize(grid, state)
    nx, ny, nz = grid.n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    in_band = band[z // B, y // B, x // B]
    seen = (state.cnt > 0).reshape(nz, ny, nx)
    return np.where(in_band, V, np.where(seen, d_t, -d_t))
