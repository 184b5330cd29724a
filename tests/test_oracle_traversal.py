"""Pins for the oracle's voxel traversal, integration, flags and bounds.

Each test checks the oracle against something other than itself: exact
rational brute force, closed forms, library routines, hand-derived cases in
the spirit of Fig. 2(b), or the literal incremental update of the
supplementary integration algorithm.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest
from scipy import ndimage

from synth.configs import Grid, get_config
from oracle import tsdf

Q = 2 ** 20


def snapped(o, v):
    o = np.asarray(o, np.float32)
    v = np.asarray(v, np.float32)
    O = [int(np.rint(np.float64(x) * Q)) for x in o]
    V = [int(np.rint(np.float64(x) * Q)) for x in v]
    return O, V


def brute_force_walk(grid, o, v):
    """Voxels whose slab interval has positive length after max(0, entry),
    ordered by entry parameter; exact rationals on the snapped ray."""
    O, V = snapped(o, v)
    LO = [int(round(x * Q)) for x in grid.lo]
    H = int(round(grid.h * Q))
    nx, ny, nz = grid.n

    def axis_interval(a, i):
        b0 = LO[a] + i * H
        b1 = b0 + H
        if V[a] == 0:
            return (Fr(-10 ** 30), Fr(10 ** 30)) if b0 <= O[a] < b1 else None
        t0 = Fr(b0 - O[a], V[a])
        t1 = Fr(b1 - O[a], V[a])
        return (min(t0, t1), max(t0, t1))

    res = []
    for z in range(nz):
        iz = axis_interval(2, z)
        if iz is None:
            continue
        for y in range(ny):
            iy = axis_interval(1, y)
            if iy is None:
                continue
            for x in range(nx):
                ix = axis_interval(0, x)
                if ix is None:
                    continue
                t_in = max(ix[0], iy[0], iz[0], Fr(0))
                t_out = min(ix[1], iy[1], iz[1])
                if t_out > t_in:
                    res.append((t_in, t_out, x + nx * (y + ny * z)))
    res.sort()
    return res


def f32(q):
    return np.float32(float(q))


@pytest.mark.parametrize("seed", range(12))
def test_walk_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    grid = Grid((8, 8, 8), (-0.5, -0.5, -0.5), 1.0 / 8, 3.0 / 8, 1.0 / 8)
    if seed % 3 == 0:   # camera inside the grid
        o = rng.uniform(-0.45, 0.45, 3)
    else:               # camera outside, aimed at the grid
        o = rng.normal(size=3)
        o = 1.5 * o / np.linalg.norm(o)
    target = rng.uniform(-0.4, 0.4, 3)
    v = target - o
    v /= np.linalg.norm(v)
    o, v = o.astype(np.float32), v.astype(np.float32)
    got = tsdf.walk(grid, o, v)
    exp = brute_force_walk(grid, o, v)
    assert got is not None
    vox, te, tx = got
    assert list(vox) == [e[2] for e in exp]
    assert np.array_equal(te, np.array([f32(e[0]) for e in exp], np.float32))
    assert np.array_equal(tx, np.array([f32(e[1]) for e in exp], np.float32))
    # 6-connected walk: one more voxel than the index distance travelled
    i0 = np.unravel_index(vox[0], (8, 8, 8))
    i1 = np.unravel_index(vox[-1], (8, 8, 8))
    assert len(vox) == 1 + sum(abs(int(a) - int(b)) for a, b in zip(i0, i1))


def test_walk_axis_aligned_by_hand():
    grid = Grid((4, 4, 4), (0.0, 0.0, 0.0), 0.25, 0.75, 0.25)
    o = np.array([-1.0, 0.375, 0.625], np.float32)
    v = np.array([1.0, 0.0, 0.0], np.float32)
    vox, te, tx = tsdf.walk(grid, o, v)
    # y index 1, z index 2: voxels x = 0..3 at linear 0+4*(1+4*2)=36..39
    assert list(vox) == [36, 37, 38, 39]
    assert list(te) == [1.0, 1.25, 1.5, 1.75]
    assert list(tx) == [1.25, 1.5, 1.75, 2.0]
    # moving the other way from inside the grid, starting exactly on a face
    o = np.array([0.5, 0.375, 0.625], np.float32)
    v = np.array([-1.0, 0.0, 0.0], np.float32)
    vox, te, tx = tsdf.walk(grid, o, v)
    assert list(vox) == [37, 36] and list(te) == [0.0, 0.25] and list(tx) == [0.25, 0.5]


def test_walk_misses_and_invalid():
    grid = Grid((4, 4, 4), (0.0, 0.0, 0.0), 0.25, 0.75, 0.25)
    assert len(tsdf.walk(grid, np.float32([2, 2, 2]), np.float32([1, 0, 0]))[0]) == 0
    # grid behind the camera
    assert len(tsdf.walk(grid, np.float32([2, 0.5, 0.5]), np.float32([1, 0, 0]))[0]) == 0
    # not a unit direction
    assert tsdf.walk(grid, np.float32([-1, 0.5, 0.5]), np.float32([2, 0, 0])) is None
    assert tsdf.walk(grid, np.float32([-1, 0.5, 0.5]), np.float32([np.nan, 0, 0])) is None


def test_integration_parallel_rays_closed_form():
    """Rays along +z onto the plane z = z0: V(c) = clamp(z0 - c_z, -D_T, D_T)."""
    h = 1.0 / 16
    grid = Grid((8, 8, 16), (0.0, 0.0, 0.0), h, 3 * h, h)
    z0 = 0.53                                    # between voxel centres
    xs = (np.arange(8) + 0.5) * h
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    reps = 3
    o = np.stack([np.tile(X.ravel(), reps), np.tile(Y.ravel(), reps),
                  np.full(64 * reps, -0.25)], 1).astype(np.float32)
    v = np.tile(np.float32([0, 0, 1]), (o.shape[0], 1))
    depth = (z0 - o[:, 2]).astype(np.float32)
    st = tsdf.integrate(grid, o, v, depth)
    V = tsdf.finalize(grid, st)
    cz = (np.arange(16) + 0.5) * h
    s_exact = np.clip(float(np.float32(z0) - np.float32(-0.25)) - 0.25 - cz, -3 * h, 3 * h)
    updated = s_exact > -3 * h
    for z in range(16):
        col = V[z]
        if updated[z]:
            np.testing.assert_allclose(col, s_exact[z], rtol=0, atol=1e-12)
            assert (st.cnt.reshape(16, 8, 8)[z] == reps).all()
        else:
            assert (col == -np.float32(3 * h)).all()
            assert (st.cnt.reshape(16, 8, 8)[z] == 0).all()


def test_integration_literal_running_average_and_order_invariance():
    """The supplementary algorithm's incremental update V <- (W V + w s)/(W + w),
    W <- W + w with w = 1, driven by an exact rational traversal, equals the
    oracle's mean; shuffling the rays changes nothing."""
    grid = Grid((8, 8, 8), (-0.5, -0.5, -0.5), 1.0 / 8, 2.0 / 8, 1.0 / 8)
    rng = np.random.default_rng(7)
    R = 40
    o = rng.normal(size=(R, 3))
    o = (1.5 * o / np.linalg.norm(o, axis=1, keepdims=True)).astype(np.float32)
    tgt = rng.uniform(-0.3, 0.3, (R, 3))
    v = tgt - o
    v = (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
    depth = np.float32(np.linalg.norm(tgt - o, axis=1) + rng.uniform(-0.1, 0.1, R))
    d_t = float(np.float32(grid.d_t))
    Vlit = np.full(512, -1.0)   # "unseen"
    Wlit = np.zeros(512)
    for r in range(R):
        O, Vd = snapped(o[r], v[r])
        vq = np.array(Vd, np.float64) / Q
        oq = np.array(O, np.float64) / Q
        p_star = oq + float(depth[r]) * vq
        for _, _, X in brute_force_walk(grid, o[r], v[r]):
            x, y, z = X % 8, (X // 8) % 8, X // 64
            c = np.array(grid.lo) + (np.array([x, y, z]) + 0.5) * grid.h
            s = float(np.clip(vq @ (p_star - c), -d_t, d_t))
            if s > -d_t:
                w = 1.0
                Vlit[X] = (Wlit[X] * Vlit[X] + w * s) / (Wlit[X] + w)
                Wlit[X] += w
            else:
                break
    st = tsdf.integrate(grid, o, v, depth)
    V = tsdf.finalize(grid, st).ravel()
    seen = Wlit > 0
    assert np.array_equal(seen, st.cnt > 0)
    assert np.array_equal(Wlit[seen], st.cnt[seen])
    np.testing.assert_allclose(V[seen], Vlit[seen], rtol=0, atol=1e-12)
    assert (V[~seen] == -np.float32(d_t)).all()
    perm = rng.permutation(R)
    st2 = tsdf.integrate(grid, o[perm], v[perm], depth[perm])
    assert np.array_equal(st2.cnt, st.cnt)
    np.testing.assert_allclose(st2.sum_s, st.sum_s, rtol=0, atol=1e-12)
    assert (np.abs(V) <= d_t + 1e-15).all()


def test_flags_match_library_erosion():
    rng = np.random.default_rng(3)
    grid = Grid((12, 10, 9), (0.0, 0.0, 0.0), 1 / 16, 3 / 16, 1 / 16)
    V = rng.uniform(-0.2, 0.2, (9, 10, 12))
    V[rng.uniform(size=V.shape) < 0.3] = -0.3
    fl = tsdf.flags(grid, V)
    assert np.array_equal(fl & 1, (V <= np.float32(1 / 16)).astype(np.uint8))
    ero = ndimage.binary_erosion(V < 0, structure=np.ones((5, 5, 5), bool), border_value=1)
    assert np.array_equal((fl >> 1) & 1, ero.astype(np.uint8))


def _strip(pattern, t_far=np.inf):
    """A 32x1x1 strip with flags from `pattern` (string per voxel: '.', 's'
    surface-only, 'i' surface+inside), ray along +x from x = -1."""
    h = 1.0 / 8
    grid = Grid((32, 1, 1), (0.0, 0.0, 0.0), h, 5 * h, h, 2, 15)
    fl = np.zeros((1, 1, 32), np.uint8)
    for k, ch in enumerate(pattern.ljust(32, ".")):
        fl[0, 0, k] = {".": 0, "s": 1, "i": 3, "n": 2}[ch]
    o = np.float32([[-1.0, h / 2, h / 2]])
    v = np.float32([[1.0, 0.0, 0.0]])
    return tsdf.bounds(grid, fl, o, v, t_far)


def test_bounds_fig2_cases_by_hand():
    # narrow bound: surface at voxel 10, 15 inside voxels from 11
    b = _strip("." * 10 + "s" + "i" * 15)
    assert b["status"][0] == tsdf.ST_HIT and b["first_hit"][0] == 10
    assert b["t_n"][0] == 1 + 10 / 8 and b["t_f"][0] == 1 + 26 / 8 and b["n_vox"][0] == 16
    # grazing ray: a surface voxel at an object's periphery must not end the bound
    b = _strip("....." + "s" + "...." + "s" + "i" * 20)
    assert b["first_hit"][0] == 5 and b["t_n"][0] == 1 + 5 / 8
    assert b["t_f"][0] == 1 + 26 / 8 and b["n_vox"][0] == 21
    # a thin object (never "inside") before the true surface, as in the middle ray
    b = _strip("...." + "s" + "." * 7 + "i" * 16)
    assert b["first_hit"][0] == 4 and b["t_f"][0] == 1 + 27 / 8 and b["n_vox"][0] == 23
    # interrupted run: m restarts, only the second run of 15 counts
    b = _strip("s" + "i" * 14 + "s" + "i" * 15)
    assert b["t_f"][0] == 1 + 31 / 8 and b["status"][0] == tsdf.ST_HIT
    # the first-hit voxel itself counts for the run (phase 2 starts there)
    b = _strip("." * 3 + "i" * 15)
    assert b["t_n"][0] == 1 + 3 / 8 and b["t_f"][0] == 1 + 18 / 8 and b["n_vox"][0] == 15


def test_bounds_no_far_miss_and_t_far():
    b = _strip("." * 10 + "i" * 11 + "." * 11)
    assert b["status"][0] == tsdf.ST_NO_FAR and b["t_f"][0] == 1 + 32 / 8 and b["n_vox"][0] == 22
    b = _strip("." * 32)
    assert b["status"][0] == tsdf.ST_MISS and b["first_hit"][0] == -1 and b["n_vox"][0] == 0
    b = _strip("." * 10 + "i" * 20, t_far=np.float32(2.6))
    # voxels entered at t < 2.6 are visited: 10 (2.25), 11 (2.375), 12 (2.5)
    assert b["status"][0] == tsdf.ST_NO_FAR and b["t_f"][0] == np.float32(2.6) and b["n_vox"][0] == 3
    b = _strip("." * 10 + "i" * 20, t_far=np.float32(2.25))
    assert b["status"][0] == tsdf.ST_MISS


def test_bounds_equal_direct_neighbourhood_reads():
    """Alg. 1 with the neighbourhood test read inline (125 voxels per step)
    gives the same bounds as the precomputed flag volume."""
    cfg = get_config("c1")
    g = cfg.grid
    o, v, d = cfg.integration_rays(views=[0, 1, 2, 3])
    st = tsdf.integrate(g, o, v, d)
    V = tsdf.finalize(g, st)
    fl = tsdf.flags(g, V)
    ro, rv = cfg.render_rays()
    idx = np.random.default_rng(0).choice(ro.shape[0], 64, replace=False)
    b = tsdf.bounds(g, fl, ro[idx], rv[idx])
    d_s = float(np.float32(g.d_s))
    nx, ny, nz = g.n
    Vp = np.pad(V, 2, constant_values=-1.0)
    for j, r in enumerate(idx):
        vox, te, tx = tsdf.walk(g, ro[r], rv[r])
        zyx = [(X // (nx * ny), (X // nx) % ny, X % nx) for X in vox]
        k0 = next((k for k, (z, y, x) in enumerate(zyx) if V[z, y, x] <= d_s), None)
        if k0 is None:
            assert b["status"][j] == tsdf.ST_MISS
            continue
        assert b["first_hit"][j] == vox[k0] and b["t_n"][j] == te[k0]
        m = 0
        t_f = None
        for k in range(k0, len(vox)):
            z, y, x = zyx[k]
            m = m + 1 if (Vp[z:z + 5, y:y + 5, x:x + 5] < 0).all() else 0
            if m == g.m_consec:
                t_f, n = tx[k], k - k0 + 1
                break
        if t_f is None:
            assert b["status"][j] == tsdf.ST_NO_FAR and b["t_f"][j] == tx[-1]
            assert b["n_vox"][j] == len(vox) - k0
        else:
            assert b["status"][j] == tsdf.ST_HIT and b["t_f"][j] == t_f and b["n_vox"][j] == n


def test_placement_invariants():
    rng = np.random.default_rng(1)
    R = 500
    t_n = rng.uniform(0, 3, R).astype(np.float32)
    t_f = (t_n + rng.uniform(0, 2, R)).astype(np.float32)
    n_vox = rng.integers(1, 80, R)
    status = rng.integers(0, 4, R).astype(np.uint8)
    p = tsdf.place(t_n, t_f, n_vox, status, 2, 3, 2, 40)
    c = p["counts"]
    assert p["offsets"][-1] == c.sum()
    ok = status <= 1
    assert (c[~ok] == 0).all()
    assert (c[ok] == np.clip(np.ceil(n_vox[ok] * 2 / 3 - 1e-9), 2, 40)).all()
    for r in np.flatnonzero(ok)[:50]:
        s, e = p["offsets"][r], p["offsets"][r + 1]
        t = p["t"][s:e]
        assert (np.diff(t) > 0).all() or t_f[r] == t_n[r]
        assert t[0] >= t_n[r] and t[-1] <= t_f[r]
        np.testing.assert_allclose(p["dt"][s:e].sum(), float(t_f[r]) - float(t_n[r]), atol=1e-12)
    # naive variant: a fixed count per ray
    q = tsdf.place(t_n, t_f, n_vox, status, 1, 1, 6, 6)
    assert (q["counts"][ok] == 6).all()


def test_containment_counting_by_hand():
    """Table 1's counting on hand-made rays: statuses, a depth on each bound
    (inside), just past them (failures), rays without depth ignored, lengths
    summed in 2^-24 m units."""
    st = np.array([0, 1, 0, 0, 2, 3, 0], np.uint8)
    b = dict(status=st, t_n=np.float32([1, 1, 1, 1, 0, 0, 2]), t_f=np.float32([2, 5, 2, 2, 0, 0, 3]))
    depth = np.float32([1.0, 5.0, np.nextafter(np.float32(2), np.float32(3)), 1.5, 1.0, 1.0, np.inf])
    t_in = np.float32([0.5] * 7)
    t_out = np.float32([4.5] * 7)
    c = tsdf.containment(t_in, t_out, b, depth)
    assert c["rays"] == 6 and c["failed"] == 3          # the 2.0000002, MISS and INVALID rays
    assert c["original_q"] == 6 * 4 * (1 << 24)
    assert c["reduced_q"] == (1 + 4 + 1 + 1) * (1 << 24)


def test_frontier_by_hand():
    """A 4x3x2 grid: one free voxel, one surface voxel, the rest unseen.  The
    frontier is the unseen 6-neighbours of the free voxel only, each with a
    ray from the free voxel's centre along the axis towards it."""
    from synth.configs import Grid
    g = Grid((4, 3, 2), (-1.0, 0.5, 0.0), 0.25, 0.75, 0.25)
    cnt = np.zeros((2, 3, 4), np.int64)
    fl = np.ones((2, 3, 4), np.uint8)          # unseen voxels read V = -D_T <= D_s
    cnt[0, 1, 1] = 3
    fl[0, 1, 1] = 0                            # free (V > D_s)
    cnt[0, 1, 2] = 2                           # seen surface voxel: not free, not unseen
    idx, o, v = tsdf.frontier(g, cnt.ravel(), fl.ravel())
    lin = lambda x, y, z: x + 4 * (y + 3 * z)
    assert idx.tolist() == sorted([lin(0, 1, 0), lin(1, 0, 0), lin(1, 2, 0), lin(1, 1, 1)])
    c = np.float32([-1.0 + 1.5 * 0.25, 0.5 + 1.5 * 0.25, 0.5 * 0.25])   # centre of (1, 1, 0)
    assert (o == c).all()
    d = {lin(0, 1, 0): (-1, 0, 0), lin(1, 0, 0): (0, -1, 0), lin(1, 2, 0): (0, 1, 0), lin(1, 1, 1): (0, 0, 1)}
    for i, vv in zip(idx, v):
        assert tuple(vv) == d[i]


def test_frontier_fill_covers_free_space_small_scene():
    """Filling the small scene's unseen voxels (Sec. 4.3) from the oracle's
    frontier, with depths read by a sensor at each ray's origin: the rounds
    end with an empty frontier, every voxel whose centre is in free space
    has been updated, and no updated voxel lies deeper inside an object than
    the truncation D_T plus a voxel diagonal (integration stops at s <= -D_T)."""
    from synth.scenes import sensor_depth
    cfg = get_config("c1")
    g, sc = cfg.grid, cfg.scene()
    o, v, d = cfg.integration_rays()
    st = tsdf.integrate(g, o, v, d, tie_eps=1e-9)
    nx, ny, nz = g.n
    i = np.arange(g.n_vox)
    c = np.stack([i % nx, (i // nx) % ny, i // (nx * ny)], 1) * g.h + np.array(g.lo) + 0.5 * g.h
    cl = sc.clearance(c)
    assert ((st.cnt == 0) & (cl > g.h)).any()      # the views leave free space unseen
    sizes = []
    for _ in range(4):
        fl = tsdf.flags(g, tsdf.finalize(g, st))
        idx, fo, fv = tsdf.frontier(g, st.cnt, fl)
        sizes.append(idx.size)
        if idx.size == 0:
            break
        st.add(fo, fv, sensor_depth(sc, fo, fv), 1e-9)
    assert sizes[0] > 0 and sizes[-1] == 0
    seen = st.cnt > 0
    assert not (~seen & (cl > 0)).any()
    assert not (seen & (cl < -(g.d_t + np.sqrt(3.0) * g.h))).any()
    assert (~seen & (cl < -(g.d_t + np.sqrt(3.0) * g.h))).sum() > 1000   # interiors stay unseen


def slab_range(grid, o, v):
    """[t_in, t_out] of the snapped ray inside the grid box by the slab test
    on exact rationals, t_in clipped at 0; None when the interval is empty."""
    O, V = snapped(o, v)
    LO = [int(round(x * Q)) for x in grid.lo]
    H = int(round(grid.h * Q))
    t0, t1 = Fr(0), None
    for a in range(3):
        b0, b1 = LO[a], LO[a] + grid.n[a] * H
        if V[a] == 0:
            if not b0 <= O[a] < b1:
                return None
            continue
        lo_t, hi_t = sorted((Fr(b0 - O[a], V[a]), Fr(b1 - O[a], V[a])))
        t0 = max(t0, lo_t)
        t1 = hi_t if t1 is None else min(t1, hi_t)
    return (t0, t1) if t1 is not None and t1 > t0 else None


@pytest.mark.parametrize("seed", range(6))
def test_ray_range_is_the_slab_interval(seed):
    """The oracle's grid range equals the exact slab interval of the snapped
    ray rounded once to FP32 (0, 0 when the ray misses the box)."""
    rng = np.random.default_rng(100 + seed)
    grid = Grid((8, 6, 5), (-0.5, -0.375, -0.25), 1.0 / 8, 3.0 / 8, 1.0 / 8)
    R = 64
    o = rng.normal(size=(R, 3)) * (0.3 if seed % 2 else 1.5)
    v = rng.normal(size=(R, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    o, v = o.astype(np.float32), v.astype(np.float32)
    t_in, t_out = tsdf.ray_range(grid, o, v)
    hits = 0
    for r in range(R):
        e = slab_range(grid, o[r], v[r])
        if e is None:
            assert t_in[r] == 0 and t_out[r] == 0
        else:
            hits += 1
            assert t_in[r] == f32(e[0]) and t_out[r] == f32(e[1])
    assert hits > 0


def test_ray_range_by_hand():
    grid = Grid((4, 4, 4), (0.0, 0.0, 0.0), 0.25, 0.75, 0.25)
    o = np.array([[-1.0, 0.375, 0.625],    # from outside along +x: [1, 2]
                  [0.5, 0.5, 0.5],          # from inside along +z: [0, 0.5]
                  [2.0, 2.0, 2.0],          # misses
                  [2.0, 0.5, 0.5],          # box behind the camera
                  [-1.0, -1.0, 0.5]],       # diagonal in the xy plane: [sqrt2, 2 sqrt2]
                 np.float32)
    s = np.float32(np.sqrt(0.5))
    v = np.array([[1, 0, 0], [0, 0, 1], [1, 0, 0], [1, 0, 0], [s, s, 0]], np.float32)
    t_in, t_out = tsdf.ray_range(grid, o, v)
    assert list(t_in[:4]) == [1.0, 0.0, 0.0, 0.0] and list(t_out[:4]) == [2.0, 0.5, 0.0, 0.0]
    # the snapped diagonal direction is rne(2^20 sqrt(1/2)) per axis
    Vq = np.rint(np.float64(s) * Q)
    assert t_in[4] == np.float32(Q / Vq) and t_out[4] == np.float32(2 * Q / Vq)
