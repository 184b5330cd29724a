"""Pin the integrated TSDF against the analytic scene (C1): the zero crossing
of the trilinearly interpolated volume along novel rays lies close to the
exact ray-sphere / ray-box hit, and the Alg. 1 bounds contain the training
depths (the counting of the paper's Table 1).

The projective distance v.(p* - c) averaged over views is not the Euclidean
SDF (it overestimates it for oblique views), so the crossing is not exact:
for |cos| >= 0.5 away from creases and box edges the median error is ~0.1 h,
90% are within h/2 and none exceeds 1.5 h.  A half-voxel offset of the voxel
centres, a flipped sign or a dropped depth term moves the median by h/2 or
more and fails this test."""
import numpy as np
import pytest

from synth.configs import get_config
from synth.scenes import surface_normal
from oracle import tsdf


@pytest.fixture(scope="module")
def c1_volume():
    cfg = get_config("c1")
    o, v, d = cfg.integration_rays()
    st = tsdf.integrate(cfg.grid, o, v, d)
    V = tsdf.finalize(cfg.grid, st)
    return cfg, V, tsdf.flags(cfg.grid, V), (o, v, d)


def trilinear(grid, V, p):
    """V at points p [N,3] from values at voxel centres (edge-clamped)."""
    nz, ny, nx = V.shape
    u = (p - np.asarray(grid.lo)) / grid.h - 0.5
    i0 = np.floor(u).astype(int)
    fr = u - i0
    out = np.zeros(p.shape[0])
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                ix = np.clip(i0[:, 0] + dx, 0, nx - 1)
                iy = np.clip(i0[:, 1] + dy, 0, ny - 1)
                iz = np.clip(i0[:, 2] + dz, 0, nz - 1)
                wgt = ((fr[:, 0] if dx else 1 - fr[:, 0]) * (fr[:, 1] if dy else 1 - fr[:, 1])
                       * (fr[:, 2] if dz else 1 - fr[:, 2]))
                out += wgt * V[iz, iy, ix]
    return out


def test_zero_crossing_within_half_voxel(c1_volume):
    cfg, V, _, _ = c1_volume
    g, sc = cfg.grid, cfg.scene()
    ro, rv = cfg.render_rays()
    idx, depth = sc.hit_prim(ro.astype(np.float64), rv.astype(np.float64))
    t_in, t_out = tsdf.ray_range(g, ro, rv)
    errs = []
    for r in np.flatnonzero(np.isfinite(depth)):
        prim = sc.prims[idx[r]]
        p_hit = ro[r] + depth[r] * rv[r]
        n = surface_normal(prim, p_hit)[0]
        if abs(n @ rv[r]) < 0.5:
            continue
        other = [q for q in sc.prims if q is not prim]
        if min(abs(q.sdf(p_hit[None])[0]) for q in other) < 2 * g.h:
            continue       # union crease: the along-ray TSDF mixes two surfaces
        if hasattr(prim, "lo"):   # keep away from box edges
            lo, hi = np.asarray(prim.lo), np.asarray(prim.hi)
            a = int(np.abs(n).argmax())
            rest = [b for b in range(3) if b != a]
            if min(min(p_hit[b] - lo[b], hi[b] - p_hit[b]) for b in rest) < 2 * g.h:
                continue
        ts = np.arange(t_in[r], t_out[r], g.h / 16)
        vals = trilinear(g, V, ro[r][None].astype(np.float64) + ts[:, None] * rv[r][None])
        k = np.flatnonzero((vals[:-1] > 0) & (vals[1:] <= 0))
        assert k.size > 0
        k = k[0]
        t0 = ts[k] + (ts[k + 1] - ts[k]) * vals[k] / (vals[k] - vals[k + 1])
        errs.append(t0 - depth[r])
    errs = np.abs(np.asarray(errs)) / g.h
    assert errs.size > 500
    assert np.median(errs) < 0.2 and np.percentile(errs, 90) < 0.5 and errs.max() < 1.5, \
        np.percentile(errs, [50, 90, 100])


def test_bounds_contain_training_depths(c1_volume):
    """Table 1's counting: training rays whose integration depth is not inside
    [t_n, t_f].  On this coarse 64^3 volume of a sphere 16 voxels in radius,
    a few percent of rays get t_n just past the surface: the voxel holding the
    surface point can average projective distances above D_s = 1h, so the
    surface group starts one voxel later.  Every failure is of that kind
    (within two voxels), and the far bound never ends before the surface."""
    cfg, V, fl, (o, v, d) = c1_volume
    h = cfg.grid.h
    b = tsdf.bounds(cfg.grid, fl, o, v)
    hit = np.isfinite(d)
    assert (b["status"][hit] != tsdf.ST_MISS).all()
    late = hit & (b["t_n"] > d)
    assert late.sum() / hit.sum() < 0.10
    assert ((b["t_n"] - d)[late] < 2 * h).all()
    assert (b["t_f"][hit] >= d[hit]).all()
