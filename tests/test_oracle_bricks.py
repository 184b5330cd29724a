"""Oracle pins of the two-level volume (bricks of 8^3 voxels; per-voxel sums
only where the truncation band reaches): hand-derived band bricks of single
axis-aligned rays (also on a grid whose size is not a multiple of 8), and on
the small scene the invariants that make the two-level volume equal to the
dense one."""
import numpy as np

from synth.configs import Grid, get_config
from oracle import tsdf


def _row_ray(x0, y, z, depth):
    o = np.array([[x0, y, z]], np.float32)
    v = np.array([[1.0, 0.0, 0.0]], np.float32)
    return o, v, np.array([depth], np.float32)


def test_single_ray_band_bricks_by_hand():
    # h = 1/16, D_T = 3h; the ray runs along x through the centres of row
    # (y, z) = (3, 4) from x = -h/4, so voxel i has t = (i + 3/4) h and
    # s = d - t.  With d = 12 h: s_i = (11.25 - i) h; updated while s > -3h
    # (i <= 14), inside the band where s < 3h (i >= 9).
    h = 1.0 / 16
    g = Grid((16, 8, 8), (0.0, 0.0, 0.0), h, 3 * h, h)
    st = tsdf.integrate(g, *_row_ray(-h / 4, 3.5 * h, 4.5 * h, 12 * h))
    band, seen = tsdf.bricks(g, st)
    assert band.shape == (1, 1, 2)
    assert band.tolist() == [[[False, True]]]       # voxels 0..7 only clamped, 9..14 in band
    row = 16 * (3 + 8 * 4)
    assert np.flatnonzero(seen).tolist() == list(range(row, row + 15))
    V2 = tsdf.bricks_expand(g, st, band)
    V = tsdf.finalize(g, st)
    assert np.array_equal(V2, V)                    # brick 0's seen voxels hold exactly D_T
    assert (V[4, 3, :8] == np.float32(3 * h)).all()


def test_ragged_grid_band_brick_by_hand():
    # 12 voxels along x: the second brick column holds voxels 8..11 only.
    # d = 11 h: s_i = (10.25 - i) h, band for i >= 8.
    h = 1.0 / 16
    g = Grid((12, 8, 8), (0.0, 0.0, 0.0), h, 3 * h, h)
    st = tsdf.integrate(g, *_row_ray(-h / 4, 3.5 * h, 4.5 * h, 11 * h))
    band, seen = tsdf.bricks(g, st)
    assert band.tolist() == [[[False, True]]]
    assert int(seen.sum()) == 12
    # a depth nearer the start puts the band in the first brick as well
    st2 = tsdf.integrate(g, *_row_ray(-h / 4, 3.5 * h, 4.5 * h, 7 * h))
    band2, _ = tsdf.bricks(g, st2)
    assert band2.tolist() == [[[True, True]]]       # s_i = (6.25 - i) h: band for 4 <= i <= 9


def test_two_level_volume_equals_dense_small_scene():
    cfg = get_config("c1")
    g = cfg.grid
    o, v, d = cfg.integration_rays()
    st = tsdf.integrate(g, o, v, d, tie_eps=1e-9)
    V = tsdf.finalize(g, st)
    band, seen = tsdf.bricks(g, st)
    nx, ny, nz = g.n
    d_t = float(np.float32(g.d_t))
    # outside the band bricks every seen voxel holds exactly D_T
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    in_band = band[z // 8, y // 8, x // 8]
    s3 = seen.reshape(nz, ny, nx)
    assert (V[~in_band & s3] == d_t).all()
    # every band brick holds a voxel below D_T
    below = s3 & (V < d_t)
    for bz, by, bx in zip(*np.nonzero(band)):
        assert below[8 * bz: 8 * bz + 8, 8 * by: 8 * by + 8, 8 * bx: 8 * bx + 8].any()
    V2 = tsdf.bricks_expand(g, st, band)
    assert np.array_equal(V2, V)
    assert np.array_equal(tsdf.flags(g, V2), tsdf.flags(g, V))
    # the band bricks are a minority: the pool is far smaller than a dense state
    assert 0 < band.sum() < 0.5 * band.size
