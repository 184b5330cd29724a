"""Property tests of the oracle on random inputs drawn by hypothesis: the
voxel walk visits 6-connected voxels with contiguous, ordered crossing
parameters; integration does not depend on the order of the rays;
compositing weights are non-negative, sum to at most one and leave a
non-increasing transmittance; placement puts ascending samples inside the
bound whose sections tile it."""
import numpy as np
from hypothesis import given, settings, strategies as st, HealthCheck

from synth.configs import Grid, get_config
from oracle import tsdf, render

FAST = settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
G = Grid((8, 6, 5), (-1.0, -0.75, -0.5), 0.25, 0.75, 0.25)
unit = st.floats(-1.0, 1.0, allow_nan=False)


@FAST
@given(ox=st.floats(-2.0, 2.0), oy=st.floats(-2.0, 2.0), oz=st.floats(-2.0, 2.0),
       dx=unit, dy=unit, dz=unit)
def test_walk_is_a_connected_ordered_path(ox, oy, oz, dx, dy, dz):
    d = np.array([dx, dy, dz])
    if np.linalg.norm(d) < 1e-3:
        return
    v = (d / np.linalg.norm(d)).astype(np.float32)
    w = tsdf.walk(G, np.float32([ox, oy, oz]), v)
    if w is None or w[0].size == 0:
        return
    vox, te, tx = w
    nx, ny, nz = G.n
    xyz = np.stack([vox % nx, (vox // nx) % ny, vox // (nx * ny)], 1)
    assert (np.abs(np.diff(xyz, axis=0)).sum(1) == 1).all()        # one face per step
    assert te[0] >= 0 and (te <= tx).all()
    assert np.array_equal(tx[:-1], te[1:])                           # contiguous intervals
    assert len(set(vox.tolist())) == vox.size                         # no voxel twice


_C1 = None


def _c1():
    global _C1
    if _C1 is None:
        cfg = get_config("c1")
        _C1 = (cfg.grid,) + cfg.integration_rays()
    return _C1


@settings(max_examples=8, deadline=None)
@given(seed=st.integers(0, 2 ** 31 - 1))
def test_integration_ignores_ray_order(seed):
    g, o, v, d = _c1()
    rng = np.random.default_rng(seed)
    pick = rng.choice(o.shape[0], 400, replace=False)
    perm = rng.permutation(pick)
    a = tsdf.integrate(g, o[pick], v[pick], d[pick], tie_eps=1e-9)
    b = tsdf.integrate(g, o[perm], v[perm], d[perm], tie_eps=1e-9)
    assert np.array_equal(a.cnt, b.cnt) and a.updates == b.updates
    assert np.allclose(a.sum_s, b.sum_s, rtol=0, atol=1e-12)


@FAST
@given(n=st.integers(1, 40), s=st.floats(1.0, 200.0), seed=st.integers(0, 2 ** 31 - 1))
def test_compositing_weights(n, s, seed):
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0.1, 3.0, n))
    dt = np.full(n, 0.05)
    f = rng.uniform(-0.3, 0.3, n)
    grad = rng.normal(size=(n, 3))
    rgb = rng.uniform(size=(n, 3))
    v = np.float32([[0.0, 0.0, 1.0]])
    out = render.composite(np.array([0, n]), v, t, dt, f, grad, rgb, s)
    w = out["w"]
    assert (w >= 0).all() and w.sum() <= 1.0 + 1e-12
    assert abs(w.sum() - out["acc"][0]) <= 1e-12
    # transmittance before sample i: 1 - (weights of the samples before it)
    T = 1.0 - np.concatenate([[0.0], np.cumsum(w)[:-1]])
    assert (np.diff(T) <= 1e-12).all() and T.min() >= -1e-12


@FAST
@given(tn=st.floats(0.0, 5.0), length=st.floats(1e-3, 5.0), n_vox=st.integers(0, 300),
       status=st.sampled_from([tsdf.ST_HIT, tsdf.ST_NO_FAR, tsdf.ST_MISS, tsdf.ST_INVALID]))
def test_placement_inside_the_bound(tn, length, n_vox, status):
    tf = tn + length
    p = tsdf.place(np.array([tn]), np.array([tf]), np.array([n_vox]), np.array([status], np.uint8),
                   1, 2, 1, 64)
    c = int(p["counts"][0])
    if status in (tsdf.ST_HIT, tsdf.ST_NO_FAR):
        assert c == min(max(-(-n_vox // 2), 1), 64)
        t, dt = p["t"], p["dt"]
        assert (np.diff(t) > 0).all() and t[0] > tn and t[-1] < tf
        assert abs(dt.sum() - length) <= 1e-12 * max(1.0, tf)
        assert np.allclose(t - dt / 2, tn + np.arange(c) * dt[0], rtol=0, atol=1e-12)
    else:
        assert c == 0 and p["t"].size == 0
