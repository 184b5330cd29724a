"""GPU parity of the two-level volume (bricks of 8^3 voxels; per-voxel sums
and counts only in band bricks), through the C ABI: band bricks, their slots
and every seen bit exact against the oracle, pool counts equal to the
oracle's and pool sums and counts equal to the dense integration, finalized
flags bit-exact and V equal to the dense V (exactly D_T where the dense V is
D_T up to FP32 rounding), on the small scene (exact and NeRF-mode depths, and
a grid whose size is not a multiple of 8) and on the room volume."""
import os
from dataclasses import replace

import numpy as np
import pytest
import torch

from synth.configs import get_config
from oracle import tsdf as OT

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def voxel_maps(g):
    """Per voxel (linear order): brick index, voxel inside the brick, and the
    seen word / bit that hold it."""
    nx, ny, nz = g.n
    nb = [(x + 7) // 8 for x in g.n]
    i = np.arange(nx * ny * nz, dtype=np.int64)
    x, y, z = i % nx, (i // nx) % ny, i // (nx * ny)
    b = x // 8 + nb[0] * (y // 8 + nb[1] * (z // 8))
    local = (x & 7) + 8 * (y & 7) + 64 * (z & 7)
    return b, local, z & 7, (8 * (y & 7) + (x & 7)).astype(np.uint64)


def gpu_seen(views, g):
    b, _, word, bit = voxel_maps(g)
    w = host(views["seen"]).view(np.uint64)
    return ((w[b, word] >> bit) & np.uint64(1)).astype(bool)


def build(g, o, v, d):
    from paper_2311_17878_amd import ops
    grid = ops.make_grid(g.n, g.lo, g.h, g.d_t, g.d_s, g.nb_radius, g.m_consec)
    nup = torch.zeros(1, dtype=torch.int64, device="cuda")
    sp = ops.sparse_integrate(grid, [(dev(o), dev(v), dev(d))], nup)
    st = ops.new_state(grid)
    nup_d = torch.zeros(1, dtype=torch.int64, device="cuda")
    ops.integrate(grid, st, dev(o), dev(v), dev(d), nup_d)
    Vd, fld = ops.finalize(grid, st)
    V2, fl2 = ops.sparse_finalize(grid, sp)
    torch.cuda.synchronize()
    return dict(grid=grid, sp=sp, views=ops.sparse_views(grid, sp), st=st, nup=int(nup.item()),
                nup_d=int(nup_d.item()), Vd=host(Vd), fld=host(fld), V2=host(V2), fl2=host(fl2))


def check_against_dense(g, r):
    """Pool sums and counts equal the dense state's at every voxel of a band
    brick; V and flags of the two-level volume equal the dense ones."""
    from paper_2311_17878_amd import ops
    vw = r["views"]
    slot = host(vw["slot"])
    b, local, _, _ = voxel_maps(g)
    dsum, dcnt = (host(x) for x in ops.state_views(r["grid"], r["st"]))
    in_band = slot[b] >= 0
    psum, pcnt = host(vw["psum"]), host(vw["pcnt"])
    assert np.array_equal(psum[slot[b[in_band]], local[in_band]], dsum[in_band])
    assert np.array_equal(pcnt[slot[b[in_band]], local[in_band]], dcnt[in_band])
    assert int(pcnt.astype(np.int64).sum()) == int(dcnt[in_band].astype(np.int64).sum())
    assert r["nup"] == r["nup_d"]
    assert np.array_equal(r["fl2"], r["fld"])
    d_t = np.float32(g.d_t)
    same = r["V2"] == r["Vd"]
    # where they differ, the voxel lies outside the band bricks, is seen, holds
    # exactly D_T in the two-level volume and D_T within an FP32 rounding of
    # the sum in the dense one
    assert (~in_band[~same]).all() and (r["V2"][~same] == d_t).all()
    assert (np.abs(r["Vd"][~same] - d_t) <= 4 * np.spacing(d_t)).all()
    return in_band


@pytest.mark.parametrize("name", ["c1", "c1n", "ragged"])
def test_two_level_volume_matches_oracle(name):
    cfg = get_config("c1" if name == "ragged" else name)
    g = cfg.grid if name != "ragged" else replace(cfg.grid, n=(60, 52, 44))
    o, v, d = cfg.integration_rays()
    r = build(g, o, v, d)
    st = OT.integrate(g, o, v, d, tie_eps=1e-9)
    assert st.ties == 0
    band, seen = OT.bricks(g, st)
    vw = r["views"]
    assert vw["n_bricks"] == tuple((x + 7) // 8 for x in g.n)
    assert np.array_equal(host(vw["band"]).reshape(band.shape) != 0, band)
    assert r["sp"]["n_band"] == int(band.sum())
    slot = host(vw["slot"])
    exp_slot = np.full(band.size, -1, np.int64)
    exp_slot[band.ravel()] = np.arange(int(band.sum()))
    assert np.array_equal(slot, exp_slot)
    assert np.array_equal(gpu_seen(vw, g), seen)
    in_band = check_against_dense(g, r)
    b, local, _, _ = voxel_maps(g)
    pcnt = host(vw["pcnt"])
    assert np.array_equal(pcnt[slot[b[in_band]], local[in_band]].astype(np.int64), st.cnt[in_band])
    assert r["nup"] == st.updates
    assert np.array_equal(r["fl2"].reshape(g.n[2], g.n[1], g.n[0]),
                          OT.flags(g, OT.bricks_expand(g, st, band)))
    dense_bytes = 12 * g.n_vox
    two_level = r["sp"]["meta"].numel() + r["sp"]["pool"].numel()
    print("%s: %d of %d bricks in the band; two-level %d bytes, dense state %d bytes"
          % (name, r["sp"]["n_band"], band.size, two_level, dense_bytes))
    assert two_level < dense_bytes


def test_two_level_volume_room():
    """The 256^3 room: flags equal to the oracle's (stored fixture), and to
    the dense volume; sampled counts and V against the oracle; every brick
    holding a voxel whose integer sum is below count x D_T is a band brick."""
    cfg = get_config("c2")
    g = cfg.grid
    o, v, d = cfg.integration_rays(tile=8)   # by 8x8 pixel blocks; same volume
    r = build(g, o, v, d)
    gold = np.load(os.path.join(HERE, "golden", "c2_volume.npz"))
    N = int(gold["n_vox"])
    fl = (np.unpackbits(gold["flag0"])[:N] | (np.unpackbits(gold["flag1"])[:N] << 1)).astype(np.uint8)
    assert np.array_equal(r["fl2"], fl)
    assert r["nup"] == int(gold["updates"])
    in_band = check_against_dense(g, r)
    from paper_2311_17878_amd import ops
    dsum, dcnt = (host(x) for x in ops.state_views(r["grid"], r["st"]))
    dt32 = int(round(float(np.float32(g.d_t)) * 2.0 ** 32))
    below = (dcnt != 0) & (dsum < dcnt.astype(np.uint32).astype(np.int64) * dt32)
    assert in_band[below].all()
    idx = gold["sample_idx"]
    seen = gpu_seen(r["views"], g)
    assert np.array_equal(seen[idx], gold["sample_cnt"] > 0)
    assert np.abs(r["V2"][idx] - gold["sample_V"]).max() <= 1e-5 * float(np.float32(g.d_t))
    nb = r["sp"]["n_band"]
    nbr = int(np.prod(r["views"]["n_bricks"]))
    two_level = r["sp"]["meta"].numel() + r["sp"]["pool"].numel()
    print("room: %d of %d bricks in the band (%.1f%%); two-level %.1f MB, dense state %.1f MB"
          % (nb, nbr, 100.0 * nb / nbr, two_level / 1e6, 12 * g.n_vox / 1e6))
    assert two_level < 0.5 * 12 * g.n_vox


def test_two_level_edge_cases():
    from paper_2311_17878_amd import ops, _lib as L
    cfg = get_config("c1")
    g = cfg.grid
    grid = ops.make_grid(g.n, g.lo, g.h, g.d_t, g.d_s, g.nb_radius, g.m_consec)
    # no rays: nothing seen, no band brick, every voxel unseen
    e = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    sp = ops.sparse_integrate(grid, [(e, e, torch.empty(0, device="cuda"))])
    assert sp["n_band"] == 0
    V, fl = ops.sparse_finalize(grid, sp)
    assert (host(V) == -np.float32(g.d_t)).all() and (host(fl) == 3).all()
    # bad arguments are rejected on the host
    lib = L.load()
    import ctypes
    assert lib.tsdf_sparse_pool_bytes(-1, ctypes.byref(ctypes.c_size_t(0))) != 0
    assert lib.tsdf_sparse_alloc(ctypes.byref(grid), None, None, None, 0, None) != 0


def test_render_from_two_level_volume_equals_dense():
    """The renderer fed by the two-level volume renders the small scene's
    view exactly as from the dense volume (same flags, same kernels)."""
    from paper_2311_17878_amd import ops
    from paper_2311_17878_amd.pipeline import TsdfRenderer
    cfg = get_config("c1")
    g, s = cfg.grid, cfg.sampling
    grid = ops.make_grid(g.n, g.lo, g.h, g.d_t, g.d_s, g.nb_radius, g.m_consec)
    F = ops.Field(cfg.sdf.width, cfg.sdf.n_hidden, cfg.sdf.pe_freqs, cfg.sdf.skip_at,
                  cfg.sdf.n_feat, cfg.color.n_hidden, cfg.sdf.beta, cfg.in_center,
                  cfg.in_scale, cfg.sdf_params(), cfg.color_params())
    o, v, d = cfg.integration_rays()
    ro, rv = (dev(x) for x in cfg.render_rays())
    Rd = TsdfRenderer(grid, F, s.rho_num, s.rho_den, s.n_min, s.n_max, cfg.neus_s)
    Rd.integrate(dev(o), dev(v), dev(d))
    Rd.finalize()
    Rt = TsdfRenderer(grid, F, s.rho_num, s.rho_den, s.n_min, s.n_max, cfg.neus_s)
    half = o.shape[0] // 2           # two batches: every batch is marked before any is added
    Rt.fuse_two_level([(dev(o[:half]), dev(v[:half]), dev(d[:half])),
                       (dev(o[half:]), dev(v[half:]), dev(d[half:]))], want_v=True)
    assert Rt.state is None and Rt.two_level["n_band"] > 0
    assert torch.equal(Rt.flags, Rd.flags)
    a, b = Rd.render(ro, rv), Rt.render(ro, rv)
    for k in ("rgb", "depth", "normal", "acc"):
        assert torch.equal(a[k], b[k]), k
