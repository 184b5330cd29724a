"""GPU parity of the NeRF-mode bounds (D_T = 39h, D_s = 27h, 7^3
neighbourhood, M = 15) on the small scene fused from density-field-like
depths (seeded noise and floaters), and of Table 1's counting, through the
C ABI: integration counts and flags exact, bounds of the training and render
rays bit-exact, the counting (rays, failures, summed ranges) exact."""
import numpy as np
import pytest
import torch

from synth.configs import get_config
from oracle import tsdf as OT

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", params=["c1", "c1n"])
def vol(request):
    from paper_2311_17878_amd import ops
    cfg = get_config(request.param)
    g = cfg.grid
    o, v, d = cfg.integration_rays()
    st = OT.integrate(g, o, v, d, tie_eps=1e-9)
    V = OT.finalize(g, st)
    fl = OT.flags(g, V)
    grid = ops.make_grid(g.n, g.lo, g.h, g.d_t, g.d_s, g.nb_radius, g.m_consec)
    return dict(cfg=cfg, g=g, grid=grid, rays=(o, v, d), st=st, fl=fl)


def test_nerf_mode_flags_and_bounds(vol):
    from paper_2311_17878_amd import ops
    g, grid, (o, v, d) = vol["g"], vol["grid"], vol["rays"]
    st = ops.new_state(grid)
    nup = torch.zeros(1, dtype=torch.int64, device="cuda")
    ops.integrate(grid, st, dev(o), dev(v), dev(d), nup)
    torch.cuda.synchronize()
    assert vol["st"].ties == 0
    assert int(nup.item()) == vol["st"].updates
    _, flg = ops.finalize(grid, st)
    assert np.array_equal(host(flg).reshape(vol["fl"].shape), vol["fl"])
    ro, rv = vol["cfg"].render_rays()
    for oo, vv in ((o, v), (ro, rv)):
        ob = OT.bounds(g, vol["fl"], oo, vv)
        gb = ops.ray_bounds(grid, dev(vol["fl"].ravel()), dev(oo), dev(vv), steps=True)
        for k in ("t_n", "t_f", "first_hit", "n_vox", "status", "n_steps"):
            assert np.array_equal(host(gb[k]), ob[k]), k


def test_containment_counting(vol):
    """Table 1's counting of the training rays on the GPU equals the
    oracle's exactly; the failure rate and the range reduction are stated."""
    from paper_2311_17878_amd import ops
    g, grid, (o, v, d) = vol["g"], vol["grid"], vol["rays"]
    ob = OT.bounds(g, vol["fl"], o, v)
    t_in, t_out = OT.ray_range(g, o, v)
    ref = OT.containment(t_in, t_out, ob, d)
    gi, go = ops.ray_range(grid, dev(o), dev(v))
    gb = {k: dev(ob[k]) for k in ("t_n", "t_f", "status")}
    out = host(ops.bound_stats(gi, go, gb, dev(d)))
    assert out.tolist() == [ref["rays"], ref["failed"], ref["original_q"], ref["reduced_q"]]
    q = float(1 << 24)
    print("%s: %d rays with depth, %d failed (%.3f%%), original range %.3f m, reduced %.3f m"
          % (vol["cfg"].name, ref["rays"], ref["failed"], 100.0 * ref["failed"] / ref["rays"],
             ref["original_q"] / q / ref["rays"], ref["reduced_q"] / q / ref["rays"]))
    # the bound is a reduction of the range
    assert ref["reduced_q"] < ref["original_q"]
    # empty input
    e = torch.empty(0, device="cuda")
    eb = {"t_n": e, "t_f": e, "status": torch.empty(0, dtype=torch.uint8, device="cuda")}
    assert host(ops.bound_stats(e, e, eb, e)).tolist() == [0, 0, 0, 0]
