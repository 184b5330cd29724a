"""A render recorded as a HIP graph and replayed: every replay equals the
eager render of the rays the input tensors hold at that time, with eager
work and synchronisations between the replays (small scene, 64x64 view)."""
import numpy as np
import pytest
import torch

from synth.configs import get_config

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def test_graph_replays_equal_eager():
    from paper_2311_17878_amd import ops
    from paper_2311_17878_amd.pipeline import TsdfRenderer
    cfg = get_config("c1")
    g, s = cfg.grid, cfg.sampling
    grid = ops.make_grid(g.n, g.lo, g.h, g.d_t, g.d_s, g.nb_radius, g.m_consec)
    F = ops.Field(cfg.sdf.width, cfg.sdf.n_hidden, cfg.sdf.pe_freqs, cfg.sdf.skip_at,
                  cfg.sdf.n_feat, cfg.color.n_hidden, cfg.sdf.beta, cfg.in_center,
                  cfg.in_scale, cfg.sdf_params(), cfg.color_params())
    R = TsdfRenderer(grid, F, s.rho_num, s.rho_den, s.n_min, s.n_max, cfg.neus_s)
    o, v, d = cfg.integration_rays()
    R.integrate(dev(o), dev(v), dev(d))
    R.finalize()
    ro, rv = cfg.render_rays()
    # a second ray set of the same size: the view seen from the opposite side
    ro2, rv2 = -ro, -rv
    o_in, v_in = dev(ro), dev(rv)
    graph, out = R.capture(o_in, v_in)
    keys = ("rgb", "depth", "normal", "acc")
    for k, (a, b) in enumerate([(ro, rv), (ro2, rv2), (ro, rv), (ro2, rv2)]):
        ref = R.render(dev(a), dev(b))             # eager work between the replays
        torch.cuda.synchronize()
        o_in.copy_(dev(a))
        v_in.copy_(dev(b))
        graph.replay()
        torch.cuda.synchronize()
        for key in keys:
            assert torch.equal(out[key], ref[key]), (k, key)
        assert int(out["s_total"].item()) == int(ref["s_total"].item())
