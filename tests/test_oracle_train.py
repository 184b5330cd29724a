"""Pin the training-step oracle: weight gradients vs central finite
differences on 32 seeded weights, in FP64, and the eikonal special case.

The loss is only piecewise smooth (ReLU units of the colour network and the
clamp cos = min(v . grad f, 0) of the NeuS opacity), so a step of 1e-4 can
straddle a kink for some weights, and softplus with beta = 100 makes the
third derivative large (the central-difference truncation error grows as
beta^2 h^2).  The pin uses h = 1e-6: truncation ~1e-7 relative, rounding
~eps64 L / h ~ 1e-11 absolute, both well inside the stated tolerance."""
import numpy as np
import pytest
import torch

from synth.configs import get_config
from oracle import tsdf, train as TR, field as F


def make_batch(cfg, n_rays, n_eik, seed=0, views=None):
    g = cfg.grid
    o, v, d = cfg.integration_rays(views=views)
    st = tsdf.integrate(g, o, v, d)
    fl = tsdf.flags(g, tsdf.finalize(g, st))
    ro, rv, target = cfg.training_batch(n_rays, seed)
    b = tsdf.bounds(g, fl, ro, rv)
    s = cfg.sampling
    p = tsdf.place(b["t_n"], b["t_f"], b["n_vox"], b["status"], s.rho_num, s.rho_den, s.n_min, s.n_max)
    return dict(o=ro, v=rv, offsets=p["offsets"], t=p["t"], dt=p["dt"], target=target,
                eik_x=cfg.eikonal_points(n_eik, seed), eik_lambda=0.1)


@pytest.mark.parametrize("name,n_rays", [("c1", 48), ("c2", 6)])
def test_weight_gradients_match_central_differences(name, n_rays):
    cfg = get_config(name)
    views = None if name == "c1" else [0, 1]
    batch = make_batch(cfg, n_rays, 16, views=views)
    assert batch["offsets"][-1] > 0
    ps, pc = cfg.sdf_params(), cfg.color_params()
    L, gs, gc = TR.loss_and_grads(cfg, ps, pc, batch)
    assert L == pytest.approx(TR.loss_value(cfg, ps.astype(np.float64), pc.astype(np.float64), batch),
                              rel=1e-14)
    rng = np.random.default_rng(5)
    # 32 seeded weights: 24 in the SDF network (incl. second-order paths), 8 in colour
    pick_s = rng.choice(np.flatnonzero(np.abs(gs) > 1e-8 * np.abs(gs).max()), 24, replace=False)
    pick_c = rng.choice(np.flatnonzero(np.abs(gc) > 1e-8 * np.abs(gc).max()), 8, replace=False)
    h = 1e-6
    base_s, base_c = ps.astype(np.float64), pc.astype(np.float64)
    for which, idxs, grad in (("s", pick_s, gs), ("c", pick_c, gc)):
        for i in idxs:
            a, b = base_s.copy(), base_c.copy()
            tgt = a if which == "s" else b
            tgt[i] += h
            lp = TR.loss_value(cfg, a, b, batch)
            tgt[i] -= 2 * h
            lm = TR.loss_value(cfg, a, b, batch)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grad[i]) <= 1e-4 * abs(grad[i]) + 1e-10 * max(1.0, abs(L)), \
                (which, i, fd, grad[i])


def test_eikonal_zero_for_exact_distance():
    """A one-layer 'network' f = scale * (w . x_hat + b) with |w| = 1 has
    |grad f| = 1 everywhere: the eikonal term and its gradient vanish."""
    from synth.weights import SdfNet
    net = SdfNet(width=1, n_hidden=0, pe_freqs=0, skip_at=-1, n_feat=0)
    w = np.array([0.6, 0.0, 0.8, -0.1], np.float32)   # W [1,3], b [1]
    layers = F.as_layers(w, [(3, 1)], requires_grad=True)
    x = torch.tensor(np.random.default_rng(0).uniform(-1, 1, (20, 3)), requires_grad=True)
    f, _, _ = F.sdf_forward(net, layers, x, (0.0, 0.0, 0.0), 1.0)
    (g,) = torch.autograd.grad(f.sum(), x, create_graph=True)
    eik = ((torch.linalg.norm(g, dim=-1) - 1) ** 2).mean()
    gw = torch.autograd.grad(eik, [layers[0][0], layers[0][1]], allow_unused=True)
    assert eik.item() < 1e-14
    assert all(t is None or t.abs().max().item() < 1e-7 for t in gw)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are g and g^2 at
    every step, so each step moves p by lr g / (|g| + eps)."""
    from oracle import train as OTR
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p = np.array([1.0, 1.0, 1.0, 1.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 1e-2, 1e-8
    for t in range(1, 6):
        p, m, v = OTR.adam(p, g, m, v, lr, 0.9, 0.999, eps, t)
    np.testing.assert_allclose(p, 1.0 - 5 * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-12)
