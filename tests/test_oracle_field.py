"""Pins for the oracle's network, gradient, compositing and HS baseline."""
import math

import numpy as np
import pytest
import torch

from synth.configs import get_config
from synth.weights import SdfNet, ColorNet, sdf_params
from oracle import field as F
from oracle import render as Rn


def test_softplus_textbook_values():
    beta = 100.0
    z = torch.tensor([0.0, 0.5, -0.5, 1e-3, -30.0], dtype=torch.float64)
    sp = F.softplus_beta(z, beta)
    assert sp[0].item() == pytest.approx(math.log(2.0) / beta, abs=1e-18)
    assert sp[1].item() == pytest.approx(0.5 + math.exp(-50) / beta, rel=1e-15)
    assert sp[2].item() == pytest.approx(math.exp(-50) / beta, rel=1e-12)
    assert sp[3].item() == pytest.approx(math.log(1 + math.exp(0.1)) / beta, rel=1e-14)
    assert sp[4].item() == 0.0 or sp[4].item() < 1e-300


def test_one_hidden_unit_closed_form_and_gradient():
    """y0 = softplus_beta(x_hat_0) for a 1-unit network, f = scale * y0:
    f(center) = scale ln2/beta and df/dx = sigmoid(beta x_hat_0) = 1/2 there."""
    net = SdfNet(width=1, n_hidden=1, pe_freqs=0, skip_at=-1, n_feat=0, beta=100.0)
    params = np.array([1.0, 0.0, 0.0, 0.0, 1.0, 0.0], np.float32)  # W0=[1,0,0], b0, W1=[1], b1
    layers = F.as_layers(params, net.layer_dims())
    scale = 2.0
    p = torch.tensor([[0.0, 0.3, -0.2], [1.0, 0.0, 0.0]], dtype=torch.float64, requires_grad=True)
    f, feat, _ = F.sdf_forward(net, layers, p, (0.0, 0.0, 0.0), scale)
    (g,) = torch.autograd.grad(f.sum(), p)
    assert f[0].item() == pytest.approx(scale * math.log(2) / 100, rel=1e-15)
    assert g[0, 0].item() == pytest.approx(0.5, rel=1e-15)
    assert g[0, 1].item() == 0.0 and g[0, 2].item() == 0.0
    assert f[1].item() == pytest.approx(scale * (0.5 + math.log1p(math.exp(-50)) / 100), rel=1e-15)
    assert g[1, 0].item() == pytest.approx(1 / (1 + math.exp(-50)), rel=1e-15)


def test_encoding_values():
    x = torch.tensor([[math.pi / 2, 0.0, math.pi]], dtype=torch.float64)
    g = F.encode(x, 2)
    assert g.shape == (1, 15)
    exp = [math.pi / 2, 0, math.pi, 1, 0, 0, 0, 1, -1, 0, 0, 0, -1, 1, 1]
    np.testing.assert_allclose(g[0].numpy(), exp, atol=1e-15)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_gradient_matches_finite_differences(name):
    cfg = get_config(name)
    layers = F.as_layers(cfg.sdf_params(), cfg.sdf.layer_dims())
    rng = np.random.default_rng(0)
    c = np.asarray(cfg.in_center)
    p = torch.tensor(c + cfg.in_scale * rng.uniform(-0.8, 0.8, (16, 3)), dtype=torch.float64,
                     requires_grad=True)
    f, _, _ = F.sdf_forward(cfg.sdf, layers, p, cfg.in_center, cfg.in_scale)
    (g,) = torch.autograd.grad(f.sum(), p)
    eps = 1e-6 * cfg.in_scale
    with torch.no_grad():
        for a in range(3):
            d = torch.zeros(3, dtype=torch.float64)
            d[a] = eps
            fp = F.sdf_forward(cfg.sdf, layers, p + d, cfg.in_center, cfg.in_scale)[0]
            fm = F.sdf_forward(cfg.sdf, layers, p - d, cfg.in_center, cfg.in_scale)[0]
            fd = (fp - fm) / (2 * eps)
            np.testing.assert_allclose(g[:, a].numpy(), fd.numpy(), rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_geometric_init_is_close_to_a_sphere(name):
    cfg = get_config(name)
    rng = np.random.default_rng(1)
    xh = rng.uniform(-0.9, 0.9, (2000, 3))
    p = np.asarray(cfg.in_center) + cfg.in_scale * xh
    f = F.sdf_only(cfg, cfg.sdf_params(), p) / cfg.in_scale
    r = np.linalg.norm(xh, axis=1)
    sign = -1.0 if cfg.sdf.inside_out else 1.0
    err = f - sign * (r - cfg.sdf.sphere_r)
    # finite-width networks only approximate the sphere: loose statement
    assert np.abs(err).mean() < (0.1 if cfg.sdf.width >= 256 else 0.25)
    assert sign * np.corrcoef(f, r)[0, 1] > (0.9 if cfg.sdf.width >= 256 else 0.5)


def _plane_rays(s, n_sec, t0, t1, cos=-1.0, f0=0.7):
    """One ray through the plane f(t) = f0 + cos t, sections of [t0, t1]."""
    edges = np.linspace(t0, t1, n_sec + 1)
    t = 0.5 * (edges[:-1] + edges[1:])
    dt = np.diff(edges)
    f = f0 + cos * t
    v = np.array([[1.0, 0.0, 0.0]], np.float32)
    grad = np.tile([cos, 0.0, 0.0], (n_sec, 1))
    rgb = np.tile([0.2, 0.4, 0.6], (n_sec, 1))
    return edges, t, dt, f, v, grad, rgb


def test_composite_plane_telescopes_exactly():
    s = 64.0
    edges, t, dt, f, v, grad, rgb = _plane_rays(s, 37, 0.3, 1.1)
    out = Rn.composite([0, 37], v, t, dt, f, grad, rgb, s)
    phi = lambda x: 1 / (1 + np.exp(-s * x))
    fe = 0.7 - edges
    # contiguous sections telescope: T_k = Phi(f(a_k)) / Phi(f(a_0))
    assert out["acc"][0] == pytest.approx(1 - phi(fe[-1]) / phi(fe[0]), rel=1e-13)
    np.testing.assert_allclose(out["w"], (phi(fe[:-1]) - phi(fe[1:])) / phi(fe[0]), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(out["rgb"][0], out["acc"][0] * np.array([0.2, 0.4, 0.6]), rtol=1e-13)
    np.testing.assert_allclose(out["normal"][0], [-1, 0, 0], atol=1e-15)


def test_composite_depth_symmetric_window_is_the_hit():
    """Cells symmetric about the zero crossing t* give depth exactly t*."""
    s = 64.0
    t_star = 0.7
    edges, t, dt, f, v, grad, rgb = _plane_rays(s, 40, t_star - 0.4, t_star + 0.4)
    out = Rn.composite([0, 40], v, t, dt, f, grad, rgb, s)
    assert out["depth"][0] == pytest.approx(t_star, abs=1e-13)


def test_composite_dense_full_range_vs_bounded():
    """Dense brute force over the full range converges to the bounded result."""
    s = 64.0
    res = []
    for t0, t1, n in ((0.0, 10.0, 4096 * 4), (0.45, 0.95, 64)):
        edges, t, dt, f, v, grad, rgb = _plane_rays(s, n, t0, t1)
        res.append(Rn.composite([0, n], v, t, dt, f, grad, rgb, s))
    assert res[0]["acc"][0] == pytest.approx(res[1]["acc"][0], abs=1e-6)
    assert res[0]["depth"][0] == pytest.approx(res[1]["depth"][0], abs=1e-6)


def test_composite_weights_bounded_random():
    rng = np.random.default_rng(2)
    R = 50
    counts = rng.integers(0, 30, R)
    off = np.concatenate([[0], np.cumsum(counts)])
    S = off[-1]
    t = rng.uniform(0, 5, S)
    dt = rng.uniform(0, 0.2, S)
    f = rng.normal(0, 0.3, S)
    grad = rng.normal(size=(S, 3))
    rgb = rng.uniform(size=(S, 3))
    v = rng.normal(size=(R, 3)).astype(np.float32)
    out = Rn.composite(off, v, t, dt, f, grad, rgb, 64.0)
    assert (out["w"] >= 0).all()
    assert (out["acc"] <= 1 + 1e-12).all()
    assert (out["acc"][counts == 0] == 0).all() and (out["depth"][counts == 0] == 0).all()


def test_hs_upsample_uniform_weights_are_stratified():
    z = np.linspace(0.5, 2.0, 64)[None]
    fine = Rn.hs_upsample(z, np.full((1, 64), 3.0), 64.0, 64)  # far outside: alpha = 0
    u = (np.arange(64) + 0.5) / 64
    np.testing.assert_allclose(fine[0], 0.5 + u * 1.5, rtol=0, atol=1e-12)


def test_hs_upsample_concentrates_at_the_surface():
    z = np.linspace(0.0, 4.0, 64)[None]
    f = 1.3 - z                       # plane crossing at t = 1.3
    fine = Rn.hs_upsample(z, f, 64.0, 64)
    assert np.median(fine) == pytest.approx(1.3, abs=4.0 / 63)
    assert (np.diff(fine[0]) >= 0).all()
    t, dt = Rn.hs_sections(z, fine, np.array([4.0]))
    assert (dt >= 0).all() and dt.sum() == pytest.approx(4.0, abs=1e-12)


def test_full_upsample_ragged_closed_forms():
    """Coarse + fine inside the bound, ragged coarse sets: with zero opacity
    the coarse weights are uniform, so the fine points are the stratified
    quantiles z_0 + u_m (z_{n-1} - z_0) of each ray's own range; rays with
    fewer than two coarse points keep them; the sections tile [z_0, t_f]."""
    n_fine = 8
    ns = [0, 1, 2, 5, 17, 64, 3]
    lengths = np.array([0.0, 2.0, 3.0, 5.5, 9.0, 4.0, 1.0])
    t_f = 0.25 * np.arange(len(ns)) + lengths
    t_c, dt_c, f_c, off = [], [], [], [0]
    for r, n in enumerate(ns):
        d = lengths[r] / max(n, 1)
        z = 0.25 * r + (np.arange(n) + 0.5) * d
        t_c.append(z)
        dt_c.append(np.full(n, d))
        f_c.append(np.full(n, 5.0))                # far outside every surface: alpha = 0
        off.append(off[-1] + n)
    t_c, dt_c, f_c = map(np.concatenate, (t_c, dt_c, f_c))
    counts, o2, t, dt, rid = Rn.full_upsample(np.array(off), t_c, dt_c, f_c, t_f, 64.0, n_fine)
    u = (np.arange(n_fine) + 0.5) / n_fine
    for r, n in enumerate(ns):
        a, b = o2[r], o2[r + 1]
        assert (rid[a:b] == r).all()
        zc = t_c[off[r]:off[r + 1]]
        if n < 2:
            assert counts[r] == n
            np.testing.assert_array_equal(t[a:b], zc)
            np.testing.assert_array_equal(dt[a:b], dt_c[off[r]:off[r + 1]])
            continue
        assert counts[r] == n + n_fine
        fine = zc[0] + u * (zc[-1] - zc[0])
        y = np.sort(np.concatenate([zc, fine]))
        e = np.append(y[1:], t_f[r])
        np.testing.assert_allclose(t[a:b], 0.5 * (y + e), rtol=0, atol=1e-12)
        np.testing.assert_allclose(dt[a:b], e - y, rtol=0, atol=1e-12)
        assert dt[a:b].sum() == pytest.approx(t_f[r] - zc[0], abs=1e-12)


def test_full_upsample_concentrates_at_the_crossing():
    """A plane crossing inside a ray's bound: half the fine points fall
    within one coarse spacing of it."""
    n, n_fine = 12, 32
    z = 1.0 + (np.arange(n) + 0.5) * 0.25
    f = 2.3 - z                                    # crossing at t = 2.3
    counts, o2, t, dt, rid = Rn.full_upsample(np.array([0, n]), z, np.full(n, 0.25), f,
                                              np.array([4.0]), 64.0, n_fine)
    edges = np.append(t - dt / 2, 4.0)
    fine = np.setdiff1d(np.round(edges[:-1], 12), np.round(z, 12))
    assert fine.size == n_fine
    assert np.median(fine) == pytest.approx(2.3, abs=0.25)


def test_recover_select_and_merge_by_hand():
    """Selection is strict (acc == tau stays), takes NaN, keeps ray order;
    the merge replaces exactly the selected rows."""
    acc = np.array([1.0, 0.95, 0.9499999, 0.0, np.nan, 0.2, 0.99])
    idx = Rn.recover_select(acc, 0.95)
    assert idx.tolist() == [2, 3, 4, 5]
    assert Rn.recover_select(np.zeros(0), 0.95).size == 0
    out = {"acc": acc.copy(), "rgb": np.arange(21.0).reshape(7, 3)}
    sub = {"acc": np.array([0.5, 0.6, 0.7, 0.8]), "rgb": -np.ones((4, 3))}
    m = Rn.recover_merge(out, idx, sub)
    assert m["acc"].tolist()[:2] == [1.0, 0.95] and m["acc"][6] == 0.99
    assert m["acc"][idx].tolist() == [0.5, 0.6, 0.7, 0.8]
    assert (m["rgb"][idx] == -1).all() and (m["rgb"][[0, 1, 6]] == out["rgb"][[0, 1, 6]]).all()
    assert np.isnan(out["acc"][4])            # the input is untouched


# ----------------------------------------------------------------------------
# Closed-form pins of the network composition (Sec. 3.1, below Eq. 1; the
# supplementary normal): tiny networks with chosen weights whose outputs
# follow by hand, so that a swapped concatenation, a missing 1/sqrt(2), a
# wrong activation or a wrong input order each changes a checked value.

class _Cfg:
    """The fields of a workload configuration that the oracle field reads."""

    def __init__(self, sdf, color, center, scale):
        self.sdf, self.color, self.in_center, self.in_scale = sdf, color, center, scale


def _sp(z, beta=100.0):
    return math.log1p(math.exp(-beta * abs(z))) / beta + max(z, 0.0)


def _sig(z):
    return 1.0 / (1.0 + math.exp(-z))


def _skip_net():
    """PE(1) (9-d encoding), two hidden layers, the second one's input the
    concatenation [h_0, gamma] / sqrt(2); width 10 so layer 0 has 1 unit."""
    net = SdfNet(width=10, n_hidden=2, pe_freqs=1, skip_at=1, n_feat=2, beta=100.0)
    assert net.layer_dims() == [(9, 1), (10, 10), (10, 3)]
    W0 = np.zeros((1, 9)); W0[0, 4] = 2.0          # 2 sin(x_hat_1)
    b0 = np.array([-0.3125])
    W1 = np.zeros((10, 10)); b1 = np.zeros(10)
    W1[0, 0] = 1.0                                  # h_0 / sqrt(2)
    W1[1, 1] = 1.0                                  # gamma_0 / sqrt(2) = x_hat_0 / sqrt(2)
    W1[2, 8] = 1.0                                  # gamma_7 / sqrt(2) = cos(x_hat_1) / sqrt(2)
    W1[3, 6] = -1.0; b1[3] = 0.0625                 # -sin(x_hat_2)/sqrt(2) + 1/16
    W2 = np.zeros((3, 10)); b2 = np.array([0.125, 0.0, 0.25])
    W2[0, :4] = [1.0, 2.0, -1.0, 0.5]               # y0
    W2[1, 1] = 3.0                                  # feat_0
    W2[2, 4] = 1.0                                  # feat_1 = softplus(0) + 0.25
    params = np.concatenate([W0.ravel(), b0, W1.ravel(), b1, W2.ravel(), b2]).astype(np.float32)
    return net, params


def _skip_net_by_hand(xh, beta=100.0):
    x0, x1, x2 = xh
    z0 = 2.0 * math.sin(x1) - 0.3125
    h0 = _sp(z0, beta)
    r = 1.0 / math.sqrt(2.0)
    z1 = [r * h0, r * x0, r * math.cos(x1), -r * math.sin(x2) + 0.0625]
    h1 = [_sp(z, beta) for z in z1]
    y0 = h1[0] + 2.0 * h1[1] - h1[2] + 0.5 * h1[3] + 0.125
    feat = [3.0 * h1[1], _sp(0.0, beta) + 0.25]
    # d y0 / d x_hat by the chain rule (softplus_beta' = sigmoid(beta z))
    s = [_sig(beta * z) for z in z1]
    g = [2.0 * s[1] * r,
         s[0] * r * _sig(beta * z0) * 2.0 * math.cos(x1) - s[2] * r * (-math.sin(x1)),
         0.5 * s[3] * (-r * math.cos(x2))]
    return y0, feat, g


def test_skip_and_encoding_composition_closed_form():
    net, params = _skip_net()
    layers = F.as_layers(params, net.layer_dims())
    center, scale = (0.5, -0.25, 0.125), 2.0
    xh = np.array([[0.013, 0.161, -0.027], [-0.004, 0.3, 0.2], [0.02, -0.05, 0.9]])
    p = torch.tensor(np.asarray(center) + scale * xh, dtype=torch.float64, requires_grad=True)
    f, feat, x_hat = F.sdf_forward(net, layers, p, center, scale)
    (g,) = torch.autograd.grad(f.sum(), p)
    for i in range(xh.shape[0]):
        y0, ft, gg = _skip_net_by_hand(x_hat[i].detach().numpy())
        assert f[i].item() == pytest.approx(scale * y0, rel=1e-13, abs=1e-15)
        np.testing.assert_allclose(feat[i].detach().numpy(), ft, rtol=1e-13, atol=1e-15)
        # grad f with respect to world p: f = scale y0(x_hat), x_hat = (p - c)/scale
        np.testing.assert_allclose(g[i].numpy(), gg, rtol=1e-11, atol=1e-14)


def test_skip_composition_detects_plausible_mistakes():
    """The closed form above separates the right composition from a swapped
    concatenation, a missing 1/sqrt(2) and ReLU in place of softplus."""
    xh = (0.013, 0.161, -0.027)
    y_ok = _skip_net_by_hand(xh)[0]
    x0, x1, x2 = xh
    h0 = _sp(2.0 * math.sin(x1) - 0.3125)
    gam = [x0, x1, x2, math.sin(x0), math.sin(x1), math.sin(x2), math.cos(x0), math.cos(x1),
           math.cos(x2)]

    def y(u, act):
        z = [u[0], u[1], u[8], -u[6] + 0.0625]
        h = [act(v) for v in z]
        return h[0] + 2.0 * h[1] - h[2] + 0.5 * h[3] + 0.125

    r = 1.0 / math.sqrt(2.0)
    variants = {
        "swapped": y([r * v for v in gam + [h0]], _sp),
        "no sqrt2": y([h0] + gam, _sp),
        "relu": y([r * v for v in [max(2.0 * math.sin(x1) - 0.3125, 0.0)] + gam],
                  lambda v: max(v, 0.0)),
    }
    for name, yv in variants.items():
        assert abs(yv - y_ok) > 1e-4, name


def _feature_net():
    """SDF net with one hidden unit and one feature: y0 = softplus(x_hat_0),
    feat = 2 y0 + 0.5; grad f = (sigmoid(beta x_hat_0), 0, 0)."""
    net = SdfNet(width=1, n_hidden=1, pe_freqs=0, skip_at=-1, n_feat=1, beta=100.0)
    params = np.array([1.0, 0.0, 0.0, 0.0, 1.0, 2.0, 0.0, 0.5], np.float32)
    return net, params


@pytest.mark.parametrize("j", range(10))
def test_color_input_order_relu_sigmoid_closed_form(j):
    """Colour network [x_hat, v, grad f, feat] -> ReLU -> sigmoid(3): a
    hidden layer that selects input j (+ and - copies), through the oracle's
    whole field evaluation, equals the hand-computed sigmoid of the chosen
    input's ReLU'd value."""
    snet, sparams = _feature_net()
    cnet = ColorNet(width=2, n_hidden=1, n_feat=1)
    assert cnet.layer_dims() == [(10, 2), (2, 3)]
    W0 = np.zeros((2, 10)); W0[0, j] = 1.0; W0[1, j] = -1.0
    b0 = np.zeros(2)
    W1 = np.array([[1.0, 0.0], [0.0, 1.0], [2.0, -1.0]]); b1 = np.array([0.125, -0.1875, 0.0])
    cparams = np.concatenate([W0.ravel(), b0, W1.ravel(), b1]).astype(np.float32)
    center, scale = (0.25, 0.5, -0.5), 1.5
    cfg = _Cfg(snet, cnet, center, scale)
    sl = F.as_layers(sparams, snet.layer_dims())
    cl = F.as_layers(cparams, cnet.layer_dims())
    xh = np.array([0.004, -0.3, 0.45])
    v = np.array([0.48, -0.6, 0.64])
    p = torch.tensor([np.asarray(center) + scale * xh], dtype=torch.float64)
    f, g, rgb = F.field(cfg, sl, cl, p, torch.tensor([v], dtype=torch.float64))
    h = _sp(xh[0])
    grad = [_sig(100.0 * xh[0]), 0.0, 0.0]
    assert f[0].item() == pytest.approx(scale * h, rel=1e-13)
    np.testing.assert_allclose(g[0].numpy(), grad, rtol=1e-13, atol=1e-16)
    inputs = list(xh) + list(v) + grad + [2.0 * h + 0.5]
    a = inputs[j]
    hid = (max(a, 0.0), max(-a, 0.0))
    exp = [_sig(hid[0] + 0.125), _sig(hid[1] - 0.1875), _sig(2.0 * hid[0] - hid[1])]
    np.testing.assert_allclose(rgb[0].numpy(), exp, rtol=1e-13, atol=1e-16)
    # every other input order gives a different value for this j
    others = [k for k in range(10) if inputs[k] != a]
    assert others and all(abs(_sig(max(inputs[k], 0) + 0.125) - exp[0]) > 1e-6 or
                          abs(_sig(max(-inputs[k], 0) - 0.1875) - exp[1]) > 1e-6 for k in others)
