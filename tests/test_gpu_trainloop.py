"""GPU tests of the multi-step TSDF-bounded training loop pieces, through the
C ABI: the device repack of the packed forward operands (equal to packing at
creation), the Adam step against the FP64 oracle, and a short loop on the
small configuration that lowers the loss."""
import numpy as np
import pytest
import torch

from synth.configs import get_config
from oracle import train as OTR

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def make_field(cfg, sdf_params=None, color_params=None):
    from paper_2311_17878_amd import ops
    return ops.Field(cfg.sdf.width, cfg.sdf.n_hidden, cfg.sdf.pe_freqs, cfg.sdf.skip_at,
                     cfg.sdf.n_feat, cfg.color.n_hidden, cfg.sdf.beta, cfg.in_center,
                     cfg.in_scale, cfg.sdf_params() if sdf_params is None else sdf_params,
                     cfg.color_params() if color_params is None else color_params)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_repack_equals_packing_at_creation(name):
    """Repacking unchanged parameters changes nothing; parameters changed in
    place and repacked give bit for bit the outputs of a field created from
    the changed parameters, FP32, BF16 and FP32 operands as three-part BF16
    products (whose weight copies the repack splits anew)."""
    from paper_2311_17878_amd import _lib as L
    cfg = get_config(name)
    rng = np.random.default_rng(5)
    n = 3000
    o = np.tile(np.float32(cfg.in_center), (n, 1))
    v = rng.normal(size=(n, 3)).astype(np.float32)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    t = rng.uniform(0.1, 1.5 * cfg.in_scale, n).astype(np.float32)
    rid = np.arange(n, dtype=np.int32)
    args = (dev(o), dev(v), dev(t), dev(rid))
    F = make_field(cfg)
    precs = (L.FP32, L.BF16, L.BF16X6)
    before = {p: [x.clone() for x in F.forward(*args, precision=p)] for p in precs}
    F.repack()
    for p in precs:
        for a, b in zip(before[p], F.forward(*args, precision=p)):
            assert torch.equal(a, b)
    # change every parameter in place, repack, compare with a fresh field
    sp = cfg.sdf_params().astype(np.float32)
    cp = cfg.color_params().astype(np.float32)
    scale = np.float32(0.75)
    view = F.params_tensor()
    assert view.numel() == sp.size + cp.size
    assert np.array_equal(view.cpu().numpy(), np.concatenate([sp, cp]))
    view.mul_(float(scale))
    F.repack()
    G = make_field(cfg, sp * scale, cp * scale)
    for p in precs:
        for a, b in zip(F.forward(*args, precision=p), G.forward(*args, precision=p)):
            assert torch.equal(a, b)


def test_adam_step_matches_oracle():
    from paper_2311_17878_amd import ops
    rng = np.random.default_rng(11)
    n = 100003
    p = rng.normal(size=n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    pd, md, vd = dev(p), dev(m), dev(v)
    pr, mr, vr = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    gmax = np.zeros(n)
    for t in range(1, 4):
        g = (rng.normal(size=n) * 10.0 ** rng.uniform(-6, 1, n)).astype(np.float32)
        gmax = np.maximum(gmax, np.abs(g.astype(np.float64)))
        ops.adam_step(pd.data_ptr(), dev(g), md, vd, 1e-3, 0.9, 0.999, 1e-8, t)
        pr, mr, vr = OTR.adam(pr, g, mr, vr, 1e-3, 0.9, 0.999, 1e-8, t)
    torch.cuda.synchronize()
    # FP32 state: a few roundings per step, each relative to the size of the
    # terms (m cancels when gradients change sign, so bound it by max |g|)
    assert np.abs(pd.cpu().numpy() - pr).max() <= 1e-6
    assert (np.abs(md.cpu().numpy() - mr) <= 1e-6 * gmax).all()
    assert (np.abs(vd.cpu().numpy() - vr) <= 1e-6 * gmax * gmax).all()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x6"])
def test_training_loop_lowers_the_loss(prec):
    """Twenty TSDF-bounded steps on one fixed batch of the small scene (Adam,
    lr 1e-3): the photometric loss falls, the eikonal term stays finite."""
    from paper_2311_17878_amd import ops, _lib as L
    from paper_2311_17878_amd.autograd import train, Adam
    from paper_2311_17878_amd.pipeline import TsdfRenderer
    cfg = get_config("c1")
    g, s = cfg.grid, cfg.sampling
    grid = ops.make_grid(g.n, g.lo, g.h, g.d_t, g.d_s, g.nb_radius, g.m_consec)
    R = TsdfRenderer(grid, make_field(cfg), s.rho_num, s.rho_den, s.n_min, s.n_max, cfg.neus_s)
    o, v, d = cfg.integration_rays()
    R.integrate(dev(o), dev(v), dev(d))
    R.finalize()
    bo, bv, target = cfg.training_batch(2048, seed=3)
    eik = cfg.eikonal_points(2048, seed=3)
    batch = (dev(bo), dev(bv), dev(target), dev(eik))
    precision = {"fp32": L.FP32, "bf16": L.BF16, "bf16x6": L.BF16X6}[prec]
    hist, opt = train(R, lambda k: batch, 20, precision=precision, opt=Adam(R.field, lr=1e-3))
    losses = [a for a, _ in hist]
    print("%s loop: rgb loss %.5f -> %.5f, eikonal %.4f -> %.4f"
          % (prec, losses[0], losses[-1], hist[0][1], hist[-1][1]))
    assert opt.t == 20
    assert losses[-1] < 0.8 * losses[0]
    assert all(np.isfinite(x) for x in losses) and np.isfinite(hist[-1][1])
