"""GPU parity of the fused field kernels (FP32, BF16 and FP32 operands as
three-part BF16 products, through the C ABI)
at ragged sample counts: one sample, the tile size and its neighbours, sizes
that leave a ragged last tile.  A sample's outputs do not depend on the other
samples of its launch, so every small launch must equal, bit for bit, the same
samples inside one larger launch (also when shifted to other tile positions),
and the FP32 outputs must match the FP64 oracle.  The device-side sample
count is checked below, at and above the capacity: entries past it are left
untouched."""
import ctypes
import dataclasses

import numpy as np
import pytest
import torch

from synth.configs import get_config
from oracle import field as OF

pytestmark = pytest.mark.gpu

SIZES = [1, 31, 127, 128, 129, 255, 257, 1000]
N_BIG = 1300


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def make_field(cfg):
    from paper_2311_17878_amd import ops
    return ops.Field(cfg.sdf.width, cfg.sdf.n_hidden, cfg.sdf.pe_freqs, cfg.sdf.skip_at,
                     cfg.sdf.n_feat, cfg.color.n_hidden, cfg.sdf.beta, cfg.in_center,
                     cfg.in_scale, cfg.sdf_params(), cfg.color_params())


def samples(cfg, n, seed=7):
    """n samples on n/4 seeded rays through the network's input box."""
    rng = np.random.default_rng(seed)
    nr = max(n // 4, 1)
    o = (np.float32(cfg.in_center) + rng.uniform(-0.5, 0.5, (nr, 3)) * cfg.in_scale).astype(np.float32)
    v = rng.normal(size=(nr, 3))
    v = (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
    rid = rng.integers(0, nr, n).astype(np.int32)
    t = rng.uniform(0, 0.5 * cfg.in_scale, n).astype(np.float32)
    return o, v, t, rid


PRECISIONS = ["fp32", "bf16", "bf16x6"]


def _precision(L, prec):
    return {"fp32": L.FP32, "bf16": L.BF16, "bf16x6": L.BF16X6}[prec]


@pytest.mark.parametrize("name", ["c1", "c2"])
@pytest.mark.parametrize("prec", PRECISIONS)
def test_ragged_sizes_equal_one_large_launch(name, prec):
    from paper_2311_17878_amd import _lib as L
    cfg = get_config(name)
    precision = _precision(L, prec)
    o, v, t, rid = samples(cfg, N_BIG)
    F = make_field(cfg)
    od, vd = dev(o), dev(v)
    big = [x.clone() for x in F.forward(od, vd, dev(t), dev(rid), precision=precision)]
    for n in SIZES:
        for k in (0, 37):            # the same samples at other tile positions
            sl = slice(k, k + n)
            out = F.forward(od, vd, dev(t[sl]), dev(rid[sl]), precision=precision)
            for a, b, what in zip(out, big, ("f", "grad f", "rgb")):
                assert a.shape[0] == n
                assert torch.equal(a, b[sl]), "%s: n=%d shift=%d differs in %s" % (prec, n, k, what)
    if prec != "bf16":
        of, og, orgb = OF.eval_samples(cfg, cfg.sdf_params(), cfg.color_params(), o, v, t, rid)
        ef = np.abs(host(big[0]) - of).max()
        eg = np.abs(host(big[1]) - og).max()
        ec = np.abs(host(big[2]) - orgb).max()
        print("%s %s at %d samples: max abs err f %.3g grad %.3g rgb %.3g" % (name, prec, N_BIG, ef, eg, ec))
        assert ef <= 1e-4 and eg <= 2e-4 and ec <= 2e-5


@pytest.mark.parametrize("prec", PRECISIONS)
def test_device_sample_count(prec):
    """s_count_dev below, at and above s_cap: min(count, cap) samples are
    evaluated, equal to a plain launch of that many; the rest of the outputs
    keep what they held."""
    from paper_2311_17878_amd import _lib as L, ops
    cfg = get_config("c2")
    precision = _precision(L, prec)
    cap = 300
    o, v, t, rid = samples(cfg, cap, seed=11)
    F = make_field(cfg)
    args = (dev(o), dev(v), dev(t), dev(rid))
    ref = [x.clone() for x in F.forward(*args, precision=precision)]
    ws = F.workspace()
    lib = L.load()
    for count in (0, 129, cap, cap + 77):
        cnt = torch.tensor([count], dtype=torch.int64, device="cuda")
        f = torch.full((cap,), float("nan"), device="cuda")
        g = torch.full((cap, 3), float("nan"), device="cuda")
        rgb = torch.full((cap, 3), float("nan"), device="cuda")
        L.check(lib.sdf_mlp_fwd(F.handle, *(ctypes.c_void_p(a.data_ptr()) for a in args), cap,
                                ctypes.c_void_p(cnt.data_ptr()), precision,
                                ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                ctypes.c_void_p(rgb.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                ws.numel(), ops._stream()))
        torch.cuda.synchronize()
        m = min(count, cap)
        for a, b in zip((f, g, rgb), ref):
            assert torch.equal(a[:m], b[:m]), (prec, count)
            assert bool(torch.isnan(a[m:]).all()), (prec, count)


def test_unknown_precision_is_refused():
    """sdf_mlp_fwd and sdf_mlp_bwd refuse a precision value past the last
    mode (TSDFS_EUNSUPPORTED)."""
    from paper_2311_17878_amd import _lib as L
    cfg = get_config("c1")
    o, v, t, rid = samples(cfg, 64, seed=3)
    F = make_field(cfg)
    args = (dev(o), dev(v), dev(t), dev(rid))
    with pytest.raises(L.TsdfsError) as e:
        F.forward(*args, precision=L.BF16X6 + 1)
    assert e.value.code == L.TSDFS_EUNSUPPORTED
    f, g, rgb = F.forward(*args, precision=L.BF16X6)
    with pytest.raises(L.TsdfsError) as e:
        F.backward(*args, d_f=torch.ones_like(f), d_grad=torch.zeros_like(g),
                   d_rgb=torch.zeros_like(rgb), precision=L.BF16X6 + 1)
    assert e.value.code == L.TSDFS_EUNSUPPORTED


@pytest.mark.parametrize("width", [96, 160, 224])
@pytest.mark.parametrize("prec", PRECISIONS)
def test_other_widths(width, prec):
    """Networks of other supported widths (3, 5 and 7 row tiles per layer,
    each kernel's other work shares), a 2-frequency encoding and a skip
    layer at 2: FP32 products and FP32 operands as three-part BF16 products
    against the FP64 oracle; BF16 products bit-identical between a ragged
    launch and the same samples inside a larger one."""
    from paper_2311_17878_amd import _lib as L
    from synth.weights import SdfNet, ColorNet
    base = get_config("c2")
    cfg = dataclasses.replace(
        base, sdf=SdfNet(width=width, n_hidden=5, pe_freqs=2, skip_at=2, n_feat=width,
                         inside_out=True),
        color=ColorNet(width=width, n_hidden=2, n_feat=width))
    precision = _precision(L, prec)
    o, v, t, rid = samples(cfg, 700, seed=21)
    F = make_field(cfg)
    od, vd = dev(o), dev(v)
    big = [x.clone() for x in F.forward(od, vd, dev(t), dev(rid), precision=precision)]
    sl = slice(37, 37 + 259)
    part = F.forward(od, vd, dev(t[sl]), dev(rid[sl]), precision=precision)
    for a, b in zip(part, big):
        assert torch.equal(a, b[sl])
    if prec != "bf16":
        of, og, orgb = OF.eval_samples(cfg, cfg.sdf_params(), cfg.color_params(), o, v, t, rid)
        ef = np.abs(host(big[0]) - of).max()
        eg = np.abs(host(big[1]) - og).max()
        ec = np.abs(host(big[2]) - orgb).max()
        print("width %d %s: max abs err f %.3g grad %.3g rgb %.3g" % (width, prec, ef, eg, ec))
        assert ef <= 1e-4 and eg <= 2e-4 and ec <= 2e-5
