"""torch.autograd.Function wrappers around the hand-written backward, and one
TSDF-bounded training step (the paper's future-work direction of Sec. 5,
moving the TSDF bounds into training).

All arithmetic runs in libtsdfs.so: forward through sdf_mlp_fwd / composite,
backward through composite_bwd / sdf_mlp_bwd (activations recomputed there).
"""
from __future__ import annotations

import torch

from . import ops
from ._lib import FP32


class FieldFn(torch.autograd.Function):
    """(f, grad f, rgb) at p = o[ray_id] + t v[ray_id] as a function of the
    network weights.  `sdf_w`, `col_w` are the device leaves holding the
    parameters the field was created from; their gradients come from
    sdf_mlp_bwd (same precision as the forward), including the second-order
    terms through grad f."""

    @staticmethod
    def forward(ctx, sdf_w, col_w, field, o, v, t, ray_id, precision=FP32):
        f, g, rgb = field.forward(o, v, t, ray_id, precision=precision)
        ctx.field = field
        ctx.precision = precision
        ctx.save_for_backward(o, v, t, ray_id)
        return f, g, rgb

    @staticmethod
    def backward(ctx, d_f, d_g, d_rgb):
        o, v, t, ray_id = ctx.saved_tensors
        S = t.shape[0]
        dev = t.device
        d_f = d_f.contiguous() if d_f is not None else torch.zeros(S, device=dev)
        d_g = d_g.contiguous() if d_g is not None else torch.zeros((S, 3), device=dev)
        d_rgb = d_rgb.contiguous() if d_rgb is not None else torch.zeros((S, 3), device=dev)
        d_sdf, d_col, _ = ctx.field.backward(o, v, t, ray_id, d_f, d_g, d_rgb,
                                             precision=ctx.precision)
        return d_sdf, d_col, None, None, None, None, None, None


class CompositeFn(torch.autograd.Function):
    """Per-ray colour (Eq. 1), depth (Eq. 2), normal and weight sum as
    functions of the samples' f, grad f and rgb."""

    @staticmethod
    def forward(ctx, f, g, rgb, offsets, v, t, dt, s):
        out = ops.composite(offsets, v, t, dt, f, g, rgb, s)
        ctx.save_for_backward(f, g, rgb, offsets, v, t, dt)
        ctx.s = s
        return out["rgb"], out["depth"], out["normal"], out["acc"]

    @staticmethod
    def backward(ctx, d_rgb, d_depth, d_normal, d_acc):
        f, g, rgb, offsets, v, t, dt = ctx.saved_tensors
        c = lambda x: None if x is None else x.contiguous()
        d_f, d_g, d_c = ops.composite_bwd(offsets, v, t, dt, f, g, rgb, ctx.s, c(d_rgb), c(d_depth),
                                          c(d_normal), c(d_acc))
        return d_f, d_g, d_c, None, None, None, None, None


def train_step(renderer, o, v, target, eik_x, eik_lambda=0.1, precision=FP32):
    """One TSDF-bounded training step on a batch of rays (C ABI only):
    Alg. 1 bounds -> placement -> field -> compositing -> photometric loss,
    then the compositing adjoint and the network backward with the eikonal
    term on eik_x.  precision selects FP32 products, BF16-input products or
    FP32 operands as three-part BF16 products for the field forward and the
    network backward.  Returns (loss_rgb, loss_eik,
    d_sdf, d_col, n_samples)."""
    R = renderer
    b = ops.ray_bounds(R.grid, R.flags, o, v, R.t_far)
    p = ops.place(b, R.rho[0], R.rho[1], R.n_min, R.n_max, sync=True)
    f, g, rgb = R.field.forward(o, v, p["t"], p["ray_id"], precision=precision)
    out = ops.composite(p["offsets"], v, p["t"], p["dt"], f, g, rgb, R.s)
    loss, d_out = ops.rgb_loss(out["rgb"], target)
    d_f, d_g, d_c = ops.composite_bwd(p["offsets"], v, p["t"], p["dt"], f, g, rgb, R.s, d_out)
    d_sdf, d_col, eik = R.field.backward(o, v, p["t"], p["ray_id"], d_f, d_g, d_c,
                                         eik_x=eik_x, eik_lambda=eik_lambda, precision=precision)
    return loss, eik, d_sdf, d_col, p["S"]


class Adam:
    """Adam over a field's plain parameters (SDF block and colour block, one
    device array), with the packed forward operands rebuilt after each step.
    The update runs in libtsdfs.so (adam_step, tsdfs_field_repack)."""

    def __init__(self, field, lr=5e-4, betas=(0.9, 0.999), eps=1e-8):
        self.field = field
        self.ptr, self.n_sdf, self.n_col = field.params()
        n = self.n_sdf + self.n_col
        d = torch.device("cuda")
        self.m = torch.zeros(n, dtype=torch.float32, device=d)
        self.v = torch.zeros(n, dtype=torch.float32, device=d)
        self.lr, self.betas, self.eps = float(lr), betas, float(eps)
        self.t = 0

    def step(self, d_sdf, d_col):
        self.t += 1
        b1, b2 = self.betas
        ops.adam_step(self.ptr, d_sdf, self.m[:self.n_sdf], self.v[:self.n_sdf], self.lr, b1, b2,
                      self.eps, self.t)
        ops.adam_step(self.ptr + 4 * self.n_sdf, d_col, self.m[self.n_sdf:], self.v[self.n_sdf:],
                      self.lr, b1, b2, self.eps, self.t)
        self.field.repack()


def train(renderer, batches, n_steps, eik_lambda=0.1, precision=FP32, opt=None):
    """A TSDF-bounded training loop: for each step, batches(step) gives
    device (o, v, target, eik_x); one train_step, then one Adam update of the
    field.  Returns the per-step (loss_rgb, loss_eik) as floats and the
    optimiser."""
    opt = opt or Adam(renderer.field)
    hist = []
    for k in range(n_steps):
        o, v, target, eik_x = batches(k)
        loss, eik, d_sdf, d_col, _ = train_step(renderer, o, v, target, eik_x, eik_lambda, precision)
        opt.step(d_sdf, d_col)
        hist.append((loss, eik))
    return [(float(a.item()), float(b.item())) for a, b in hist], opt

