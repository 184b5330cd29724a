"""Oracle: loss and weight gradients of one training step on bounded samples.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper only envisions moving the TSDF bounds into training (Sec. 5,
"Limitations and Future Work"); the step here is the workload's definition:

  L = (1/B) sum_rays |C_hat - C*|^2  +  lambda (1/P) sum_points (|grad f| - 1)^2

with C_hat from Eq. 1 over the TSDF-bounded samples, grad f the analytic SDF
gradient (which also feeds the colour network and the NeuS opacity), and the
eikonal points uniform in the grid cube.  Gradients w.r.t. every weight are
taken by FP64 reverse-mode differentiation of these plain CPU operations,
including the second-order path weights -> grad f -> (colour, opacity,
eikonal).
"""
from __future__ import annotations

import numpy as np
import torch

from . import field as F
from . import render as Rn

DT = torch.float64


def _flat(layers):
    return torch.cat([torch.cat([W.reshape(-1), b]) for W, b in layers])


def loss_t(cfg, sdf_layers, color_layers, batch):
    o = torch.as_tensor(np.asarray(batch["o"], np.float32).astype(np.float64))
    v = torch.as_tensor(np.asarray(batch["v"], np.float32).astype(np.float64))
    off = np.asarray(batch["offsets"], np.int64)
    rid = torch.as_tensor(np.repeat(np.arange(off.size - 1), np.diff(off)))
    t = torch.as_tensor(np.asarray(batch["t"], np.float64))
    dt = torch.as_tensor(np.asarray(batch["dt"], np.float64))
    p = o[rid] + t[:, None] * v[rid]
    f, grad, rgb = F.field(cfg, sdf_layers, color_layers, p, v[rid], create_graph=True)
    out = Rn.composite_t(off, batch["v"], t, dt, f, grad, rgb, float(cfg.neus_s))
    target = torch.as_tensor(np.asarray(batch["target"], np.float64))
    l_rgb = ((out["rgb"] - target) ** 2).sum(-1).mean()
    x = torch.as_tensor(np.asarray(batch["eik_x"], np.float32).astype(np.float64)).requires_grad_(True)
    fe, _, _ = F.sdf_forward(cfg.sdf, sdf_layers, x, cfg.in_center, cfg.in_scale)
    (ge,) = torch.autograd.grad(fe.sum(), x, create_graph=True)
    l_eik = ((torch.linalg.norm(ge, dim=-1) - 1.0) ** 2).mean()
    return l_rgb + float(batch["eik_lambda"]) * l_eik


def loss_and_grads(cfg, sdf_params, color_params, batch):
    """Loss (float) and flat FP64 gradients in the parameter layout."""
    sl = F.as_layers(sdf_params, cfg.sdf.layer_dims(), requires_grad=True)
    cl = F.as_layers(color_params, cfg.color.layer_dims(), requires_grad=True)
    L = loss_t(cfg, sl, cl, batch)
    ps = [x for W, b in sl for x in (W, b)]
    pc = [x for W, b in cl for x in (W, b)]
    gs = torch.autograd.grad(L, ps + pc, allow_unused=True)
    gs = [torch.zeros_like(p) if g is None else g for p, g in zip(ps + pc, gs)]
    g_sdf = torch.cat([g.reshape(-1) for g in gs[:len(ps)]]).numpy()
    g_col = torch.cat([g.reshape(-1) for g in gs[len(ps):]]).numpy()
    return float(L.detach()), g_sdf, g_col


def loss_value(cfg, sdf_params64, color_params64, batch):
    """Loss at FP64 parameter vectors (used for finite differences)."""
    def layers(par, dims):
        out, k = [], 0
        for d_in, d_out in dims:
            W = torch.as_tensor(par[k:k + d_in * d_out].reshape(d_out, d_in))
            k += d_in * d_out
            b = torch.as_tensor(par[k:k + d_out])
            k += d_out
            out.append((W, b))
        return out
    sl = layers(np.asarray(sdf_params64, np.float64), cfg.sdf.layer_dims())
    cl = layers(np.asarray(color_params64, np.float64), cfg.color.layer_dims())
    return float(loss_t(cfg, sl, cl, batch))


def adam(p, g, m, v, lr, beta1, beta2, eps, t):
    """One Adam update in FP64 (the optimiser of the NeuS-family training
    the method builds on): returns (p, m, v) after step t >= 1."""
    p, g, m, v = (np.asarray(x, np.float64) for x in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

