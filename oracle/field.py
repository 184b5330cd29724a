"""Oracle: neural SDF and colour networks in FP64 (plain PyTorch CPU ops).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper evaluates a pre-trained network at each sample, (sigma, c) =
MLP(p(t_i), v) (Sec. 3.1, below Eq. 1), and renders normals from the
normalised analytic gradient of the SDF network (supplementary, "Normal
Estimation").  The architecture is the workload's (NeuS/IDR-style):

  x_hat = (p - center) / scale
  gamma(x_hat) = [x_hat, sin(2^k x_hat), cos(2^k x_hat)]_{k=0..L-1}
  hidden layer l: z_l = W_l h_{l-1} + b_l,  h_l = softplus_beta(z_l);
    the skip layer's input is [h, gamma] / sqrt(2)
  output: [y0, feat] = W_out h + b_out; the SDF in world units is
    f = scale * y0 (the network works in normalised coordinates)
  grad f = d f / d p = d y0 / d x_hat   (analytic, reverse-mode)
  colour: [x_hat, v, grad f, feat] -> ReLU hidden layers -> sigmoid(3)

softplus_beta(z) = log(1 + exp(beta z)) / beta, evaluated as
z + log1p(exp(-beta z)) / beta for z > 0 (the same function, no overflow).
"""
from __future__ import annotations

import math
import numpy as np
import torch

from synth.weights import split_layers

DT = torch.float64


def softplus_beta(z, beta):
    # two overflow-free branches of the same function; each branch only ever
    # sees arguments on its own side of 0, so autograd stays exact (also at 0)
    zp = torch.clamp(z, min=0.0)
    zn = torch.clamp(z, max=0.0)
    return torch.where(z > 0, zp + torch.log1p(torch.exp(-beta * zp)) / beta,
                       torch.log1p(torch.exp(beta * zn)) / beta)


def encode(x_hat, n_freqs):
    parts = [x_hat]
    for k in range(n_freqs):
        parts.append(torch.sin((2.0 ** k) * x_hat))
        parts.append(torch.cos((2.0 ** k) * x_hat))
    return torch.cat(parts, dim=-1)


def as_layers(params, dims, requires_grad=False):
    out = []
    for W, b in split_layers(np.asarray(params, np.float32), dims):
        Wt = torch.tensor(W.astype(np.float64), dtype=DT, requires_grad=requires_grad)
        bt = torch.tensor(b.astype(np.float64), dtype=DT, requires_grad=requires_grad)
        out.append((Wt, bt))
    return out


def sdf_forward(sdf_net, layers, p, center, scale):
    """f [S], feat [S, n_feat] at world points p [S,3] (torch FP64)."""
    c = torch.tensor(np.asarray(center, np.float32).astype(np.float64), dtype=DT)
    x_hat = (p - c) / float(np.float32(scale))
    gamma = encode(x_hat, sdf_net.pe_freqs)
    h = gamma
    for l in range(sdf_net.n_hidden):
        if l == sdf_net.skip_at:
            h = torch.cat([h, gamma], dim=-1) / math.sqrt(2.0)
        W, b = layers[l]
        h = softplus_beta(h @ W.T + b, sdf_net.beta)
    W, b = layers[-1]
    y = h @ W.T + b
    return float(np.float32(scale)) * y[:, 0], y[:, 1:], x_hat


def color_forward(color_layers, x_hat, v, grad, feat):
    h = torch.cat([x_hat, v, grad, feat], dim=-1)
    for W, b in color_layers[:-1]:
        h = torch.relu(h @ W.T + b)
    W, b = color_layers[-1]
    return torch.sigmoid(h @ W.T + b)


def field(cfg, sdf_layers, color_layers, p, v, create_graph=False):
    """f, grad f (w.r.t. world p), rgb at points p [S,3] seen along v [S,3]."""
    p = p.detach().clone().requires_grad_(True)
    f, feat, x_hat = sdf_forward(cfg.sdf, sdf_layers, p, cfg.in_center, cfg.in_scale)
    (grad,) = torch.autograd.grad(f.sum(), p, create_graph=True)
    rgb = color_forward(color_layers, x_hat, v, grad, feat)
    if not create_graph:
        return f.detach(), grad.detach(), rgb.detach()
    return f, grad, rgb


def eval_samples(cfg, sdf_params, color_params, o, v, t, ray_id, chunk=65536):
    """Oracle field at p = o[ray] + t v[ray]; numpy FP64 outputs."""
    sl = as_layers(sdf_params, cfg.sdf.layer_dims())
    cl = as_layers(color_params, cfg.color.layer_dims())
    o64 = np.asarray(o, np.float32).astype(np.float64)
    v64 = np.asarray(v, np.float32).astype(np.float64)
    t64 = np.asarray(t, np.float64)
    S = t64.size
    f = np.zeros(S)
    g = np.zeros((S, 3))
    rgb = np.zeros((S, 3))
    for s in range(0, S, chunk):
        e = min(S, s + chunk)
        rid = ray_id[s:e]
        vv = torch.tensor(v64[rid], dtype=DT)
        p = torch.tensor(o64[rid], dtype=DT) + torch.tensor(t64[s:e, None], dtype=DT) * vv
        fi, gi, ci = field(cfg, sl, cl, p, vv)
        f[s:e] = fi.numpy()
        g[s:e] = gi.numpy()
        rgb[s:e] = ci.numpy()
    return f, g, rgb


def sdf_only(cfg, sdf_params, p, chunk=65536):
    """f at world points p [S,3] (no gradient, no colour), numpy FP64."""
    sl = as_layers(sdf_params, cfg.sdf.layer_dims())
    p = np.asarray(p, np.float64)
    out = np.zeros(p.shape[0])
    with torch.no_grad():
        for s in range(0, p.shape[0], chunk):
            f, _, _ = sdf_forward(cfg.sdf, sl, torch.tensor(p[s:s + chunk], dtype=DT),
                                  cfg.in_center, cfg.in_scale)
            out[s:s + chunk] = f.numpy()
    return out
