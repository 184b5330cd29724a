"""Oracle: NeuS opacity, volume rendering (Eq. 1, Eq. 2, normal) and the
hierarchical-sampling baseline, in FP64 (plain PyTorch CPU ops).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Volume rendering (Sec. 3.1, Eq. 1): C = sum_i T_i alpha_i c_i with
T_i = prod_{j<i} (1 - alpha_j); depth (Eq. 2): D = sum w_i t_i / sum w_i with
w_i = T_i alpha_i; normal (supplementary, "Normal Estimation"):
N = sum w_i n_i / sum w_i, n = grad f / |grad f|.

Coarse + fine sampling inside the TSDF bound (the "Ours (full)" rows of the
experiment tables; the supplementary ray-distribution analysis): the
adaptive samples of a ray are its coarse set, fine points are drawn from the
coarse weight distribution by inverse transform sampling (the hierarchical
sampling paragraph: normalised coarse weights), and the merged points are
rendered.  full_upsample applies the baseline's hs_upsample / hs_sections to
each ray's own coarse set.

Recovery (Sec. 3.3, last paragraph; Sec. 4.6; supplementary Sec. B.3): a
ray whose weights in the bound sum to less than tau is rendered again over
its initial (whole-grid) range with the conventional sampler, here the 64+64
hierarchical baseline; recover_select gives those rays, recover_merge puts
their new outputs in place.

Opacity from the SDF (below Eq. 1 the paper turns the SDF into the density
of Eq. 1 without fixing the map; taken here): the NeuS
discrete opacity of a section [t - dt/2, t + dt/2],
alpha = max((Phi(f_prev) - Phi(f_next)) / Phi(f_prev), 0),  Phi(x) = sigmoid(s x),
with the section-end SDFs extrapolated from the midpoint along the ray,
f_prev/next = f -/+ cos dt/2, cos = min(v . grad f, 0).  Since cos <= 0,
f_next <= f_prev and 1 - alpha = Phi(f_next)/Phi(f_prev), so
log(1 - alpha) = logsigmoid(s f_next) - logsigmoid(s f_prev) exactly.
When sum w = 0 the normalised depth and normal are reported as 0.
"""
from __future__ import annotations

import numpy as np
import torch

from . import field as F

DT = torch.float64


def _dense(offsets, values, n_max, fill=0.0):
    """Scatter a ragged per-sample array into [R, n_max] (row = ray)."""
    offsets = np.asarray(offsets, np.int64)
    counts = np.diff(offsets)
    R = counts.size
    rid = np.repeat(np.arange(R), counts)
    k = np.arange(offsets[-1]) - offsets[:-1][rid]
    shape = (R, n_max) + tuple(values.shape[1:])
    out = torch.full(shape, fill, dtype=DT)
    out[torch.as_tensor(rid), torch.as_tensor(k)] = values
    mask = torch.zeros((R, n_max), dtype=torch.bool)
    mask[torch.as_tensor(rid), torch.as_tensor(k)] = True
    return out, mask, rid, k


def composite_t(offsets, v_ray, t, dt, f, grad, rgb, s):
    """Differentiable FP64 compositing of ragged samples; per-ray outputs and w."""
    offsets = np.asarray(offsets, np.int64)
    counts = np.diff(offsets)
    n_max = max(1, int(counts.max()) if counts.size else 1)
    R = counts.size
    rid = np.repeat(np.arange(R), counts)
    v = torch.as_tensor(np.asarray(v_ray, np.float32).astype(np.float64))[torch.as_tensor(rid)]
    cos = torch.clamp((v * grad).sum(-1), max=0.0)
    f_prev = f - cos * dt * 0.5
    f_next = f + cos * dt * 0.5
    log1m_alpha = torch.nn.functional.logsigmoid(s * f_next) - torch.nn.functional.logsigmoid(s * f_prev)
    L, mask, _, _ = _dense(offsets, log1m_alpha, n_max)
    logT = torch.cumsum(L, dim=1) - L               # exclusive prefix sum
    T = torch.exp(logT)
    alpha = -torch.expm1(L)
    w = torch.where(mask, T * alpha, torch.zeros_like(T))
    tt, _, _, _ = _dense(offsets, t, n_max)
    cc, _, _, _ = _dense(offsets, rgb, n_max)
    gn = torch.linalg.norm(grad, dim=-1, keepdim=True)
    n_hat = torch.where(gn > 0, grad / torch.where(gn > 0, gn, torch.ones_like(gn)), torch.zeros_like(grad))
    nn_, _, _, _ = _dense(offsets, n_hat, n_max)
    acc = w.sum(1)
    out_rgb = (w[..., None] * cc).sum(1)
    safe = torch.where(acc > 0, acc, torch.ones_like(acc))
    depth = torch.where(acc > 0, (w * tt).sum(1) / safe, torch.zeros_like(acc))
    normal = torch.where(acc[:, None] > 0, (w[..., None] * nn_).sum(1) / safe[:, None],
                         torch.zeros((R, 3), dtype=DT))
    w_flat = w[mask]
    return dict(rgb=out_rgb, depth=depth, normal=normal, acc=acc, w=w_flat)


def composite(offsets, v_ray, t, dt, f, grad, rgb, s):
    """numpy-in / numpy-out wrapper of composite_t (FP64)."""
    T = lambda a: torch.as_tensor(np.asarray(a, np.float64))
    with torch.no_grad():
        out = composite_t(offsets, v_ray, T(t), T(dt), T(f), T(grad), T(rgb), float(s))
    return {k: v.numpy() for k, v in out.items()}


# ------------------------------------------------ hierarchical sampling ----

def hs_coarse(t_in, t_out, n_coarse):
    """n_coarse midpoints of equal sections of each ray's grid range [R, n]."""
    t0 = np.asarray(t_in, np.float64)[:, None]
    t1 = np.asarray(t_out, np.float64)[:, None]
    k = np.arange(n_coarse, dtype=np.float64)[None]
    return t0 + (k + 0.5) * (t1 - t0) / n_coarse


def hs_cdf(z, f, s):
    """Knots of the coarse-weight CDF: value at z_k is sum_{j<k} pdf_j.

    Interval k = [z_k, z_{k+1}] gets alpha_k = max((Phi(f_k) - Phi(f_{k+1})) /
    Phi(f_k), 0) from the SDF at its two ends, w_k = T_k alpha_k, and
    probability (w_k + 1e-5) / sum_j (w_j + 1e-5).
    """
    f = np.asarray(f, np.float64)
    R, n = f.shape
    phi = 1.0 / (1.0 + np.exp(-s * f))
    alpha = np.clip((phi[:, :-1] - phi[:, 1:]) / phi[:, :-1], 0.0, 1.0)
    T = np.cumprod(np.concatenate([np.ones((R, 1)), 1.0 - alpha[:, :-1]], axis=1), axis=1)
    w = T * alpha + 1e-5
    pdf = w / w.sum(1, keepdims=True)
    cdf = np.concatenate([np.zeros((R, 1)), np.cumsum(pdf, axis=1)], axis=1)  # [R, n]
    return pdf, cdf


def hs_upsample(z, f, s, n_fine):
    """Fine samples by inverse transform of the coarse weight distribution:
    the quantiles u_m = (m + 1/2) / n_fine of the piecewise-uniform density
    of hs_cdf."""
    z = np.asarray(z, np.float64)
    R, n = z.shape
    pdf, cdf = hs_cdf(z, f, s)
    u = (np.arange(n_fine) + 0.5) / n_fine
    fine = np.zeros((R, n_fine))
    for r in range(R):
        k = np.searchsorted(cdf[r], u, side="right") - 1
        k = np.clip(k, 0, n - 2)
        frac = (u - cdf[r, k]) / pdf[r, k]
        fine[r] = z[r, k] + frac * (z[r, k + 1] - z[r, k])
    return fine


def hs_sections(z_coarse, z_fine, t_out):
    """Merge coarse and fine points; sections [y_i, y_{i+1}] and [y_last, t_out].

    Returns midpoints t and lengths dt, both [R, n_coarse + n_fine].
    """
    y = np.sort(np.concatenate([z_coarse, z_fine], axis=1), axis=1)
    ends = np.concatenate([y[:, 1:], np.asarray(t_out, np.float64)[:, None]], axis=1)
    return 0.5 * (y + ends), ends - y


def full_upsample(offsets, t_c, dt_c, f_c, t_f, s, n_fine):
    """Fine samples inside the TSDF bound for ragged coarse sets.

    Ray r owns coarse samples offsets[r] .. offsets[r+1]-1 (positions t_c
    ascending, lengths dt_c, SDF f_c).  A ray with n >= 2 coarse points gets
    n_fine fine points (hs_upsample of its n points), and its samples become
    the sections of the merged points (hs_sections, the last ending at
    t_f[r]); a ray with n < 2 keeps its coarse samples.  Returns counts,
    offsets [R+1], t, dt, ray_id (ray order).
    """
    offsets = np.asarray(offsets, np.int64)
    t_c = np.asarray(t_c, np.float64)
    dt_c = np.asarray(dt_c, np.float64)
    f_c = np.asarray(f_c, np.float64)
    t_f = np.asarray(t_f, np.float64)
    R = offsets.shape[0] - 1
    counts = np.zeros(R, np.int64)
    ts, dts, rids = [], [], []
    for r in range(R):
        a, b = offsets[r], offsets[r + 1]
        n = b - a
        if n < 2:
            t_r, dt_r = t_c[a:b], dt_c[a:b]
        else:
            z = t_c[a:b][None]
            fine = hs_upsample(z, f_c[a:b][None], s, n_fine)
            t_r, dt_r = hs_sections(z, fine, t_f[r:r + 1])
            t_r, dt_r = t_r[0], dt_r[0]
        counts[r] = t_r.shape[0]
        ts.append(t_r)
        dts.append(dt_r)
        rids.append(np.full(t_r.shape[0], r, np.int64))
    off = np.concatenate([[0], np.cumsum(counts)])
    cat = lambda x: np.concatenate(x) if x else np.zeros(0)
    return counts, off, cat(ts), cat(dts), cat(rids).astype(np.int64)


def recover_select(acc, tau):
    """Rays to recover, ascending: those whose weight sum is not >= tau
    (NaN included)."""
    acc = np.asarray(acc, np.float64)
    return np.flatnonzero(~(acc >= tau))


def recover_merge(out, idx, sub):
    """Copy of the render outputs `out` (dict of per-ray arrays) with rows idx
    replaced by the recovered rays' outputs `sub` (same keys, len(idx) rows)."""
    res = {k: np.array(v, copy=True) for k, v in out.items()}
    for k in res:
        res[k][idx] = sub[k]
    return res
