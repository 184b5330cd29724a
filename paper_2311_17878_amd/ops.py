"""Thin torch-facing wrappers over the C ABI (argument marshalling only).

Every function takes device tensors, allocates outputs with torch (device
memory and the current stream are all torch provides) and calls one entry
point of libtsdfs.so; all arithmetic runs in the HIP kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    return ctypes.c_void_p(t.data_ptr())


def _dev():
    return torch.device("cuda", torch.cuda.current_device())


def make_grid(n, lo, h, d_t, d_s, nb_radius=2, m_consec=15):
    g = L.Grid()
    g.n[:] = [int(x) for x in n]
    g.lo[:] = [float(x) for x in lo]
    g.h, g.d_t, g.d_s = float(h), float(d_t), float(d_s)
    g.nb_radius, g.m_consec = int(nb_radius), int(m_consec)
    return g


def n_voxels(g):
    return int(g.n[0]) * int(g.n[1]) * int(g.n[2])


def state_bytes(g):
    b = ctypes.c_size_t(0)
    L.check(L.load().tsdfs_state_bytes(ctypes.byref(g), ctypes.byref(b)))
    return b.value


def new_state(g):
    st = torch.empty(state_bytes(g), dtype=torch.uint8, device=_dev())
    L.check(L.load().tsdf_reset(ctypes.byref(g), _p(st), _stream()))
    return st


def state_views(g, st):
    """(sum [N] int64 in 2^-32 m, count [N] int32-as-uint32) views of a state."""
    N = n_voxels(g)
    s = st[: 8 * N].view(torch.int64)
    c = st[8 * N: 12 * N].view(torch.int32)
    return s, c


def integrate(g, st, o, v, depth, n_updates=None):
    L.check(L.load().tsdf_integrate(ctypes.byref(g), _p(st), _p(o), _p(v), _p(depth), o.shape[0],
                                    _p(n_updates), _stream()))


def finalize(g, st, want_v=True):
    N = n_voxels(g)
    V = torch.empty(N, dtype=torch.float32, device=_dev()) if want_v else None
    fl = torch.empty(N, dtype=torch.uint8, device=_dev())
    L.check(L.load().tsdf_finalize(ctypes.byref(g), _p(st), _p(V), _p(fl), _stream()))
    return V, fl


def sparse_integrate(g, batches, n_updates=None):
    """Two-level volume from the rays of `batches` (a list of (o, v, depth)
    device tensors): reset, mark every batch, allocate the band bricks (one
    host read of their number), then accumulate every batch into a pool of
    exactly that many bricks.  Returns dict(meta, pool, n_band)."""
    d = _dev()
    lib = L.load()
    b = ctypes.c_size_t(0)
    L.check(lib.tsdf_sparse_meta_bytes(ctypes.byref(g), ctypes.byref(b)))
    meta = torch.empty(b.value, dtype=torch.uint8, device=d)
    L.check(lib.tsdf_sparse_reset(ctypes.byref(g), _p(meta), _stream()))
    for o, v, depth in batches:
        L.check(lib.tsdf_sparse_mark(ctypes.byref(g), _p(meta), _p(o), _p(v), _p(depth),
                                     o.shape[0], _stream()))
    L.check(lib.tsdf_sparse_alloc_ws_bytes(ctypes.byref(g), ctypes.byref(b)))
    ws = torch.empty(b.value, dtype=torch.uint8, device=d)
    n_band = torch.zeros(1, dtype=torch.int64, device=d)
    L.check(lib.tsdf_sparse_alloc(ctypes.byref(g), _p(meta), _p(n_band), _p(ws), ws.numel(),
                                  _stream()))
    cap = int(n_band.item())
    L.check(lib.tsdf_sparse_pool_bytes(cap, ctypes.byref(b)))
    pool = torch.empty(max(b.value, 8), dtype=torch.uint8, device=d)
    L.check(lib.tsdf_sparse_pool_reset(cap, _p(pool), _stream()))
    for o, v, depth in batches:
        L.check(lib.tsdf_sparse_accumulate(ctypes.byref(g), _p(meta), _p(pool), cap, _p(o), _p(v),
                                           _p(depth), o.shape[0], _p(n_updates), _stream()))
    return dict(meta=meta, pool=pool, n_band=cap)


def sparse_views(g, sp):
    """seen words [n_bricks, 8] int64 (bit patterns), band [n_bricks] int32,
    slot [n_bricks] int32, pool sums [cap, 512] int64 and counts [cap, 512]
    int32 (uint32 bit patterns) of a two-level volume; bricks x fastest."""
    nb = [(int(x) + 7) // 8 for x in g.n]
    nbr = nb[0] * nb[1] * nb[2]
    m = sp["meta"]
    seen = m[: 64 * nbr].view(torch.int64).view(nbr, 8)
    band = m[64 * nbr: 68 * nbr].view(torch.int32)
    slot = m[68 * nbr: 72 * nbr].view(torch.int32)
    cap = sp["n_band"]
    psum = sp["pool"][: 4096 * cap].view(torch.int64).view(cap, 512)
    pcnt = sp["pool"][4096 * cap: 6144 * cap].view(torch.int32).view(cap, 512)
    return dict(seen=seen, band=band, slot=slot, psum=psum, pcnt=pcnt, n_bricks=tuple(nb))


def sparse_finalize(g, sp, want_v=True):
    N = n_voxels(g)
    V = torch.empty(N, dtype=torch.float32, device=_dev()) if want_v else None
    fl = torch.empty(N, dtype=torch.uint8, device=_dev())
    L.check(L.load().tsdf_sparse_finalize(ctypes.byref(g), _p(sp["meta"]), _p(sp["pool"]),
                                          sp["n_band"], _p(V), _p(fl), _stream()))
    return V, fl


def ray_bounds(g, flags, o, v, t_far=float("inf"), steps=False):
    R = o.shape[0]
    d = _dev()
    out = dict(t_n=torch.empty(R, dtype=torch.float32, device=d),
               t_f=torch.empty(R, dtype=torch.float32, device=d),
               first_hit=torch.empty(R, dtype=torch.int32, device=d),
               n_vox=torch.empty(R, dtype=torch.int32, device=d),
               status=torch.empty(R, dtype=torch.uint8, device=d))
    out["n_steps"] = torch.empty(R, dtype=torch.int32, device=d) if steps else None
    L.check(L.load().tsdf_ray_bounds(ctypes.byref(g), _p(flags), _p(o), _p(v), R, float(t_far),
                                     _p(out["t_n"]), _p(out["t_f"]), _p(out["first_hit"]),
                                     _p(out["n_vox"]), _p(out["status"]), _p(out["n_steps"]),
                                     _stream()))
    return out


def ray_range(g, o, v):
    R = o.shape[0]
    t_in = torch.empty(R, dtype=torch.float32, device=_dev())
    t_out = torch.empty(R, dtype=torch.float32, device=_dev())
    L.check(L.load().tsdf_ray_range(ctypes.byref(g), _p(o), _p(v), R, _p(t_in), _p(t_out),
                                    _stream()))
    return t_in, t_out


def place_ws_bytes(n_rays):
    b = ctypes.c_size_t(0)
    L.check(L.load().place_samples_ws_bytes(n_rays, ctypes.byref(b)))
    return b.value


def place(bounds, rho_num, rho_den, n_min, n_max, s_cap=None, sync=True, ws=None, noalloc=False):
    """Adaptive placement.  With sync=True the total is read back and the
    sample arrays are trimmed to it; otherwise arrays of s_cap are returned
    together with the device total.  noalloc=True calls the entry point
    whose scan partials live in the library's static device array (no
    workspace)."""
    R = bounds["t_n"].shape[0]
    d = _dev()
    if s_cap is None:
        s_cap = R * n_max
    counts = torch.empty(R, dtype=torch.int32, device=d)
    offsets = torch.empty(R + 1, dtype=torch.int32, device=d)
    t = torch.empty(max(s_cap, 1), dtype=torch.float32, device=d)
    dt = torch.empty(max(s_cap, 1), dtype=torch.float32, device=d)
    ray_id = torch.empty(max(s_cap, 1), dtype=torch.int32, device=d)
    s_total = torch.zeros(1, dtype=torch.int64, device=d)
    host_total = ctypes.c_int64(-1)
    args = (_p(bounds["t_n"]), _p(bounds["t_f"]), _p(bounds["n_vox"]), _p(bounds["status"]), R,
            rho_num, rho_den, n_min, n_max, _p(counts), _p(offsets), _p(t), _p(dt), _p(ray_id),
            s_cap, _p(s_total), ctypes.byref(host_total) if sync else None)
    if noalloc:
        L.check(L.load().place_samples_noalloc(*args, _stream()))
    else:
        if ws is None:
            ws = torch.empty(max(place_ws_bytes(R), 8), dtype=torch.uint8, device=d)
        L.check(L.load().place_samples(*args, _p(ws), ws.numel(), _stream()))
    out = dict(counts=counts, offsets=offsets, t=t, dt=dt, ray_id=ray_id, s_total=s_total)
    if sync:
        S = host_total.value
        out.update(t=t[:S], dt=dt[:S], ray_id=ray_id[:S], S=S)
    return out


def place_fine(place, f_coarse, t_f, n_fine, s, s_cap=None, sync=True, ws=None):
    """Coarse + fine inside the TSDF bound: `place` is the adaptive placement
    (its samples are the coarse sets), f_coarse the SDF at them.  With
    sync=True the total is read back, checked against s_cap and the arrays
    trimmed; otherwise arrays of s_cap come back with the device total."""
    R = t_f.shape[0]
    d = _dev()
    if s_cap is None:
        s_cap = int(place["t"].shape[0]) + R * int(n_fine)
    offsets = torch.empty(R + 1, dtype=torch.int32, device=d)
    t = torch.empty(max(s_cap, 1), dtype=torch.float32, device=d)
    dt = torch.empty(max(s_cap, 1), dtype=torch.float32, device=d)
    ray_id = torch.empty(max(s_cap, 1), dtype=torch.int32, device=d)
    s_total = torch.zeros(1, dtype=torch.int64, device=d)
    if ws is None:
        b = ctypes.c_size_t(0)
        L.check(L.load().place_fine_samples_ws_bytes(R, ctypes.byref(b)))
        ws = torch.empty(max(b.value, 8), dtype=torch.uint8, device=d)
    L.check(L.load().place_fine_samples(_p(place["offsets"]), _p(place["t"]), _p(place["dt"]),
                                        _p(f_coarse), _p(t_f), R, int(n_fine), float(s),
                                        _p(offsets), _p(t), _p(dt), _p(ray_id), s_cap,
                                        _p(s_total), _p(ws), ws.numel(), _stream()))
    out = dict(offsets=offsets, t=t, dt=dt, ray_id=ray_id, s_total=s_total)
    if sync:
        S = int(s_total.item())
        if S > s_cap:
            raise RuntimeError("place_fine: %d samples exceed s_cap = %d" % (S, s_cap))
        out.update(t=t[:S], dt=dt[:S], ray_id=ray_id[:S], S=S)
    return out


def bound_stats(t_in, t_out, bounds, depth):
    """Table 1's counting (device int64 [4]: rays with depth, failures, summed
    original and reduced range in 2^-24 m units)."""
    out = torch.empty(4, dtype=torch.int64, device=_dev())
    L.check(L.load().tsdf_bound_stats(_p(t_in), _p(t_out), _p(bounds["t_n"]), _p(bounds["t_f"]),
                                      _p(bounds["status"]), _p(depth), depth.shape[0], _p(out),
                                      _stream()))
    return out


def frontier(grid, state, flags, cap):
    """Unseen voxels bordering observed free space and the rays that fill
    them: dict idx, o, v (room for cap) and the device count n."""
    d = _dev()
    idx = torch.empty(max(cap, 1), dtype=torch.int32, device=d)
    o = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=d)
    v = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=d)
    n = torch.zeros(1, dtype=torch.int64, device=d)
    b = ctypes.c_size_t(0)
    L.check(L.load().tsdf_frontier_ws_bytes(ctypes.byref(grid), ctypes.byref(b)))
    ws = torch.empty(max(b.value, 8), dtype=torch.uint8, device=d)
    L.check(L.load().tsdf_frontier(ctypes.byref(grid), _p(state), _p(flags), cap, _p(idx), _p(o),
                                   _p(v), _p(n), _p(ws), ws.numel(), _stream()))
    return dict(idx=idx, o=o, v=v, n=n)


def select_rays(acc, tau):
    """Rays to recover (weight sum not >= tau), ascending; returns the index
    array (room for every ray) and the device count."""
    R = acc.shape[0]
    d = _dev()
    idx = torch.empty(max(R, 1), dtype=torch.int32, device=d)
    n_sel = torch.zeros(1, dtype=torch.int64, device=d)
    b = ctypes.c_size_t(0)
    L.check(L.load().select_rays_ws_bytes(R, ctypes.byref(b)))
    ws = torch.empty(max(b.value, 8), dtype=torch.uint8, device=d)
    L.check(L.load().select_rays(_p(acc), R, float(tau), _p(idx), _p(n_sel), _p(ws), ws.numel(),
                                 _stream()))
    return idx, n_sel


def gather_rays(idx, n_sel, o, v, cap):
    d = _dev()
    o_sub = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=d)
    v_sub = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=d)
    L.check(L.load().gather_rays(_p(idx), _p(n_sel), cap, _p(o), _p(v), _p(o_sub), _p(v_sub),
                                 _stream()))
    return o_sub[:cap], v_sub[:cap]


def scatter_rays(idx, n_sel, cap, sub, out):
    """out[k][idx[i]] = sub[k][i] for rgb, depth, normal, acc (in place)."""
    L.check(L.load().scatter_rays(_p(idx), _p(n_sel), cap, _p(sub["rgb"]), _p(sub["depth"]),
                                  _p(sub["normal"]), _p(sub["acc"]), _p(out["rgb"]),
                                  _p(out["depth"]), _p(out["normal"]), _p(out["acc"]), _stream()))
    return out


def hs_coarse(t_in, t_out, n_coarse=64):
    R = t_in.shape[0]
    t = torch.empty(R * n_coarse, dtype=torch.float32, device=_dev())
    rid = torch.empty(R * n_coarse, dtype=torch.int32, device=_dev())
    L.check(L.load().hs_coarse(_p(t_in), _p(t_out), R, n_coarse, _p(t), _p(rid), _stream()))
    return t, rid


def hs_upsample(t_coarse, f_coarse, t_out, s, n_coarse=64, n_fine=64):
    R = t_out.shape[0]
    n = R * (n_coarse + n_fine)
    d = _dev()
    t = torch.empty(n, dtype=torch.float32, device=d)
    dt = torch.empty(n, dtype=torch.float32, device=d)
    rid = torch.empty(n, dtype=torch.int32, device=d)
    off = torch.empty(R + 1, dtype=torch.int32, device=d)
    L.check(L.load().hs_upsample(_p(t_coarse), _p(f_coarse), _p(t_out), R, n_coarse, n_fine,
                                 float(s), _p(t), _p(dt), _p(rid), _p(off), _stream()))
    return dict(t=t, dt=dt, ray_id=rid, offsets=off)


def adam_step(params_ptr, grad, m, v, lr, beta1=0.9, beta2=0.999, eps=1e-8, step=1):
    """One Adam update of the n = grad.numel() device floats at params_ptr
    (m, v: device FP32 state of the same size)."""
    n = grad.numel()
    L.check(L.load().adam_step(ctypes.c_void_p(params_ptr), _p(grad), _p(m), _p(v), n, float(lr),
                               float(beta1), float(beta2), float(eps), int(step), _stream()))


class Field:
    """Device copy of the SDF + colour networks (packed for MFMA)."""

    def __init__(self, width, n_hidden, pe_freqs, skip_at, n_feat, col_hidden, beta, center,
                 scale, sdf_params, color_params):
        import numpy as np
        d = L.FieldDesc()
        d.width, d.n_hidden, d.pe_freqs, d.skip_at = width, n_hidden, pe_freqs, skip_at
        d.n_feat, d.col_hidden, d.beta = n_feat, col_hidden, float(beta)
        d.center[:] = [float(x) for x in center]
        d.scale = float(scale)
        self._sp = np.ascontiguousarray(sdf_params, dtype=np.float32)
        self._cp = np.ascontiguousarray(color_params, dtype=np.float32)
        h = ctypes.c_void_p(None)
        L.check(L.load().tsdfs_field_create(ctypes.byref(d), self._sp.ctypes.data_as(ctypes.c_void_p),
                                            self._cp.ctypes.data_as(ctypes.c_void_p),
                                            ctypes.byref(h)))
        self.handle = h
        b = ctypes.c_size_t(0)
        L.check(L.load().sdf_mlp_fwd_ws_bytes(self.handle, ctypes.byref(b)))
        self.ws_bytes = b.value
        self._ws = None

    def params(self):
        """(device pointer, n_sdf, n_color) of the plain FP32 parameters (SDF
        block then colour block), updated in place by a training loop."""
        ptr = ctypes.c_void_p(None)
        ns, nc = ctypes.c_size_t(0), ctypes.c_size_t(0)
        L.check(L.load().tsdfs_field_params(self.handle, ctypes.byref(ptr), ctypes.byref(ns),
                                            ctypes.byref(nc)))
        return ptr.value, ns.value, nc.value

    def params_tensor(self):
        """The plain parameters as a torch view of the field's own memory."""
        ptr, ns, nc = self.params()

        class _View:
            __cuda_array_interface__ = {"shape": (ns + nc,), "typestr": "<f4", "data": (ptr, False),
                                        "version": 3, "strides": None}
        return torch.as_tensor(_View(), device=_dev())

    def repack(self):
        """Rebuild the packed forward operands from the plain parameters."""
        L.check(L.load().tsdfs_field_repack(self.handle, _stream()))

    def workspace(self):
        if self._ws is None:
            self._ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=_dev())
        return self._ws

    def forward(self, o, v, t, ray_id, s_count=None, precision=L.FP32, full=True, s_cap=None):
        S = t.shape[0] if s_cap is None else s_cap
        d = _dev()
        f = torch.empty(max(S, 1), dtype=torch.float32, device=d)
        g = torch.empty((max(S, 1), 3), dtype=torch.float32, device=d) if full else None
        rgb = torch.empty((max(S, 1), 3), dtype=torch.float32, device=d) if full else None
        ws = self.workspace()
        L.check(L.load().sdf_mlp_fwd(self.handle, _p(o), _p(v), _p(t), _p(ray_id), S, _p(s_count),
                                     precision, _p(f), _p(g), _p(rgb), _p(ws), ws.numel(),
                                     _stream()))
        return f[:S], (g[:S] if full else None), (rgb[:S] if full else None)

    def backward(self, o, v, t, ray_id, d_f, d_grad, d_rgb, eik_x=None, eik_lambda=0.0,
                 d_sdf=None, d_col=None, precision=L.FP32):
        """Accumulate weight gradients (FP32 outputs; products in FP32, with
        BF16 inputs, or with FP32 operands as three-part BF16 products) into
        d_sdf / d_col (allocated zeroed when None); returns (d_sdf, d_col,
        eikonal loss tensor)."""
        d = _dev()
        S = t.shape[0] if t is not None else 0
        P = eik_x.shape[0] if eik_x is not None else 0
        if d_sdf is None:
            d_sdf = torch.zeros(self._sp.size, dtype=torch.float32, device=d)
        if d_col is None:
            d_col = torch.zeros(self._cp.size, dtype=torch.float32, device=d)
        b = ctypes.c_size_t(0)
        L.check(L.load().sdf_mlp_bwd_ws_bytes(self.handle, S + P, ctypes.byref(b)))
        ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=d)
        eik = torch.zeros(1, dtype=torch.float32, device=d)
        L.check(L.load().sdf_mlp_bwd(self.handle, _p(o), _p(v), _p(t), _p(ray_id), S, _p(eik_x), P,
                                     float(eik_lambda), _p(d_f), _p(d_grad), _p(d_rgb), precision,
                                     _p(d_sdf), _p(d_col), _p(eik), _p(ws), ws.numel(), _stream()))
        return d_sdf, d_col, eik

    def close(self):
        if self.handle:
            L.load().tsdfs_field_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def composite(offsets, v, t, dt, f, grad, rgb, s, want_w=False):
    R = offsets.shape[0] - 1
    d = _dev()
    out = dict(rgb=torch.empty((R, 3), dtype=torch.float32, device=d),
               depth=torch.empty(R, dtype=torch.float32, device=d),
               normal=torch.empty((R, 3), dtype=torch.float32, device=d),
               acc=torch.empty(R, dtype=torch.float32, device=d))
    out["w"] = torch.empty(max(t.shape[0], 1), dtype=torch.float32, device=d) if want_w else None
    L.check(L.load().composite(_p(offsets), R, _p(v), _p(t), _p(dt), _p(f), _p(grad), _p(rgb),
                               float(s), _p(out["rgb"]), _p(out["depth"]), _p(out["normal"]),
                               _p(out["acc"]), _p(out["w"]), _stream()))
    return out


def composite_bwd(offsets, v, t, dt, f, grad, rgb, s, d_out_rgb=None, d_out_depth=None,
                  d_out_normal=None, d_out_acc=None):
    """Per-sample adjoints (d_f, d_grad_f, d_rgb) of composite() from the
    per-ray adjoints of its outputs (None = zero)."""
    S = f.shape[0]
    d = _dev()
    d_f = torch.empty(max(S, 1), dtype=torch.float32, device=d)
    d_g = torch.empty((max(S, 1), 3), dtype=torch.float32, device=d)
    d_c = torch.empty((max(S, 1), 3), dtype=torch.float32, device=d)
    L.check(L.load().composite_bwd(_p(offsets), offsets.shape[0] - 1, _p(v), _p(t), _p(dt), _p(f),
                                   _p(grad), _p(rgb), float(s), _p(d_out_rgb), _p(d_out_depth),
                                   _p(d_out_normal), _p(d_out_acc), _p(d_f), _p(d_g), _p(d_c),
                                   _stream()))
    return d_f[:S], d_g[:S], d_c[:S]


def rgb_loss(rgb, target):
    R = rgb.shape[0]
    d_rgb = torch.empty_like(rgb)
    loss = torch.empty(1, dtype=torch.float32, device=_dev())
    L.check(L.load().rgb_loss(_p(rgb), _p(target), R, _p(d_rgb), _p(loss), _stream()))
    return loss, d_rgb
