"""The TSDF-Sampling render path and the hierarchical baseline, as sequences
of C-ABI calls on torch's current stream.

Render (Sec. 3.3-3.4 + Eq. 1/2): Alg. 1 bounds -> adaptive placement ->
field (SDF, grad f, colour) -> compositing.  The placement total stays on the
device (no host synchronisation inside a frame): the field reads the sample
count from device memory and the compositing reads the ray offsets.
"""
from __future__ import annotations

import torch

from . import ops
from ._lib import FP32


class _Marks:
    """Records consecutive (start, end) event pairs per stage name."""

    def __init__(self, events):
        self.events = events
        self.cur = None

    def __call__(self, name):
        if self.events is None:
            return
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        if self.cur is not None:
            self.events.setdefault(self.cur[0], []).append((self.cur[1], e))
        self.cur = (name, e) if name is not None else None


class TsdfRenderer:
    def __init__(self, grid, field, rho_num, rho_den, n_min, n_max, s, t_far=float("inf"),
                 precision=FP32):
        self.grid = grid
        self.field = field
        self.rho = (int(rho_num), int(rho_den))
        self.n_min, self.n_max = int(n_min), int(n_max)
        self.s = float(s)
        self.t_far = float(t_far)
        self.precision = precision
        self.state = None
        self.two_level = None
        self.V = None
        self.flags = None

    # ---------------------------------------------------------- volume ----
    def integrate(self, o, v, depth, batch=1 << 22, n_updates=None):
        """Fuse training rays (device tensors) into the TSDF state."""
        if self.state is None:
            self.state = ops.new_state(self.grid)
        R = o.shape[0]
        for s in range(0, R, batch):
            e = min(R, s + batch)
            ops.integrate(self.grid, self.state, o[s:e], v[s:e], depth[s:e], n_updates)
        return self.state

    def finalize(self, want_v=True):
        self.V, self.flags = ops.finalize(self.grid, self.state, want_v)
        return self.V, self.flags

    def fuse_two_level(self, batches, want_v=False, n_updates=None):
        """Build the volume as the two-level form (bricks of 8^3 voxels,
        integration sums only where the truncation band reaches) from every
        (o, v, depth) batch, and finalize it to V and the flags Alg. 1
        reads.  Keeps the two-level buffers in self.two_level; the dense
        state is not allocated."""
        self.two_level = ops.sparse_integrate(self.grid, batches, n_updates)
        self.V, self.flags = ops.sparse_finalize(self.grid, self.two_level, want_v)
        return self.V, self.flags

    def fill_unseen(self, depth_of, max_iter=4, cap=1 << 20):
        """Cast more rays into the voxels no ray has updated (Sec. 4.3): each
        round finds the frontier (unseen voxels next to observed free space)
        and its rays on the device, takes their depths from depth_of(o, v)
        (host arrays; the scene's depth source) and integrates them, until the
        frontier is empty or max_iter rounds ran.  A ray origin is a voxel
        centre that fusion calls free, which near silhouettes can lie just
        inside a solid: depth_of must then report a short valid depth (a
        blocked sensor), since a missing reading integrates as free space and
        would open the solid's interior.  Returns the frontier sizes and
        leaves the volume finalized."""
        sizes = []
        for _ in range(max_iter):
            self.finalize(want_v=False)
            fr = ops.frontier(self.grid, self.state, self.flags, cap)
            n = int(fr["n"].item())
            sizes.append(n)
            if n == 0:
                break
            k = min(n, cap)
            o, v = fr["o"][:k], fr["v"][:k]
            d = torch.as_tensor(depth_of(o.cpu().numpy(), v.cpu().numpy()), dtype=torch.float32)
            self.integrate(o, v, d.to(o.device), batch=k)
        self.finalize()
        return sizes

    # ---------------------------------------------------------- render ----
    def capture(self, o, v):
        """Record one render of the rays in o, v (device tensors whose shapes
        stay fixed) as a HIP graph.  Returns (graph, out): graph.replay()
        renders whatever rays o, v hold at replay time into the tensors of
        out (overwritten by every replay).  The render path has no host
        synchronisation and no memset; a warm-up render first allocates the
        workspaces outside the capture."""
        self.render(o, v)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            out = self.render(o, v)
        return graph, out

    def render(self, o, v, sync=False, keep=False, events=None):
        """Render rays o, v [R,3].  `events`: optional dict that receives
        (start, end) torch.cuda.Event pairs per stage, recorded on the
        stream the kernels run on."""
        mark = _Marks(events)
        mark("bounds")
        b = ops.ray_bounds(self.grid, self.flags, o, v, self.t_far)
        mark("place")
        R = o.shape[0]
        p = ops.place(b, self.rho[0], self.rho[1], self.n_min, self.n_max, s_cap=R * self.n_max,
                      sync=sync)
        s_count = None if sync else p["s_total"]
        mark("field")
        f, g, rgb = self.field.forward(o, v, p["t"], p["ray_id"], s_count=s_count,
                                       precision=self.precision, s_cap=p["t"].shape[0])
        mark("composite")
        out = ops.composite(p["offsets"], v, p["t"], p["dt"], f, g, rgb, self.s)
        mark(None)
        if keep:
            out.update(bounds=b, place=p, f=f, grad=g, rgb_s=rgb)
        out["s_total"] = p["s_total"]
        return out

    def render_full(self, o, v, n_fine, sync=False, keep=False, events=None):
        """Coarse + fine inside the TSDF bound ("Ours (full)"): Alg. 1 bounds
        -> adaptive placement (the coarse sets) -> SDF at the coarse samples ->
        n_fine fine points per ray from the coarse weights -> field at the
        merged sections -> compositing.  No host synchronisation unless
        sync=True."""
        mark = _Marks(events)
        mark("bounds")
        b = ops.ray_bounds(self.grid, self.flags, o, v, self.t_far)
        mark("place")
        R = o.shape[0]
        pc = ops.place(b, self.rho[0], self.rho[1], self.n_min, self.n_max, s_cap=R * self.n_max,
                       sync=sync)
        mark("field_coarse")
        fc, _, _ = self.field.forward(o, v, pc["t"], pc["ray_id"],
                                      s_count=None if sync else pc["s_total"],
                                      precision=self.precision, full=False, s_cap=pc["t"].shape[0])
        mark("upsample")
        cap = R * (min(self.n_max, 64) + int(n_fine))
        p = ops.place_fine(pc, fc, b["t_f"], n_fine, self.s, s_cap=cap, sync=sync)
        mark("field")
        f, g, rgb = self.field.forward(o, v, p["t"], p["ray_id"],
                                       s_count=None if sync else p["s_total"],
                                       precision=self.precision, s_cap=p["t"].shape[0])
        mark("composite")
        out = ops.composite(p["offsets"], v, p["t"], p["dt"], f, g, rgb, self.s)
        mark(None)
        if keep:
            out.update(bounds=b, coarse=pc, f_coarse=fc, place=p, f=f, grad=g, rgb_s=rgb)
        out["s_total"] = p["s_total"]
        return out

    def render_recover(self, o, v, tau=0.95, n_fine=0, keep=False, events=None):
        """TSDF-bounded render (with n_fine fine samples per ray when > 0),
        then recovery: rays whose weights sum to less than tau are rendered
        again over their initial range with the 64+64 hierarchical sampler
        and their outputs replace the bounded ones.  One host
        synchronisation (the number of recovered rays sizes the re-render)."""
        mark = _Marks(events)
        out = self.render_full(o, v, n_fine) if n_fine > 0 else self.render(o, v)
        mark("select")
        idx, n_sel = ops.select_rays(out["acc"], tau)
        n = int(n_sel.item())
        out["n_recovered"] = n
        if n > 0:
            mark("gather")
            o_s, v_s = ops.gather_rays(idx, n_sel, o, v, n)
            rec = self.render_hs(o_s, v_s)
            mark("scatter")
            ops.scatter_rays(idx, n_sel, n, rec, out)
        mark(None)
        if keep:
            out.update(recovered=idx[:n])
        return out

    def render_hs(self, o, v, keep=False, events=None):
        mark = _Marks(events)
        mark("range+coarse")
        t_in, t_out = ops.ray_range(self.grid, o, v)
        tc, rid = ops.hs_coarse(t_in, t_out, 64)
        mark("field_coarse")
        fc, _, _ = self.field.forward(o, v, tc, rid, precision=self.precision, full=False)
        mark("upsample")
        up = ops.hs_upsample(tc, fc, t_out, self.s)
        mark("field")
        f, g, rgb = self.field.forward(o, v, up["t"], up["ray_id"], precision=self.precision)
        mark("composite")
        out = ops.composite(up["offsets"], v, up["t"], up["dt"], f, g, rgb, self.s)
        mark(None)
        if keep:
            out.update(t_in=t_in, t_out=t_out, t_coarse=tc, f_coarse=fc, up=up, f=f, grad=g,
                       rgb_s=rgb)
        return out
