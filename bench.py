#!/usr/bin/env python3
"""Benchmark: rays/s of TSDF-bounded rendering on one MI355X.

Workload (default, "c2"): a 6x6x3 m synthetic room (20 boxes, four 2 cm
slabs); a 256^3 TSDF fused from 100 seeded 384x384 depth maps (14.7 M rays);
one 640x480 novel view (307 200 rays); SDF network 8x256 (6-frequency
encoding, skip at layer 4, 257 outputs) and colour network 4x256, FP32.

A timed step is one TSDF-bounded render of the view with the volume resident:
Alg. 1 bounds -> adaptive placement -> field (SDF + grad f + colour) ->
compositing.  Also reported on the same GPU: dense 64+64 hierarchical
sampling, the BF16 field, the field with FP32 operands as three-part BF16
products (FP32 accuracy on the BF16 matrix cores), the integration
throughput, the field kernel's roofline fraction and the CPU oracle on a
bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0}
HBM_PEAK_GBS = 8000.0

# HBM traffic of one 6.02 M-sample field launch on the c2 view, from the
# FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch) of the kernel built from
# the sources whose digest is given; scaled by a plain copy's counters
# (fetch x 2, write x 1).  Reported only while the sources still match.
FIELD_SOURCES = {"k_field_fp32": ["field_fp32.hip", "field_common.hpp", "common.hpp", "field.hip"],
                 "k_field_fp32_split": ["field_fp32.hip", "field_common.hpp", "common.hpp",
                                        "field.hip"],
                 "k_field_bf16": ["field_bf16.hip", "field_bf16_layout.hpp", "field_common.hpp",
                                  "common.hpp", "field.hip"]}
TRAFFIC = {
    "k_field_fp32": {"sha256_16": "87ddab944ac78476", "fetch_kib": 3.6421e+07, "write_kib": 5.7854e+07},
    "k_field_fp32_split": {"sha256_16": "87ddab944ac78476", "fetch_kib": 3.9673e+07,
                           "write_kib": 5.8033e+07},
    "k_field_bf16": {"sha256_16": "143471f6598e3903", "fetch_kib": 1.3242e+07, "write_kib": 2.1042e+07},
}
COPY_SCALE = {"fetch": 2.0, "write": 1.0}


def field_traffic_bytes(kernel, workload):
    """Measured HBM bytes per launch, or None when the kernel changed since."""
    import hashlib
    t = TRAFFIC.get(kernel)
    if t is None or workload != "c2":
        return None
    m = hashlib.sha256()
    for f in FIELD_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2311_17878_amd", "csrc", f), "rb") as fh:
            m.update(fh.read())
    if m.hexdigest()[:16] != t["sha256_16"]:
        return None
    return 1024.0 * (t["fetch_kib"] * COPY_SCALE["fetch"] + t["write_kib"] * COPY_SCALE["write"])


def field_flops_per_sample(sdf, col):
    """Algorithmic FLOP of one full field evaluation: SDF forward, reverse
    pass for d f / d x (all hidden layers, f row only at the output), colour
    forward.  Padding and recomputation are not counted."""
    dims = sdf.layer_dims()
    fwd = sum(i * o for i, o in dims)
    rev = dims[-1][0] + sum(i * o for i, o in dims[:-1])
    colour = sum(i * o for i, o in col.layer_dims())
    return 2 * (fwd + rev + colour), 2 * fwd


def train_flops_per_row(sdf, col):
    """Algorithmic FLOP per row (sample or eikonal point) of the training
    backward as implemented: the forward recomputed (hidden F_h + output
    W n_y), the reverse pass for d f / d x (F_h), the colour forward and its
    backward (3 C), the adjoint of the reverse pass (2 F_h) and first-order
    backprop (2 F_h + 2 W n_y less the first layer's input gradient):
    6 F_h + 3 W n_y + 3 C - d_gamma d_out0 multiply-adds."""
    dims = sdf.layer_dims()
    f_h = sum(i * o for i, o in dims[:-1])
    w_ny = dims[-1][0] * dims[-1][1]
    c = sum(i * o for i, o in col.layer_dims())
    return 2 * (6 * f_h + 3 * w_ny + 3 * c - dims[0][0] * dims[0][1])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(cfg, ro, rv, n_rays, seed=0):
    """The FP64 oracle's render path on a seeded subset of the view's rays,
    with the oracle's own volume (stored flags written by the oracle)."""
    import torch
    from oracle import tsdf as OT, field as OF, render as OR
    gold = np.load(os.path.join(ROOT, "tests", "golden", f"{cfg.name}_volume.npz"))
    N = int(gold["n_vox"])
    f0 = np.unpackbits(gold["flag0"])[:N]
    f1 = np.unpackbits(gold["flag1"])[:N]
    fl = (f0 | (f1 << 1)).astype(np.uint8)
    idx = np.sort(np.random.default_rng(seed).choice(ro.shape[0], n_rays, replace=False))
    o, v = ro[idx], rv[idx]
    s = cfg.sampling
    t0 = time.perf_counter()
    b = OT.bounds(cfg.grid, fl, o, v, s.t_far)
    p = OT.place(b["t_n"], b["t_f"], b["n_vox"], b["status"], s.rho_num, s.rho_den, s.n_min, s.n_max)
    f, g, rgb = OF.eval_samples(cfg, cfg.sdf_params(), cfg.color_params(), o, v, p["t"], p["ray_id"])
    OR.composite(p["offsets"], v, p["t"], p["dt"], f, g, rgb, cfg.neus_s)
    dt = time.perf_counter() - t0
    return dict(value=n_rays / dt, unit="rays/s", cores=torch.get_num_threads(), kind="oracle",
                cpu_model=cpu_model(),
                sample=f"{n_rays} seeded rays of the view through the FP64 oracle render path "
                       f"(bounds, placement, field, compositing) with the oracle's stored flags; "
                       f"{int(p['offsets'][-1])} samples; {dt:.1f} s")


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def panorama_leg(steps, warmup, tile=8):
    """The large panorama workload in BF16: the 512^3 volume fused from all
    300 views of 512^2 (78.6 M rays), one equirectangular 2048 x 1024 view
    (2.1 M rays, 1 to 64 samples per ray, the ragged samples in one
    persistent field launch), timed like the main step; the field kernel's
    MFMA fraction from the field stage's events."""
    import torch
    from synth.configs import get_config
    from paper_2311_17878_amd import ops, _lib
    from paper_2311_17878_amd.pipeline import TsdfRenderer
    cfg = get_config("c5")
    g, s = cfg.grid, cfg.sampling
    t0 = time.time()
    o, v, d = cfg.integration_rays(progress=lambda k, n: log(f"c5 depth maps {k}/{n}"), tile=tile)
    ro, rv = cfg.render_rays()
    log(f"c5 inputs: {o.shape[0]} training rays, {ro.shape[0]} render rays "
        f"({time.time() - t0:.1f} s)")
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    grid = ops.make_grid(g.n, g.lo, g.h, g.d_t, g.d_s, g.nb_radius, g.m_consec)
    field = ops.Field(cfg.sdf.width, cfg.sdf.n_hidden, cfg.sdf.pe_freqs, cfg.sdf.skip_at,
                      cfg.sdf.n_feat, cfg.color.n_hidden, cfg.sdf.beta, cfg.in_center,
                      cfg.in_scale, cfg.sdf_params(), cfg.color_params())
    R = TsdfRenderer(grid, field, s.rho_num, s.rho_den, s.n_min, s.n_max, cfg.neus_s, s.t_far,
                     _lib.BF16)
    o_d, v_d, d_d = dev(o), dev(v), dev(d)
    del o, v, d
    nup = torch.zeros(1, dtype=torch.int64, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    R.integrate(o_d, v_d, d_d, batch=1 << 24, n_updates=nup)
    e1.record()
    torch.cuda.synchronize()
    integ_ms = e0.elapsed_time(e1)
    n_train = o_d.shape[0]
    del o_d, v_d, d_d
    R.finalize(want_v=False)
    ro_d, rv_d = dev(ro), dev(rv)
    n_rays = ro.shape[0]
    for _ in range(warmup):
        R.render(ro_d, rv_d)
    torch.cuda.synchronize()
    ev = {}
    e0.record()
    for _ in range(steps):
        out = R.render(ro_d, rv_d, events=ev)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    stage_ms = {k: float(np.mean([a.elapsed_time(b) for a, b in v_])) for k, v_ in ev.items()}
    S = int(out["s_total"].item())
    chk = R.render(ro_d, rv_d, keep=True)
    counts = chk["place"]["counts"].cpu().numpy()
    fl_sample, _ = field_flops_per_sample(cfg.sdf, cfg.color)
    achieved = S * fl_sample / (stage_ms["field"] * 1e-3) / 1e12
    res = {
        "workload": f"c5: one {n_rays}-ray equirectangular view; {cfg.notes}; TSDF {g.n[0]}^3, "
                    f"h={g.h:.6f} m; networks as the room's; BF16 products, FP32 accumulation",
        "precision": "bf16",
        "integrate": {"rays": n_train, "ms": integ_ms, "rays_per_s": n_train / (integ_ms * 1e-3),
                      "voxel_updates": int(nup.item()),
                      "ray_order": "8x8 pixel blocks per view" if tile == 8 else "row by row"},
        "ms_per_step": ms, "rays_per_s": n_rays / (ms * 1e-3),
        "samples_per_ray": {"mean": S / n_rays, "min": int(counts.min()),
                            "p50": float(np.percentile(counts, 50)),
                            "p99": float(np.percentile(counts, 99)), "max": int(counts.max()),
                            "samples": S},
        "stage_ms": stage_ms,
        "roofline": {"kernel": "k_field_bf16", "bound": "mfma", "achieved": achieved,
                     "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS["bf16"], "flop_per_sample": fl_sample},
    }
    log(f"c5 panorama (bf16): {ms:.2f} ms/step, {n_rays / ms * 1e3:.0f} rays/s, "
        f"{S / n_rays:.2f} samples/ray, field {achieved:.0f} TFLOP/s")
    del R, field, chk, out, ro_d, rv_d
    torch.cuda.empty_cache()
    return res


def stage_hbm(stage_ms, n_rays, S, total_steps):
    work = {
        "bounds": 24 * n_rays + 17 * n_rays + total_steps,       # o, v in; t_n, t_f, ids out; 1 B/step
        "place": 13 * n_rays + 8 * n_rays + 12 * S,              # bounds in; count, offset; t, dt, ray_id
        "composite": 36 * S + 32 * n_rays,                       # t, dt, f, grad f, rgb; ray outputs
    }
    out = {}
    for k, b in work.items():
        if k in stage_ms and stage_ms[k] > 0:
            gbs = b / (stage_ms[k] * 1e-3) / 1e9
            out[k] = {"bytes": b, "GB_per_s": gbs, "frac": gbs / HBM_PEAK_GBS}
    out["dda_steps"] = total_steps
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--hs-steps", type=int, default=2)
    ap.add_argument("--cpu-rays", type=int, default=16384,
                    help="rays of the view in the CPU oracle sample (about 10-30 s of host work)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hs", action="store_true")
    ap.add_argument("--no-other", action="store_true", help="skip the other-precision leg")
    ap.add_argument("--no-split", dest="split", action="store_false",
                    help="skip the leg with FP32 operands as three-part BF16 products")
    ap.add_argument("--no-train", action="store_true", help="skip the training-step leg")
    ap.add_argument("--no-table1", action="store_true",
                    help="skip Table 1's counting on the training rays and the NeRF-mode leg")
    ap.add_argument("--recover-tau", type=float, default=0.95,
                    help="weight-sum threshold of the recovery leg (0: skip the leg)")
    ap.add_argument("--full-fine", type=int, default=8,
                    help="fine samples per ray of the coarse + fine leg (0: skip the leg)")
    ap.add_argument("--fill-rounds", type=int, default=2,
                    help="rounds of filling unseen voxels on a copy of the volume (0: skip)")
    ap.add_argument("--ray-order", default="tile8", choices=["row", "tile8"],
                    help="order of the training rays within each view: by 8x8 pixel blocks "
                         "(default) or row by row; the fused volume is the same bit for bit")
    ap.add_argument("--no-graph", dest="graph", action="store_false",
                    help="skip the recorded-graph leg")
    ap.add_argument("--no-rho-sweep", dest="rho_sweep", action="store_false",
                    help="skip the sampling-density sweep")
    ap.add_argument("--no-two-level", dest="two_level", action="store_false",
                    help="skip the two-level volume leg")
    ap.add_argument("--no-c5", dest="c5", action="store_false",
                    help="skip the panorama leg (512^3 volume from 300 views, 2.1 M-ray view, BF16)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (to scale HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_calibration}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the library has no "
              "multi-GPU path; the figure is the throughput of one GPU", file=sys.stderr)
        sys.exit(2)

    import torch
    from synth.configs import get_config
    from paper_2311_17878_amd import ops, _lib
    from paper_2311_17878_amd.pipeline import TsdfRenderer

    torch.cuda.set_device(0)
    cfg = get_config(args.workload)
    g, s = cfg.grid, cfg.sampling
    prec = _lib.BF16 if args.precision == "bf16" else _lib.FP32
    t0 = time.time()
    o, v, d = cfg.integration_rays(progress=lambda k, n: log(f"depth maps {k}/{n}"),
                                   tile=8 if args.ray_order == "tile8" else 0)
    ro, rv = cfg.render_rays()
    log(f"inputs: {o.shape[0]} training rays, {ro.shape[0]} render rays ({time.time() - t0:.1f} s)")
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    grid = ops.make_grid(g.n, g.lo, g.h, g.d_t, g.d_s, g.nb_radius, g.m_consec)
    field = ops.Field(cfg.sdf.width, cfg.sdf.n_hidden, cfg.sdf.pe_freqs, cfg.sdf.skip_at,
                      cfg.sdf.n_feat, cfg.color.n_hidden, cfg.sdf.beta, cfg.in_center,
                      cfg.in_scale, cfg.sdf_params(), cfg.color_params())
    R = TsdfRenderer(grid, field, s.rho_num, s.rho_den, s.n_min, s.n_max, cfg.neus_s, s.t_far, prec)
    o_d, v_d, d_d = dev(o), dev(v), dev(d)
    ro_d, rv_d = dev(ro), dev(rv)
    n_rays = ro.shape[0]

    # ---- integration throughput (one pass over all training rays, resident)
    nup = torch.zeros(1, dtype=torch.int64, device="cuda")
    R.state = ops.new_state(grid)
    R.integrate(o_d, v_d, d_d, batch=o.shape[0])        # warm-up pass
    torch.cuda.synchronize()
    R.state = ops.new_state(grid)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    R.integrate(o_d, v_d, d_d, batch=o.shape[0], n_updates=nup)
    e1.record()
    torch.cuda.synchronize()
    integ_ms = e0.elapsed_time(e1)
    e0.record()
    R.finalize()
    e1.record()
    torch.cuda.synchronize()
    fin_ms = e0.elapsed_time(e1)
    updates = int(nup.item())
    log(f"integrate: {integ_ms:.2f} ms, {updates} updates; finalize {fin_ms:.2f} ms")

    # ---- TSDF-bounded render: warm-up, then exactly K timed steps
    for _ in range(args.warmup):
        R.render(ro_d, rv_d)
    torch.cuda.synchronize()
    ev = {}
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        out = R.render(ro_d, rv_d, events=ev)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    stage_ms = {k: float(np.mean([a.elapsed_time(b) for a, b in v_])) for k, v_ in ev.items()}
    S = int(out["s_total"].item())
    chk = R.render(ro_d, rv_d, keep=True)
    counts = chk["place"]["counts"].cpu().numpy()
    status = chk["bounds"]["status"].cpu().numpy()
    nz = counts[counts > 0]
    nsteps = ops.ray_bounds(R.grid, R.flags, ro_d, rv_d, R.t_far, steps=True)["n_steps"]
    total_steps = int(nsteps.sum().item())
    fl_sample, fl_sdf_only = field_flops_per_sample(cfg.sdf, cfg.color)
    field_ms = stage_ms["field"]
    achieved = S * fl_sample / (field_ms * 1e-3) / 1e12
    dtype = "bf16" if prec == _lib.BF16 else "f32"
    log(f"render: {ms:.3f} ms/step, {n_rays / ms * 1e3:.0f} rays/s, S={S}, stages {stage_ms}")

    result = {
        "metric": "rays/sec and samples/ray, TSDF-bounded vs 64+64 hierarchical; BF16 vs FP32",
        "value": n_rays / (ms * 1e-3),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name}: one {ro.shape[0]}-ray novel view; {cfg.notes}; "
                        f"TSDF {g.n[0]}^3, h={g.h:.6f} m, D_T=5h, D_s=1h, 5^3 neighbourhood, M=15; "
                        f"SDF {cfg.sdf.n_hidden}x{cfg.sdf.width} PE{cfg.sdf.pe_freqs} skip{cfg.sdf.skip_at}, "
                        f"colour {cfg.color.n_hidden}x{cfg.color.width}; NeuS s={cfg.neus_s:g}",
            "rays": n_rays,
            "rho": f"{s.rho_num}/{s.rho_den} samples per traversed voxel",
            "n_min": s.n_min, "n_max": s.n_max,
            "precision": dtype,
        },
        "samples_per_ray": {
            "mean": S / n_rays,
            "mean_nonzero": float(nz.mean()) if nz.size else 0.0,
            "min": int(counts.min()), "p50": float(np.percentile(counts, 50)),
            "p99": float(np.percentile(counts, 99)), "max": int(counts.max()),
            "status_counts": {k: int((status == i).sum()) for i, k in
                              enumerate(["hit", "no_far", "miss", "invalid"])},
            "samples": S,
        },
        "stage_ms": stage_ms,
        # algorithmic bytes of the HBM-bound stages (per ray / sample / DDA step), their GB/s
        # over the stage's event time, and the fraction of the 8 TB/s HBM peak
        "stage_hbm": stage_hbm(stage_ms, n_rays, S, total_steps),
        "roofline": {
            "kernel": "k_field_fp32" if prec == _lib.FP32 else "k_field_bf16",
            "bound": "mfma",
            "achieved": achieved,
            "peak": PEAK_TFLOPS[dtype],
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS[dtype],
            "traffic": field_traffic_bytes("k_field_fp32" if prec == _lib.FP32 else "k_field_bf16",
                                           cfg.name),
            "traffic_unit": "bytes per launch (HBM, counters)",
            "flop_per_sample": fl_sample,
        },
        "integrate": {
            "rays": int(o.shape[0]), "ms": integ_ms, "rays_per_s": o.shape[0] / (integ_ms * 1e-3),
            "voxel_updates": updates, "updates_per_s": updates / (integ_ms * 1e-3),
            # 28 B per ray + a 12 B read-modify-write (int64 sum, uint32 count) per update
            "hbm_GB_per_s": (28 * o.shape[0] + 24 * updates) / (integ_ms * 1e-3) / 1e9,
            "hbm_frac": (28 * o.shape[0] + 24 * updates) / (integ_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "finalize_ms": fin_ms,
            "ray_order": "8x8 pixel blocks per view" if args.ray_order == "tile8" else "row by row",
            "paper_context": "1.445e6 rays/s (0.692 us/ray, 39.0 M rays in 27.02 s, GPU unnamed)",
        },
    }

    # ---- the small scene (64^3 volume, 64-wide networks) and its 4096-ray
    # view: eager renders against replays of one recorded HIP graph, host
    # wall clock over 100 back-to-back renders each, and the median latency
    # of single frames (launch, run, wait)
    if args.graph:
        cs = get_config("c1")
        gs_, ss_ = cs.grid, cs.sampling
        grid_s = ops.make_grid(gs_.n, gs_.lo, gs_.h, gs_.d_t, gs_.d_s, gs_.nb_radius,
                               gs_.m_consec)
        field_s = ops.Field(cs.sdf.width, cs.sdf.n_hidden, cs.sdf.pe_freqs, cs.sdf.skip_at,
                            cs.sdf.n_feat, cs.color.n_hidden, cs.sdf.beta, cs.in_center,
                            cs.in_scale, cs.sdf_params(), cs.color_params())
        Rs = TsdfRenderer(grid_s, field_s, ss_.rho_num, ss_.rho_den, ss_.n_min, ss_.n_max,
                          cs.neus_s, ss_.t_far, prec)
        so, sv, sd = cs.integration_rays()
        Rs.integrate(dev(so), dev(sv), dev(sd))
        Rs.finalize(want_v=False)
        o_s, v_s = (dev(x) for x in cs.render_rays())
        for _ in range(5):
            Rs.render(o_s, v_s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(100):
            Rs.render(o_s, v_s)
        torch.cuda.synchronize()
        eager_ms = (time.perf_counter() - t0) / 100 * 1e3
        graph_r, out_g = Rs.capture(o_s, v_s)
        graph_r.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(100):
            graph_r.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) / 100 * 1e3
        # latency of one frame: launch, run and wait, one at a time
        lat = {}
        for name_, fn_ in (("eager", lambda: Rs.render(o_s, v_s)), ("graph", graph_r.replay)):
            ts_ = []
            for _ in range(50):
                t0 = time.perf_counter()
                fn_()
                torch.cuda.synchronize()
                ts_.append((time.perf_counter() - t0) * 1e3)
            lat[name_] = float(np.median(ts_))
        ref_s = Rs.render(o_s, v_s)
        torch.cuda.synchronize()
        result["graph"] = {"workload": "c1: 4096-ray view of the 64^3 volume, 64-wide networks",
                           "eager_ms": eager_ms, "graph_ms": graph_ms,
                           "speedup": eager_ms / graph_ms,
                           "frame_latency_ms": lat,
                           "rays_per_s_graph": 4096 / (graph_ms * 1e-3),
                           "equal_to_eager": bool(torch.equal(out_g["rgb"], ref_s["rgb"]))}
        log(f"graph: {result['graph']}")
        del graph_r, out_g, Rs, field_s

    # ---- sampling density swept over the paper's 13-28 samples per ray:
    # rho samples per traversed voxel (the default rho is the main step)
    sweep = {}
    rho0 = R.rho
    for num, den in ((1, 3), (rho0[0], rho0[1]), (5, 8), (5, 7)) if args.rho_sweep else ():
        R.rho = (num, den)
        for _ in range(args.warmup):
            R.render(ro_d, rv_d)
        torch.cuda.synchronize()
        start.record()
        for _ in range(args.steps):
            out_s = R.render(ro_d, rv_d)
        end.record()
        torch.cuda.synchronize()
        ms_s = start.elapsed_time(end) / args.steps
        sweep[f"{num}/{den}"] = {"ms_per_step": ms_s, "rays_per_s": n_rays / (ms_s * 1e-3),
                                 "samples_per_ray": int(out_s["s_total"].item()) / n_rays}
    R.rho = rho0
    if sweep:
        result["rho_sweep"] = sweep
    log(f"rho sweep: {sweep}")

    # ---- the other precision on the same step
    other = _lib.FP32 if prec == _lib.BF16 else _lib.BF16
    if args.no_other:
        other = None
    if other is not None:
        oname = "f32" if other == _lib.FP32 else "bf16"
        R.precision = other
        for _ in range(args.warmup):
            R.render(ro_d, rv_d)
        ev_o = {}
        torch.cuda.synchronize()
        start.record()
        for _ in range(args.steps):
            R.render(ro_d, rv_d, events=ev_o)
        end.record()
        torch.cuda.synchronize()
        R.precision = prec
        ms_o = start.elapsed_time(end) / args.steps
        field_o = float(np.mean([a.elapsed_time(b) for a, b in ev_o["field"]]))
        ach_o = S * fl_sample / (field_o * 1e-3) / 1e12
        result[oname] = {
            "ms_per_step": ms_o, "rays_per_s": n_rays / (ms_o * 1e-3), "field_ms": field_o,
            "roofline": {"kernel": "k_field_bf16" if other == _lib.BF16 else "k_field_fp32",
                         "bound": "mfma", "achieved": ach_o, "peak": PEAK_TFLOPS[oname],
                         "unit": "TFLOP/s", "frac": ach_o / PEAK_TFLOPS[oname],
                         "traffic": field_traffic_bytes(
                             "k_field_bf16" if other == _lib.BF16 else "k_field_fp32", cfg.name)},
        }
        log(f"{oname}: {ms_o:.3f} ms/step")

    # ---- FP32 operands as three-part BF16 products (FP32 accuracy on the
    # BF16 matrix cores: six BF16 products per FP32 product) on the same step
    if args.split:
        R.precision = _lib.BF16X6
        for _ in range(args.warmup):
            R.render(ro_d, rv_d)
        ev_x = {}
        torch.cuda.synchronize()
        start.record()
        for _ in range(args.steps):
            R.render(ro_d, rv_d, events=ev_x)
        end.record()
        torch.cuda.synchronize()
        R.precision = prec
        ms_x = start.elapsed_time(end) / args.steps
        field_x = float(np.mean([a.elapsed_time(b) for a, b in ev_x["field"]]))
        alg_x = S * fl_sample / (field_x * 1e-3) / 1e12
        field_f32 = field_ms if prec == _lib.FP32 else result.get("f32", {}).get("field_ms")
        result["f32_bf16x6"] = {
            "ms_per_step": ms_x, "rays_per_s": n_rays / (ms_x * 1e-3), "field_ms": field_x,
            "field_speedup_vs_f32": (field_f32 / field_x) if field_f32 else None,
            "fp32_equivalent_TFLOP_s": alg_x,
            "roofline": {"kernel": "k_field_fp32 (three-part BF16 products)", "bound": "mfma",
                         "achieved": 6 * alg_x, "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                         "frac": 6 * alg_x / PEAK_TFLOPS["bf16"],
                         "work": "6 BF16 MFMA products per FP32 product",
                         "traffic": field_traffic_bytes("k_field_fp32_split", cfg.name)},
        }
        log(f"f32 as bf16x6: {ms_x:.3f} ms/step, field {field_x:.2f} ms")

    # ---- coarse + fine inside the TSDF bound ("Ours (full)"): the adaptive
    # samples as coarse sets (SDF only), n_fine fine points per ray, the field
    # at the merged sections, compositing
    full_ms = None
    if args.full_fine > 0:
        nf = args.full_fine
        for _ in range(args.warmup):
            R.render_full(ro_d, rv_d, nf)
        ev_f = {}
        torch.cuda.synchronize()
        start.record()
        for _ in range(args.steps):
            out_f = R.render_full(ro_d, rv_d, nf, events=ev_f)
        end.record()
        torch.cuda.synchronize()
        full_ms = start.elapsed_time(end) / args.steps
        S_f = int(out_f["s_total"].item())
        result[f"full_{nf}"] = {
            "ms_per_step": full_ms, "rays_per_s": n_rays / (full_ms * 1e-3), "n_fine": nf,
            "precision": dtype,
            "samples_per_ray": {"coarse_sdf_only": S / n_rays, "rendered": S_f / n_rays,
                                "field_evaluations": (S + S_f) / n_rays},
            "stage_ms": {k: float(np.mean([a.elapsed_time(b) for a, b in v_]))
                         for k, v_ in ev_f.items()},
        }
        log(f"full (+{nf} fine): {full_ms:.3f} ms/step, {S_f / n_rays:.2f} rendered samples/ray")

    # ---- Table 1's counting on the training rays (this workload's bounds),
    # then the same scene fused from density-field-like depths in NeRF mode
    # (D_T = 39h, D_s = 27h, 7^3 neighbourhood): counting, integration and
    # a render of the view with those bounds
    def table1(rr, o_, v_, d_):
        bt = ops.ray_bounds(rr.grid, rr.flags, o_, v_, rr.t_far)
        ti, to = ops.ray_range(rr.grid, o_, v_)
        c = ops.bound_stats(ti, to, bt, d_).cpu().numpy().tolist()
        q = float(1 << 24)
        return {"rays_with_depth": c[0], "failed": c[1], "failed_frac": c[1] / max(c[0], 1),
                "original_range_m": c[2] / q / max(c[0], 1), "reduced_range_m": c[3] / q / max(c[0], 1)}
    nerf_name = cfg.name + "n"
    if not args.no_table1:
        result["table1"] = {cfg.name: table1(R, o_d, v_d, d_d)}
        try:
            cfg_n = get_config(nerf_name)
        except KeyError:
            cfg_n = None
        if cfg_n is not None:
            gn = cfg_n.grid
            _, _, dn = cfg_n.integration_rays(tile=8 if args.ray_order == "tile8" else 0)
            dn_d = dev(dn)
            grid_n = ops.make_grid(gn.n, gn.lo, gn.h, gn.d_t, gn.d_s, gn.nb_radius, gn.m_consec)
            Rn = TsdfRenderer(grid_n, field, s.rho_num, s.rho_den, s.n_min, s.n_max, cfg.neus_s,
                              s.t_far, prec)
            nup_n = torch.zeros(1, dtype=torch.int64, device="cuda")
            Rn.state = ops.new_state(grid_n)
            torch.cuda.synchronize()
            e0.record()
            Rn.integrate(o_d, v_d, dn_d, batch=o.shape[0], n_updates=nup_n)
            e1.record()
            torch.cuda.synchronize()
            integ_n = e0.elapsed_time(e1)
            Rn.finalize()
            t1n = table1(Rn, o_d, v_d, dn_d)
            for _ in range(args.warmup):
                Rn.render(ro_d, rv_d)
            torch.cuda.synchronize()
            start.record()
            for _ in range(args.steps):
                out_n = Rn.render(ro_d, rv_d)
            end.record()
            torch.cuda.synchronize()
            ms_n = start.elapsed_time(end) / args.steps
            S_n = int(out_n["s_total"].item())
            t1n.update({"integrate_ms": integ_n, "voxel_updates": int(nup_n.item()),
                        "render_ms_per_step": ms_n, "render_rays_per_s": n_rays / (ms_n * 1e-3),
                        "samples_per_ray": S_n / n_rays,
                        "bounds": f"D_T={gn.d_t / gn.h:g}h, D_s={gn.d_s / gn.h:g}h, "
                                  f"{2 * gn.nb_radius + 1}^3, M={gn.m_consec}",
                        "depths": "exact depths plus seeded N(0, (2h)^2) error, 1% floaters "
                                  "uniform in [0.3, 1] x depth"})
            result["table1"][nerf_name] = t1n
            log(f"table1 {cfg.name}: {result['table1'][cfg.name]}; {nerf_name}: {t1n}")
            del Rn, dn_d

    # ---- recovery: bounded render, then rays with weight sum < tau rendered
    # again over their initial range by the 64+64 hierarchical sampler
    if args.recover_tau > 0:
        tau = args.recover_tau
        for _ in range(args.warmup):
            R.render_recover(ro_d, rv_d, tau)
        ev_r = {}
        torch.cuda.synchronize()
        start.record()
        for _ in range(args.steps):
            out_r = R.render_recover(ro_d, rv_d, tau, events=ev_r)
        end.record()
        torch.cuda.synchronize()
        rec_ms = start.elapsed_time(end) / args.steps
        n_rec = int(out_r["n_recovered"])
        result["recover"] = {
            "tau": tau, "ms_per_step": rec_ms, "rays_per_s": n_rays / (rec_ms * 1e-3),
            "rays_recovered": n_rec, "frac_recovered": n_rec / n_rays,
            "samples_per_ray_total": (S + 192 * n_rec) / n_rays,
            "stage_ms": {k: float(np.mean([a.elapsed_time(b) for a, b in v_]))
                         for k, v_ in ev_r.items()},
        }
        log(f"recover (tau {tau}): {rec_ms:.3f} ms/step, {n_rec} rays recovered")

    # ---- one TSDF-bounded training step (8192 rays + 8192 eikonal points)
    if cfg.name in ("c2", "c3", "c4") and not args.no_train:
        from paper_2311_17878_amd.autograd import train_step
        tro, trv, ttarget = cfg.training_batch(8192, seed=0)
        teik = cfg.eikonal_points(8192, seed=0)
        tro, trv, ttarget, teik = dev(tro), dev(trv), dev(ttarget), dev(teik)
        n_t = max(1, min(args.steps, 5))
        for tname, tprec in (("train_step", _lib.FP32), ("train_step_bf16", _lib.BF16),
                             ("train_step_bf16x6", _lib.BF16X6)):
            out_t = train_step(R, tro, trv, ttarget, teik, precision=tprec)   # warm-up
            torch.cuda.synchronize()
            start.record()
            for _ in range(n_t):
                out_t = train_step(R, tro, trv, ttarget, teik, precision=tprec)
            end.record()
            torch.cuda.synchronize()
            tms = start.elapsed_time(end) / n_t
            S_t = int(out_t[4])
            t_flop = S_t * fl_sample + (S_t + 8192) * train_flops_per_row(cfg.sdf, cfg.color)
            t_peak = PEAK_TFLOPS["f32" if tprec == _lib.FP32 else "bf16"]
            # the split form runs six BF16 products per FP32 one
            t_work = 6 if tprec == _lib.BF16X6 else 1
            result[tname] = {
                "rays": 8192, "eikonal_points": 8192, "samples": S_t, "ms_per_step": tms,
                "rays_per_s": 8192 / (tms * 1e-3),
                "flop_per_step": t_flop, "tflop_per_s": t_flop / (tms * 1e-3) / 1e12,
                "mfma_frac": t_work * t_flop / (tms * 1e-3) / 1e12 / t_peak,
                "loss_rgb": float(out_t[0].item()), "loss_eik": float(out_t[1].item()),
                "precision": {_lib.FP32: "f32 (forward and backward)",
                              _lib.BF16: "bf16 product inputs, f32 accumulation (forward and "
                                         "backward)",
                              _lib.BF16X6: "f32 operands as three-part bf16 products (six per "
                                           "f32 product, f32 accumulation; forward and "
                                           "backward)"}[tprec],
            }
            log(f"{tname}: {tms:.2f} ms")
        # a multi-step training loop: train_step, Adam over the field's
        # parameters, repack of the forward operands, on 10 pre-uploaded
        # batches in turn (a separate field, so the render legs keep theirs)
        from paper_2311_17878_amd.autograd import train, Adam
        bl = []
        for k in range(10):
            bo, bv, bt = cfg.training_batch(8192, seed=100 + k)
            bl.append((dev(bo), dev(bv), dev(bt), dev(cfg.eikonal_points(8192, seed=100 + k))))
        n_loop = max(2, min(args.steps, 10))
        for lname, lprec in (("train_loop", _lib.FP32), ("train_loop_bf16", _lib.BF16),
                             ("train_loop_bf16x6", _lib.BF16X6)):
            fl = ops.Field(cfg.sdf.width, cfg.sdf.n_hidden, cfg.sdf.pe_freqs, cfg.sdf.skip_at,
                           cfg.sdf.n_feat, cfg.color.n_hidden, cfg.sdf.beta, cfg.in_center,
                           cfg.in_scale, cfg.sdf_params(), cfg.color_params())
            saved = R.field
            R.field = fl
            opt = Adam(fl, lr=5e-4)
            train(R, lambda k: bl[k % 10], 1, precision=lprec, opt=opt)       # warm-up
            torch.cuda.synchronize()
            start.record()
            hist, _ = train(R, lambda k: bl[(k + 1) % 10], n_loop, precision=lprec, opt=opt)
            end.record()
            torch.cuda.synchronize()
            R.field = saved
            lms = start.elapsed_time(end) / n_loop
            result[lname] = {
                "steps": n_loop, "ms_per_step": lms, "rays_per_s": 8192 / (lms * 1e-3),
                "loss_rgb_first": hist[0][0], "loss_rgb_last": hist[-1][0],
                "optimizer": "Adam lr 5e-4 (device), packed operands rebuilt every step",
            }
            log(f"{lname}: {lms:.2f} ms/step, loss {hist[0][0]:.5f} -> {hist[-1][0]:.5f}")

    # ---- filling unseen voxels (Sec. 4.3) on a copy of the fused volume:
    # per round the flags, the frontier and its rays on the device, depths
    # from a sensor at each ray's origin (host, not timed), and the fill
    # rays fused; then the render step on the filled volume
    if args.fill_rounds > 0:
        from synth.scenes import sensor_depth
        scene = cfg.scene()
        Rf = TsdfRenderer(grid, field, s.rho_num, s.rho_den, s.n_min, s.n_max, cfg.neus_s,
                          s.t_far, prec)
        Rf.state = R.state.clone()
        N = g.n_vox
        seen = lambda st: int((st[8 * N: 12 * N].view(torch.int32) != 0).sum().item())
        rounds = []
        seen0 = seen(Rf.state)
        cap = 1 << 22
        for _ in range(args.fill_rounds):
            torch.cuda.synchronize()
            e0.record()
            Rf.finalize(want_v=False)
            e1.record()
            e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e2.record()
            fr = ops.frontier(grid, Rf.state, Rf.flags, cap)
            e3.record()
            n = int(fr["n"].item())
            r_ = {"frontier": n, "finalize_ms": e0.elapsed_time(e1),
                  "frontier_ms": e2.elapsed_time(e3)}
            if n == 0:
                rounds.append(r_)
                break
            k = min(n, cap)
            h0 = time.time()
            dfill = sensor_depth(scene, fr["o"][:k].cpu().numpy(), fr["v"][:k].cpu().numpy())
            r_["host_depth_s"] = time.time() - h0
            dfill = dev(dfill)
            nup_f = torch.zeros(1, dtype=torch.int64, device="cuda")
            torch.cuda.synchronize()
            e0.record()
            Rf.integrate(fr["o"][:k], fr["v"][:k], dfill, batch=k, n_updates=nup_f)
            e1.record()
            torch.cuda.synchronize()
            r_.update(integrate_ms=e0.elapsed_time(e1), voxel_updates=int(nup_f.item()),
                      seen_after=seen(Rf.state))
            rounds.append(r_)
        Rf.finalize()
        for _ in range(args.warmup):
            Rf.render(ro_d, rv_d)
        torch.cuda.synchronize()
        start.record()
        for _ in range(args.steps):
            out_fl = Rf.render(ro_d, rv_d)
        end.record()
        torch.cuda.synchronize()
        ms_fl = start.elapsed_time(end) / args.steps
        result["fill_unseen"] = {
            "voxels": N, "seen_before": seen0, "rounds": rounds,
            "render_ms_per_step": ms_fl, "render_rays_per_s": n_rays / (ms_fl * 1e-3),
            "samples_per_ray": int(out_fl["s_total"].item()) / n_rays,
        }
        log(f"fill unseen: {rounds}; render after {ms_fl:.3f} ms/step")
        del Rf, fr

    # ---- two-level volume (bricks of 8^3 voxels; integration sums only
    # where the truncation band reaches) of the room at this grid's
    # resolution and with 4x finer voxels: time, memory against the dense
    # state, flags checked equal to the dense volume's, and the bounds of the
    # view on each resolution
    if args.two_level:
        from dataclasses import replace as _replace
        tl = {}
        o_b = [(o_d, v_d, d_d)]
        for fac in (1, 4):
            gg = g if fac == 1 else _replace(g, n=tuple(x * fac for x in g.n), h=g.h / fac,
                                             d_t=g.d_t / fac, d_s=g.d_s / fac)
            grid_t = ops.make_grid(gg.n, gg.lo, gg.h, gg.d_t, gg.d_s, gg.nb_radius, gg.m_consec)
            ops.sparse_integrate(grid_t, o_b)                     # warm-up
            torch.cuda.synchronize()
            e0.record()
            sp = ops.sparse_integrate(grid_t, o_b)
            e1.record()
            torch.cuda.synchronize()
            t_int = e0.elapsed_time(e1)
            e0.record()
            _, fl_t = ops.sparse_finalize(grid_t, sp, want_v=False)
            e1.record()
            torch.cuda.synchronize()
            t_fin = e0.elapsed_time(e1)
            st_t = ops.new_state(grid_t)
            torch.cuda.synchronize()
            e0.record()
            ops.integrate(grid_t, st_t, o_d, v_d, d_d)
            e1.record()
            torch.cuda.synchronize()
            t_dense = e0.elapsed_time(e1)
            _, fl_dense = ops.finalize(grid_t, st_t, want_v=False)
            same = bool(torch.equal(fl_t, fl_dense))
            del st_t, fl_dense
            bt = ops.ray_bounds(grid_t, fl_t, ro_d, rv_d, s.t_far)
            hit = bt["status"] == 0
            nbr = sp["meta"].numel() // 72
            tl[f"{gg.n[0]}^3"] = {
                "h_m": gg.h, "bricks": nbr, "band_bricks": sp["n_band"],
                "band_frac": sp["n_band"] / nbr,
                "two_level_bytes": sp["meta"].numel() + sp["pool"].numel(),
                "dense_state_bytes": 12 * gg.n_vox, "flag_bytes": gg.n_vox,
                "integrate_ms": t_int, "finalize_ms": t_fin, "dense_integrate_ms": t_dense,
                "flags_equal_dense": same,
                "mean_bound_m": float((bt["t_f"] - bt["t_n"])[hit].mean().item()),
                "mean_bound_voxels": float(bt["n_vox"][hit].float().mean().item()),
            }
            if fac > 1:
                # the view rendered on the finer flags (same field, same rules)
                Rt = TsdfRenderer(grid_t, field, s.rho_num, s.rho_den, s.n_min, s.n_max,
                                  cfg.neus_s, s.t_far, prec)
                Rt.flags = fl_t
                for _ in range(args.warmup):
                    Rt.render(ro_d, rv_d)
                torch.cuda.synchronize()
                start.record()
                for _ in range(args.steps):
                    out_t = Rt.render(ro_d, rv_d)
                end.record()
                torch.cuda.synchronize()
                ms_t = start.elapsed_time(end) / args.steps
                tl[f"{gg.n[0]}^3"].update(
                    render_ms_per_step=ms_t, render_rays_per_s=n_rays / (ms_t * 1e-3),
                    render_samples_per_ray=int(out_t["s_total"].item()) / n_rays)
                del Rt, out_t
            del sp, fl_t, bt
            torch.cuda.empty_cache()
        result["two_level"] = tl
        log(f"two-level volume: {tl}")

    if not args.no_hs:
        for _ in range(1):
            R.render_hs(ro_d, rv_d)
        torch.cuda.synchronize()
        ev_hs = {}
        start.record()
        for _ in range(args.hs_steps):
            R.render_hs(ro_d, rv_d, events=ev_hs)
        end.record()
        torch.cuda.synchronize()
        hs_ms = start.elapsed_time(end) / args.hs_steps
        result["hs_64_64"] = {
            "ms_per_step": hs_ms, "rays_per_s": n_rays / (hs_ms * 1e-3), "samples_per_ray": 192,
            "stage_ms": {k: float(np.mean([a.elapsed_time(b) for a, b in v_]))
                         for k, v_ in ev_hs.items()},
            "speedup_tsdf_vs_hs": hs_ms / ms,
            "speedup_full_vs_hs": hs_ms / full_ms if full_ms else None,
        }
        for v_ in result.get("rho_sweep", {}).values():
            v_["speedup_vs_hs"] = hs_ms / v_["ms_per_step"]
        log(f"hs 64+64: {hs_ms:.2f} ms/step")

    if args.c5 and cfg.name in ("c2", "c3", "c4"):
        result["c5_panorama_bf16"] = panorama_leg(max(3, args.steps // 2), 1,
                                                  8 if args.ray_order == "tile8" else 0)

    if not args.no_cpu_baseline:
        try:
            result["cpu_baseline"] = cpu_baseline(cfg, ro, rv, args.cpu_rays)
        except FileNotFoundError as e:
            result["cpu_baseline"] = None
            log(f"cpu baseline skipped: {e}")

    print(json.dumps(result))


if __name__ == "__main__":
    main()
