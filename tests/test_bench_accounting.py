"""The benchmark's accounting, checked on the CPU: the algorithmic FLOP of a
field evaluation and of a training row written out here by hand from the
room network's shapes (one term per product of the implemented backward),
the traffic figure's tie to the kernel sources, and the one-GPU guard."""
import hashlib
import os
import subprocess
import sys

from synth.configs import get_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

# room network: encoding 39 -> 256, 256, 256 -> 217 (the layer before the
# skip leaves room for the 39 re-injected inputs) -> 256 x 4 -> 257 outputs;
# colour 265 -> 256 x 4 -> 3
SDF = [(39, 256), (256, 256), (256, 256), (256, 217), (256, 256), (256, 256), (256, 256),
       (256, 256)]
OUT = (256, 257)
COL = [(265, 256), (256, 256), (256, 256), (256, 256), (256, 3)]


def test_field_flop_per_sample_room():
    fwd = sum(i * o for i, o in SDF) + OUT[0] * OUT[1]
    rev = sum(i * o for i, o in SDF) + OUT[0]            # only the f row goes back
    col = sum(i * o for i, o in COL)
    assert (fwd, rev, col) == (524544, 459008, 265216)
    cfg = get_config("c2")
    assert cfg.sdf.layer_dims() == SDF + [OUT] and cfg.color.layer_dims() == COL
    assert bench.field_flops_per_sample(cfg.sdf, cfg.color) == (2 * (fwd + rev + col), 2 * fwd)
    assert 2 * (fwd + rev + col) == 2497536


def test_training_flop_per_row_room():
    io = lambda d: d[0] * d[1]
    terms = []
    terms += [io(d) for d in SDF] + [io(OUT)]                     # forward recomputed
    terms += [io(d) for d in SDF[1:]] + [io(SDF[0])]              # reverse pass, encoding rows
    terms += [io(d) for d in COL]                                 # colour forward
    terms += [2 * io(d) for d in COL]                             # colour dW and dX
    terms += [2 * io(SDF[0])] + [2 * io(d) for d in SDF[1:]]      # adjoint of the reverse pass
    terms += [2 * io(OUT)] + [io(d) for d in SDF] + [io(d) for d in SDF[1:]]  # first order
    macs = sum(terms)
    assert macs == 3735552
    cfg = get_config("c2")
    assert bench.train_flops_per_row(cfg.sdf, cfg.color) == 2 * macs


def test_traffic_follows_the_kernel_sources(monkeypatch):
    m = hashlib.sha256()
    for f in bench.FIELD_SOURCES["k_field_bf16"]:
        with open(os.path.join(ROOT, "paper_2311_17878_amd", "csrc", f), "rb") as fh:
            m.update(fh.read())
    ok = {"sha256_16": m.hexdigest()[:16], "fetch_kib": 100.0, "write_kib": 50.0}
    monkeypatch.setitem(bench.TRAFFIC, "k_field_bf16", ok)
    assert bench.field_traffic_bytes("k_field_bf16", "c2") == 1024.0 * (100.0 * 2 + 50.0)
    assert bench.field_traffic_bytes("k_field_bf16", "c1") is None       # other workload
    monkeypatch.setitem(bench.TRAFFIC, "k_field_bf16", dict(ok, sha256_16="0" * 16))
    assert bench.field_traffic_bytes("k_field_bf16", "c2") is None       # sources changed


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
