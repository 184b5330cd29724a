"""The oracle's C code (voxel walk, integration, Alg. 1 bounds, grid ranges)
built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host code
only) and driven through its Python wrappers in a child process on rays of
the small scene, including rays that miss, start inside the grid, or carry
invalid depths: no sanitizer report."""
import os
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
from oracle import _native
_native.LIB = sys.argv[2]
_native._lib = None
from oracle import tsdf
from synth.configs import get_config
cfg = get_config("c1")
g = cfg.grid
o, v, d = cfg.integration_rays(views=[0, 3])
rng = np.random.default_rng(0)
pick = rng.choice(o.shape[0], 3000, replace=False)
o, v, d = o[pick], v[pick], d[pick]
d[::17] = np.nan
d[::23] = -1.0
d[::29] = np.inf
o2 = rng.uniform(-1.2, 1.2, (500, 3)).astype(np.float32)        # inside and around the grid
v2 = rng.normal(size=(500, 3))
v2 = (v2 / np.linalg.norm(v2, axis=1, keepdims=True)).astype(np.float32)
v2[::50] = 0.0                                                    # invalid directions
st = tsdf.integrate(g, np.concatenate([o, o2]), np.concatenate([v, v2]),
                    np.concatenate([d, np.full(500, 0.7, np.float32)]))
fl = tsdf.flags(g, tsdf.finalize(g, st))
b = tsdf.bounds(g, fl, np.concatenate([o, o2]), np.concatenate([v, v2]))
t_in, t_out = tsdf.ray_range(g, o2, v2)
for k in range(0, 500, 25):
    tsdf.walk(g, o2[k], v2[k])
print("ok", st.updates, int((b["status"] == 0).sum()))
'''


def test_oracle_c_code_under_sanitizers():
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    ubsan = subprocess.check_output(["gcc", "-print-file-name=libubsan.so"], text=True).strip()
    with tempfile.TemporaryDirectory() as tmp:
        lib = os.path.join(tmp, "_tsdf_oracle_san.so")
        subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                               "-fno-omit-frame-pointer", "-o", lib,
                               os.path.join(ROOT, "oracle", "tsdf_oracle.c"), "-lm"])
        env = dict(os.environ, LD_PRELOAD=asan + ":" + ubsan,
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([sys.executable, "-c", CHILD, ROOT, lib], env=env, capture_output=True,
                           text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    assert r.stdout.startswith("ok")
