"""Write the oracle's full-size TSDF flags for a workload (tests/golden/).

Calls only the CPU oracle (oracle/) on the seeded synthetic inputs (synth/):
integrates every training ray, finalises V, builds the Alg. 1 voxel flags and
stores them bit-packed, together with V and the update count at a seeded
sample of voxels and the integration totals.  Usage:

    python tests/golden/make_volume_golden.py c2
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synth.configs import get_config  # noqa: E402
from oracle import tsdf  # noqa: E402


def main(name, n_sample=200_000, views_per_batch=10):
    cfg = get_config(name)
    g = cfg.grid
    n_views = len(cfg.integ_views(cfg.scene()))
    st = tsdf.Integration(g)
    t0 = time.time()
    for s in range(0, n_views, views_per_batch):
        o, v, d = cfg.integration_rays(views=range(s, min(n_views, s + views_per_batch)))
        st.add(o, v, d, tie_eps=2.0 ** -36)
        print(f"views {s}..{s + views_per_batch}: {st.updates} updates, {time.time() - t0:.0f} s",
              flush=True)
    V = tsdf.finalize(g, st)
    fl = tsdf.flags(g, V).ravel()
    rng = np.random.Generator(np.random.PCG64(0))
    idx = np.sort(rng.choice(g.n_vox, n_sample, replace=False))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_volume.npz")
    np.savez_compressed(out, flag0=np.packbits(fl & 1), flag1=np.packbits((fl >> 1) & 1),
                        sample_idx=idx, sample_V=V.ravel()[idx], sample_cnt=st.cnt[idx],
                        updates=st.updates, ties=st.ties, invalid=st.invalid,
                        n_vox=g.n_vox)
    print("wrote", out, os.path.getsize(out), "bytes; ties", st.ties)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c2")
