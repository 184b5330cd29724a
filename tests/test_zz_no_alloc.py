"""The placement entry point without a workspace (its scan partials in the
library's static device array) against place_samples with a caller
workspace: bit-identical outputs on two calls in a row, the second with
fewer rays, and the size limit of the static array rejected on the host."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _bounds(R, seed):
    """Seeded bounds of R rays: every status, bound lengths of 0..300 voxels."""
    rng = np.random.default_rng(seed)
    status = rng.choice([0, 0, 0, 1, 2, 3], R).astype(np.uint8)
    n_vox = rng.integers(0, 300, R).astype(np.int32)
    t_n = rng.uniform(0.0, 4.0, R).astype(np.float32)
    t_f = (t_n + rng.uniform(0.0, 3.0, R)).astype(np.float32)
    dev = lambda a: torch.as_tensor(a).cuda()
    return dict(t_n=dev(t_n), t_f=dev(t_f), n_vox=dev(n_vox), status=dev(status))


@pytest.mark.parametrize("sizes", [(300_001, 4_097), (1_000, 1)])
def test_place_noalloc_matches_place(sizes):
    from paper_2311_17878_amd import ops
    for k, R in enumerate(sizes):
        b = _bounds(R, seed=10 + k)
        ref = ops.place(b, 1, 2, 1, 64, sync=True)
        got = ops.place(b, 1, 2, 1, 64, sync=True, noalloc=True)
        torch.cuda.synchronize()
        assert got["S"] == ref["S"]
        for key in ("counts", "offsets", "t", "dt", "ray_id"):
            assert torch.equal(got[key], ref[key]), (R, key)
        assert int(got["s_total"].item()) == ref["S"]


def test_place_noalloc_size_limit():
    from paper_2311_17878_amd import _lib as L
    lib = L.load()
    z = torch.zeros(16, device="cuda")
    p = ctypes.c_void_p(z.data_ptr())
    R = 4 * 1024 * 1024 + 1      # one ray above the static array's limit
    rc = lib.place_samples_noalloc(p, p, p, p, R, 1, 2, 1, 1, p, p, p, p, p, 0, p, None, None)
    assert rc == L.TSDFS_EINVAL
    assert b"exceeds" in L.load().tsdfs_last_error()
