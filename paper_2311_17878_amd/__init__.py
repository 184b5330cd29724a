"""TSDF-Sampling hot path on AMD MI355X (gfx950).

libtsdfs.so (HIP kernels behind a C ABI, see include/tsdfs.h) does all the
work; this package only marshals torch device tensors into its calls.
"""
from ._lib import TsdfsError, load, lib_path  # noqa: F401
