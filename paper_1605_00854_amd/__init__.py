"""MI355X-native simulator of probabilistic Boolean networks (arXiv:1605.00854).

The package is a thin binding over the C-ABI library libpbn_amd.so (HIP kernels
for gfx950 plus host-side preparation).  Import `api` for the calls.
"""
__all__ = ["api"]
