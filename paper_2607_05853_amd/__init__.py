"""MI355X (gfx950) dual-k-mesh Tamm-Dancoff BSE hot path.

The compute path lives in libbse.so (HIP kernels behind a C ABI, declared
in include/bse.h); `bse` is its thin ctypes binding and `autograd` wraps the
apply and its adjoint as torch.autograd.Functions.
"""
__all__ = ["bse"]
