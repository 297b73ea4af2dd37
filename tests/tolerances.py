"""Parity bounds of the GPU tests, in one place.

Applies are compared on their kernel part: the error max |Y - Y_ref| is divided by the largest element of
the oracle's kernel part Y_ref - D X (D the diagonal of transition energies, which every precision
evaluates in FP64), not by max |Y|, which the diagonal dominates.  Each bound sits about ten times above
what the split kernels measure, and far below what a plain bf16 product gives (numpy emulation of the
direct term's dataflow at the 4x4x4 workload, tests/test_tolerance_emulation.py: kernel-part error
2.9e-3 for bf16 hi parts only, 4.1e-6 for the two-term split, 4.6e-8 for FP32 storage):

* FP64: sums of <= 10^5 FP64 terms in another order;
* FP32: 2^-24 per stored operand plus FP32 accumulation inside a tile;
* BF16x3: the two-term split keeps 16 significant bits per operand (2^-17 relative rounding).

Gradients with respect to W(q) / W(R) have no diagonal and are compared relative to their largest element.
"""
import numpy as np

import oracle as O

KERNEL_TOL = {"f64": 1e-11, "f32": 2e-6, "bf16x3": 5e-5}
GRAD_TOL = {"f64": 1e-11, "f32": 1e-5, "bf16x3": 1e-4}


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def kernel_err(Y, ref, DX):
    """max |Y - ref| / max |ref - DX|: error relative to the kernel part of the reference."""
    Y, ref, DX = np.asarray(Y), np.asarray(ref), np.asarray(DX)
    return np.abs(Y - ref).max() / np.abs(ref - DX).max()


def diag_times(prob, X, rows=None):
    """D X for the transition energies of a problem (rows: the k rows to keep, in order)."""
    te = O.transition_energies(prob)                       # [Nk][(c v)]
    X = np.asarray(X).reshape(prob.Nk, te.shape[1], -1)
    out = te[:, :, None] * X
    if rows is not None:
        out = out[list(rows)]
    return out.reshape(-1, X.shape[2])
