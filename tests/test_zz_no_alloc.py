"""The allocation-free interpolation entry point against the allocating one, through the C ABI: two calls in
a row on the shared static workspace, the second with a smaller input, each equal to bse_interpolate_W
(the same kernels; FP64 bound 1e-12 of the largest element, in practice identical)."""
import numpy as np
import pytest
import torch

from synth import dense_kmesh, make_problem

pytestmark = pytest.mark.gpu


def T(a, dt=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a)).to(torch.device("cuda:0"), dt)


def rel(a, b):
    return ((a - b).abs().max() / b.abs().max()).item()


def test_interpolate_noalloc_matches_allocating_entry_point():
    from paper_2607_05853_amd import bse as B
    cases = [(make_problem("mesh8_ao64", 0, "G2"), "f64"),               # 512 q x 125 R, N_aux 256
             (make_problem("mesh4_ao16", 1, "G2", coarse=(3, 3, 2)), "f32")]  # 64 q x 27 R, N_aux 64
    for p, prec in cases:
        kq = dense_kmesh(p.nk)
        W_R = T(p.W_R)
        ref = B.interpolate_W(W_R, p.R, p.w_R, kq, out_prec=prec)
        out = torch.full_like(ref, float("nan"))
        B.interpolate_W_noalloc(W_R, p.R, p.w_R, kq, out, out_prec=prec)
        torch.cuda.synchronize()
        err = rel(out, ref)
        print("[noalloc %s, %d q x %d R] rel diff %.1e, identical %s" %
              (prec, len(kq), len(p.R), err, torch.equal(out, ref)), flush=True)
        assert err < 1e-12
