"""GPU parity at the largest workload: 16x16x16 dense mesh (4096 k) from a 6x6x6 coarse mesh, N_ao = 128,
n_v = n_c = 8, N_aux = 512, W(R) within |R| <= 3 cells, BSE dim 262144, blocks of 16 vectors, BF16x3
apply and adjoint.

The explicit H (262144^2) is out of reach, so the oracle evaluates sampled outputs one at a time from
their definition (its row-at-a-time forms, pinned against the block forms on small meshes): two k rows
of H X and the W(q) gradient at one pair {q, -q}; the energy gradient is checked everywhere.  Bounds as for
every BF16x3 result (tests/tolerances.py): the apply on its kernel part, the gradient relative to its
largest element.  The module takes a few minutes, most of it the oracle on the host cores."""
import time

import numpy as np
import pytest
import torch

import oracle as O
from synth import dense_kmesh, make_problem, random_block
from tolerances import GRAD_TOL, KERNEL_TOL, diag_times, kernel_err

pytestmark = pytest.mark.gpu

ROWS = [0, 2731]   # k = Gamma and a generic k
QS = [1234, 3134]  # a q with q != -q on the mesh and its partner -q (the gradient of the pair comes from the
                   # pair densities of one of them)


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.fixture(scope="module")
def big():
    from paper_2607_05853_amd import bse as B
    t0 = time.time()
    p = make_problem("mesh16_ao128", 0, "G1")
    kq = dense_kmesh(p.nk)
    dev = torch.device("cuda:0")

    def T(a, dt=torch.complex128):
        return torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)

    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, kq)
    plan = B.plan_from_problem(p, Wq, prec="bf16x3", max_nb=16)
    plan.set_R(p.R, p.w_R)
    del Wq
    torch.cuda.empty_cache()
    print("\n[largest] problem and plan %.1f s, plan %.1f GB, pairs %s, conduction route %s" %
          (time.time() - t0, plan.bytes / 2**30, plan.pairs, plan.conduction), flush=True)
    W = O.interpolate_W_matmul(p.W_R, p.R, p.w_R, kq)
    print("[largest] oracle W(q) %.1f s" % (time.time() - t0), flush=True)
    yield dict(B=B, p=p, plan=plan, W=W, T=T)
    plan.close()


def test_largest_apply_sampled_rows(big):
    p, plan, T = big["p"], big["plan"], big["T"]
    nt = p.nv * p.nc
    X = random_block(p.N, 16, seed=41)
    t0 = time.time()
    Y = plan.apply(T(X))
    torch.cuda.synchronize()
    got = np.vstack([Y[k * nt:(k + 1) * nt].cpu().numpy() for k in ROWS])
    print("[largest] GPU apply %.1f s" % (time.time() - t0), flush=True)
    del Y
    t0 = time.time()
    ref = O.apply_H_rows_allpairs(p, big["W"], X, ROWS)
    err = kernel_err(got, ref, diag_times(p, X, ROWS))
    print("[largest] oracle rows %.1f s, kernel-part err %.2e (of max |Y|: %.2e)" %
          (time.time() - t0, err, rel(got, ref)), flush=True)
    assert err < KERNEL_TOL["bf16x3"]


def test_largest_adjoint_sampled_q(big):
    B, p, plan, T = big["B"], big["p"], big["plan"], big["T"]
    Yb, X = random_block(p.N, 16, seed=42), random_block(p.N, 16, seed=43)
    t0 = time.time()
    g = plan.apply_adjoint(T(Yb), T(X), want_WR=True, want_Wq=True, want_eps=True)
    torch.cuda.synchronize()
    print("[largest] GPU adjoint %.1f s" % (time.time() - t0), flush=True)
    # g_WR is the interpolation adjoint of g_Wq (FP64 on both sides)
    gr = B.interpolate_W_adjoint(g["W_q"], p.R, p.w_R, dense_kmesh(p.nk))
    assert (g["W_R"] - gr).abs().max().item() <= 1e-12 * gr.abs().max().item()
    gq = g["W_q"][QS].cpu().numpy()
    ge = g["eps"].cpu().numpy()
    del g, gr
    torch.cuda.empty_cache()
    assert rel(ge, O.grad_eps(p, Yb, X)) < 1e-13
    t0 = time.time()
    ref = O.grad_Wq_at(p, Yb, X, QS)
    err = rel(gq, ref)
    print("[largest] oracle g_W(q) %.1f s, rel err %.2e" % (time.time() - t0, err), flush=True)
    assert err < GRAD_TOL["bf16x3"]
