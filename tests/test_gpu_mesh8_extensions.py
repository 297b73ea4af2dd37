"""Sampled parity of the two-centre apply and of the coupling block at the timed 8^3 workload (mesh8_ao64:
N_ao = 64, nv = 4, nc = 8, N_aux = 256, blocks of 8, BF16x3 as in bench.py --mode two_centre / full_bse):
two k rows of the GPU result against the oracle's row-at-a-time forms (pinned against the block forms in
tests/test_oracle_rows.py)."""
import numpy as np
import pytest
import torch

import oracle as O
from synth import dense_kmesh, make_problem, random_block
from tolerances import KERNEL_TOL, diag_times, kernel_err

pytestmark = pytest.mark.gpu

ROWS = [5, 300]


def T(a, dt=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a)).to(torch.device("cuda:0"), dt)


def rows_of(Y, p, rows):
    nt = p.nv * p.nc
    return np.vstack([Y[k * nt:(k + 1) * nt] for k in rows])


@pytest.fixture(scope="module")
def B():
    from paper_2607_05853_amd import bse
    return bse


def test_mesh8_two_centre_apply_sampled_rows(B):
    p = make_problem("mesh8_ao64", 0, "G1", two_centre=True)
    print("[mesh8 two-centre apply, bf16x3, rows %s]" % ROWS, flush=True)
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
    plan = B.plan_from_problem(p, Wq, prec="bf16x3", max_nb=8)
    X = random_block(p.N, 8, seed=31)
    Y = plan.apply(T(X)).cpu().numpy()
    plan.close()
    ref = O.apply_rows_twosided(p, O.interpolate_W_matmul(p.W_R, p.R, p.w_R, dense_kmesh(p.nk)), X, ROWS, "A")
    err = kernel_err(rows_of(Y, p, ROWS), ref, diag_times(p, X, ROWS))
    print("    kernel-part err %.2e" % err, flush=True)
    assert err < KERNEL_TOL["bf16x3"]


def test_mesh8_coupling_sampled_rows(B):
    p = make_problem("mesh8_ao64", 0, "G1")
    print("[mesh8 coupling block, bf16x3, rows %s]" % ROWS, flush=True)
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
    plan = B.plan_from_problem(p, Wq, prec="bf16x3", max_nb=16)
    X = random_block(p.N, 8, seed=32)
    Y = plan.apply_coupling(T(X)).cpu().numpy()
    plan.close()
    ref = O.apply_rows_twosided(p, O.interpolate_W_matmul(p.W_R, p.R, p.w_R, dense_kmesh(p.nk)), X, ROWS, "B")
    err = np.abs(rows_of(Y, p, ROWS) - ref).max() / np.abs(ref).max()   # B has no diagonal
    print("    rel err %.2e" % err, flush=True)
    assert err < KERNEL_TOL["bf16x3"]
