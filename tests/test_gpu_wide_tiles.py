"""GPU parity of the BF16x3 kernels for large shapes: the 128 x 256 three-stage W-step tile, the fused W
step + direct block (P kept on chip) and the persistent streaming kernel of the pair densities, against the
oracle's explicit A and against the kernels they replace.

The wide tile and the streaming kernel give results identical to the tiled kernels (same MFMA sequence per
accumulator); the fused kernel forms T = M_c P^T on 16x16x32 MFMA in another summation order, so it is held
to the BF16x3 bound of the kernel part.  BSE_WIDE_TILES=0 / BSE_FUSED_WSTEP=0 / BSE_STREAM_PD=0 select the
previous kernels at the next apply; BSE_FRAG_HALVES=0 at plan creation keeps the halves in row order.
"""
import os

import numpy as np
import pytest
import torch

import oracle as O
from synth import dense_kmesh, make_problem, random_block
from tolerances import KERNEL_TOL, diag_times, kernel_err

pytestmark = pytest.mark.gpu

# n_v = n_c = 8: the fused kernel; N_aux 256 (one 256-column tile of P) and 512 (two, T parked between them)
FUSED_256 = dict(cfg_id=70, coarse=(2, 2, 2), dense=(2, 2, 2), n_ao=16, nv=8, nc=8, n_aux=256)
FUSED_512 = dict(cfg_id=71, coarse=(2, 2, 2), dense=(2, 2, 2), n_ao=16, nv=8, nc=8, n_aux=512)
# ragged wide tile: 18 k x 9 rows = 162 rows (128 + 34), N_aux = 272 (256 + 16)
# streaming pair densities: K = N_ao of 64 and 128; rows q x n_band ragged (n_v = 3, n_c = 5), columns
# n_band x N_aux of 1200 / 2000 (ragged 256-column tiles)
STREAM_64 = dict(cfg_id=73, coarse=(2, 2, 2), dense=(2, 2, 3), n_ao=64, nv=3, nc=5, n_aux=400)
STREAM_128 = dict(cfg_id=74, coarse=(2, 2, 2), dense=(2, 2, 3), n_ao=128, nv=3, nc=5, n_aux=400)
WIDE_RAGGED = dict(cfg_id=72, coarse=(2, 2, 2), dense=(3, 3, 2), n_ao=16, nv=3, nc=4, n_aux=272)
# halves in fragment order (N_ao = 128, N_aux a multiple of 32, n_v^2 a multiple of 8): columns
# n_band x N_aux of 1664 / 2496, so the last 256-column tile holds 4 / 6 of the 8 waves' 32-column blocks
FRAG_128 = dict(cfg_id=75, coarse=(2, 2, 2), dense=(2, 2, 3), n_ao=128, nv=4, nc=6, n_aux=416)
FRAG_64 = dict(cfg_id=79, coarse=(2, 2, 2), dense=(2, 2, 3), n_ao=64, nv=4, nc=6, n_aux=416)
# T.X with 16-row tiles: n_c n_v of 16, 32 and 64 (the last two with compile-time band counts)
TX_16 = dict(cfg_id=76, coarse=(2, 2, 2), dense=(2, 3, 2), n_ao=16, nv=4, nc=4, n_aux=40)
TX_32 = dict(cfg_id=77, coarse=(2, 2, 2), dense=(2, 3, 2), n_ao=16, nv=4, nc=8, n_aux=40)
TX_64 = dict(cfg_id=78, coarse=(2, 2, 2), dense=(2, 2, 2), n_ao=16, nv=8, nc=8, n_aux=48)


def dev():
    return torch.device("cuda:0")


def T(a, dt=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dev(), dt)


def H_(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def B():
    from paper_2607_05853_amd import bse
    return bse


def _apply_with(plan, X, var, value):
    old = os.environ.get(var)
    os.environ[var] = value
    try:
        return H_(plan.apply(T(X)))
    finally:
        if old is None:
            del os.environ[var]
        else:
            os.environ[var] = old


@pytest.mark.parametrize("wgen", ["G1", "G2"])
@pytest.mark.parametrize("cfg", ["FUSED_256", "FUSED_512"])
def test_fused_direct_block(B, cfg, wgen):
    conf = {"FUSED_256": FUSED_256, "FUSED_512": FUSED_512}[cfg]
    p = make_problem(conf, 1, wgen)
    kq = dense_kmesh(p.nk)
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, kq)
    plan = B.plan_from_problem(p, Wq, prec="bf16x3", max_nb=6, check_hermitian=True, conduction="mc")
    assert plan.conduction == "mc"
    X = random_block(p.N, 6, seed=4)
    H = O.build_H(p, O.interpolate_W_matmul(p.W_R, p.R, p.w_R, kq))
    DX = diag_times(p, X)
    ref = H @ X
    Yf = _apply_with(plan, X, "BSE_FUSED_WSTEP", "1")
    Yu = _apply_with(plan, X, "BSE_FUSED_WSTEP", "0")
    ef, eu = kernel_err(Yf, ref, DX), kernel_err(Yu, ref, DX)
    d = kernel_err(Yf, Yu, DX)
    # a second call reuses the workspaces and the parked T tiles: it must repeat the first bit for bit
    Yf2 = _apply_with(plan, X, "BSE_FUSED_WSTEP", "1")
    print("[fused %s %s] kernel-part err fused %.2e, two-kernel %.2e, between them %.2e" % (cfg, wgen, ef, eu, d),
          flush=True)
    assert np.array_equal(Yf, Yf2)
    assert max(ef, eu) < KERNEL_TOL["bf16x3"]
    assert d < KERNEL_TOL["bf16x3"]
    plan.close()


@pytest.mark.parametrize("all_pairs", [False, True])
def test_wide_tile_ragged_identical(B, all_pairs):
    p = make_problem(WIDE_RAGGED, 2, "G2")
    kq = dense_kmesh(p.nk)
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, kq)
    plan = B.plan_from_problem(p, Wq, prec="bf16x3", max_nb=5, conduction="mc", all_pairs=all_pairs)
    X = random_block(p.N, 5, seed=6)
    Yw = _apply_with(plan, X, "BSE_WIDE_TILES", "1")
    Yn = _apply_with(plan, X, "BSE_WIDE_TILES", "0")
    H = O.build_H(p, O.interpolate_W_matmul(p.W_R, p.R, p.w_R, kq))
    err = kernel_err(Yw, H @ X, diag_times(p, X))
    print("[wide tile ragged, all pairs %s] kernel-part err %.2e, identical to the 64 x 128 tile: %s" %
          (all_pairs, err, np.array_equal(Yw, Yn)), flush=True)
    assert np.array_equal(Yw, Yn)
    assert err < KERNEL_TOL["bf16x3"]
    plan.close()


@pytest.mark.parametrize("all_pairs", [False, True])
@pytest.mark.parametrize("cfg", ["STREAM_64", "STREAM_128"])
def test_stream_pair_densities_identical(B, cfg, all_pairs):
    p = make_problem({"STREAM_64": STREAM_64, "STREAM_128": STREAM_128}[cfg], 3, "G2")
    kq = dense_kmesh(p.nk)
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, kq)
    plan = B.plan_from_problem(p, Wq, prec="bf16x3", max_nb=4, conduction="mc", all_pairs=all_pairs)
    X = random_block(p.N, 4, seed=7)
    Ys = _apply_with(plan, X, "BSE_STREAM_PD", "1")
    Yt = _apply_with(plan, X, "BSE_STREAM_PD", "0")
    H = O.build_H(p, O.interpolate_W_matmul(p.W_R, p.R, p.w_R, kq))
    err = kernel_err(Ys, H @ X, diag_times(p, X))
    print("[stream %s, all pairs %s] kernel-part err %.2e, identical to the tiled kernel: %s" %
          (cfg, all_pairs, err, np.array_equal(Ys, Yt)), flush=True)
    assert np.array_equal(Ys, Yt)
    assert err < KERNEL_TOL["bf16x3"]
    plan.close()


def _plan_with(B, p, Wq, frag, **kw):
    old = os.environ.get("BSE_FRAG_HALVES")
    os.environ["BSE_FRAG_HALVES"] = "1" if frag else "0"
    try:
        return B.plan_from_problem(p, Wq, prec="bf16x3", max_nb=4, **kw)
    finally:
        if old is None:
            del os.environ["BSE_FRAG_HALVES"]
        else:
            os.environ["BSE_FRAG_HALVES"] = old


@pytest.mark.parametrize("all_pairs", [False, True])
@pytest.mark.parametrize("cfg", ["FRAG_128", "FRAG_64"])
def test_fragment_order_halves_identical(B, cfg, all_pairs):
    # the streaming kernel on halves in fragment order against the row layout (streaming and tiled kernels):
    # apply, adjoint (every pair-density product of the gradient) and the coupling block, bit for bit
    p = make_problem({"FRAG_128": FRAG_128, "FRAG_64": FRAG_64}[cfg], 5, "G2")
    kq = dense_kmesh(p.nk)
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, kq)
    pf = _plan_with(B, p, Wq, True, conduction="mc", all_pairs=all_pairs)
    pr = _plan_with(B, p, Wq, False, conduction="mc", all_pairs=all_pairs)
    assert pf.frag and not pr.frag
    X = random_block(p.N, 4, seed=11)
    Yb = random_block(p.N, 4, seed=12)
    Yf = H_(pf.apply(T(X)))
    Yr = _apply_with(pr, X, "BSE_STREAM_PD", "1")
    Yt = _apply_with(pr, X, "BSE_STREAM_PD", "0")
    H = O.build_H(p, O.interpolate_W_matmul(p.W_R, p.R, p.w_R, kq))
    err = kernel_err(Yf, H @ X, diag_times(p, X))
    gf = pf.apply_adjoint(T(Yb), T(X), want_WR=False, want_Wq=True)
    gr = pr.apply_adjoint(T(Yb), T(X), want_WR=False, want_Wq=True)
    Bf = H_(pf.apply_coupling(T(X)))
    Br = H_(pr.apply_coupling(T(X)))
    print("[fragment-order halves %s, all pairs %s] kernel-part err %.2e; identical: apply %s / %s, g_W(q) %s, "
          "g_eps %s, coupling %s" % (cfg, all_pairs, err, np.array_equal(Yf, Yr), np.array_equal(Yf, Yt),
                                      torch.equal(gf["W_q"], gr["W_q"]), torch.equal(gf["eps"], gr["eps"]),
                                      np.array_equal(Bf, Br)), flush=True)
    assert err < KERNEL_TOL["bf16x3"]
    assert np.array_equal(Yf, Yr) and np.array_equal(Yf, Yt)
    assert torch.equal(gf["W_q"], gr["W_q"]) and torch.equal(gf["eps"], gr["eps"])
    assert np.array_equal(Bf, Br)
    pf.close()
    pr.close()


def test_fragment_order_only_where_it_applies(B):
    # row layout for shapes the fragment order does not cover (N_aux = 400; n_v^2 odd) and for FP32
    for cfg, prec in ((STREAM_64, "bf16x3"), (STREAM_128, "bf16x3"), (FRAG_128, "f32")):
        p = make_problem(cfg, 3, "G2")
        Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
        pl = B.plan_from_problem(p, Wq, prec=prec, max_nb=2)
        assert not pl.frag, (cfg, prec)
        pl.close()


@pytest.mark.parametrize("nb", [3, 8, 16])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("cfg", ["TX_16", "TX_32", "TX_64"])
def test_tx_restaged_kernel(B, cfg, prec, nb):
    # the restaged T.X kernel against the oracle and against the previous kernel (BSE_TX2=0: FP32 matrix
    # cores for c64 T, FP64 vector units for c128 T): the sums run over k in another order, so they agree to
    # the rounding of the product precision
    p = make_problem({"TX_16": TX_16, "TX_32": TX_32, "TX_64": TX_64}[cfg], 4, "G2")
    kq = dense_kmesh(p.nk)
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, kq)
    plan = B.plan_from_problem(p, Wq, prec=prec, max_nb=16)
    X = random_block(p.N, nb, seed=13)
    Y2 = _apply_with(plan, X, "BSE_TX2", "1")
    Y1 = _apply_with(plan, X, "BSE_TX2", "0")
    H = O.build_H(p, O.interpolate_W_matmul(p.W_R, p.R, p.w_R, kq))
    DX = diag_times(p, X)
    e2, e1 = kernel_err(Y2, H @ X, DX), kernel_err(Y1, H @ X, DX)
    d = kernel_err(Y2, Y1, DX)
    print("[T.X %s %s nb=%d] kernel-part err restaged %.2e, previous %.2e, between them %.2e" %
          (cfg, prec, nb, e2, e1, d), flush=True)
    assert e2 < KERNEL_TOL[prec]
    assert d < (1e-13 if prec == "f64" else 1e-6)
    plan.close()
