"""GPU parity: every C-ABI entry point against the FP64 oracle on seeded inputs.

Applies are held to the bounds of tests/tolerances.py on their kernel part (the error relative to the
largest element of the oracle's A X - D X, D the FP64 diagonal); interpolation and FP64 results to 1e-12
of the largest reference element.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
from synth import dense_kmesh, make_problem, polarisations, random_block
from tolerances import GRAD_TOL, KERNEL_TOL, diag_times, kernel_err

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12}  # interpolation: FP64 whatever the output precision
RAGGED = dict(cfg_id=93, coarse=(3, 3, 3), dense=(3, 2, 5), n_ao=12, nv=3, nc=5, n_aux=40)


def dev():
    return torch.device("cuda:0")


def T(a, dt=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dev(), dt)


def H_(t):
    return t.detach().cpu().numpy()


def OW(p):
    """The oracle's own W(q) on the dense mesh (oracle inputs never come from the GPU path)."""
    return O.interpolate_W_matmul(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.fixture(scope="module")
def B():
    from paper_2607_05853_amd import bse
    print("\n[gpu] libbse", bse.version(), flush=True)
    return bse


# ---------------------------------------------------------------------------
# interpolation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n_aux,n_R,n_q", [(5, 3, 7), (17, 27, 64), (64, 125, 33)])
def test_interpolate_small(B, n_aux, n_R, n_q):
    rng = np.random.default_rng(n_aux)
    W_R = rng.standard_normal((n_R, n_aux, n_aux)) + 1j * rng.standard_normal((n_R, n_aux, n_aux))
    R = rng.integers(-3, 4, size=(n_R, 3)).astype(np.int32)
    w = rng.random(n_R)
    q = rng.random((n_q, 3))
    ref = O.interpolate_W(W_R, R, w, q)
    out = H_(B.interpolate_W(T(W_R), R, w, q))
    assert rel(out, ref) < TOL["f64"]
    out32 = H_(B.interpolate_W(T(W_R), R, w, q, out_prec="f32"))
    assert rel(out32, ref) < 1e-6


@pytest.mark.parametrize("cfg", ["mesh4_ao16", "mesh8_ao64"])
def test_interpolate_configs(B, cfg):
    p = make_problem(cfg, 0, "G2")
    kq = dense_kmesh(p.nk)
    got = H_(B.interpolate_W(T(p.W_R), p.R, p.w_R, kq))
    idx = np.arange(len(kq)) if cfg == "mesh4_ao16" else np.array([0, 1, 7, 63, 64, 200, 511])
    ref = O.interpolate_W(p.W_R, p.R, p.w_R, kq[idx])
    assert rel(got[idx], ref) < TOL["f64"]
    # Hermitian W(q) for the G2 generator, at every q
    assert np.abs(got - np.conj(np.transpose(got, (0, 2, 1)))).max() < 1e-13 * np.abs(got).max()


def test_interpolate_large_sampled(B):
    # the largest workload's table: 4096 q x 512^2, checked on sampled q against the oracle
    p = make_problem("mesh16_ao128", 0, "G1")
    kq = dense_kmesh(p.nk)
    got = B.interpolate_W(T(p.W_R), p.R, p.w_R, kq)
    idx = np.array([0, 1, 255, 1000, 4095])
    ref = O.interpolate_W(p.W_R, p.R, p.w_R, kq[idx])
    assert rel(H_(got[torch.as_tensor(idx, device=dev())]), ref) < TOL["f64"]
    del got


def test_coarse_round_trip_on_gpu(B):
    # coarse W(k) -> R (adjoint with weights 1/N_c) -> back onto the coarse points: exact
    from synth import ws_rset
    coarse = (4, 4, 4)
    R, w = ws_rset(coarse)
    qc = dense_kmesh(coarse)
    rng = np.random.default_rng(11)
    Wqc = rng.standard_normal((len(qc), 6, 6)) + 1j * rng.standard_normal((len(qc), 6, 6))
    W_R = B.interpolate_W_adjoint(T(Wqc), R, np.full(len(R), 1.0 / len(qc)), qc)
    assert rel(H_(W_R), O.coarse_to_R(Wqc, coarse, R)) < TOL["f64"]
    back = H_(B.interpolate_W(W_R, R, w, qc))
    assert rel(back, Wqc) < TOL["f64"]


def test_interpolate_adjoint_matches_oracle(B):
    p = make_problem("mesh4_ao16", 0, "G2", coarse=(3, 3, 2))
    kq = dense_kmesh(p.nk)
    rng = np.random.default_rng(4)
    g = rng.standard_normal((len(kq), p.n_aux, p.n_aux)) + 1j * rng.standard_normal((len(kq), p.n_aux, p.n_aux))
    got = H_(B.interpolate_W_adjoint(T(g), p.R, p.w_R, kq))
    ref = O.grad_WR_from_Wq(g, p.R, p.w_R, kq)
    assert rel(got, ref) < TOL["f64"]


# ---------------------------------------------------------------------------
# apply
# ---------------------------------------------------------------------------
def _plan(B, p, prec="f64", nb=8, Wq=None):
    if Wq is None:
        Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
    return B.plan_from_problem(p, Wq, prec=prec, max_nb=nb, check_hermitian=True), Wq


@pytest.mark.parametrize("wgen", ["G1", "G2"])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_apply_c1(B, wgen, prec):
    p = make_problem("mesh4_ao16", 0, wgen, coarse=(3, 3, 2) if wgen == "G2" else (2, 2, 2))
    plan, Wq = _plan(B, p, prec, nb=3)
    H = O.build_H(p, OW(p))
    X = random_block(p.N, 3, seed=1)
    Y = H_(plan.apply(T(X)))
    err = kernel_err(Y, H @ X, diag_times(p, X))
    print("[c1 %s %s] kernel-part err %.3e (of max |Y|: %.3e)" % (wgen, prec, err, rel(Y, H @ X)), flush=True)
    assert err < KERNEL_TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_apply_complex_hermitian_vbar(B, prec):
    # the generators' Vbar is real symmetric (real auxiliary functions), but the ABI takes any Hermitian
    # Vbar: with a complex one the orientation of the exchange term (mu on the density at k, nu on the one
    # at k') is observable, and the apply must follow the oracle's (pinned by the AO-kernel brute force)
    p = make_problem("mesh4_ao16", 0, "G2", coarse=(3, 3, 2))
    A = np.random.default_rng(8).standard_normal((p.n_aux, p.n_aux))
    p = dataclasses.replace(p, Vbar=p.Vbar + 0.1j * (A - A.T))
    plan, Wq = _plan(B, p, prec, nb=3)
    H = O.build_H(p, OW(p))
    X = random_block(p.N, 3, seed=1)
    DX = diag_times(p, X)
    HT = O.build_H(dataclasses.replace(p, Vbar=p.Vbar.T), OW(p))
    assert kernel_err(HT @ X, H @ X, DX) > 1e3 * KERNEL_TOL[prec]   # the transposed Vbar is far outside
    err = kernel_err(H_(plan.apply(T(X))), H @ X, DX)
    plan.close()
    print("[complex Vbar %s] kernel-part err %.3e" % (prec, err), flush=True)
    assert err < KERNEL_TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_apply_ragged_and_triplet(B, prec):
    # sizes that are not multiples of any tile: 30 k, 3+5 bands, 40 aux, 12 AOs, 5 vectors
    p = make_problem(RAGGED, 2, "G2")
    plan, Wq = _plan(B, p, prec, nb=5)
    X = random_block(p.N, 5, seed=3)
    H = O.build_H(p, OW(p))
    DX = diag_times(p, X)
    e1 = kernel_err(H_(plan.apply(T(X))), H @ X, DX)
    p.alpha = 0.0
    plan0, _ = _plan(B, p, prec, nb=5, Wq=Wq)
    H0 = O.build_H(p, OW(p))
    e2 = kernel_err(H_(plan0.apply(T(X))), H0 @ X, DX)
    # nb smaller than max_nb, single vector
    e3 = kernel_err(H_(plan.apply(T(X[:, :1].copy()))), H @ X[:, :1], DX[:, :1])
    print("[ragged %s] kernel-part err singlet %.2e triplet %.2e one vector %.2e" % (prec, e1, e2, e3), flush=True)
    assert max(e1, e2, e3) < KERNEL_TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_apply_c2_sampled_rows(B, prec):
    # the timed workload (8x8x8 dense mesh, N_aux = 256, blocks of 8) in every precision, two k rows
    # of the oracle's matrix-free apply (one row per q batch boundary region and one interior)
    p = make_problem("mesh8_ao64", 0, "G2")
    plan, Wq = _plan(B, p, prec, nb=8)
    X = random_block(p.N, 8, seed=5)
    Y = H_(plan.apply(T(X)))
    rows = [0, 301, 511]
    ref = O.apply_H_rows(p, OW(p), X, rows)
    nt = p.nc * p.nv
    got = np.concatenate([Y[k * nt:(k + 1) * nt] for k in rows])
    err = kernel_err(got, ref, diag_times(p, X, rows))
    print("[c2 sampled %s] kernel-part err %.3e (of max |Y|: %.3e)" % (prec, err, rel(got, ref)), flush=True)
    assert err < KERNEL_TOL[prec]


# n_aux a multiple of 16 selects the direct-to-LDS kernels.  DMA: n_ao = 80 > 64 takes the 128-row
# conduction-side tile with ragged rows and the matrix-core epilogue, nv = 5 gives 25 columns per q (5 q
# per column group, 2 q per epilogue pass).  DMA_MT: nc = 17 needs two 16-row tiles of conduction bands
# in the matrix-core epilogue, nv = 2 puts 32 q in a column group.  DMA_ODD: n_ao = 20 (not a multiple
# of 8) keeps the vector-unit epilogue and the register-staged valence pair-density GEMM
DMA = dict(cfg_id=94, coarse=(2, 2, 2), dense=(2, 2, 3), n_ao=80, nv=5, nc=3, n_aux=48)
DMA_MT = dict(cfg_id=95, coarse=(2, 2, 2), dense=(2, 3, 1), n_ao=40, nv=2, nc=17, n_aux=32)
DMA_ODD = dict(cfg_id=98, coarse=(2, 2, 2), dense=(3, 1, 2), n_ao=20, nv=3, nc=4, n_aux=32)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("shape", ["DMA", "DMA_MT", "DMA_ODD"])
def test_apply_dma_shapes(B, prec, shape):
    p = make_problem({"DMA": DMA, "DMA_MT": DMA_MT, "DMA_ODD": DMA_ODD}[shape], 0, "G2", coarse=(3, 3, 2))
    plan, Wq = _plan(B, p, prec, nb=4)
    X = random_block(p.N, 4, seed=8)
    H = O.build_H(p, OW(p))
    err = kernel_err(H_(plan.apply(T(X))), H @ X, diag_times(p, X))
    print("[dma shapes %s %s] kernel-part err %.3e" % (shape, prec, err), flush=True)
    assert err < KERNEL_TOL[prec]


@pytest.mark.parametrize("route", ["mc", "u"])
@pytest.mark.parametrize("shape", ["mesh4_ao16", "RAGGED", "DMA", "DMA_MT", "DMA_ODD"])
def test_bf16x3_conduction_routes(B, shape, route):
    # the two BF16x3 routes of the conduction side: forming M_cc' and T = M_c P^T (the split GEMM; N_aux = 40
    # in RAGGED takes its register-staged fallback) or the B_c(k) contraction of direct_b3
    conf = {"mesh4_ao16": "mesh4_ao16", "RAGGED": RAGGED, "DMA": DMA, "DMA_MT": DMA_MT, "DMA_ODD": DMA_ODD}[shape]
    p = make_problem(conf, 2, "G2", coarse=(3, 3, 2))
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
    plan = B.plan_from_problem(p, Wq, prec="bf16x3", max_nb=4, conduction=route)
    assert plan.conduction == route
    X = random_block(p.N, 4, seed=9)
    err = kernel_err(H_(plan.apply(T(X))), O.build_H(p, OW(p)) @ X, diag_times(p, X))
    print("[conduction %s %s] kernel-part err %.3e" % (shape, route, err), flush=True)
    assert err < KERNEL_TOL["bf16x3"]


def test_apply_c3_oracle_rows_and_properties(B):
    # 12x12x12 dense mesh, N_ao = 96, n_v = 6, n_c = 10, N_aux = 384 (BSE dim 103680), the precision form:
    # the FP64 and BF16x3 applies on sampled k rows against the oracle's row-at-a-time A X, the BF16x3 apply
    # against the FP64 one on every row, Hermiticity of the BF16x3 apply and the closed form of the zero
    # kernel
    p = make_problem("mesh12_ao96", 0, "G2")
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
    X1h = random_block(p.N, 4, seed=11)
    X1, X2 = T(X1h), T(random_block(p.N, 4, seed=12))
    rows = [0, 1000]
    nt = p.nc * p.nv
    ref = O.apply_H_rows_allpairs(p, OW(p), X1h, rows)
    DX = diag_times(p, X1h, rows)
    take = lambda Y: np.concatenate([Y[k * nt:(k + 1) * nt] for k in rows])
    planf = B.plan_from_problem(p, Wq, prec="f64", max_nb=4)
    Yf1 = planf.apply(X1)
    planf.close()
    planb = B.plan_from_problem(p, Wq, prec="bf16x3", max_nb=4)
    Yb1, Yb2 = planb.apply(X1), planb.apply(X2)
    lhs = torch.sum(torch.conj(X1) * Yb2).item()
    rhs = torch.sum(torch.conj(Yb1) * X2).item()
    herm = abs(lhs - rhs) / (torch.linalg.norm(Yb1).item() * torch.linalg.norm(X2).item())
    planb.close()
    e_f = kernel_err(take(H_(Yf1)), ref, DX)
    e_b = kernel_err(take(H_(Yb1)), ref, DX)
    DX_all = T(diag_times(p, X1h))
    e_bf = ((Yb1 - Yf1).abs().max() / (Yf1 - DX_all).abs().max()).item()
    print("[c3] oracle rows: f64 %.2e bf16x3 %.2e; bf16x3 vs f64 (all rows) %.2e; hermiticity defect %.2e" %
          (e_f, e_b, e_bf, herm), flush=True)
    assert e_f < KERNEL_TOL["f64"]
    assert e_b < KERNEL_TOL["bf16x3"] and e_bf < KERNEL_TOL["bf16x3"]
    assert herm < 1e-8
    # zero screened and bare interaction: H = diag(e_c - e_v) exactly
    p0 = dataclasses.replace(p, Vbar=np.zeros_like(p.Vbar))
    Wz = torch.zeros_like(Wq)
    planz = B.plan_from_problem(p0, Wz, prec="bf16x3", max_nb=4)
    Yz = H_(planz.apply(X1))
    planz.close()
    te = O.transition_energies(p0).reshape(-1)
    assert rel(Yz, te[:, None] * X1h) < 1e-14


def test_apply_hermitian_and_deterministic(B):
    p = make_problem(RAGGED, 4, "G2")
    plan, _ = _plan(B, p, "f64", nb=4)
    X1 = T(random_block(p.N, 4, seed=7))
    X2 = T(random_block(p.N, 4, seed=8))
    HX2 = plan.apply(X2)
    HX1 = plan.apply(X1)
    lhs = torch.sum(torch.conj(X1) * HX2).item()
    rhs = torch.sum(torch.conj(HX1) * X2).item()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    again = plan.apply(X2)
    assert torch.equal(again, HX2)


def test_zero_kernel_is_diagonal(B):
    p = make_problem(RAGGED, 1)
    p.Vbar = p.Vbar * 0
    Wq = torch.zeros((p.Nk, p.n_aux, p.n_aux), dtype=torch.complex128, device=dev())
    plan, _ = _plan(B, p, "f64", nb=2, Wq=Wq)
    X = random_block(p.N, 2, seed=2)
    te = O.transition_energies(p).ravel()
    assert rel(H_(plan.apply(T(X))), te[:, None] * X) < 1e-15


# ---------------------------------------------------------------------------
# start vectors and Haydock
# ---------------------------------------------------------------------------
def test_velocity_start(B):
    p = make_problem(RAGGED, 0)
    plan, _ = _plan(B, p, "f64", nb=4)
    pol = polarisations(4)
    got = H_(plan.velocity_start(T(p.vel), T(p.eps_ks, torch.float64), pol))
    assert rel(got, O.velocity_start(p, pol)) < 1e-14


def test_haydock_c1(B):
    p = make_problem("mesh4_ao16", 0, "G2", coarse=(3, 3, 2))
    plan, Wq = _plan(B, p, "f64", nb=3)
    H = O.build_H(p, OW(p))
    pol = polarisations(3)
    P = plan.velocity_start(T(p.vel), T(p.eps_ks, torch.float64), pol)
    te = O.transition_energies(p)
    w = np.linspace(te.min() - 1, te.max() + 1, 2001)
    m = 200
    out = plan.haydock(P, m, w, 0.1)
    P_or = O.velocity_start(p, pol)
    Sa, Aa, Ba, st = O.haydock_spectrum(lambda x: H @ x, P_or, m, w, 0.1, p.Nk)
    assert (out["steps"] == m).all()
    assert np.abs(out["a"][:, :50] - Aa[:, :50]).max() < 1e-10
    assert np.abs(out["b"][:, :51] - Ba[:, :51]).max() < 1e-10 * Ba[:, 0].max()
    Sref, _, _ = O.eig_spectrum(H, P_or, w, 0.1, p.Nk)
    e_eig = rel(out["S"], Sref)
    print("[haydock c1] spectrum rel err vs eigh %.3e" % e_eig, flush=True)
    assert e_eig < 1e-8
    assert rel(out["S"], Sa) < 1e-8


def test_haydock_full_krylov_and_breakdown(B):
    p = make_problem(dict(cfg_id=94, coarse=(2, 2, 2), dense=(2, 2, 2), n_ao=8, nv=2, nc=2, n_aux=12), 0)
    plan, Wq = _plan(B, p, "f64", nb=2)
    H = O.build_H(p, OW(p))
    P = O.velocity_start(p, np.eye(3))[:, :2]
    w = np.linspace(1.0, 5.0, 101)
    out = plan.haydock(T(P), p.N, w, 0.1)
    Sref, _, _ = O.eig_spectrum(H, P, w, 0.1, p.Nk)
    # m = dim: exact up to rounding unless an invariant subspace ends the chain first
    assert rel(out["S"], Sref) < 1e-9
    # W = Vbar = 0 and a one-entry start vector: b_1 = 0, chain stops after one step
    p.Vbar = p.Vbar * 0
    plan0, _ = _plan(B, p, "f64", nb=1, Wq=torch.zeros_like(Wq))
    e = np.zeros((p.N, 1), dtype=complex)
    e[5, 0] = 0.6 + 0.8j
    out0 = plan0.haydock(T(e), 10, w, 0.1)
    assert out0["breakdown"] and out0["steps"][0] == 1
    te = O.transition_energies(p).ravel()
    ref = (0.1 / np.pi) / ((w - te[5]) ** 2 + 0.01) / p.Nk
    assert rel(out0["S"][0], ref) < 1e-13
    # three entries with distinct energies: the Krylov space is invariant after three steps, and the chain
    # stops there however large or small the start vector is (the test is against the chain's own scale of A)
    idx = [1, 6, 11]
    assert len(set(np.round(te[idx], 12))) == 3
    v = np.zeros((p.N, 1), dtype=complex)
    v[idx, 0] = [0.6, -0.3 + 0.2j, 0.5j]
    runs = [plan0.haydock(T(sp * v), 10, w, 0.1) for sp in (1.0, 1e-20, 1e20)]
    ref3 = (0.1 / np.pi) * sum(abs(v[i, 0]) ** 2 / ((w - te[i]) ** 2 + 0.01) for i in idx) / p.Nk
    for sp, r in zip((1.0, 1e-20, 1e20), runs):
        assert r["breakdown"] and r["steps"][0] == 3, (sp, r["steps"])
        assert np.abs(r["a"][0, :3] - runs[0]["a"][0, :3]).max() < 1e-13 * te.max()
        assert np.abs(r["b"][0, 1:3] - runs[0]["b"][0, 1:3]).max() < 1e-13 * te.max()
        assert rel(r["S"][0] / sp ** 2, ref3) < 1e-12


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_apply_adjoint(B, prec):
    p = make_problem(RAGGED, 5, "G2")
    plan, Wq = _plan(B, p, prec, nb=3)
    plan.set_R(p.R, p.w_R)
    rng = np.random.default_rng(12)
    Yb = rng.standard_normal((p.N, 3)) + 1j * rng.standard_normal((p.N, 3))
    X = rng.standard_normal((p.N, 3)) + 1j * rng.standard_normal((p.N, 3))
    g = plan.apply_adjoint(T(Yb), T(X), want_WR=True, want_Wq=True, want_eps=True)
    ge, gq = O.grad_apply(p, OW(p), Yb, X)
    gr = O.grad_WR_from_Wq(gq, p.R, p.w_R, dense_kmesh(p.nk))
    eq, er = rel(H_(g["W_q"]), gq), rel(H_(g["W_R"]), gr)
    print("[adjoint %s] W_q %.2e W_R %.2e" % (prec, eq, er), flush=True)
    assert rel(H_(g["eps"]), ge) < 1e-13
    assert eq < GRAD_TOL[prec] and er < GRAD_TOL[prec]


# BF16x3 adjoint on the k-major kernel (n_v^2 and N_aux multiples of 8): ADJ_TN has ragged 40 x 40
# W-gradient tiles and a 9-deep Z product (one partial k step); ADJ_SPLIT has n_v = 8 and a 2048-deep
# W-gradient reduction split over two k ranges
ADJ_TN = dict(cfg_id=80, coarse=(2, 2, 2), dense=(3, 2, 2), n_ao=16, nv=4, nc=3, n_aux=40)
ADJ_SPLIT = dict(cfg_id=81, coarse=(2, 2, 2), dense=(4, 4, 2), n_ao=16, nv=8, nc=2, n_aux=24)
# N_aux = 72 > 64: the W-gradient product takes the 128-row tiles (Z keeps the 64-row ones)
ADJ_WIDE = dict(cfg_id=82, coarse=(2, 2, 2), dense=(3, 2, 2), n_ao=16, nv=4, nc=3, n_aux=72)


@pytest.mark.parametrize("all_pairs", [False, True])
@pytest.mark.parametrize("cfg", ["ADJ_TN", "ADJ_SPLIT", "ADJ_WIDE"])
def test_apply_adjoint_kmajor(B, cfg, all_pairs):
    # all_pairs=False: the gradient of each q pair {q, -q} from one set of pair densities
    conf = {"ADJ_TN": ADJ_TN, "ADJ_SPLIT": ADJ_SPLIT, "ADJ_WIDE": ADJ_WIDE}[cfg]
    p = make_problem(conf, 6, "G2", coarse=(3, 3, 2))
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
    plan = B.plan_from_problem(p, Wq, prec="bf16x3", max_nb=4, all_pairs=all_pairs)
    assert (plan.pairs[0] < p.Nk) == (not all_pairs)
    plan.set_R(p.R, p.w_R)
    Yb, X = random_block(p.N, 4, seed=31), random_block(p.N, 4, seed=32)
    g = plan.apply_adjoint(T(Yb), T(X), want_WR=True, want_Wq=True, want_eps=True)
    ge, gq = O.grad_apply(p, OW(p), Yb, X)
    gr = O.grad_WR_from_Wq(gq, p.R, p.w_R, dense_kmesh(p.nk))
    eq, er = rel(H_(g["W_q"]), gq), rel(H_(g["W_R"]), gr)
    print("[adjoint k-major %s all_pairs=%s] W_q %.2e W_R %.2e" % (cfg, all_pairs, eq, er), flush=True)
    assert rel(H_(g["eps"]), ge) < 1e-13
    assert eq < GRAD_TOL["bf16x3"] and er < GRAD_TOL["bf16x3"]


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
@pytest.mark.parametrize("cfg", ["mesh4_ao16", "RAGGED", "DMA"])
def test_pair_symmetry_against_all_pairs(B, prec, cfg):
    # the apply forms the direct blocks of about half of the q and takes the rest from
    # D(k, k-q) = D(k-q, k)^dagger; both modes must give the oracle's H X
    conf = {"mesh4_ao16": "mesh4_ao16", "RAGGED": RAGGED, "DMA": DMA}[cfg]
    p = make_problem(conf, 1, "G2", coarse=(3, 3, 2))
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
    X = random_block(p.N, 4, seed=21)
    H = O.build_H(p, OW(p))
    ref = H @ X
    half = B.plan_from_problem(p, Wq, prec=prec, max_nb=4)
    full = B.plan_from_problem(p, Wq, prec=prec, max_nb=4, all_pairs=True)
    formed, total = half.pairs
    assert total == p.Nk and full.pairs == (p.Nk, p.Nk)
    neg = [int(np.ravel_multi_index(tuple((-np.array(np.unravel_index(q, p.nk))) % np.array(p.nk)), p.nk))
           for q in range(p.Nk)]
    assert formed == sum(1 for q in range(p.Nk) if q <= neg[q])
    DX = diag_times(p, X)
    eh, ef = kernel_err(H_(half.apply(T(X))), ref, DX), kernel_err(H_(full.apply(T(X))), ref, DX)
    print("[pair symmetry %s %s] formed %d of %d, kernel-part err %.2e (all pairs %.2e)" %
          (cfg, prec, formed, total, eh, ef), flush=True)
    assert eh < KERNEL_TOL[prec] and ef < KERNEL_TOL[prec]


def test_pair_symmetry_off_for_general_W(B):
    # a W_q without W(-q) = conj W(q) must fall back to forming every block (and still match the oracle,
    # whose H is then not Hermitian)
    p = make_problem("mesh4_ao16", 2, "G2", coarse=(3, 3, 2))
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
    rng = np.random.default_rng(4)
    bump = (rng.standard_normal((p.n_aux, p.n_aux)) + 1j * rng.standard_normal((p.n_aux, p.n_aux))) * 1e-3
    Wq[5] += T(bump)
    plan = B.plan_from_problem(p, Wq, prec="f64", max_nb=3)
    assert plan.pairs == (p.Nk, p.Nk)
    X = random_block(p.N, 3, seed=22)
    W_or = OW(p)
    W_or[5] += bump
    H = O.build_H(p, W_or)
    assert kernel_err(H_(plan.apply(T(X))), H @ X, diag_times(p, X)) < KERNEL_TOL["f64"]


def test_plan_refuses_non_hermitian_inputs(B):
    # the plan reads M_v'v(k',k) and M_v'c'(k',k') as conjugates of the pair densities it forms, which holds
    # only for Hermitian C^mu: other coefficients, or a non-Hermitian Vbar, are refused with BSE_ENOTHERM
    # instead of applying an operator different from the oracle's A
    p = make_problem("mesh4_ao16", 3, "G2", coarse=(3, 3, 2))
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
    rng = np.random.default_rng(41)
    bump = 1e-6 * (rng.standard_normal((p.n_ao, p.n_ao)) + 1j * rng.standard_normal((p.n_ao, p.n_ao)))
    C_bad = p.C.copy()
    C_bad[7] += bump
    V_bad = p.Vbar.copy()
    V_bad[2, 5] += 1e-6j
    for q, what in [(dataclasses.replace(p, C=C_bad), "C^mu"), (dataclasses.replace(p, Vbar=V_bad), "Vbar")]:
        for prec in ("f64", "bf16x3"):
            with pytest.raises(B.BSEError) as e:
                B.plan_from_problem(q, Wq, prec=prec, max_nb=2)
            assert e.value.status == 5, what
            assert what + " is not Hermitian" in str(e.value)
    # asymmetry at the rounding level of the inputs (1e-15 of max |C|) is accepted, and the plan applies the
    # oracle's A of those coefficients
    C_ok = p.C + 1e-15 * np.abs(p.C).max() * (rng.standard_normal(p.C.shape) + 1j * rng.standard_normal(p.C.shape))
    q = dataclasses.replace(p, C=C_ok)
    plan = B.plan_from_problem(q, Wq, prec="f64", max_nb=2)
    X = random_block(p.N, 2, seed=42)
    assert kernel_err(H_(plan.apply(T(X))), O.build_H(q, OW(q)) @ X, diag_times(q, X)) < KERNEL_TOL["f64"]
