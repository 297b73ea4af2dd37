"""GPU tests of the drivers and gradients: block LOBPCG against the oracle's
eigen-decomposition, Hellmann-Feynman and spectrum gradients against the
oracle's gradients and against central finite differences of the GPU path."""
import numpy as np
import pytest
import torch

import oracle as O
from synth import dense_kmesh, make_problem, random_block

pytestmark = pytest.mark.gpu

SMALL = dict(cfg_id=96, coarse=(3, 3, 2), dense=(3, 2, 2), n_ao=10, nv=2, nc=3, n_aux=20)
DMA_LOB = dict(cfg_id=77, coarse=(3, 3, 2), dense=(4, 4, 2), n_ao=16, nv=4, nc=4, n_aux=48)


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
    return bse


def _plan(B, p, W_R=None, eps=None, prec="f64", nb=4):
    W_R = T(p.W_R) if W_R is None else W_R
    eps = T(p.eps_qp, torch.float64) if eps is None else eps
    Wq = B.interpolate_W(W_R, p.R, p.w_R, dense_kmesh(p.nk))
    plan = B.Plan(p.nk, p.n_ao, p.nv, p.nc, p.n_aux, eps, T(p.psi), T(p.C), T(p.Vbar), Wq, alpha=p.alpha,
                  prec=prec, max_nb=nb)
    plan.set_R(p.R, p.w_R)
    return plan, Wq


def _admissible(p, seed, scale=1e-2):
    rng = np.random.default_rng(seed)
    idx = {tuple(r): i for i, r in enumerate(p.R)}
    d = np.zeros(p.W_R.shape)
    for i, r in enumerate(p.R):
        j = idx[tuple(-r)]
        if j < i:
            continue
        A = rng.standard_normal(p.W_R.shape[1:]) * scale
        if i == j:
            A = A + A.T
        d[i] = A
        d[j] = A.T
    return d.astype(complex)


@pytest.mark.parametrize("cfg,wgen", [("mesh4_ao16", "G1"), (SMALL, "G2")])
def test_lobpcg_lowest(B, cfg, wgen):
    p = make_problem(cfg, 0, wgen) if cfg == "mesh4_ao16" else make_problem(cfg, 0, wgen)
    plan, Wq = _plan(B, p, nb=4)
    H = O.build_H(p, OW(p))
    ev, Z = np.linalg.eigh(H)
    om, x, it = plan.lowest_excitons(n_block=4, tol=1e-10, max_iter=500)
    print("[lobpcg] iterations %d, omega %s" % (it, om), flush=True)
    assert np.abs(om - ev[:4]).max() < 1e-8 * abs(ev[0])
    r = H @ H_(x) - H_(x) * om
    assert np.abs(r).max() < 1e-8


def test_lowest_gradient_vs_oracle_and_fd(B):
    from paper_2607_05853_amd import autograd as AG
    p = make_problem(SMALL, 1, "G2")
    W_R = T(p.W_R).requires_grad_(True)
    eps = T(p.eps_qp, torch.float64).requires_grad_(True)
    plan, Wq = _plan(B, p, W_R.detach(), eps.detach(), nb=4)
    om1 = AG.lowest_exciton_energy(plan, W_R, eps, n_block=4, tol=1e-12)
    om1.backward()
    Om_ref, ge_ref, gq_ref = O.grad_lowest(p, OW(p))
    gr_ref = O.grad_WR_from_Wq(gq_ref, p.R, p.w_R, dense_kmesh(p.nk))
    assert abs(om1.item() - Om_ref) < 1e-10
    assert rel(H_(eps.grad), ge_ref) < 1e-7
    assert rel(H_(W_R.grad), gr_ref) < 1e-7
    # central finite differences of the GPU path along an admissible direction
    h = 1e-6
    dW = _admissible(p, 5)

    def f(Wr):
        pl, _ = _plan(B, p, T(Wr), nb=4)
        om, _, _ = pl.lowest_excitons(n_block=4, tol=1e-13, max_iter=800, allow_unconverged=True)
        pl.close()
        return om[0]

    fd = (f(p.W_R + h * dW) - f(p.W_R - h * dW)) / (2 * h)
    an = np.real(np.vdot(H_(W_R.grad), dW))
    print("[grad Omega1] fd %.10e adjoint %.10e" % (fd, an), flush=True)
    assert abs(fd - an) < 1e-4 * max(abs(an), 1e-8)


def test_apply_autograd_matches_explicit(B):
    from paper_2607_05853_amd import autograd as AG
    p = make_problem(SMALL, 2, "G2")
    W_R = T(p.W_R).requires_grad_(True)
    eps = T(p.eps_qp, torch.float64).requires_grad_(True)
    plan, Wq = _plan(B, p, W_R.detach(), eps.detach(), nb=3)
    X = T(random_block(p.N, 3, seed=4)).requires_grad_(True)
    Yb_h = random_block(p.N, 3, seed=6)
    Yb = T(Yb_h)
    Y = AG.apply(plan, X, W_R, eps)
    L = torch.real(torch.sum(torch.conj(Yb) * Y))
    L.backward()
    H = O.build_H(p, OW(p))
    ge, gq = O.grad_apply(p, OW(p), Yb_h, random_block(p.N, 3, seed=4))
    gr = O.grad_WR_from_Wq(gq, p.R, p.w_R, dense_kmesh(p.nk))
    assert rel(H_(X.grad), H @ Yb_h) < 1e-12
    assert rel(H_(eps.grad), ge) < 1e-12
    assert rel(H_(W_R.grad), gr) < 1e-11


def test_spectrum_vjp_full_krylov_vs_oracle(B):
    # with m = dim the Lanczos resolvent is exact, so the VJP equals the oracle's
    # exact-resolvent gradient
    from paper_2607_05853_amd import autograd as AG
    p = make_problem(dict(cfg_id=97, coarse=(3, 3, 2), dense=(2, 2, 2), n_ao=8, nv=2, nc=2, n_aux=12), 0, "G2")
    W_R = T(p.W_R).requires_grad_(True)
    eps = T(p.eps_qp, torch.float64).requires_grad_(True)
    plan, Wq = _plan(B, p, W_R.detach(), eps.detach(), nb=2)
    P = O.velocity_start(p, np.eye(3))[:, :2]
    w = np.linspace(1.6, 3.2, 17)
    eta = 0.1
    gamma = np.random.default_rng(3).standard_normal((2, len(w)))
    S = AG.haydock_spectrum(plan, T(P), W_R, eps, p.N, w, eta)
    torch.sum(T(gamma, torch.float64) * S).backward()
    ge, gq = O.grad_spectrum(p, OW(p), P, w, eta, gamma)
    gr = O.grad_WR_from_Wq(gq, p.R, p.w_R, dense_kmesh(p.nk))
    print("[spectrum vjp] eps %.2e W_R %.2e" % (rel(H_(eps.grad), ge), rel(H_(W_R.grad), gr)), flush=True)
    assert rel(H_(eps.grad), ge) < 1e-7
    assert rel(H_(W_R.grad), gr) < 1e-7


def test_spectrum_vjp_fd_converged_chain(B):
    # fewer steps than the dimension: compare with FD of the Haydock output itself
    from paper_2607_05853_amd import autograd as AG
    p = make_problem(SMALL, 3, "G2")
    W_R = T(p.W_R).requires_grad_(True)
    eps = T(p.eps_qp, torch.float64).requires_grad_(True)
    plan, _ = _plan(B, p, W_R.detach(), eps.detach(), nb=2)
    P = T(O.velocity_start(p, np.eye(3))[:, :2])
    w = np.linspace(1.8, 3.0, 13)
    m = p.N  # 72: exact Krylov space
    gamma = np.random.default_rng(9).standard_normal((2, len(w)))
    S = AG.haydock_spectrum(plan, P, W_R, eps, m, w, 0.1)
    torch.sum(T(gamma, torch.float64) * S).backward()
    h = 1e-6
    de = np.random.default_rng(1).standard_normal(p.eps_qp.shape)

    def f(e):
        pl, _ = _plan(B, p, eps=T(e, torch.float64), nb=2)
        out = pl.haydock(P, m, w, 0.1)
        pl.close()
        return np.sum(gamma * out["S"])

    fd = (f(p.eps_qp + h * de) - f(p.eps_qp - h * de)) / (2 * h)
    an = float(np.sum(H_(eps.grad) * de))
    assert abs(fd - an) < 1e-4 * max(abs(an), 1e-8)


# BF16x3 gradients against the oracle's exact FP64 gradients, to the 1e-4 the mixed-precision path is held
# to.  SMALL (N_aux = 20) runs the BF16x3 adjoint on the register-staged kernels, TN_GRAD (n_v^2 and N_aux
# multiples of 8) on the k-major kernel with the pair-symmetric gradient
TN_GRAD = dict(cfg_id=84, coarse=(3, 3, 2), dense=(3, 2, 2), n_ao=16, nv=4, nc=3, n_aux=40)
TN_SPEC = dict(cfg_id=85, coarse=(3, 3, 2), dense=(2, 2, 2), n_ao=12, nv=4, nc=2, n_aux=24)


@pytest.mark.parametrize("cfg", ["SMALL", "TN_GRAD"])
def test_bf16x3_lowest_gradient_vs_oracle(B, cfg):
    # Hellmann-Feynman gradient of Omega_1 through the BF16x3 adjoint, with the eigenvector of the FP64
    # LOBPCG (on the BF16x3 operator the residual cannot fall below its rounding, ~4e-8 of |A|; the gradient
    # only needs x)
    p = make_problem({"SMALL": SMALL, "TN_GRAD": TN_GRAD}[cfg], 1, "G2")
    plan64, _ = _plan(B, p, prec="f64", nb=4)
    om, X, _ = plan64.lowest_excitons(n_block=4, tol=1e-12, max_iter=500)
    x = X[:, :1].contiguous()
    plan, _ = _plan(B, p, prec="bf16x3", nb=4)
    g = plan.apply_adjoint(x, x, want_WR=True, want_eps=True)
    om16 = torch.real(torch.sum(torch.conj(x) * plan.apply(x))).item()
    Om_ref, ge_ref, gq_ref = O.grad_lowest(p, OW(p))
    gr_ref = O.grad_WR_from_Wq(gq_ref, p.R, p.w_R, dense_kmesh(p.nk))
    e_om, e_e, e_w = abs(om16 - Om_ref) / abs(Om_ref), rel(H_(g["eps"]), ge_ref), rel(H_(g["W_R"]), gr_ref)
    print("[bf16x3 grad Omega1 %s] Omega %.1e eps %.1e W_R %.1e" % (cfg, e_om, e_e, e_w), flush=True)
    assert e_om < 1e-6 and e_e < 1e-4 and e_w < 1e-4


@pytest.mark.parametrize("cfg", ["SPEC", "TN_SPEC"])
def test_bf16x3_spectrum_vjp_vs_oracle(B, cfg):
    from paper_2607_05853_amd import autograd as AG
    conf = {"SPEC": dict(cfg_id=97, coarse=(3, 3, 2), dense=(2, 2, 2), n_ao=8, nv=2, nc=2, n_aux=12),
            "TN_SPEC": TN_SPEC}[cfg]
    p = make_problem(conf, 0, "G2")
    W_R = T(p.W_R).requires_grad_(True)
    eps = T(p.eps_qp, torch.float64).requires_grad_(True)
    plan, _ = _plan(B, p, W_R.detach(), eps.detach(), prec="bf16x3", nb=2)
    P = O.velocity_start(p, np.eye(3))[:, :2]
    w = np.linspace(1.6, 3.2, 17)
    gamma = np.random.default_rng(3).standard_normal((2, len(w)))
    S = AG.haydock_spectrum(plan, T(P), W_R, eps, p.N, w, 0.1)  # full Krylov space: exact resolvent
    torch.sum(T(gamma, torch.float64) * S).backward()
    ge, gq = O.grad_spectrum(p, OW(p), P, w, 0.1, gamma)
    gr = O.grad_WR_from_Wq(gq, p.R, p.w_R, dense_kmesh(p.nk))
    e_e, e_w = rel(H_(eps.grad), ge), rel(H_(W_R.grad), gr)
    print("[bf16x3 spectrum vjp %s] eps %.1e W_R %.1e" % (cfg, e_e, e_w), flush=True)
    assert e_e < 1e-4 and e_w < 1e-4


@pytest.mark.parametrize("prec", ["bf16x3", "f32"])
def test_lobpcg_lowest_reduced_precision(B, prec):
    # Rayleigh-Ritz on a reduced-precision operator must drop nearly dependent directions at a threshold
    # above the apply's rounding; otherwise the rounding turns into spurious Ritz values
    p = make_problem(DMA_LOB, 0, "G2")
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
    plan = B.plan_from_problem(p, Wq, prec=prec, max_nb=16)
    ev = np.linalg.eigvalsh(O.build_H(p, OW(p)))
    om, _, it = plan.lowest_excitons(n_block=4, tol=1e-6, max_iter=300, want_vectors=False)
    print("[lobpcg %s] iterations %d, omega %s, ref %s" % (prec, it, om, ev[:4]), flush=True)
    assert np.abs(om - ev[:4]).max() < 1e-6 * abs(ev[0])
    plan.close()


def test_lobpcg_mesh8_bf16x3_matches_f64(B):
    # at the timed 8^3 workload the BF16x3 iteration once produced Ritz values near -1e24 (directions
    # kept down to 1e-12 of the Gram spectrum); it must converge to the FP64 plan's lowest excitons
    p = make_problem("mesh8_ao64", 0, "G1")
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
    om = {}
    for prec, tol in [("f64", 1e-9), ("bf16x3", 1e-6)]:
        plan = B.plan_from_problem(p, Wq, prec=prec, max_nb=8)
        om[prec], _, it = plan.lowest_excitons(n_block=4, tol=tol, max_iter=300, want_vectors=False)
        print("[lobpcg mesh8 %s] iterations %d, omega %s" % (prec, it, om[prec]), flush=True)
        plan.close()
    assert np.abs(om["bf16x3"] - om["f64"]).max() < 1e-6 * om["f64"][0]


def test_bf16x3_autograd_lowest_energy_vs_oracle(B):
    # the differentiable lowest exciton energy on a BF16x3 plan end to end: LOBPCG to the tolerance the plan's
    # precision can reach (its default), Hellmann-Feynman backward through the BF16x3 adjoint
    from paper_2607_05853_amd import autograd as AG
    p = make_problem(DMA_LOB, 1, "G2")
    W_R = T(p.W_R).requires_grad_(True)
    eps = T(p.eps_qp, torch.float64).requires_grad_(True)
    plan, _ = _plan(B, p, W_R.detach(), eps.detach(), prec="bf16x3", nb=4)
    om1 = AG.lowest_exciton_energy(plan, W_R, eps, n_block=4)
    om1.backward()
    Om_ref, ge_ref, gq_ref = O.grad_lowest(p, OW(p))
    gr_ref = O.grad_WR_from_Wq(gq_ref, p.R, p.w_R, dense_kmesh(p.nk))
    e_om, e_e, e_w = abs(om1.item() - Om_ref) / abs(Om_ref), rel(H_(eps.grad), ge_ref), rel(H_(W_R.grad), gr_ref)
    print("[bf16x3 autograd Omega1] Omega %.1e eps %.1e W_R %.1e" % (e_om, e_e, e_w), flush=True)
    assert e_om < 1e-6 and e_e < 1e-4 and e_w < 1e-4
