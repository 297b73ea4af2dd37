"""Pins of the oracle's gradients against finite differences and the first-moment identity."""
import numpy as np
import pytest

import oracle as O
from synth import make_problem, dense_kmesh


def _setup(cfg):
    p = make_problem(cfg, 0, "G2", coarse=(3, 3, 2))
    kq = dense_kmesh(p.nk)
    return p, kq


def _admissible_dWR(p, seed):
    # real delta W(R) with delta W(-R) = delta W(R)^T keeps H Hermitian
    rng = np.random.default_rng(seed)
    idx = {tuple(r): i for i, r in enumerate(p.R)}
    d = np.zeros(p.W_R.shape)
    for i, r in enumerate(p.R):
        j = idx[tuple(-r)]
        if j < i:
            continue
        A = rng.standard_normal(p.W_R.shape[1:]) * 1e-2
        if i == j:
            A = A + A.T
        d[i] = A
        d[j] = A.T
    return d.astype(complex)


def test_apply_gradient_is_exact_linear_response(tiny_cfg):
    _linear_response(tiny_cfg)


def test_apply_gradient_linear_response_where_q_differs_from_minus_q(small_cfg):
    # on the 2x2x2 mesh every q is its own negative, so the phase sign of the W(R) gradient and which of
    # q, -q a pair's contribution goes to are invisible there; the 3x2x2 mesh shows both
    _linear_response(small_cfg)


def _linear_response(cfg):
    # L = Re <Ybar, H(W) X> is linear in W(R) and eps: its derivative along any direction
    # equals the difference quotient exactly (up to rounding)
    p, kq = _setup(cfg)
    rng = np.random.default_rng(1)
    Yb = rng.standard_normal((p.N, 2)) + 1j * rng.standard_normal((p.N, 2))
    X = rng.standard_normal((p.N, 2)) + 1j * rng.standard_normal((p.N, 2))
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, kq)
    g_eps, g_Wq = O.grad_apply(p, Wq, Yb, X)
    g_WR = O.grad_WR_from_Wq(g_Wq, p.R, p.w_R, kq)

    def L(W_R, eps):
        q = O.interpolate_W(W_R, p.R, p.w_R, kq)
        p.eps_qp, old = eps, p.eps_qp
        val = np.real(np.vdot(Yb, O.build_H(p, q) @ X))
        p.eps_qp = old
        return val

    # general complex direction in W(R) (L is real-linear in W)
    dW = rng.standard_normal(p.W_R.shape) + 1j * rng.standard_normal(p.W_R.shape)
    fd = L(p.W_R + dW, p.eps_qp) - L(p.W_R, p.eps_qp)
    assert abs(fd - np.real(np.vdot(g_WR, dW))) < 1e-10 * max(1, abs(fd))
    de = rng.standard_normal(p.eps_qp.shape)
    fd = L(p.W_R, p.eps_qp + de) - L(p.W_R, p.eps_qp)
    assert abs(fd - np.sum(g_eps * de)) < 1e-10 * max(1, abs(fd))


def test_first_moment_identity(tiny_cfg):
    # d(p^H H p)/d theta = p^H (dH/d theta) p with dH from two explicit Hamiltonians
    p, kq = _setup(tiny_cfg)
    P = O.velocity_start(p, np.eye(3))[:, :1]
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, kq)
    g_eps, g_Wq = O.grad_apply(p, Wq, P, P)
    dWq = np.random.default_rng(4).standard_normal(Wq.shape) * 1e-3 + 0j
    dH = O.build_H(p, Wq + dWq) - O.build_H(p, Wq)
    lhs = np.real(np.vdot(P[:, 0], dH @ P[:, 0]))
    assert abs(lhs - np.real(np.vdot(g_Wq, dWq))) < 1e-12 * max(abs(lhs), 1e-12) + 1e-16


def test_lowest_exciton_gradient_fd(small_cfg):
    p, kq = _setup(small_cfg)
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, kq)
    Om1, g_eps, g_Wq = O.grad_lowest(p, Wq)
    g_WR = O.grad_WR_from_Wq(g_Wq, p.R, p.w_R, kq)
    # closed form for eps: dOmega_1/de_ck = sum_v |x_cvk|^2, checked by FD
    h = 1e-6
    for (k, n) in [(0, 0), (3, p.nv), (5, p.nv + 1)]:
        e = p.eps_qp.copy()
        e[k, n] += h
        p.eps_qp, old = e, p.eps_qp
        up = np.linalg.eigvalsh(O.build_H(p, Wq))[0]
        e2 = old.copy()
        e2[k, n] -= h
        p.eps_qp = e2
        dn = np.linalg.eigvalsh(O.build_H(p, Wq))[0]
        p.eps_qp = old
        assert abs((up - dn) / (2 * h) - g_eps[k, n]) < 1e-7
    dW = _admissible_dWR(p, 3)
    f = lambda W: np.linalg.eigvalsh(O.build_H(p, O.interpolate_W(W, p.R, p.w_R, kq)))[0]
    fd = (f(p.W_R + h * dW) - f(p.W_R - h * dW)) / (2 * h)
    assert abs(fd - np.real(np.vdot(g_WR, dW))) < 1e-7 * max(1.0, abs(fd))


def test_spectrum_gradient_fd(tiny_cfg):
    p, kq = _setup(tiny_cfg)
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, kq)
    P = O.velocity_start(p, np.eye(3))[:, :2]
    w = np.linspace(1.8, 3.0, 9)
    eta = 0.1
    gamma = np.random.default_rng(8).standard_normal((2, len(w)))
    g_eps, g_Wq = O.grad_spectrum(p, Wq, P, w, eta, gamma)
    g_WR = O.grad_WR_from_Wq(g_Wq, p.R, p.w_R, kq)

    def L(W_R, eps):
        p.eps_qp, old = eps, p.eps_qp
        S = O.eig_spectrum(O.build_H(p, O.interpolate_W(W_R, p.R, p.w_R, kq)), P, w, eta, p.Nk)[0]
        p.eps_qp = old
        return np.sum(gamma * S)

    h = 1e-6
    dW = _admissible_dWR(p, 9)
    fd = (L(p.W_R + h * dW, p.eps_qp) - L(p.W_R - h * dW, p.eps_qp)) / (2 * h)
    assert abs(fd - np.real(np.vdot(g_WR, dW))) < 1e-6 * max(1.0, abs(fd))
    de = np.random.default_rng(2).standard_normal(p.eps_qp.shape)
    fd = (L(p.W_R, p.eps_qp + h * de) - L(p.W_R, p.eps_qp - h * de)) / (2 * h)
    assert abs(fd - np.sum(g_eps * de)) < 1e-6 * max(1.0, abs(fd))
