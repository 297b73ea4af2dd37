"""Pins of the oracle's full BSE (coupling block B of Eq. (Hamiltonian), the paired eigenproblem of
Eqs. (right)/(left) and the spectrum of Eq. (full_BSE_epsilon2))."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from synth import dense_kmesh, make_problem, polarisations

SMALL = dict(cfg_id=83, coarse=(3, 3, 2), dense=(3, 2, 2), n_ao=8, nv=2, nc=3, n_aux=12)


def _Wq(p):
    return O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))


def _ao_bruteforce_B(p, Wq):
    """Coupling block through the 4-index AO kernels (pure Python loops, bands contracted last).

    K^W_{s't',st}(q) = sum_munu C^mu_{s't'} W_munu(q) C^nu_{st},  K^V likewise with Vbar;
    B = -(1/N_k) sum conj(psi_c'(k')_s') psi_v(k)_t' K^W(k'-k) conj(psi_c(k)_s) psi_v'(k')_t
        + (alpha/N_k) sum conj(psi_c(k)_s') psi_v(k)_t' K^V conj(psi_c'(k')_s) psi_v'(k')_t
    """
    nv, nc, Nk, na = p.nv, p.nc, p.Nk, p.n_ao
    KW = np.zeros((Nk, na, na, na, na), dtype=complex)
    for q in range(Nk):
        for a in range(na):
            for b_ in range(na):
                KW[q, a, b_] = np.tensordot(p.C[:, a, b_] @ Wq[q], p.C, axes=(0, 0))
    KV = np.zeros((na, na, na, na), dtype=complex)
    for a in range(na):
        for b_ in range(na):
            KV[a, b_] = np.tensordot(p.C[:, a, b_] @ p.Vbar, p.C, axes=(0, 0))
    B = np.zeros((p.N, p.N), dtype=complex)
    for k in range(Nk):
        for kp in range(Nk):
            q = O.q_index(p.nk, k, kp)
            for c in range(nc):
                for v in range(nv):
                    I = (k * nc + c) * nv + v
                    for c2 in range(nc):
                        for v2 in range(nv):
                            J = (kp * nc + c2) * nv + v2
                            ld = np.conj(p.psi[kp, nv + c2])[:, None] * p.psi[k, v][None, :]
                            rd = np.conj(p.psi[k, nv + c])[:, None] * p.psi[kp, v2][None, :]
                            d = np.einsum("ab,abcd,cd->", ld, KW[q], rd)
                            lx = np.conj(p.psi[k, nv + c])[:, None] * p.psi[k, v][None, :]
                            rx = np.conj(p.psi[kp, nv + c2])[:, None] * p.psi[kp, v2][None, :]
                            x = np.einsum("ab,abcd,cd->", lx, KV, rx)
                            B[I, J] = -d / Nk + p.alpha * x / Nk
    return B


@pytest.mark.parametrize("complex_vbar", [False, True])
@pytest.mark.parametrize("dense", [(2, 2, 1), (3, 2, 1)])
@pytest.mark.parametrize("wgen", ["G1", "G2"])
def test_coupling_block_bruteforce(wgen, dense, complex_vbar):
    # the 3x2x1 mesh has q != -q, where G2's W(q) is not symmetric, so which of W(q), W(-q) = W(q)^T the
    # direct term takes shows; a complex Hermitian Vbar shows the orientation of the exchange term (the
    # generators' Vbar is real symmetric)
    p = make_problem(dict(cfg_id=82, coarse=(3, 3, 2), dense=dense, n_ao=4, nv=2, nc=2, n_aux=6), 1, wgen)
    if complex_vbar:
        A = np.random.default_rng(8).standard_normal((p.n_aux, p.n_aux))
        p = dataclasses.replace(p, Vbar=p.Vbar + 0.1j * (A - A.T))
    Wq = _Wq(p)
    B = O.build_B(p, Wq)
    Bb = _ao_bruteforce_B(p, Wq)
    assert np.abs(B - Bb).max() < 1e-13 * np.abs(B).max()


@pytest.mark.parametrize("two_centre", [False, True])
@pytest.mark.parametrize("wgen", ["G1", "G2"])
def test_coupling_block_is_symmetric(wgen, two_centre):
    # B^T = B (and A^H = A) for real W(R) with W(-R) = W(R)^T and a real symmetric Vbar
    p = make_problem(SMALL, 2, wgen, two_centre=two_centre)
    Wq = _Wq(p)
    B = O.build_B(p, Wq)
    assert np.abs(B - B.T).max() < 1e-14 * np.abs(B).max()
    assert np.abs(B - B.conj().T).max() > 1e-3 * np.abs(B).max()   # complex symmetric, not Hermitian


def test_paired_eigenproblem():
    p = make_problem(SMALL, 3, "G2")
    Wq = _Wq(p)
    A, B = O.build_H(p, Wq), O.build_B(p, Wq)
    H = O.build_full(p, Wq)
    Om, X, Y = O.full_bse_eig(A, B)
    N = p.N
    Z = np.vstack([X, Y])
    # right eigenvectors of the explicit Hamiltonian, normalisation X^H X - Y^H Y = I (all S at once)
    assert np.abs(H @ Z - Z * Om[None, :]).max() < 1e-11 * np.abs(H).max()
    assert np.abs(X.conj().T @ X - Y.conj().T @ Y - np.eye(N)).max() < 1e-10
    # the negative branch: (Y*, X*) with -Omega; left eigenvectors (X^H, -Y^H) of Eq. (left)
    Zm = np.vstack([Y.conj(), X.conj()])
    assert np.abs(H @ Zm + Zm * Om[None, :]).max() < 1e-11 * np.abs(H).max()
    L = np.hstack([X.conj().T, -Y.conj().T])
    assert np.abs(L @ H - Om[:, None] * L).max() < 1e-11 * np.abs(H).max()
    # the library's general eigensolver gives the same +-Omega pairs
    ev = np.sort(np.linalg.eigvals(H).real)
    assert np.abs(ev[N:] - Om).max() < 1e-10 and np.abs(ev[:N] + Om[::-1]).max() < 1e-10
    # stable ground state: the coupling lowers every excitation relative to the TDA one at the bottom
    assert Om[0] < np.linalg.eigvalsh(A)[0]


def test_no_coupling_is_tda():
    p = make_problem(SMALL, 4, "G1")
    A = O.build_H(p, _Wq(p))
    Om, X, Y = O.full_bse_eig(A, np.zeros_like(A))
    assert np.abs(Om - np.linalg.eigvalsh(A)).max() < 1e-12
    assert np.abs(Y).max() < 1e-12
    w = np.linspace(1.0, 5.0, 81)
    P = O.velocity_start(p, polarisations(2))
    S = O.full_bse_spectrum(p, polarisations(2), Om, X, Y, w, 0.1)
    ref = O.eig_spectrum(A, P, w, 0.1, p.Nk)[0]
    assert np.abs(S - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("b", [0.3, 0.2 + 0.5j, -0.9j])
def test_two_level_closed_form(b):
    # one transition: Omega = sqrt(a^2 - |b|^2), |X|^2 = (a + Omega) / (2 Omega), |Y|^2 = (a - Omega) / (2 Omega)
    a = 2.0
    Om, X, Y = O.full_bse_eig(np.array([[a]], dtype=complex), np.array([[b]], dtype=complex))
    w = np.sqrt(a * a - abs(b) ** 2)
    assert abs(Om[0] - w) < 1e-14
    assert abs(abs(X[0, 0]) ** 2 - (a + w) / (2 * w)) < 1e-13
    assert abs(abs(Y[0, 0]) ** 2 - (a - w) / (2 * w)) < 1e-13
    assert abs(Y[0, 0] / X[0, 0] + np.conj(b) / (a + w)) < 1e-13


def test_spectrum_resolvent_identity():
    # with v = [p; p*] and J = diag(I, -I):
    #   -(1/pi) Im v^H J (omega + i eta - H)^{-1} v / N_k = sum_S |a_S|^2 [L(omega - Omega_S) - L(omega + Omega_S)] / N_k
    # which fixes the signs of the X and Y terms of Eq. (full_BSE_epsilon2) against the operator
    p = make_problem(SMALL, 5, "G2")
    Wq = _Wq(p)
    A, B = O.build_H(p, Wq), O.build_B(p, Wq)
    H = O.build_full(p, Wq)
    Om, X, Y = O.full_bse_eig(A, B)
    pol = polarisations(3)
    P = O.velocity_start(p, pol)
    w = np.linspace(0.5, 5.0, 31)
    eta = 0.15
    S = O.full_bse_spectrum(p, pol, Om, X, Y, w, eta)
    amp = np.abs(O.full_bse_amplitudes(p, pol, X, Y)) ** 2
    tail = (amp.T @ O.lorentzian(w[None, :] + Om[:, None], eta)) / p.Nk
    N = p.N
    J = np.r_[np.ones(N), -np.ones(N)]
    for e in range(len(pol)):
        v = np.r_[P[:, e], P[:, e].conj()]
        f = np.array([np.vdot(v, J * np.linalg.solve((x + 1j * eta) * np.eye(2 * N) - H, v)) for x in w])
        assert np.abs(-f.imag / np.pi / p.Nk - (S[e] - tail[e])).max() < 1e-10 * np.abs(S[e]).max()


def test_planted_amplitude_sign_fails_the_identity():
    # the Y term with the wrong sign (or without the conjugate) breaks the resolvent identity
    p = make_problem(SMALL, 5, "G2")
    Wq = _Wq(p)
    A, B = O.build_H(p, Wq), O.build_B(p, Wq)
    H = O.build_full(p, Wq)
    Om, X, Y = O.full_bse_eig(A, B)
    P = O.velocity_start(p, polarisations(1))[:, 0]
    N = p.N
    J = np.r_[np.ones(N), -np.ones(N)]
    x, eta = Om[0], 0.15
    v = np.r_[P, P.conj()]
    f = np.vdot(v, J * np.linalg.solve((x + 1j * eta) * np.eye(2 * N) - H, v))
    L = lambda d: O.lorentzian(d, eta)
    for amp in [P.conj() @ X + P @ Y, P.conj() @ X - P.conj() @ Y]:
        val = np.sum(np.abs(amp) ** 2 * (L(x - Om) - L(x + Om))) / p.Nk
        assert abs(-f.imag / np.pi / p.Nk - val) > 1e-4 * abs(val)
