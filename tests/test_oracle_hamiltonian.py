"""Pins of the oracle's explicit TDA Hamiltonian (Eq. (Hamiltonian) through Eq. (W_LRI))."""
import dataclasses
import json
import os

import numpy as np
import pytest

import oracle as O
from synth import make_problem, dense_kmesh
from synth.crystal import Problem

with open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")) as _f:
    GOLD = json.load(_f)


def _Wq(p):
    return O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))


def _manual_problem(nk, eps_v, eps_c, C, Vbar, R, W_R, alpha):
    Nk = int(np.prod(nk))
    psi = np.zeros((Nk, 2, C.shape[1]), dtype=complex)
    psi[:, 0, 0] = 1.0
    psi[:, 1, 1] = 1.0
    eps = np.tile([eps_v, eps_c], (Nk, 1)).astype(float)
    return Problem(name="hand", nk=tuple(nk), coarse=tuple(nk), n_ao=C.shape[1], nv=1, nc=1,
                   n_aux=C.shape[0], alpha=alpha, eps_ks=eps, eps_qp=eps, psi=psi,
                   vel=np.zeros((3, Nk, 1, 1), dtype=complex), C=C, Vbar=Vbar,
                   R=np.asarray(R, dtype=np.int32), w_R=np.ones(len(R)), W_R=W_R)


def test_hand_one_k():
    g = GOLD["one_k"]
    C = np.array([[[complex(*x) for x in row] for row in g["C"]]])
    p = _manual_problem((1, 1, 1), g["eps_v"], g["eps_c"], C, np.array([[g["Vbar"]]], dtype=complex),
                        [[0, 0, 0]], np.array([[[g["W0"]]]], dtype=complex), g["alpha"])
    H = O.build_H(p, _Wq(p))
    Ccv, Cvv, Ccc = C[0, 1, 0], C[0, 0, 0], C[0, 1, 1]
    expect = (g["eps_c"] - g["eps_v"]) + g["alpha"] * g["Vbar"] * abs(Ccv) ** 2 - Cvv * g["W0"] * Ccc
    assert H.shape == (1, 1)
    assert abs(H[0, 0] - expect) < 1e-15


def test_hand_three_k_phase_orientation():
    g = GOLD["three_k"]
    b = complex(*g["b"])
    C = np.array([[[g["a"], b], [np.conj(b), g["d"]]]], dtype=complex)
    R = [[0, 0, 0], [1, 0, 0]]
    W_R = np.array([[[g["W_R0"]]], [[g["W_Rx"]]]], dtype=complex)
    p = _manual_problem(g["dense"], g["eps_v"], g["eps_c"], C, np.array([[g["Vbar"]]], dtype=complex),
                        R, W_R, g["alpha"])
    H = O.build_H(p, _Wq(p))
    expect = np.zeros((3, 3), dtype=complex)
    for k in range(3):
        for kp in range(3):
            q = (kp - k) / 3.0
            expect[k, kp] = (g["alpha"] * g["Vbar"] * abs(b) ** 2 / 3
                             - g["a"] * g["d"] * (g["W_R0"] + g["W_Rx"] * np.exp(2j * np.pi * q)) / 3)
        expect[k, k] += g["eps_c"] - g["eps_v"]
    assert np.abs(H - expect).max() < 1e-15


def _ao_bruteforce_H(p, Wq):
    """Independent factorisation through the 4-index AO kernels (pure Python loops).

    K^W_{s't',st}(q) = sum_munu C^mu_{s't'} W_munu(q) C^nu_{st},
    K^V_{s't',st}    = sum_munu C^mu_{s't'} Vbar_munu C^nu_{st},
    A = diag - (1/N_k) sum conj(psi_v'(k')_s') psi_v(k)_t' K^W conj(psi_c(k)_s) psi_c'(k')_t
             + (alpha/N_k) sum conj(psi_c(k)_s') psi_v(k)_t' K^V conj(psi_v'(k')_s) psi_c'(k')_t
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
    N = p.N
    H = np.zeros((N, N), dtype=complex)
    te = O.transition_energies(p)
    for k in range(Nk):
        for kp in range(Nk):
            q = O.q_index(p.nk, k, kp)
            for c in range(nc):
                for v in range(nv):
                    I = (k * nc + c) * nv + v
                    for c2 in range(nc):
                        for v2 in range(nv):
                            J = (kp * nc + c2) * nv + v2
                            lv = np.conj(p.psi[kp, v2])[:, None] * p.psi[k, v][None, :]          # (s', t')
                            rc = np.conj(p.psi[k, nv + c])[:, None] * p.psi[kp, nv + c2][None, :]  # (s, t)
                            d = np.einsum("ab,abcd,cd->", lv, KW[q], rc)
                            lx = np.conj(p.psi[k, nv + c])[:, None] * p.psi[k, v][None, :]
                            rx = np.conj(p.psi[kp, v2])[:, None] * p.psi[kp, nv + c2][None, :]
                            x = np.einsum("ab,abcd,cd->", lx, KV, rx)
                            H[I, J] = -d / Nk + p.alpha * x / Nk
            if k == kp:
                for c in range(nc):
                    for v in range(nv):
                        I = (k * nc + c) * nv + v
                        H[I, I] += te[k, c * nv + v]
    return H


@pytest.mark.parametrize("complex_vbar", [False, True])
@pytest.mark.parametrize("dense", [(2, 2, 1), (3, 2, 1)])
@pytest.mark.parametrize("wgen", ["G1", "G2"])
def test_bruteforce_ao_kernel(wgen, dense, complex_vbar):
    # On the 2x2x1 mesh every q is its own negative, so W(q) = W(-q) = W(q)^T even for G2 and the mu <-> nu
    # orientation of W in the direct term is invisible; the 3x2x1 mesh has q != -q, where G2's W(q) is not
    # symmetric and the brute force fixes which pair density carries mu (the valence one) and which nu.
    # The generators' Vbar is real symmetric (real auxiliary functions); a complex Hermitian Vbar fixes the
    # orientation of the exchange term the same way (mu on the density at k, nu on the one at k').
    p = make_problem(dict(cfg_id=92, coarse=(3, 3, 2), dense=dense, n_ao=4, nv=2, nc=2, n_aux=6), 1, wgen)
    if complex_vbar:
        A = np.random.default_rng(8).standard_normal((p.n_aux, p.n_aux))
        p = dataclasses.replace(p, Vbar=p.Vbar + 0.1j * (A - A.T))
        assert np.abs(p.Vbar.imag).max() > 1e-2
    Wq = _Wq(p)
    H = O.build_H(p, Wq)
    Hb = _ao_bruteforce_H(p, Wq)
    assert np.abs(H - Hb).max() < 1e-13 * np.abs(H).max()


@pytest.mark.parametrize("wgen", ["G1", "G2"])
def test_hermitian(tiny_cfg, wgen):
    p = make_problem(tiny_cfg, 0, wgen, coarse=(3, 3, 2))
    H = O.build_H(p, _Wq(p))
    assert np.abs(H - H.conj().T).max() <= 1e-14 * np.abs(H).max()


def test_zero_kernel_is_transition_energies(small_cfg):
    p = make_problem(small_cfg, 0)
    p.W_R = p.W_R * 0
    p.Vbar = p.Vbar * 0
    H = O.build_H(p, _Wq(p))
    te = O.transition_energies(p).ravel()
    assert np.abs(H - np.diag(te)).max() == 0.0
    # the diagonal is E^QP_ck - E^QP_vk in the row order (k, c, v), written out here without the oracle; the
    # scissor makes the Kohn-Sham differences another diagonal, and n_c != n_v another (v, c) order
    nv = p.nv
    te_ref = np.array([p.eps_qp[k, nv + c] - p.eps_qp[k, v]
                       for k in range(p.Nk) for c in range(p.nc) for v in range(nv)])
    assert np.array_equal(np.diag(H).real, te_ref)
    assert np.abs((p.eps_qp - p.eps_ks)[:, nv:]).min() > 0.1 and p.nc != p.nv
    # IPA limit of the spectrum: peaks at e_c - e_v with weight |p_I|^2 / N_k
    P = O.velocity_start(p, np.eye(3))
    w = np.linspace(1.0, 6.0, 101)
    S, Om, Z = O.eig_spectrum(H, P, w, 0.1, p.Nk)
    ipa = np.array([[np.sum(np.abs(P[:, e]) ** 2 * (0.1 / np.pi) / ((x - te) ** 2 + 0.01)) for x in w]
                    for e in range(3)]) / p.Nk
    assert np.abs(S - ipa).max() < 1e-12 * np.abs(ipa).max()


def test_exchange_psd_low_rank_and_alpha(small_cfg):
    p = make_problem(small_cfg, 0)
    p.W_R = p.W_R * 0
    te = np.diag(O.transition_energies(p).ravel())
    Hx = O.build_H(p, _Wq(p)) - te
    ev = np.linalg.eigvalsh(Hx)
    assert ev.min() > -1e-13 * ev.max()
    assert np.sum(ev > 1e-10 * ev.max()) <= p.n_aux
    # triplet channel (alpha = 0) removes exchange entirely
    H0 = O.build_H(p, _Wq(p), alpha=0.0)
    assert np.abs(H0 - te).max() == 0.0
    # linearity in alpha
    H1 = O.build_H(p, _Wq(p), alpha=1.0) - te
    assert np.abs(2 * H1 - Hx).max() < 1e-14 * np.abs(te).max()


def test_linearity_in_W(tiny_cfg):
    p = make_problem(tiny_cfg, 0, "G2", coarse=(3, 3, 2))
    Wq = _Wq(p)
    te = np.diag(O.transition_energies(p).ravel())
    H1 = O.build_H(p, Wq)
    H2 = O.build_H(p, 2.0 * Wq)
    H0 = O.build_H(p, 0 * Wq)
    assert np.abs((H2 - H0) - 2 * (H1 - H0)).max() < 1e-14 * np.abs(H1).max()


def test_gauge_covariance(small_cfg):
    # psi_nk -> exp(i phi_nk) psi_nk is a unitary change of the transition basis:
    # eigenvalues and the spectrum are unchanged
    p = make_problem(small_cfg, 0, "G2", coarse=(3, 3, 2))
    Wq = _Wq(p)
    P = O.velocity_start(p, np.eye(3))
    w = np.linspace(1.5, 5.0, 57)
    S, Om, _ = O.eig_spectrum(O.build_H(p, Wq), P, w, 0.1, p.Nk)
    rng = np.random.default_rng(5)
    ph = np.exp(2j * np.pi * rng.random(p.psi.shape[:2]))
    p.psi = p.psi * ph[:, :, None]
    nv = p.nv
    p.vel = p.vel * np.conj(ph[None, :, nv:, None]) * ph[None, :, None, :nv]
    S2, Om2, _ = O.eig_spectrum(O.build_H(p, Wq), O.velocity_start(p, np.eye(3)), w, 0.1, p.Nk)
    assert np.abs(Om - Om2).max() < 1e-12
    assert np.abs(S - S2).max() < 1e-11 * np.abs(S).max()


def test_q_index_is_the_mesh_index_of_the_difference():
    # q_index(k, k') is the position in the mesh of k' - k (mod 1), found here by coordinates on a mesh with
    # three different sizes, so that a swapped axis or a reversed difference shows; the oracle's mesh is the
    # one the inputs are generated on
    nk = (3, 2, 5)
    km = O.kmesh(nk)
    assert np.array_equal(km, dense_kmesh(nk))
    for i in range(len(km)):
        for j in range(len(km)):
            d = (km[j] - km[i]) % 1.0
            hit = np.flatnonzero(np.all(np.abs(((km - d) + 0.5) % 1.0 - 0.5) < 1e-12, axis=1))
            assert len(hit) == 1 and O.q_index(nk, i, j) == hit[0]


def test_lowest_exciton_is_the_lowest_eigenpair(small_cfg):
    # (Omega_1, x) is an eigenpair of A with |x| = 1, and A - Omega_1 is positive semi-definite (a Cholesky
    # factorisation of A - Omega_1 + 1e-9 succeeds, of A - Omega_1 - 1e-9 fails)
    p = make_problem(small_cfg, 0, "G2", coarse=(3, 3, 2))
    H = O.build_H(p, _Wq(p))
    Om, x = O.lowest_exciton(H)
    assert x.shape == (p.N,)
    assert abs(np.linalg.norm(x) - 1.0) < 1e-13
    assert np.abs(H @ x - Om * x).max() < 1e-12 * np.abs(H).max()
    eye = np.eye(p.N)

    def positive_definite(M):
        try:
            np.linalg.cholesky(M)
            return True
        except np.linalg.LinAlgError:
            return False

    assert positive_definite(H - (Om - 1e-9) * eye)
    assert not positive_definite(H - (Om + 1e-9) * eye)


def test_apply_rows_match_explicit(small_cfg):
    p = make_problem(small_cfg, 0, "G2", coarse=(3, 3, 2))
    Wq = _Wq(p)
    H = O.build_H(p, Wq)
    X = np.random.default_rng(2).standard_normal((p.N, 3)) + 0j
    nt = p.nc * p.nv
    rows = [0, 5, 11]
    Y = O.apply_H_rows(p, Wq, X, rows)
    ref = np.concatenate([H[k * nt:(k + 1) * nt] @ X for k in rows])
    assert np.abs(Y - ref).max() < 1e-13 * np.abs(ref).max()


def test_velocity_start_hand_case():
    # Eq. (abs_vel): amplitude <v k|v|c k> / (E^KS_c - E^KS_v) uses Kohn-Sham energies, not the
    # quasiparticle ones of the diagonal; p_I is the conjugate of that amplitude.
    C = np.zeros((1, 2, 2), dtype=complex)
    p = _manual_problem((1, 1, 1), -1.0, 1.5, C, np.zeros((1, 1), dtype=complex), [[0, 0, 0]],
                        np.zeros((1, 1, 1), dtype=complex), 2.0)
    p.eps_qp = p.eps_ks + np.array([[0.0, 1.0]])
    p.vel = np.zeros((3, 1, 1, 1), dtype=complex)
    p.vel[0, 0, 0, 0] = 1 + 2j
    p.vel[1, 0, 0, 0] = 3.0
    P = O.velocity_start(p, np.array([[1.0, 0, 0], [np.sqrt(0.5), np.sqrt(0.5), 0]]))
    assert abs(P[0, 0] - (0.4 + 0.8j)) < 1e-15
    assert abs(P[0, 1] - (4 + 2j) * np.sqrt(0.5) / 2.5) < 1e-15
