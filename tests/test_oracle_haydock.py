"""Pins of the oracle's Haydock recurrence and continued fraction (Lanczos, not in the paper)."""
import numpy as np
import pytest

import oracle as O
from synth import make_problem, dense_kmesh


def _setup(cfg, wgen="G2"):
    p = make_problem(cfg, 0, wgen, coarse=(3, 3, 2))
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))
    H = O.build_H(p, Wq)
    P = O.velocity_start(p, np.eye(3))
    return p, H, P


def test_full_krylov_equals_eigh(tiny_cfg):
    # With m >= dim the Lanczos continued fraction is the exact resolvent element.
    p, H, P = _setup(tiny_cfg)
    assert p.N == 32
    w = np.linspace(1.0, 5.0, 201)
    Sref, _, _ = O.eig_spectrum(H, P, w, 0.1, p.Nk)
    S, a, b, st = O.haydock_spectrum(lambda x: H @ x, P, p.N, w, 0.1, p.Nk)
    assert np.abs(S - Sref).max() < 1e-11 * np.abs(Sref).max()


def test_full_krylov_indefinite_operator(tiny_cfg):
    # the recurrence is that of any Hermitian operator: shifted so that its spectrum has both signs (and
    # Rayleigh quotients of both signs occur), the full-Krylov continued fraction is still the resolvent
    p, H, P = _setup(tiny_cfg)
    ev = np.linalg.eigvalsh(H)
    Hs = H - np.median(ev) * np.eye(p.N)
    w = np.linspace(-3.0, 3.0, 201)
    Sref, _, _ = O.eig_spectrum(Hs, P, w, 0.1, p.Nk)
    S, a, b, st = O.haydock_spectrum(lambda x: Hs @ x, P, p.N, w, 0.1, p.Nk)
    assert (a < 0).any() and (a > 0).any()
    assert np.abs(S - Sref).max() < 1e-11 * np.abs(Sref).max()


def test_moment_identities(small_cfg):
    # p^H H^n p = b_0^2 (T_m^n)_{11} for n <= 2m - 1, at every m
    p, H, P = _setup(small_cfg)
    m = 6
    a, b, st, Q = O.haydock(lambda x: H @ x, P[:, 0], m)
    T = np.diag(a[:m]) + np.diag(b[1:m], 1) + np.diag(b[1:m], -1)
    v = P[:, 0].copy()
    Tn = np.eye(m)
    for n in range(0, 2 * m):
        lhs = np.vdot(P[:, 0], v)
        rhs = b[0] ** 2 * Tn[0, 0]
        assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(lhs)), n
        v = H @ v
        Tn = Tn @ T
    assert abs(b[0] - np.linalg.norm(P[:, 0])) < 1e-15 * b[0]
    # basis orthonormal
    G = Q.conj() @ Q.T
    assert np.abs(G - np.eye(len(Q))).max() < 1e-13


def test_diagonal_closed_form_and_breakdown(small_cfg):
    p = make_problem(small_cfg, 0)
    te = O.transition_energies(p).ravel()
    H = np.diag(te).astype(complex)
    # one-entry start vector: b_1 = 0 exactly, the chain stops after one step
    e = np.zeros(p.N, dtype=complex)
    e[7] = 0.3 - 0.4j
    a, b, st, _ = O.haydock(lambda x: H @ x, e, 20)
    assert st == 1 and a[0] == te[7] and b[1] == 0.0
    w = np.linspace(1.0, 6.0, 33)
    S = O.continued_fraction(a, b, st, w, 0.1, p.Nk)
    ref = 0.25 * (0.1 / np.pi) / ((w - te[7]) ** 2 + 0.01) / p.Nk
    assert np.abs(S - ref).max() < 1e-14 * ref.max()
    # general start vector on a diagonal H: closed-form Lorentzian sum once m >= #distinct energies
    P = O.velocity_start(p, np.eye(3))
    S, a, b, st = O.haydock_spectrum(lambda x: H @ x, P, p.N, w, 0.1, p.Nk)
    ipa = np.array([[np.sum(np.abs(P[:, c]) ** 2 * (0.1 / np.pi) / ((x - te) ** 2 + 0.01)) for x in w]
                    for c in range(3)]) / p.Nk
    assert np.abs(S - ipa).max() < 1e-11 * ipa.max()


@pytest.mark.slow
def test_c1_convergence_in_m():
    # at the tiny benchmark workload (dim 1024) 200 steps are converged on the eta = 0.1 eV scale
    p = make_problem("mesh4_ao16", 0)
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))
    H = O.build_H(p, Wq)
    P = O.velocity_start(p, np.eye(3))
    te = O.transition_energies(p)
    w = np.linspace(te.min() - 1, te.max() + 1, 2001)
    Sref, _, _ = O.eig_spectrum(H, P, w, 0.1, p.Nk)
    S200 = O.haydock_spectrum(lambda x: H @ x, P, 200, w, 0.1, p.Nk)[0]
    err = np.abs(S200 - Sref).max() / np.abs(Sref).max()
    assert err < 1e-8


def test_breakdown_does_not_depend_on_the_scales(small_cfg):
    # p supported on three distinct transition energies of a diagonal H: the Krylov space is invariant after
    # three steps.  The chain must stop there whatever the size of p (b_0) or of H: a test against b_0 would
    # run on into rounding noise for a tiny p, and stop at once for a huge one
    p = make_problem(small_cfg, 0)
    te = O.transition_energies(p).ravel()
    idx = [3, 11, 20]
    assert len(set(np.round(te[idx], 12))) == 3
    v = np.zeros(p.N, dtype=complex)
    v[idx] = [0.6, -0.3 + 0.2j, 0.5j]
    ref = None
    for sp in (1.0, 1e-20, 1e20):
        for sh in (1.0, 1e-8, 1e8):
            H = np.diag(sh * te).astype(complex)
            a, b, st, _ = O.haydock(lambda x: H @ x, sp * v, 10)
            assert st == 3, (sp, sh, st)
            assert b[3] <= 1e-14 * sh * te.max()
            # the recurrence coefficients scale with H alone, b_0 with p alone
            assert abs(b[0] - sp * np.linalg.norm(v)) <= 1e-15 * b[0]
            if ref is None:
                ref = (a[:3].copy(), b[1:3].copy())
            assert np.allclose(a[:3] / sh, ref[0], rtol=1e-13, atol=0)
            assert np.allclose(b[1:3] / sh, ref[1], rtol=1e-12, atol=0)
