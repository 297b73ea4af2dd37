"""k-dependent two-centre LRI coefficients (Sec. III.A): pins of the oracle's C-tilde.

The oracle evaluates C-tilde^mu_{i ka, j kb} = sum_st conj(c^{ka}_{si}) c^{kb}_{tj} [C^mu_st(kb) + C^mu_ts(-ka)]
in reciprocal space.  The first pin rebuilds the same coefficient from real space, without that formula:
on a Born-von-Karman supercell every product of two AOs phi_s(r - a) phi_t(r - b) is expanded over the
ABFs of its two centres with the translation-invariant coefficients C^mu_st(b - a) (mu at a, on the atom
of s) and C^mu_ts(a - b) (mu at b, on the atom of t), and the Bloch sums are carried out cell by cell."""
import itertools

import numpy as np
import pytest

import oracle as O
from synth import dense_kmesh, make_problem

MESH = (3, 3, 3)          # every R of the coefficient set (|R_i| <= 1) is a distinct class mod 3
N_AO, N_AUX = 4, 6


def _coeffs(seed, complex_=False):
    p = make_problem(dict(cfg_id=87, coarse=(2, 2, 2), dense=(2, 2, 2), n_ao=N_AO, nv=2, nc=2, n_aux=N_AUX),
                     seed, "G1", two_centre=True)
    C_R = p.C_R
    if complex_:
        rng = np.random.default_rng(seed + 100)
        C_R = C_R + 1j * rng.standard_normal(C_R.shape) * (C_R != 0)
    return C_R, p.RC


def _bloch_product_brute_force(C_R, RC, k1, k2):
    """Coefficient B^mu_st of P^{k1-k2}_mu in phi^{k2 *}_s phi^{k1}_t, from real-space products.

    phi^k_s(r) = sum_a phi_s(r - a) e^{i k.a};  P^q_mu(r) = sum_L P_mu(r - L) e^{i q.L}.
    Returns the coefficient of P_mu(r - L) divided by e^{i (k1 - k2).L} for every cell L: [L][mu][s][t]."""
    n = np.array(MESH)
    cells = [np.array(c) for c in itertools.product(*(range(m) for m in MESH))]
    cls = {tuple(np.asarray(R) % n): i for i, R in enumerate(RC)}

    def C_at(d):                       # C(R) for the R of the class d mod the supercell, zero otherwise
        i = cls.get(tuple(np.asarray(d) % n))
        return None if i is None else C_R[i]

    out = np.zeros((len(cells), N_AUX, N_AO, N_AO), dtype=np.complex128)
    for a in cells:
        for b in cells:
            ph = np.exp(-2j * np.pi * np.dot(k2, a) + 2j * np.pi * np.dot(k1, b))
            Cab = C_at(b - a)          # mu at cell a: C^mu_st(b - a)
            Cba = C_at(a - b)          # mu at cell b: C^mu_ts(a - b)
            La = int(np.ravel_multi_index(tuple(a), MESH))
            Lb = int(np.ravel_multi_index(tuple(b), MESH))
            if Cab is not None:
                out[La] += ph * Cab
            if Cba is not None:
                out[Lb] += ph * np.transpose(Cba, (0, 2, 1))
    for L, c in enumerate(cells):
        out[L] *= np.exp(-2j * np.pi * np.dot(k1 - k2, c))
    return out


KPAIRS = [(0, 0), (1, 0), (5, 13), (26, 7), (14, 14)]


@pytest.mark.parametrize("i1,i2", KPAIRS)
def test_two_centre_coefficient_from_real_space(i1, i2):
    C_R, RC = _coeffs(0)
    km = dense_kmesh(MESH)
    k1, k2 = km[i1], km[i2]
    B = _bloch_product_brute_force(C_R, RC, k1, k2)
    # the same coefficient for every cell L: the expansion is a Bloch sum of P_mu at q = k1 - k2
    assert np.abs(B - B[0][None]).max() < 1e-13
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((2, 3, N_AO)) + 1j * rng.standard_normal((2, 3, N_AO))
    # C-tilde^mu_{i k2, j k1} = sum_st conj(c^{k2}_{si}) c^{k1}_{tj} B^mu_st
    ref = np.einsum("is,mst,jt->mij", psi[0].conj(), B[0], psi[1])
    got = O.pair_density_2c(psi, C_R, RC, 0, k2, [0, 1, 2], 1, k1, [0, 1, 2])
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


def _planted(kind, psi, C_R, RC, ka, k_a, bi, kb, k_b, bj):
    """Plausible mistakes in the reciprocal-space formula (each must fail the real-space pin)."""
    Ck = lambda k: O.lri_coeff_k(C_R, RC, k)
    if kind == "no_transpose":
        Ceff = Ck(k_b) + Ck(-np.asarray(k_a))
    elif kind == "phase_sign":
        Ceff = Ck(-np.asarray(k_b)) + np.transpose(Ck(k_a), (0, 2, 1))
    elif kind == "swapped_k":
        Ceff = Ck(k_a) + np.transpose(Ck(-np.asarray(k_b)), (0, 2, 1))
    elif kind == "one_centre":
        Ceff = Ck(k_b)
    a, b = psi[ka][list(bi)], psi[kb][list(bj)]
    return np.matmul(a.conj()[None], np.matmul(Ceff, b.T))


@pytest.mark.parametrize("kind", ["no_transpose", "phase_sign", "swapped_k", "one_centre"])
def test_planted_mistakes_fail_the_real_space_pin(kind):
    C_R, RC = _coeffs(0)
    km = dense_kmesh(MESH)
    k1, k2 = km[5], km[13]
    B = _bloch_product_brute_force(C_R, RC, k1, k2)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((2, 3, N_AO)) + 1j * rng.standard_normal((2, 3, N_AO))
    ref = np.einsum("is,mst,jt->mij", psi[0].conj(), B[0], psi[1])
    bad = _planted(kind, psi, C_R, RC, 0, k2, [0, 1, 2], 1, k1, [0, 1, 2])
    assert np.abs(bad - ref).max() > 1e-3 * np.abs(ref).max()


def test_single_cell_reduces_to_k_independent_form():
    # with C(R) = 0 for R != 0 the two centres give the k-independent C = C(0) + C(0)^T
    C_R, RC = _coeffs(1)
    C0 = C_R[:1]
    R0 = RC[:1]
    rng = np.random.default_rng(4)
    psi = rng.standard_normal((3, 3, N_AO)) + 1j * rng.standard_normal((3, 3, N_AO))
    Ck = C0[0] + np.transpose(C0[0], (0, 2, 1))
    for ka, kb in [(0, 1), (2, 0), (1, 1)]:
        k_a, k_b = rng.random(3), rng.random(3)
        got = O.pair_density_2c(psi, C0, R0, ka, k_a, [0, 2], kb, k_b, [1, 0, 2])
        ref = O.pair_density(psi, Ck, ka, [0, 2], kb, [1, 0, 2])
        assert np.abs(got - ref).max() < 1e-14


def test_conjugate_relation_needs_real_coefficients():
    # real C(R): C-tilde_{j kb, i ka} = conj C-tilde_{i ka, j kb}, which makes the BSE Hamiltonian Hermitian
    rng = np.random.default_rng(5)
    psi = rng.standard_normal((2, 3, N_AO)) + 1j * rng.standard_normal((2, 3, N_AO))
    k_a, k_b = rng.random(3), rng.random(3)
    for cplx, holds in [(False, True), (True, False)]:
        C_R, RC = _coeffs(2, complex_=cplx)
        m1 = O.pair_density_2c(psi, C_R, RC, 0, k_a, [0, 1, 2], 1, k_b, [0, 1])
        m2 = O.pair_density_2c(psi, C_R, RC, 1, k_b, [0, 1], 0, k_a, [0, 1, 2])
        err = np.abs(m2 - np.transpose(m1, (0, 2, 1)).conj()).max() / np.abs(m1).max()
        assert (err < 1e-14) == holds


TINY = dict(cfg_id=86, coarse=(3, 3, 2), dense=(3, 2, 2), n_ao=8, nv=2, nc=3, n_aux=12)


@pytest.mark.parametrize("over", [{}, dict(offset=(1.0 / 3, 1.0 / 3, 0.0)), dict(momentum=(0.5, 0.0, 0.25))])
def test_two_centre_hamiltonian(over):
    p = make_problem(TINY, 3, "G2", two_centre=True, **over)
    assert p.C is None and p.C_R.dtype == np.float64
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))
    H = O.build_H(p, Wq)
    assert np.abs(H - H.conj().T).max() < 1e-14 * np.abs(H).max()
    # exchange alone (W = 0, no diagonal) is positive semi-definite of rank <= n_aux
    Hx = O.build_H(p, np.zeros_like(Wq)) - np.diag(O.transition_energies(p).reshape(-1))
    ev = np.linalg.eigvalsh(Hx)
    assert ev.min() > -1e-12 * ev.max() and (ev > 1e-10 * ev.max()).sum() <= p.n_aux
    # the kernel is a moderate perturbation of the transition energies, as for the k-independent draw
    p0 = make_problem(TINY, 3, "G2", **over)
    K = H - np.diag(O.transition_energies(p).reshape(-1))
    K0 = O.build_H(p0, Wq) - np.diag(O.transition_energies(p0).reshape(-1))
    r = np.linalg.norm(K, 2) / np.linalg.norm(K0, 2)
    assert 0.2 < r < 5.0


def test_row_forms_refuse_two_centre_inputs():
    p = make_problem(TINY, 3, "G2", two_centre=True)
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))
    with pytest.raises(NotImplementedError):
        O.apply_H_rows_allpairs(p, Wq, np.zeros((p.N, 1)), [0])


def test_two_centre_gradient_is_exact_linear_response():
    # L = Re <Ybar, H(W) X> is linear in W(q): the gradient of the two-centre Hamiltonian equals the
    # difference quotient along any complex direction
    p = make_problem(TINY, 4, "G2", two_centre=True)
    kq = dense_kmesh(p.nk)
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, kq)
    rng = np.random.default_rng(6)
    Yb = rng.standard_normal((p.N, 2)) + 1j * rng.standard_normal((p.N, 2))
    X = rng.standard_normal((p.N, 2)) + 1j * rng.standard_normal((p.N, 2))
    _, g_Wq = O.grad_apply(p, Wq, Yb, X)
    dW = rng.standard_normal(Wq.shape) + 1j * rng.standard_normal(Wq.shape)
    L = lambda W: np.real(np.vdot(Yb, O.build_H(p, W) @ X))
    fd = L(Wq + dW) - L(Wq)
    assert abs(fd - np.real(np.vdot(g_Wq, dW))) < 1e-10 * max(1, abs(fd))
