"""Pins of k-offset averaging (Sec. IV.A, the k-point convergence study) in the oracle and the input
generator: the paper's four offsets and weights, the shifted meshes, and the averaged spectrum in the
zero-kernel limit against its closed form."""
import numpy as np

import oracle as O
from synth import dense_kmesh, make_problem

TINY = dict(cfg_id=86, coarse=(2, 2, 2), dense=(2, 3, 2), n_ao=8, nv=2, nc=2, n_aux=10)


def test_paper_offsets_and_weights():
    # (0,0,0) 1/27, (1/3,0,0) 8/27, (1/3,1/3,0) 6/27, (2/3,1/3,0) 12/27: the 27 points of the offset grid
    assert len(O.PAPER_OFFSETS) == 4 == len(O.PAPER_OFFSET_WEIGHTS)
    assert [round(27 * w) for w in O.PAPER_OFFSET_WEIGHTS] == [1, 8, 6, 12]
    assert abs(sum(O.PAPER_OFFSET_WEIGHTS) - 1.0) < 1e-15
    for o in O.PAPER_OFFSETS:
        assert all(abs(3 * x - round(3 * x)) < 1e-15 and 0 <= x < 1 for x in o)


def test_offset_average_of_equal_spectra_is_that_spectrum():
    S = np.random.default_rng(1).random((3, 11))
    assert np.abs(O.offset_average([S] * 4, O.PAPER_OFFSET_WEIGHTS) - S).max() < 1e-15


def test_shifted_problem_shares_everything_but_the_bands():
    p0 = make_problem(TINY, 2, "G2")
    p1 = make_problem(TINY, 2, "G2", offset=(1.0 / 3, 1.0 / 3, 0.0))
    z = make_problem(TINY, 2, "G2", offset=(0.0, 0.0, 0.0))
    assert np.array_equal(z.psi, p0.psi) and np.array_equal(z.eps_qp, p0.eps_qp)   # zero offset = unshifted
    assert np.array_equal(p1.C, p0.C) and np.array_equal(p1.W_R, p0.W_R) and np.array_equal(p1.Vbar, p0.Vbar)
    assert np.abs(p1.eps_ks - p0.eps_ks).max() > 1e-3                                # other k, other bands
    assert np.allclose(p1.kfrac, dense_kmesh(p0.nk) + np.array([1 / 3, 1 / 3, 0]) / np.array(p0.nk))
    # the scissor is the unshifted mesh's: the shifted QP energies are the KS ones plus the same constant
    d0 = p0.eps_qp[:, p0.nv:] - p0.eps_ks[:, p0.nv:]
    d1 = p1.eps_qp[:, p1.nv:] - p1.eps_ks[:, p1.nv:]
    assert np.abs(d1 - d0[0, 0]).max() < 1e-14 and np.abs(d0 - d0[0, 0]).max() < 1e-14


def test_zero_kernel_offset_average_closed_form():
    # W = Vbar = 0: each shifted spectrum is the Lorentzian sum over its transitions with weights |p|^2 / N_k,
    # and the average is the weighted sum of those closed forms
    w = np.linspace(1.0, 6.0, 101)
    eta = 0.1
    S_or, S_cf = [], []
    for o in O.PAPER_OFFSETS:
        p = make_problem(TINY, 3, "G1", offset=o)
        H = O.build_H(p, np.zeros((p.Nk, p.n_aux, p.n_aux), dtype=complex), alpha=0.0)
        P = O.velocity_start(p, np.eye(3))
        S_or.append(O.eig_spectrum(H, P, w, eta, p.Nk)[0])
        te = O.transition_energies(p).ravel()
        L = (eta / np.pi) / ((w[None, :] - te[:, None]) ** 2 + eta ** 2)
        S_cf.append((np.abs(P) ** 2).T @ L / p.Nk)
    got = O.offset_average(S_or, O.PAPER_OFFSET_WEIGHTS)
    ref = sum(wj * Sj for wj, Sj in zip(O.PAPER_OFFSET_WEIGHTS, S_cf))
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
