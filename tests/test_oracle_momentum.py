"""Finite exciton momentum Q (the extension the paper leaves to future work, transitions (v k, c k+Q)):
pins of the input recipe and of the oracle's Hamiltonian built from it.  The direct term couples
(v k, c k+Q) and (v' k', c' k'+Q) through W(k' - k), so the same W(q) serves every Q."""
import numpy as np

import oracle as O
from synth import dense_kmesh, make_problem

TINY = dict(cfg_id=88, coarse=(2, 2, 2), dense=(2, 3, 2), n_ao=8, nv=2, nc=2, n_aux=10)


def test_zero_momentum_is_the_optical_problem():
    a = make_problem(TINY, 1, "G2")
    b = make_problem(TINY, 1, "G2", momentum=(0, 0, 0))
    assert np.array_equal(a.psi, b.psi) and np.array_equal(a.eps_qp, b.eps_qp) and np.array_equal(a.vel, b.vel)


def test_mesh_momentum_moves_the_conduction_bands_by_Q():
    # Q = one mesh spacing along x: the conduction bands of k are the unshifted ones of k + Q
    p0 = make_problem(TINY, 1, "G2")
    pq = make_problem(TINY, 1, "G2", momentum=(1, 0, 0))
    n = np.array(p0.nk)
    kq = [int(np.ravel_multi_index(tuple((np.array(np.unravel_index(k, p0.nk)) + [1, 0, 0]) % n), p0.nk))
          for k in range(p0.Nk)]
    assert np.abs(pq.psi[:, :p0.nv] - p0.psi[:, :p0.nv]).max() == 0
    assert np.abs(pq.psi[:, p0.nv:] - p0.psi[kq, p0.nv:]).max() < 1e-12
    assert np.abs(pq.eps_qp[:, p0.nv:] - p0.eps_qp[kq, p0.nv:]).max() < 1e-12
    assert np.abs(pq.vel).max() == 0


def test_finite_momentum_hamiltonian():
    p = make_problem(TINY, 2, "G2", coarse=(3, 3, 2), momentum=(0.5, 0.25, 0.0))
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))
    H = O.build_H(p, Wq)
    assert np.abs(H - H.conj().T).max() < 1e-14 * np.abs(H).max()
    # zero kernel: the eigenvalues are E_c(k+Q) - E_v(k)
    H0 = O.build_H(p, np.zeros_like(Wq), alpha=0.0)
    ev = np.sort(np.linalg.eigvalsh(H0))
    te = np.sort(np.array([p.eps_qp[k, p.nv + c] - p.eps_qp[k, v]
                           for k in range(p.Nk) for c in range(p.nc) for v in range(p.nv)]))
    assert np.abs(ev - te).max() < 1e-13
