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


# ---------------------------------------------------------------------------
# momentum-resolved spectra: the start vector <c k+Q| e^{iQ.r} |v k>
# ---------------------------------------------------------------------------
def test_density_start_vanishes_at_zero_momentum():
    # bands at the same k are orthonormal
    p = make_problem(TINY, 3, "G2")
    assert np.abs(O.density_start(p)).max() < 1e-14


def test_density_start_bounded_by_completeness():
    # the conduction bands at k + Q are orthonormal, so sum_c |<u_c^{k+Q}|u_v^k>|^2 <= |u_v^k|^2 = 1; with
    # every band of k + Q (n_ao = nv + nc, all of them either side) the sum over both band sets is exactly 1
    p = make_problem(TINY, 3, "G2", momentum=(0.5, 0.25, 0.0))
    r = np.abs(O.density_start(p).reshape(p.Nk, p.nc, p.nv)) ** 2
    assert r.sum(axis=1).max() <= 1.0 + 1e-14
    full = dict(cfg_id=87, coarse=(2, 2, 2), dense=(2, 2, 2), n_ao=4, nv=2, nc=2, n_aux=6)
    q = (1.0, 0.5, 0.0)
    pc = make_problem(full, 0, "G2", momentum=q)            # valence at k, conduction at k + Q
    pv = make_problem(full, 0, "G2", offset=q)               # every band at k + Q (valence ones used)
    rho_c = O.density_start(pc).reshape(pc.Nk, pc.nc, pc.nv)
    # valence bands of k + Q against those of k, by the same definition
    rho_v = np.einsum("kas,kbs->kab", pv.psi[:, :pv.nv].conj(), pc.psi[:, :pc.nv])
    tot = (np.abs(rho_c) ** 2).sum(axis=1) + (np.abs(rho_v) ** 2).sum(axis=1)
    assert np.abs(tot - 1.0).max() < 1e-13


def test_density_start_long_wavelength_limit_is_the_velocity_form():
    # <u_c^{k+Q}|u_v^k> -> Q_cart . <c|v|v> / (E_c - E_v) as Q -> 0 (k fractional, Q_cart = 2 pi Q), with the
    # band gauge continuous in k; the error is first order in Q
    p0 = make_problem(TINY, 4, "G2")
    pvel = O.velocity_start(p0, np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]))
    errs = []
    for d in (1e-4, 1e-5):
        for axis in (0, 1):
            Q = [0.0, 0.0, 0.0]
            Q[axis] = d                                        # units of the dense-mesh spacing
            pq = make_problem(TINY, 4, "G2", momentum=tuple(Q))
            q_cart = 2.0 * np.pi * d / p0.nk[axis]
            rho = O.density_start(pq)[:, 0] / q_cart
            errs.append(np.abs(rho - pvel[:, axis]).max() / np.abs(pvel[:, axis]).max())
    print("long-wavelength limit errors", errs)
    assert max(errs) < 1e-3
    assert errs[2] < 0.2 * errs[0] and errs[3] < 0.2 * errs[1]   # first order in Q


def test_density_spectrum_zero_kernel_closed_form():
    # W = Vbar = 0: S(Q, w) = (1/N_k) sum |p_cvk(Q)|^2 L(w - (E_c(k+Q) - E_v(k)))
    import dataclasses
    p = make_problem(TINY, 5, "G2", momentum=(1.0, 0.0, 0.0))
    p = dataclasses.replace(p, Vbar=np.zeros_like(p.Vbar))
    Wq = np.zeros((p.Nk, p.n_aux, p.n_aux), complex)
    P = O.density_start(p)
    w = np.linspace(1.0, 6.0, 101)
    S, _, _ = O.eig_spectrum(O.build_H(p, Wq), P, w, 0.1, p.Nk)
    te = O.transition_energies(p).ravel()
    ref = (np.abs(P[:, 0]) ** 2) @ O.lorentzian(w[None, :] - te[:, None], 0.1) / p.Nk
    assert np.abs(S[0] - ref).max() < 1e-13 * np.abs(ref).max()
