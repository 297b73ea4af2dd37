"""Pins of the oracle's exciton binding energy (Sec. IV.B.3): E_B is the smallest direct quasiparticle gap
over the mesh (lowest conduction minus highest valence band at the same k) minus the lowest excitation
energy Omega_1 of A.

The cases are chosen so that the plausible mistakes fail one of them: Kohn-Sham instead of quasiparticle
energies (the scissor moves the gap), the indirect gap (band edges at different k), a max for the min, the
wrong band pair, or the wrong sign."""
import dataclasses

import numpy as np

import oracle as O
from synth import dense_kmesh, make_problem
from synth.crystal import Problem


def _Wq(p):
    return O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))


def test_binding_energy_hand_case():
    # two k points, 2 valence + 2 conduction bands (ascending per k).  Direct gaps c1 - v_top: 1.1 at k0,
    # 1.0 at k1; the indirect gap (lowest c1 anywhere minus highest v_top anywhere) is 0.5 - (-0.1) = 0.6;
    # the largest direct gap 1.1; the Kohn-Sham energies lack the 0.25 eV scissor on the conduction bands
    eps_qp = np.array([[-0.7, -0.1, 1.0, 1.6],
                       [-0.9, -0.5, 0.5, 2.0]])
    eps_ks = eps_qp - np.array([0.0, 0.0, 0.25, 0.25])
    p = Problem(name="hand", nk=(2, 1, 1), coarse=(1, 1, 1), n_ao=4, nv=2, nc=2, n_aux=1, alpha=2.0,
                eps_ks=eps_ks, eps_qp=eps_qp, psi=np.zeros((2, 4, 4), complex),
                vel=np.zeros((3, 2, 2, 2), complex), C=np.zeros((1, 4, 4), complex),
                Vbar=np.zeros((1, 1), complex), R=np.zeros((1, 3), np.int32), w_R=np.ones(1),
                W_R=np.zeros((1, 1, 1), complex))
    assert abs(O.binding_energy(p, 0.93) - 0.07) < 1e-15
    assert abs(O.binding_energy(p, 1.0)) < 1e-15


def test_zero_kernel_has_zero_binding_energy():
    # W = Vbar = 0: A is the diagonal of transition energies, whose smallest entry is the smallest direct
    # gap, so E_B = 0 exactly
    for cfg, wgen in [("mesh4_ao16", "G1"), (dict(cfg_id=91, coarse=(2, 2, 2), dense=(3, 2, 2), n_ao=10, nv=2,
                                                  nc=3, n_aux=16), "G2")]:
        p = make_problem(cfg, 0, wgen)
        p = dataclasses.replace(p, Vbar=np.zeros_like(p.Vbar), W_R=np.zeros_like(p.W_R))
        Om1, _ = O.lowest_exciton(O.build_H(p, _Wq(p)))
        assert O.binding_energy(p, Om1) == 0.0
        # the quasiparticle gap is the scissored one: the Kohn-Sham gap differs from it
        gap_ks = (p.eps_ks[:, p.nv] - p.eps_ks[:, p.nv - 1]).min()
        assert abs(Om1 - gap_ks) > 0.1


def test_binding_energy_convex_in_the_screened_interaction():
    # with the exchange removed (triplet, alpha = 0) A(s) = diag(te) + s D is linear in the scale s of W, so
    # Omega_1(s) = lambda_min(A(s)) is concave (a minimum of linear functions of s) and E_B(s) = gap -
    # Omega_1(s) is convex with E_B(0) = 0: E_B(s) / s does not decrease for s > 0, E_B(s) + E_B(-s) >= 0,
    # and a strong enough screened interaction binds (E_B > 0 and growing)
    base = make_problem("mesh4_ao16", 1, "G1")
    scales = (-1.0, 0.0, 1.0, 4.0, 16.0)
    eb = {}
    for s in scales:
        p = dataclasses.replace(base, W_R=s * base.W_R, alpha=0.0)
        Om1, _ = O.lowest_exciton(O.build_H(p, _Wq(p)))
        eb[s] = O.binding_energy(p, Om1)
    assert abs(eb[0.0]) < 1e-14
    assert eb[1.0] / 1.0 <= eb[4.0] / 4.0 <= eb[16.0] / 16.0
    assert eb[1.0] + eb[-1.0] >= 0.0
    assert 0.0 < eb[4.0] < eb[16.0]
    # first order in a small kernel: Omega_1 = te[i0] + D[i0, i0] + O(s^2) for the smallest transition energy
    # te[i0] (non-degenerate here), so E_B -> -D[i0, i0], of either sign, and the second-order remainder
    # (convexity) is >= 0
    for sk in (1e-3, -1e-3):
        p = dataclasses.replace(base, W_R=sk * base.W_R, alpha=0.0)
        H = O.build_H(p, _Wq(p))
        te = O.transition_energies(p).ravel()
        i0 = int(np.argmin(te))
        assert np.sort(te)[1] - te[i0] > 1e-3
        first = -(H[i0, i0].real - te[i0])
        Om1, _ = O.lowest_exciton(H)
        e = O.binding_energy(p, Om1)
        assert abs(first) > 1e-7 and abs(e / first - 1.0) < 1e-2 and e - first >= -1e-15
