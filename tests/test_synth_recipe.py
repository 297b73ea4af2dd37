"""The seeded synthetic inputs follow their stated recipe (they stand in for the paper's DFT + G0W0 front end,
Sec. II.A and the workflow of Sec. III.B): the named workloads have their sizes; the bands are orthonormal
eigenvectors of the tight-binding H(k) at the Gamma-centred mesh points, valence below conduction; the
quasiparticle energies are the Kohn-Sham ones with one scissor on the conduction bands that sets the
smallest direct gap to 2 eV; every C^mu is Hermitian (two-centre coefficients real, supported on the atom
of their first AO); Vbar is real symmetric positive semi-definite; W(R) is real, G1 a positive
semi-definite matrix times exp(-|R|/1.5) and G2 with W(-R) = W(R)^T but not symmetric; every draw is a
pure function of (workload, seed)."""
import numpy as np
import pytest

from synth import dense_kmesh, make_problem
from synth.crystal import CONFIGS

SIZES = {   # dense mesh, coarse mesh, N_ao, n_v, n_c, N_aux, |R| cut
    "mesh4_ao16": ((4, 4, 4), (2, 2, 2), 16, 4, 4, 64, None),
    "mesh8_ao64": ((8, 8, 8), (4, 4, 4), 64, 4, 8, 256, None),
    "mesh12_ao96": ((12, 12, 12), (4, 4, 4), 96, 6, 10, 384, None),
    "mesh8_ao64_grad": ((8, 8, 8), (4, 4, 4), 64, 4, 8, 256, None),
    "mesh16_ao128": ((16, 16, 16), (6, 6, 6), 128, 8, 8, 512, 3.0),
}
SMALL = dict(cfg_id=91, coarse=(3, 3, 2), dense=(3, 2, 2), n_ao=10, nv=2, nc=3, n_aux=16)


def test_named_workload_sizes():
    assert set(SIZES) == set(CONFIGS)
    for name, (dense, coarse, n_ao, nv, nc, n_aux, r_cut) in SIZES.items():
        c = CONFIGS[name]
        assert (tuple(c["dense"]), tuple(c["coarse"]), c["n_ao"], c["nv"], c["nc"], c["n_aux"], c["r_cut"]) == \
            (dense, coarse, n_ao, nv, nc, n_aux, r_cut)


def _Hk(p, k):
    H = sum(M * np.exp(2j * np.pi * np.dot(k, R)) for R, M in p.H_R.items())
    return 0.5 * (H + H.conj().T)


@pytest.mark.parametrize("wgen", ["G1", "G2"])
def test_bands_are_eigenvectors_of_the_tight_binding_model(wgen):
    p = make_problem(SMALL, 3, wgen)
    nv = p.nv
    for ik, k in enumerate(dense_kmesh(p.nk)):
        U = p.psi[ik]                                                   # rows: bands
        assert np.abs(U @ U.conj().T - np.eye(nv + p.nc)).max() < 1e-12
        Hk = _Hk(p, k)
        assert np.abs(Hk @ U.T - U.T * p.eps_ks[ik][None, :]).max() < 1e-12
        assert np.all(np.diff(p.eps_ks[ik, :nv]) >= 0) and np.all(np.diff(p.eps_ks[ik, nv:]) >= 0)
        assert p.eps_ks[ik, nv - 1] < p.eps_ks[ik, nv]


def test_scissor_sets_the_direct_gap():
    for cfg in ("mesh4_ao16", SMALL):
        p = make_problem(cfg, 1, "G2")
        nv = p.nv
        assert np.array_equal(p.eps_qp[:, :nv], p.eps_ks[:, :nv])
        shift = p.eps_qp[:, nv:] - p.eps_ks[:, nv:]
        assert np.abs(shift - shift[0, 0]).max() < 1e-12 and abs(shift[0, 0]) > 0.1   # either sign
        assert abs((p.eps_qp[:, nv] - p.eps_qp[:, nv - 1]).min() - 2.0) < 1e-12


def test_coefficients_and_bare_coulomb():
    p = make_problem("mesh4_ao16", 0, "G1")
    assert np.abs(p.C - np.conj(np.transpose(p.C, (0, 2, 1)))).max() == 0.0
    assert np.abs(p.Vbar.imag).max() == 0.0
    V = p.Vbar.real
    assert np.abs(V - V.T).max() == 0.0
    assert np.linalg.eigvalsh(V).min() > -1e-12 * np.abs(V).max()
    t = make_problem(SMALL, 0, "G1", two_centre=True)
    assert t.C is None and not np.iscomplexobj(t.C_R)
    # a coefficient is nonzero only when the auxiliary function sits on the atom of the first AO
    atom_s = np.arange(t.n_ao) * 2 // t.n_ao
    atom_mu = np.arange(t.n_aux) * 2 // t.n_aux
    off = atom_mu[:, None] != atom_s[None, :]                          # [mu][s]
    assert np.abs(t.C_R[:, off, :]).max() == 0.0 and np.abs(t.C_R).max() > 0


def test_screened_interaction_generators():
    p = make_problem(SMALL, 2, "G1")
    assert np.abs(p.W_R.imag).max() == 0.0
    rn = np.sqrt((p.R.astype(float) ** 2).sum(1))
    i0 = int(np.flatnonzero(rn == 0)[0])
    base = p.W_R[i0].real
    assert np.abs(base - base.T).max() < 1e-15 and np.linalg.eigvalsh(base).min() > -1e-12 * np.abs(base).max()
    ratio = p.W_R.real / base[None]
    assert np.abs(ratio - np.exp(-rn / 1.5)[:, None, None]).max() < 1e-12
    g = make_problem(SMALL, 2, "G2")
    assert np.abs(g.W_R.imag).max() == 0.0
    idx = {tuple(r): i for i, r in enumerate(g.R)}
    for i, r in enumerate(g.R):
        assert np.array_equal(g.W_R[idx[tuple(-r)]], g.W_R[i].T)
    assert max(np.abs(g.W_R[i] - g.W_R[i].T).max() for i in range(len(g.R))) > 1e-3


def test_draws_are_pure_functions_of_workload_and_seed():
    a, b = make_problem(SMALL, 5, "G2"), make_problem(SMALL, 5, "G2")
    for f in ("eps_ks", "eps_qp", "psi", "vel", "C", "Vbar", "W_R"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    c = make_problem(SMALL, 6, "G2")
    assert not np.array_equal(a.C, c.C) and not np.array_equal(a.W_R, c.W_R)
