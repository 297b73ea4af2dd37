"""GPU parity of k-offset averaging (Sec. IV.A, the k-point convergence study): the Haydock spectrum
averaged over the paper's four shifted dense meshes against the oracle's average of exact
(eigendecomposition) spectra, FP64 and BF16x3.  Every plan takes the same interpolated W_q."""
import numpy as np
import pytest
import torch

import oracle as O
from synth import dense_kmesh, make_problem, polarisations

pytestmark = pytest.mark.gpu


def T(a, dt=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a)).to(torch.device("cuda:0"), dt)


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.fixture(scope="module")
def B():
    from paper_2607_05853_amd import bse
    return bse


def test_offset_set_matches_the_paper(B):
    offs, wts = B.offset_set()
    assert np.abs(offs - np.array(O.PAPER_OFFSETS)).max() < 1e-15
    assert np.abs(wts - np.array(O.PAPER_OFFSET_WEIGHTS)).max() < 1e-15


@pytest.mark.parametrize("prec,tol", [("f64", 1e-7), ("bf16x3", 1e-6)])
def test_offset_averaged_spectrum(B, prec, tol):
    offs, wts = B.offset_set()
    conf = dict(cfg_id=87, coarse=(3, 3, 2), dense=(4, 4, 4), n_ao=16, nv=4, nc=4, n_aux=64)
    p0 = make_problem(conf, 0, "G2")
    Wq = B.interpolate_W(T(p0.W_R), p0.R, p0.w_R, dense_kmesh(p0.nk))  # one W_q for every offset
    W_or = O.interpolate_W_matmul(p0.W_R, p0.R, p0.w_R, dense_kmesh(p0.nk))
    te = O.transition_energies(p0)
    w = np.linspace(te.min() - 1.0, te.max() + 1.0, 501)
    pol = polarisations(3)
    plans, Ps, S_or = [], [], []
    for o in offs:
        p = make_problem(conf, 0, "G2", offset=tuple(o))
        pl = B.plan_from_problem(p, Wq, prec=prec, max_nb=3)
        plans.append(pl)
        Ps.append(pl.velocity_start(T(p.vel), T(p.eps_ks, torch.float64), pol))
        S_or.append(O.eig_spectrum(O.build_H(p, W_or), O.velocity_start(p, pol), w, 0.1, p.Nk)[0])
    out = B.offset_spectrum(plans, Ps, wts, 200, w, 0.1)
    ref = O.offset_average(S_or, O.PAPER_OFFSET_WEIGHTS)
    err = rel(out["S"], ref)
    shift = rel(S_or[0], ref)  # how far the unshifted spectrum is from the average
    print("[offsets %s] averaged spectrum rel err %.2e (unshifted vs average %.2e)" % (prec, err, shift), flush=True)
    assert (out["steps"] == 200).all()
    assert err < tol and shift > 100 * tol
    for pl in plans:
        pl.close()
