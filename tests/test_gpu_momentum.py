"""GPU parity at finite exciton momentum Q: the library takes the transitions (v k, c k+Q) through the band
arrays (conduction bands at k + Q), and its apply, pair symmetry and lowest exciton must reproduce the
oracle's Hamiltonian built from the same arrays."""
import numpy as np
import pytest
import torch

import oracle as O
from synth import dense_kmesh, make_problem
from tolerances import KERNEL_TOL, diag_times, kernel_err

pytestmark = pytest.mark.gpu

CONF = dict(cfg_id=89, coarse=(3, 3, 2), dense=(4, 4, 2), n_ao=16, nv=4, nc=4, n_aux=48)


def T(a, dt=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a)).to(torch.device("cuda:0"), dt)


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.fixture(scope="module")
def B():
    from paper_2607_05853_amd import bse
    return bse


@pytest.mark.parametrize("Q", [(1, 0, 0), (0.5, 0.25, 0.0)])
@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_finite_momentum_apply(B, Q, prec):
    p = make_problem(CONF, 3, "G2", momentum=Q)
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
    plan = B.plan_from_problem(p, Wq, prec=prec, max_nb=4, check_hermitian=True)
    assert plan.pairs[0] < p.Nk  # the pair symmetry holds at any Q
    H = O.build_H(p, O.interpolate_W_matmul(p.W_R, p.R, p.w_R, dense_kmesh(p.nk)))
    X = np.random.default_rng(5).standard_normal((p.N, 3)) + 0j
    err = kernel_err(plan.apply(T(X)).cpu().numpy(), H @ X, diag_times(p, X))
    print("[momentum %s %s] apply kernel-part err %.2e" % (Q, prec, err), flush=True)
    assert err < KERNEL_TOL[prec]
    if prec == "f64":
        om, _, _ = plan.lowest_excitons(n_block=4, tol=1e-11, max_iter=500)
        ev = np.linalg.eigvalsh(H)
        assert np.abs(om - ev[:4]).max() < 1e-8 * abs(ev[0])


def H_(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("Q", [(1, 0, 0), (0.5, 0.25, 0.0)])
@pytest.mark.parametrize("prec,tol", [("f64", 1e-9), ("bf16x3", 1e-5)])
def test_momentum_resolved_spectrum(B, Q, prec, tol):
    # S(Q, w) from the start vector <c k+Q| e^{iQ.r} |v k> on a plan built at momentum Q, at an on-mesh and
    # an off-mesh Q: the start vector against the oracle's, and the Haydock spectrum over the full Krylov
    # space against the oracle's eigendecomposition of its explicit A_Q
    p = make_problem(CONF, 6, "G2", momentum=Q)
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
    plan = B.plan_from_problem(p, Wq, prec=prec, max_nb=1)
    P = plan.density_start(T(p.psi))
    P_or = O.density_start(p)
    e_p = rel(H_(P), P_or)
    H = O.build_H(p, O.interpolate_W_matmul(p.W_R, p.R, p.w_R, dense_kmesh(p.nk)))
    te = O.transition_energies(p)
    w = np.linspace(te.min() - 1.0, te.max() + 1.0, 401)
    out = plan.haydock(P, p.N, w, 0.1)
    plan.close()
    S_ref, _, _ = O.eig_spectrum(H, P_or, w, 0.1, p.Nk)
    err = rel(out["S"], S_ref)
    print("[momentum-resolved %s %s] start vector %.1e, spectrum %.2e (%d steps)" %
          (Q, prec, e_p, err, out["steps"][0]), flush=True)
    assert e_p < 1e-14
    assert err < tol
