"""Pins of the oracle's row-at-a-time forms (used for sampled rows on the largest mesh).

Each is checked against the block-by-block oracle functions, which are themselves pinned to hand
cases, closed forms and brute force.  The comparisons use general complex inputs (C^mu, Vbar and W(q)
neither Hermitian nor symmetric, random W(q) per q) so that a transposed or conjugated operand, a
swapped k / k' or a wrong q = k' - k cannot cancel out, and chunk sizes that do not divide N_k."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from synth import dense_kmesh, make_problem, random_block

RAGGED = dict(cfg_id=93, coarse=(3, 3, 3), dense=(3, 2, 5), n_ao=12, nv=3, nc=5, n_aux=40)
WIDE_V = dict(cfg_id=81, coarse=(2, 2, 2), dense=(4, 4, 2), n_ao=16, nv=8, nc=2, n_aux=24)


def _cn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _general(p, seed):
    """The same bands with non-Hermitian C, a non-symmetric complex Vbar and a random W(q) per q."""
    rng = np.random.default_rng(seed)
    q = dataclasses.replace(p, C=_cn(rng, p.C.shape) / np.sqrt(p.n_ao), Vbar=_cn(rng, p.Vbar.shape) / p.n_aux)
    Wq = _cn(rng, (p.Nk, p.n_aux, p.n_aux)) / p.n_aux
    return q, Wq


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("cfg", ["RAGGED", "WIDE_V"])
def test_interpolate_matmul_matches_direct_sum(cfg):
    conf = {"RAGGED": RAGGED, "WIDE_V": WIDE_V}[cfg]
    p = make_problem(conf, 2, "G2", coarse=(3, 3, 2))
    q = np.vstack([dense_kmesh(p.nk), np.random.default_rng(1).random((5, 3))])  # mesh and off-mesh q
    assert rel(O.interpolate_W_matmul(p.W_R, p.R, p.w_R, q), O.interpolate_W(p.W_R, p.R, p.w_R, q)) < 1e-14


def test_interpolate_matmul_single_R_closed_form():
    rng = np.random.default_rng(3)
    R = np.array([[2, -1, 3]])
    W_R = _cn(rng, (1, 4, 4))
    q = rng.random((6, 3))
    got = O.interpolate_W_matmul(W_R, R, np.array([0.5]), q)
    for i in range(len(q)):
        assert np.abs(got[i] - 0.5 * np.exp(2j * np.pi * q[i] @ R[0]) * W_R[0]).max() < 1e-14


@pytest.mark.parametrize("cfg,chunk", [("RAGGED", 7), ("WIDE_V", 5), ("mesh4_ao16", 64)])
@pytest.mark.parametrize("alpha", [2.0, 0.0])
def test_allpairs_rows_match_blocks(cfg, chunk, alpha):
    conf = {"RAGGED": RAGGED, "WIDE_V": WIDE_V, "mesh4_ao16": "mesh4_ao16"}[cfg]
    p, Wq = _general(make_problem(conf, 4, "G1"), 11)
    X = random_block(p.N, 3, seed=12)
    rows = [0, 1, p.Nk // 2, p.Nk - 1]
    ref = O.apply_H_rows(p, Wq, X, rows, alpha=alpha)
    got = O.apply_H_rows_allpairs(p, Wq, X, rows, alpha=alpha, chunk=chunk)
    assert rel(got, ref) < 1e-13


def test_allpairs_rows_match_explicit_H():
    p = make_problem(RAGGED, 5, "G2", coarse=(3, 3, 2))
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))
    H = O.build_H(p, Wq)
    X = random_block(p.N, 2, seed=13)
    nt = p.nv * p.nc
    rows = [3, 17]
    got = O.apply_H_rows_allpairs(p, Wq, X, rows, chunk=4)
    ref = np.vstack([(H @ X)[k * nt:(k + 1) * nt] for k in rows])
    assert rel(got, ref) < 1e-13


@pytest.mark.parametrize("cfg,chunk", [("RAGGED", 7), ("WIDE_V", 64)])
def test_grad_Wq_at_matches_grad_apply(cfg, chunk):
    conf = {"RAGGED": RAGGED, "WIDE_V": WIDE_V}[cfg]
    p, Wq = _general(make_problem(conf, 6, "G1"), 14)
    Yb, X = random_block(p.N, 3, seed=15), random_block(p.N, 3, seed=16)
    _, gq = O.grad_apply(p, Wq, Yb, X)
    qs = [0, 1, p.Nk // 3, p.Nk - 1]
    assert rel(O.grad_Wq_at(p, Yb, X, qs, chunk=chunk), gq[qs]) < 1e-13


def test_grad_eps_matches_grad_apply():
    p, Wq = _general(make_problem(RAGGED, 7, "G1"), 17)
    Yb, X = random_block(p.N, 3, seed=18), random_block(p.N, 3, seed=19)
    ge, _ = O.grad_apply(p, Wq, Yb, X)
    assert np.abs(O.grad_eps(p, Yb, X) - ge).max() < 1e-13 * np.abs(ge).max()


def _general_2c(p, seed):
    """Two-centre coefficients kept real (the form assumes it), a non-symmetric complex Vbar and a random
    W(q) per q."""
    rng = np.random.default_rng(seed)
    q = dataclasses.replace(p, Vbar=_cn(rng, p.Vbar.shape) / p.n_aux)
    Wq = _cn(rng, (p.Nk, p.n_aux, p.n_aux)) / p.n_aux
    return q, Wq


@pytest.mark.parametrize("over", [{}, dict(offset=(1.0 / 3, 1.0 / 3, 0.0)), dict(momentum=(0.5, 0.25, 0.0))])
@pytest.mark.parametrize("two_centre", [False, True])
@pytest.mark.parametrize("block", ["A", "B"])
def test_twosided_rows_match_blocks(block, two_centre, over):
    base = make_problem(RAGGED, 8, "G1", two_centre=two_centre, **over)
    p, Wq = (_general_2c if two_centre else _general)(base, 21)
    X = random_block(p.N, 3, seed=22)
    rows = [0, 1, p.Nk // 2, p.Nk - 1]
    ref = O.apply_H_rows(p, Wq, X, rows) if block == "A" else O.apply_B_rows(p, Wq, X, rows)
    got = O.apply_rows_twosided(p, Wq, X, rows, block=block, chunk=7)
    assert rel(got, ref) < 1e-13


def test_twosided_rows_refuse_complex_two_centre_coefficients():
    p = make_problem(RAGGED, 8, "G1", two_centre=True)
    p = dataclasses.replace(p, C_R=p.C_R + 0j)
    with pytest.raises(ValueError):
        O.apply_rows_twosided(p, np.zeros((p.Nk, p.n_aux, p.n_aux), complex), np.zeros((p.N, 1)), [0])


@pytest.mark.parametrize("cfg,chunk", [("RAGGED", 7), ("WIDE_V", 5)])
@pytest.mark.parametrize("alpha", [2.0, 0.0])
def test_hamiltonian_rows_match_blocks(cfg, chunk, alpha):
    # the explicit rows of A, every column block at once, against hamiltonian_block one (k, k') at a time,
    # with general complex inputs so that a transposed block or a swapped (c', v') order cannot cancel
    conf = {"RAGGED": RAGGED, "WIDE_V": WIDE_V}[cfg]
    p, Wq = _general(make_problem(conf, 9, "G1"), 23)
    rows = [0, 2, p.Nk - 1]
    nt = p.nc * p.nv
    got = O.hamiltonian_rows(p, Wq, rows, alpha=alpha, chunk=chunk)
    ref = np.vstack([np.hstack([O.hamiltonian_block(p, Wq, alpha, k, kp) for kp in range(p.Nk)]) for k in rows])
    assert got.shape == (len(rows) * nt, p.N)
    assert rel(got, ref) < 1e-13


def test_hamiltonian_rows_give_build_H():
    p = make_problem(RAGGED, 5, "G2", coarse=(3, 3, 2))
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))
    H = O.build_H(p, Wq)
    got = O.hamiltonian_rows(p, Wq, list(range(p.Nk)), chunk=8)
    assert rel(got, H) < 1e-13
    assert np.abs(got - got.conj().T).max() < 1e-14 * np.abs(got).max()
