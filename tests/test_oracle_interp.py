"""Pins of the oracle's dual-k-mesh interpolation of W (Sec. III.B; phase of Eq. (W_LRI))."""
import numpy as np
import pytest

import oracle as O
from synth import make_problem, ws_rset, dense_kmesh


def test_single_R_closed_form():
    # W(R) nonzero only at R = (1, 0, 0): W(q) = w_R W(R) exp(+2 pi i q.R).
    # At q = (1/4, 0, 0) the phase is exp(i pi / 2) = +i (sign of the transform pinned).
    R = np.array([[1, 0, 0], [0, 0, 0]], dtype=np.int32)
    w = np.array([0.5, 1.0])
    W_R = np.zeros((2, 2, 2), dtype=complex)
    W_R[0] = [[1.0, 2.0], [3.0, 4.0]]
    out = O.interpolate_W(W_R, R, w, [[0.25, 0.0, 0.0], [0.75, 0.0, 0.0]])
    assert np.allclose(out[0], 0.5j * W_R[0], atol=1e-15)
    assert np.allclose(out[1], -0.5j * W_R[0], atol=1e-15)


def test_R0_only_gives_constant():
    R = np.array([[0, 0, 0]], dtype=np.int32)
    W_R = np.random.default_rng(1).standard_normal((1, 3, 3)).astype(complex)
    q = dense_kmesh((3, 2, 2))
    out = O.interpolate_W(W_R, R, np.array([1.0]), q)
    assert np.abs(out - W_R[0][None]).max() == 0.0


@pytest.mark.parametrize("coarse,dense", [((2, 2, 2), (4, 4, 4)), ((4, 4, 4), (8, 8, 8)), ((3, 3, 2), (6, 6, 5))])
def test_matches_numpy_fft_of_padded_box(coarse, dense):
    # Library routine: sum_R w_R W(R) e^{2 pi i q.R} on the dense mesh equals
    # N_dense * ifftn of the box holding w_R W(R) at R mod n_dense (images are
    # distinct mod n_dense for these meshes).
    R, w = ws_rset(coarse)
    rng = np.random.default_rng(7)
    W_R = rng.standard_normal((len(R), 2, 2)) + 1j * rng.standard_normal((len(R), 2, 2))
    box = np.zeros(tuple(dense) + (2, 2), dtype=complex)
    seen = set()
    for r, wr, Wm in zip(R, w, W_R):
        idx = tuple(int(x) % n for x, n in zip(r, dense))
        assert idx not in seen
        seen.add(idx)
        box[idx] += wr * Wm
    ref = np.fft.ifftn(box, axes=(0, 1, 2)) * np.prod(dense)
    ref = ref.reshape(-1, 2, 2)
    out = O.interpolate_W(W_R, R, w, dense_kmesh(dense))
    assert np.abs(out - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("coarse", [(2, 2, 2), (4, 4, 4), (3, 2, 2)])
def test_coarse_round_trip_exact(coarse):
    # The paper's dual-k-mesh step: W(k) on the coarse mesh -> W(R) on the BvK
    # supercell -> back to any q.  On the coarse points themselves the
    # interpolation must reproduce W(k) exactly (WS set with face weights).
    R, w = ws_rset(coarse)
    qc = dense_kmesh(coarse)
    rng = np.random.default_rng(3)
    Wqc = rng.standard_normal((len(qc), 3, 3)) + 1j * rng.standard_normal((len(qc), 3, 3))
    W_R = O.coarse_to_R(Wqc, coarse, R)
    back = O.interpolate_W(W_R, R, w, qc)
    assert np.abs(back - Wqc).max() < 1e-13 * np.abs(Wqc).max()


def test_truncated_set_weights():
    # |R| <= 3 truncation of the 6^3 supercell: 123 points, weights summing to 120.
    R, w = ws_rset((6, 6, 6), 3.0)
    assert len(R) == 123 and abs(w.sum() - 120.0) < 1e-12
    R, w = ws_rset((4, 4, 4))
    assert len(R) == 125 and abs(w.sum() - 64.0) < 1e-12


def test_Wq_hermitian_for_G2(tiny_cfg):
    # classes that are their own negative (all of them on a 2^3 supercell) carry
    # symmetric matrices, so use a supercell with 3 along two axes
    p = make_problem(tiny_cfg, 0, "G2", coarse=(3, 3, 2))
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh((4, 4, 4)))
    assert np.abs(Wq - np.conj(np.transpose(Wq, (0, 2, 1)))).max() < 1e-14
    # and G2 makes W(q) complex with W(q) != W(-q), so the orientation is testable
    assert np.abs(Wq.imag).max() > 1e-3
    assert np.abs(Wq[21] - np.transpose(Wq[21])).max() > 1e-3   # q = (1/4, 1/4, 1/4)
