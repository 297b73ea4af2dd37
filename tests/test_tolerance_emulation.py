"""The GPU parity tolerances tell a split-precision product from a plain one.

The GPU tests hold each reduced-precision apply to a bound on the error of its kernel part, Y - D X with
D the FP64 diagonal of transition energies, relative to the largest element of the oracle's kernel part
(the diagonal is FP64 at every precision, so normalising by max |Y| would let the diagonal hide the
kernel's error).  This module emulates, in numpy, the dataflow of the direct term on the 4x4x4 workload
with every stored operand rounded as the GPU stores it, and shows that

* rounding each operand to one bf16 (8 significant bits: a product of the hi parts only) misses the
  BF16x3 bound by a wide margin, and so does dropping the lo part of any single operand (the halves, the
  bands, W(q), G_v, P or M_c) while the others stay split, and
* rounding to the two-term split hi + lo of BF16x3 and to FP32 meets the bounds with room,

so the bounds reject a kernel that drops the lo terms, while the split kernels pass them."""
import numpy as np
import pytest

import oracle as O
from synth import dense_kmesh, make_problem, random_block

from tolerances import KERNEL_TOL  # the bounds of the GPU tests: max |Y - A X| / max |(A - D) X|


def _bf16(x):
    """Round float32 values to bfloat16 (round to nearest even), returned as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _round(z, mode):
    """Complex values as stored by a kernel of the given mode (real and imaginary parts separately)."""
    if mode == "none":
        return z

    def r(x):
        if mode == "f32":
            return np.asarray(x, dtype=np.float32).astype(np.float64)
        hi = _bf16(x)
        if mode == "bf16_hi":
            return hi
        lo = _bf16(np.asarray(x, dtype=np.float32).astype(np.float64) - hi)
        return hi + lo                                    # "bf16x3": hi*hi + hi*lo + lo*hi keeps hi + lo
    return r(z.real) + 1j * r(z.imag)


OPERANDS = ("Bv", "Bc", "psi", "W", "Gv", "P", "Mc")   # every operand a BF16x3 kernel stores split


def _emulated_kernel_apply(p, Wq, X, mode, hi_only=None):
    """Direct + exchange terms of A X with the pair densities formed from stored (rounded) halves and bands,
    P = conj(G_v) W(q) from rounded G_v and W(q), T = M_c P^T from rounded M_c and P, and FP64 for the
    exchange and the accumulation over k' (as on the GPU).  hi_only: the one operand (of OPERANDS) stored
    as its bf16 hi part alone, as a kernel that drops that operand's lo plane would."""
    nv, nc, Nk, na = p.nv, p.nc, p.Nk, p.n_aux
    nt = nc * nv
    md = lambda name: "bf16_hi" if name == hi_only else mode
    psi_v, psi_c = p.psi[:, :nv], p.psi[:, nv:]
    Bv = _round(np.einsum("kvs,mst->kvmt", psi_v.conj(), p.C), md("Bv"))     # psi_v(k)^H C^mu
    Bc = _round(np.einsum("kcs,mst->kcmt", psi_c.conj(), p.C), md("Bc"))
    pv, pc = _round(psi_v, md("psi")), _round(psi_c, md("psi"))
    W = _round(Wq, md("W"))
    q = O.q_index_table(p.nk)
    Xk = X.reshape(Nk, nc, nv, -1)
    Y = np.zeros((Nk, nc, nv, X.shape[1]), dtype=complex)
    for k in range(Nk):
        kp = np.arange(Nk)
        # G_v[k'][v][v'][mu] = B_v(k)[v][mu] . psi_v'(k')  = M^mu_vv'(k, k');  conj gives M^mu_v'v(k', k)
        Gv = _round(np.einsum("vmt,kpt->kvpm", Bv[k], pv[kp]), md("Gv"))
        P = _round(np.einsum("kvpm,kmn->kvpn", Gv.conj(), W[q[k, kp]]), md("P"))
        Mc = _round(np.einsum("cmt,kdt->kcdm", Bc[k], pc[kp]), md("Mc"))          # M^nu_cc'(k, k')
        T = np.einsum("kcdn,kvpn->kcvdp", Mc, P)                               # [k'][c][v][c'][v']
        Y[k] = -(1.0 / Nk) * np.einsum("kcvdp,kdpb->cvb", T, Xk)
    rho = np.einsum("kcs,mst,kvt->kcvm", psi_c.conj(), p.C, psi_v)            # FP64, as the plan keeps it
    t = np.einsum("kcvm,kcvb->mb", rho.conj(), Xk)
    Y += (p.alpha / Nk) * np.einsum("kcvm,mn,nb->kcvb", rho, p.Vbar, t)
    return Y.reshape(Nk * nt, -1)


def _kernel_err(p, Wq, X, mode, hi_only=None):
    H = O.build_H(p, Wq)
    ref = H @ X - O.transition_energies(p).reshape(-1)[:, None] * X
    got = _emulated_kernel_apply(p, Wq, X, mode, hi_only)
    return np.abs(got - ref).max() / np.abs(ref).max()


def test_emulation_is_exact_in_fp64():
    p = make_problem("mesh4_ao16", 0, "G2", coarse=(3, 3, 2))
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))
    X = random_block(p.N, 3, seed=1)
    # no rounding at all: the emulated dataflow reproduces the oracle's kernel part
    assert _kernel_err(p, Wq, X, "none") < 1e-12


def test_bounds_reject_hi_only_and_accept_split():
    p = make_problem("mesh4_ao16", 0, "G2", coarse=(3, 3, 2))
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))
    X = random_block(p.N, 3, seed=1)
    e_hi = _kernel_err(p, Wq, X, "bf16_hi")
    e_b3 = _kernel_err(p, Wq, X, "bf16x3")
    e_32 = _kernel_err(p, Wq, X, "f32")
    print("[emulation] kernel-part error: bf16 hi only %.2e, bf16x3 %.2e, f32 %.2e" % (e_hi, e_b3, e_32))
    assert e_hi > 10 * KERNEL_TOL["bf16x3"]
    assert e_b3 < 0.2 * KERNEL_TOL["bf16x3"]
    assert e_32 < 0.2 * KERNEL_TOL["f32"]
    # and an FP32 bound would also reject the split product (its 16 bits are not FP32's 24)
    assert e_b3 > KERNEL_TOL["f32"]


@pytest.mark.parametrize("operand", OPERANDS)
def test_bound_rejects_one_operand_without_its_lo_part(operand):
    # a BF16x3 kernel that loads only the hi plane of one operand (the others split) still misses the bound
    p = make_problem("mesh4_ao16", 0, "G2", coarse=(3, 3, 2))
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))
    X = random_block(p.N, 3, seed=1)
    e = _kernel_err(p, Wq, X, "bf16x3", hi_only=operand)
    print("[emulation] %s hi only: kernel-part error %.2e" % (operand, e))
    assert e > 3 * KERNEL_TOL["bf16x3"]
