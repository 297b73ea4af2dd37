"""Planted mistakes in the oracle.  Each plausible slip (a dropped term, a wrong sign, a transposed or
unconjugated operand, a wrong index, orientation or band, a missing normalisation, a dropped ragged chunk)
is planted in a copy of one oracle function for the duration of one test, and at least one of the pins
that tie that function to the paper and the mathematics (hand-derived cases, the AO-kernel brute force,
closed forms, library routines, invariants, finite differences) must then fail.  Covered: the explicit
Hamiltonian (Eq. (Hamiltonian) with the kernels of Eq. (W_LRI)), its diagonal and q indexing, the pair
densities (C-tilde of Sec. III.A), the interpolation of W and its inverse (Sec. III.B), the velocity and
finite-momentum start vectors (Eq. (abs_vel)), the exact spectrum and the Lorentzian, the Lanczos
recurrence and continued fraction, the lowest exciton and the binding energy (Sec. IV.B.3), the gradients,
and the row-at-a-time forms the large-mesh parity tests use.  The copies without a slip reproduce the
oracle and pass every pin (the "none" cases), so a failure is the pin catching the slip."""
import dataclasses

import numpy as np
import pytest

import oracle
import oracle.bse_ref as R
import test_oracle_binding as TB
import test_oracle_full_bse as TF
import test_oracle_grad as TG
import test_oracle_hamiltonian as TH
import test_oracle_haydock as TY
import test_oracle_interp as TI
import test_oracle_momentum as TM
import test_oracle_offsets as TO
import test_oracle_rows as TR
import test_oracle_two_centre as TC
from conftest import SMALL, TINY
from synth import dense_kmesh, make_problem


# ---------------------------------------------------------------------------------------------------------
# mutated copies of the oracle functions (same arithmetic as the oracle except for the planted slip)
# ---------------------------------------------------------------------------------------------------------
def _block_with(kind):
    """hamiltonian_block with one planted slip."""
    def blk(prob, W_q, alpha, k, kp, cache=None):
        val, con = R._bands(prob)
        Nk, nc, nv = prob.Nk, prob.nc, prob.nv
        Mcv = R._pairs(prob, k, con, k, val)
        Mvc = R._pairs(prob, kp, val, kp, con)
        if kind == "valence_density_unconjugated":
            Mvv = np.transpose(R._pairs(prob, k, val, kp, val), (0, 2, 1))   # M_vv'(k,k') where conj is due
        else:
            Mvv = R._pairs(prob, kp, val, k, val)
        if kind == "conduction_density_reversed":
            Mcc = np.transpose(R._pairs(prob, kp, con, k, con), (0, 2, 1))   # M_c'c(k',k) read as [c][c']
        else:
            Mcc = R._pairs(prob, k, con, kp, con)
        qi = R.q_index(prob.nk, kp, k) if kind == "W_of_minus_q" else R.q_index(prob.nk, k, kp)
        Wq = W_q[qi].T if kind == "W_transposed" else W_q[qi]
        Vb = prob.Vbar.T if kind == "Vbar_transposed" else prob.Vbar
        out = "vcpd" if kind == "transition_order" else "cvdp"
        t1 = np.einsum("mcv,mn->ncv", Mcv, Vb)
        Xb = (alpha / Nk) * np.einsum("ncv,npd->" + out, t1, Mvc)
        t2 = np.einsum("mpv,mn->npv", Mvv, Wq)
        Db = -(1.0 / Nk) * np.einsum("npv,ncd->" + out, t2, Mcc)
        if kind == "exchange_sign":
            Xb = -Xb
        elif kind == "direct_sign":
            Db = -Db
        elif kind == "dropped_exchange":
            Xb = 0.0 * Xb
        elif kind == "dropped_direct":
            Db = 0.0 * Db
        elif kind == "direct_without_1_over_Nk":
            Db = Nk * Db
        b = (Xb + Db).reshape(nc * nv, nc * nv)
        if k == kp:
            te = R.transition_energies(prob)[k]
            b = b + np.diag(-te if kind == "diagonal_sign" else te)
        return b
    return blk


def _interp_with(kind):
    def interp(W_R, Rv, w_R, q_frac):
        W_R = np.asarray(W_R, dtype=np.complex128)
        q_frac = np.atleast_2d(np.asarray(q_frac, dtype=np.float64))
        out = np.zeros((len(q_frac),) + W_R.shape[1:], dtype=np.complex128)
        sign = -1.0 if kind == "fourier_sign" else 1.0
        two_pi = 1.0 if kind == "missing_2pi" else 2.0 * np.pi
        for iq, q in enumerate(q_frac):
            for r in range(len(Rv)):
                w = 1.0 if kind == "weights_dropped" else w_R[r]
                out[iq] += w * np.exp(sign * 1j * two_pi * np.dot(q, Rv[r])) * W_R[r]
        return out
    return interp


def _velocity_with(kind):
    def vel(prob, pol):
        pol = np.atleast_2d(pol)
        nv, nc = prob.nv, prob.nc
        eps = prob.eps_qp if kind == "quasiparticle_denominator" else prob.eps_ks
        out = np.zeros((prob.N, len(pol)), dtype=np.complex128)
        for b, e in enumerate(pol):
            for k in range(prob.Nk):
                for c in range(nc):
                    for v in range(nv):
                        amp = sum(e[a] * prob.vel[a, k, c, v] for a in range(3))
                        if kind == "conjugated_amplitude":
                            amp = np.conj(amp)
                        out[(k * nc + c) * nv + v, b] = amp / (eps[k, nv + c] - eps[k, v])
        return out
    return vel


def _cf_with(kind):
    def cf(a, b, steps, omega, eta, Nk):
        z = np.asarray(omega, dtype=np.float64) + (-1j if kind == "eta_sign" else 1j) * eta
        sh = 1 if kind == "coefficient_shift" else 0
        g = z - a[steps - 1]
        for j in range(steps - 1, 0, -1):
            g = z - a[j - 1] - b[min(j + sh, steps - 1)] ** 2 / g
        f = (b[0] if kind == "b0_unsquared" else b[0] ** 2) / g
        return -np.imag(f) / (np.pi * (1 if kind == "missing_1_over_Nk" else Nk))
    return cf


def _eb_with(kind):
    def eb(prob, Omega1):
        nv = prob.nv
        e = prob.eps_ks if kind == "kohn_sham_energies" else prob.eps_qp
        if kind == "indirect_gap":
            gap = e[:, nv].min() - e[:, nv - 1].max()
        elif kind == "max_for_min":
            gap = (e[:, nv] - e[:, nv - 1]).max()
        elif kind == "wrong_bands":
            gap = (e[:, nv + 1] - e[:, nv - 2]).min()
        else:
            gap = (e[:, nv] - e[:, nv - 1]).min()
        return Omega1 - gap if kind == "wrong_sign" else gap - Omega1
    return eb


def _grad_with(kind):
    """grad_apply with one planted slip."""
    def grad(prob, W_q, Ybar, X, alpha=None):
        nv, nc, Nk = prob.nv, prob.nc, prob.Nk
        nt = nc * nv
        val, con = R._bands(prob)
        Ybar = np.asarray(Ybar).reshape(prob.N, -1)
        X = np.asarray(X).reshape(prob.N, -1)
        g_eps = np.zeros((Nk, nv + nc))
        for k in range(Nk):
            for c in range(nc):
                for v in range(nv):
                    s = np.real(np.vdot(Ybar[(k * nc + c) * nv + v], X[(k * nc + c) * nv + v]))
                    sg = -1.0 if kind == "eps_signs_swapped" else 1.0
                    g_eps[k, nv + c] += sg * s
                    g_eps[k, v] -= sg * s
        g_Wq = np.zeros((Nk, prob.n_aux, prob.n_aux), dtype=np.complex128)
        for k in range(Nk):
            for kp in range(Nk):
                Mvv = R._pairs(prob, kp, val, k, val)
                Mcc = R._pairs(prob, k, con, kp, con)
                G = (Ybar[k * nt:(k + 1) * nt] @ X[kp * nt:(kp + 1) * nt].conj().T).reshape(nc, nv, nc, nv)
                out = "nm" if kind == "W_gradient_transposed" else "mn"
                a = Mvv if kind == "valence_conjugate_dropped" else Mvv.conj()
                term = np.einsum("mpv,ncd,cvdp->" + out, a, Mcc.conj(), G)
                scale = -1.0 if kind != "W_gradient_sign" else 1.0
                if kind != "W_gradient_without_1_over_Nk":
                    scale /= Nk
                qi = R.q_index(prob.nk, kp, k) if kind == "W_gradient_at_minus_q" else R.q_index(prob.nk, k, kp)
                g_Wq[qi] += scale * term
        return g_eps, g_Wq
    return grad


def _gwr_with(kind):
    def gwr(g_Wq, Rv, w_R, q_frac):
        out = np.zeros((len(Rv),) + g_Wq.shape[1:], dtype=np.complex128)
        sign = 1.0 if kind == "phase_sign" else -1.0
        for r in range(len(Rv)):
            for iq, q in enumerate(q_frac):
                out[r] += np.exp(sign * 2j * np.pi * np.dot(q, Rv[r])) * g_Wq[iq]
            if kind != "weights_dropped":
                out[r] *= w_R[r]
        return out
    return gwr


def _pd_with(kind):
    """pair_density with one planted slip."""
    def pd(psi, C, ki, bi, kj, bj):
        a = psi[ki][list(bi)]
        b = psi[kj][list(bj)]
        if kind == "conjugate_on_the_right":
            a, b = a.conj(), b.conj()
        Cm = np.transpose(C, (0, 2, 1)) if kind == "C_transposed" else C
        if kind == "k_of_the_left_band":
            b = psi[ki][list(bj)]
        return np.matmul(a.conj()[None], np.matmul(Cm, b.T))
    return pd


def _spec_with(kind):
    def spec(Omega, Z, P, omega, eta, Nk):
        amp = np.abs((Z.T if kind == "eigenvectors_unconjugated" else Z.conj().T) @ P) ** 2
        if kind == "amplitude_unsquared":
            amp = np.sqrt(amp)
        L = R.lorentzian(np.asarray(omega)[None, :] - np.asarray(Omega)[:, None], eta)
        return (amp.T @ L) / (1 if kind == "missing_1_over_Nk" else Nk)
    return spec


def _lor_with(kind):
    def lor(x, eta):
        if kind == "full_width_for_half_width":
            eta = eta / 2
        num = eta if kind != "missing_1_over_pi" else eta * np.pi
        return (num / np.pi) / (x * x + (eta if kind == "eta_unsquared" else eta * eta))
    return lor


def _lowest_with(kind):
    def lowest(H):
        Om, Z = np.linalg.eigh(H)
        i = -1 if kind == "largest_eigenvalue" else 0
        return Om[i], (Z[i] if kind == "eigenvector_row" else Z[:, i])
    return lowest


def _c2r_with(kind):
    def c2r(W_qc, coarse, Rv):
        qc = R.coarse_mesh(coarse)
        out = np.zeros((len(Rv),) + W_qc.shape[1:], dtype=np.complex128)
        sign = 1.0 if kind == "phase_sign" else -1.0
        for r in range(len(Rv)):
            for iq in range(len(qc)):
                out[r] += np.exp(sign * 2j * np.pi * np.dot(qc[iq], Rv[r])) * W_qc[iq]
        return out if kind == "missing_1_over_Nc" else out / len(qc)
    return c2r


def _ds_with(kind):
    def ds(prob):
        nv, nc = prob.nv, prob.nc
        out = np.zeros((prob.N, 1), dtype=np.complex128)
        for k in range(prob.Nk):
            for c in range(nc):
                for v in range(nv):
                    if kind == "conjugated_element":
                        out[(k * nc + c) * nv + v, 0] = np.vdot(prob.psi[k, v], prob.psi[k, nv + c])
                    elif kind == "same_band_twice":
                        out[(k * nc + c) * nv + v, 0] = np.vdot(prob.psi[k, nv + c], prob.psi[k, nv + c])
                    else:
                        out[(k * nc + c) * nv + v, 0] = np.vdot(prob.psi[k, nv + c], prob.psi[k, v])
        return out
    return ds


def _allpairs_with(kind):
    """apply_H_rows_allpairs with one planted slip."""
    def rows_fn(prob, W_q, X, rows, alpha=None, chunk=64):
        alpha = prob.alpha if alpha is None else alpha
        nv, nc, Nk, na, no = prob.nv, prob.nc, prob.Nk, prob.n_aux, prob.n_ao
        nt = nc * nv
        val, con = R._bands(prob)
        pv, pc = prob.psi[:, val, :], prob.psi[:, con, :]
        C = prob.C
        X = np.asarray(X).reshape(Nk, nt, -1)
        nb = X.shape[2]
        Xr = X.reshape(Nk, nc, nv, nb)
        last = Nk - chunk + 1 if kind == "ragged_chunk_dropped" else Nk
        t = np.zeros((na, nb), dtype=np.complex128)
        for k0 in range(0, max(last, 1), chunk):
            ks = slice(k0, min(Nk, k0 + chunk))
            K = ks.stop - ks.start
            Cpc = np.transpose(np.tensordot(C, pc[ks], axes=([2], [2])), (2, 1, 0, 3)).reshape(K, no, -1)
            left = pv[ks] if kind == "exchange_density_unconjugated" else pv[ks].conj()
            Mvc = np.transpose(np.matmul(left, Cpc).reshape(K, nv, na, nc), (0, 2, 1, 3))
            t += np.transpose(Mvc, (1, 0, 2, 3)).reshape(na, -1) @ np.transpose(Xr[ks], (0, 2, 1, 3)).reshape(-1, nb)
        u = (prob.Vbar.T if kind == "Vbar_transposed" else prob.Vbar) @ t
        qtab = np.array([[R.q_index(prob.nk, kp, k) if kind == "q_reversed" else R.q_index(prob.nk, k, kp)
                          for kp in range(Nk)] for k in rows])
        eps_t = R.transition_energies(prob)
        out = np.zeros((len(rows), nt, nb), dtype=np.complex128)
        for i, k in enumerate(rows):
            Mcv = R.pair_density(prob.psi, C, k, con, k, val)
            out[i] += (alpha / Nk) * np.einsum("mcv,mb->cvb", Mcv, u).reshape(nt, nb)
            out[i] += eps_t[k][:, None] * X[k]
            Cv = np.matmul(C, pv[k].T)
            Bc = np.matmul(pc[k].conj()[None], C)
            for k0 in range(0, max(last, 1), chunk):
                ks = slice(k0, min(Nk, k0 + chunk))
                K = ks.stop - ks.start
                Mvv = np.transpose(np.tensordot(pv[ks].conj(), Cv, axes=([2], [1])), (0, 2, 1, 3)).reshape(K, na, nv * nv)
                Mcc = np.transpose(np.tensordot(Bc, pc[ks], axes=([2], [2])), (2, 1, 3, 0)).reshape(K, nc * nc, na)
                W = W_q[qtab[i, ks]]
                t2 = np.matmul(W if kind == "W_transposed" else np.transpose(W, (0, 2, 1)), Mvv)
                D = -(1.0 / Nk) * np.matmul(Mcc, t2)
                D = np.transpose(D.reshape(K, nc, nc, nv, nv),
                                 (0, 2, 3, 1, 4) if kind == "block_transposed" else (0, 1, 4, 2, 3)).reshape(K, nt, nt)
                out[i] += np.transpose(D, (1, 0, 2)).reshape(nt, K * nt) @ X[ks].reshape(K * nt, nb)
        return out.reshape(len(rows) * nt, nb)
    return rows_fn


def _wmm_with(kind):
    def wmm(W_R, Rv, w_R, q_frac):
        W_R = np.asarray(W_R, dtype=np.complex128)
        q_frac = np.atleast_2d(np.asarray(q_frac, dtype=np.float64))
        sign = -1.0 if kind == "phase_sign" else 1.0
        w = np.ones(len(Rv)) if kind == "weights_dropped" else np.asarray(w_R)
        ph = w[None, :] * np.exp(sign * 2j * np.pi * (q_frac @ np.asarray(Rv, dtype=np.float64).T))
        out = (ph @ W_R.reshape(len(Rv), -1)).reshape((len(q_frac),) + W_R.shape[1:])
        return np.transpose(out, (0, 2, 1)) if kind == "result_transposed" else out
    return wmm


def _geps_with(kind):
    def geps(prob, Ybar, X):
        nv, nc, Nk = prob.nv, prob.nc, prob.Nk
        yb = np.asarray(Ybar) if kind == "conjugate_dropped" else np.conj(np.asarray(Ybar))
        s = np.real(np.sum(yb * np.asarray(X), axis=1)).reshape(Nk, nc, nv)
        sg = -1.0 if kind == "signs_swapped" else 1.0
        g = np.zeros((Nk, nv + nc))
        g[:, nv:] = sg * s.sum(axis=2)
        g[:, :nv] = -sg * s.sum(axis=1)
        return g
    return geps


def _gwq_with(kind):
    """grad_Wq_at with one planted slip."""
    def gwq(prob, Ybar, X, qs, chunk=64):
        nv, nc, Nk, na, no = prob.nv, prob.nc, prob.Nk, prob.n_aux, prob.n_ao
        nt = nc * nv
        val, con = R._bands(prob)
        pv, pc = prob.psi[:, val, :], prob.psi[:, con, :]
        C = prob.C
        Ybar = np.asarray(Ybar).reshape(Nk, nt, -1)
        X = np.asarray(X).reshape(Nk, nt, -1)
        out = np.zeros((len(qs), na, na), dtype=np.complex128)
        n = np.array(prob.nk)
        kidx = np.array(np.unravel_index(np.arange(Nk), prob.nk)).T
        for i, q in enumerate(qs):
            sq = -1 if kind == "pairs_at_minus_q" else 1
            kps = np.ravel_multi_index(tuple(((kidx + sq * np.array(np.unravel_index(q, prob.nk))) % n).T), prob.nk)
            for k0 in range(0, Nk, chunk):
                ks = np.arange(k0, min(Nk, k0 + chunk))
                kp = kps[ks]
                K = len(ks)
                Cv = np.transpose(np.tensordot(C, pv[ks], axes=([2], [2])), (2, 1, 0, 3)).reshape(K, no, -1)
                Mvv = np.transpose(np.matmul(pv[kp].conj(), Cv).reshape(K, nv, na, nv), (0, 2, 1, 3))
                Cc = np.transpose(np.tensordot(C, pc[kp], axes=([2], [2])), (2, 1, 0, 3)).reshape(K, no, -1)
                Mcc = np.transpose(np.matmul(pc[ks].conj(), Cc).reshape(K, nc, na, nc), (0, 2, 1, 3))
                xk = X[kp] if kind == "X_unconjugated" else X[kp].conj()
                G = np.matmul(Ybar[ks], np.transpose(xk, (0, 2, 1)))
                G = np.transpose(G.reshape(K, nc, nv, nc, nv), (0, 1, 3, 4, 2)).reshape(K, nc * nc, nv * nv)
                Z = np.matmul(Mcc.conj().reshape(K, na, nc * nc), G)
                A = np.transpose(Mvv.conj().reshape(K, na, nv * nv), (1, 0, 2)).reshape(na, -1)
                Bz = np.transpose(Z, (1, 0, 2)).reshape(na, -1)
                term = -(1.0 / Nk) * (A @ Bz.T)
                out[i] += term.T if kind == "result_transposed" else term
        return out
    return gwq


def _haydock_with(kind):
    """haydock with one planted slip."""
    def hay(apply, p, m, tol=1e-12):
        p = np.asarray(p, dtype=np.complex128)
        b0 = np.linalg.norm(p)
        a = np.zeros(m)
        b = np.zeros(m + 1)
        b[0] = b0
        Q = [p if kind == "start_unnormalised" else p / b0]
        qprev = np.zeros_like(p)
        steps = m
        for j in range(1, m + 1):
            qj = Q[-1]
            w = apply(qj)
            a[j - 1] = np.abs(np.vdot(qj, w)) if kind == "a_modulus" else np.real(np.vdot(qj, w))
            if kind != "a_not_subtracted":
                w = w - a[j - 1] * qj
            w = w - (b[j - 1] if j > 1 else 0.0) * qprev
            Qm = np.array(Q)
            for _ in range(2):
                w = w - Qm.T @ (Qm.conj() @ w)
            b[j] = np.linalg.norm(w) ** (2 if kind == "b_squared" else 1)
            scale = max(np.abs(a[:j]).max(), b[1:j].max(initial=0.0))
            if b[j] <= tol * scale:
                steps = j
                break
            qprev = qj
            if j < m:
                Q.append(w / b[j])
        return a, b, steps, np.array(Q[:steps])
    return hay


def _gspec_with(kind):
    def gspec(prob, W_q, P, omega, eta, gamma, H=None, alpha=None):
        if H is None:
            H = R.build_H(prob, W_q, alpha)
        Om, U = np.linalg.eigh(H)
        Nk = prob.Nk
        Ys, Xs = [], []
        for e in range(P.shape[1]):
            c = U.conj().T @ P[:, e]
            for iw, w in enumerate(omega):
                z = w + 1j * eta
                y = U @ (c / (z - Om))
                yt = y if kind == "same_resolvent_both_sides" else U @ (c / (np.conj(z) - Om))
                f = -1.0 if kind == "missing_i" else -1j
                Ys.append((f * gamma[e][iw] / (np.pi * Nk)) * yt)
                Xs.append(y)
        return R.grad_apply(prob, W_q, np.array(Ys).T, np.array(Xs).T, alpha)
    return gspec


def _glow_with(kind):
    def glow(prob, W_q, H=None, alpha=None):
        if H is None:
            H = R.build_H(prob, W_q, alpha)
        Om, Z = np.linalg.eigh(H)
        x = Z[:, 1:2] if kind == "second_eigenvector" else Z[:, :1]
        if kind == "eigenvector_conjugated":
            x = x.conj()
        g_eps, g_Wq = R.grad_apply(prob, W_q, x, x, alpha)
        return Om[0], g_eps, g_Wq
    return glow


def _te_with(kind):
    def te(prob, eps=None):
        e = prob.eps_qp if eps is None else eps
        if kind == "kohn_sham" and eps is None:
            e = prob.eps_ks
        nv, nc = prob.nv, prob.nc
        out = np.empty((len(e), nc * nv))
        for k in range(len(e)):
            for c in range(nc):
                for v in range(nv):
                    d = e[k, nv + c] - e[k, v]
                    out[k, (v * nc + c) if kind == "valence_major" else (c * nv + v)] = -d if kind == "reversed" else d
        return out
    return te


def _qi_with(kind):
    def qi(nk, ik, jk):
        n1, n2, n3 = nk
        a1, a2, a3 = ik // (n2 * n3), (ik // n3) % n2, ik % n3
        b1, b2, b3 = jk // (n2 * n3), (jk // n3) % n2, jk % n3
        if kind == "k_minus_kprime":
            a1, a2, a3, b1, b2, b3 = b1, b2, b3, a1, a2, a3
        if kind == "axes_swapped":
            return (((b3 - a3) % n3) * n2 + (b2 - a2) % n2) * n1 + (b1 - a1) % n1
        return (((b1 - a1) % n1) * n2 + (b2 - a2) % n2) * n3 + (b3 - a3) % n3
    return qi


def _cb_with(kind):
    """coupling_block with one planted slip."""
    def cb(prob, W_q, alpha, k, kp):
        val, con = R._bands(prob)
        nc, nv = prob.nc, prob.nv
        Mcv = R._pairs(prob, k, con, k, val)
        Mcv2 = R._pairs(prob, kp, con, kp, val)
        if kind == "exchange_density_conjugated":
            Mcv2 = np.transpose(R._pairs(prob, kp, val, kp, con), (0, 2, 1))     # M_v'c'(k',k') read as [c'][v']
        Mcpv = R._pairs(prob, kp, con, k, val)
        Mcvp = R._pairs(prob, k, con, kp, val)
        if kind == "direct_densities_swapped":
            Mcpv, Mcvp = R._pairs(prob, k, con, kp, val), R._pairs(prob, kp, con, k, val)
        qi = R.q_index(prob.nk, kp, k) if kind == "W_of_minus_q" else R.q_index(prob.nk, k, kp)
        Wq = W_q[qi].T if kind == "W_transposed" else W_q[qi]
        Vb = prob.Vbar.T if kind == "Vbar_transposed" else prob.Vbar
        Xb = (alpha / prob.Nk) * np.einsum("mcv,mn,ndp->cvdp", Mcv, Vb, Mcv2)
        Db = -(1.0 / prob.Nk) * np.einsum("mdv,mn,ncp->cvdp", Mcpv, Wq, Mcvp)
        if kind == "direct_sign":
            Db = -Db
        elif kind == "exchange_sign":
            Xb = -Xb
        return (Xb + Db).reshape(nc * nv, nc * nv)
    return cb


def _feig_with(kind):
    """full_bse_eig with one planted slip."""
    def feig(A, B):
        import scipy.linalg
        N = A.shape[0]
        Bl = B if kind == "lower_block_unconjugated" else B.conj()
        M = np.block([[A, B], [Bl, A.conj()]])
        J = np.diag(np.r_[np.ones(N), -np.ones(N)]).astype(np.complex128)
        lam, Z = scipy.linalg.eigh(J, M)
        pos = lam < 0 if kind == "negative_branch" else lam > 0
        Om = 1.0 / np.abs(lam[pos])
        Z = Z[:, pos] * (np.sqrt(Om)[None, :] if kind != "normalised_in_M" else 1.0)
        order = np.argsort(Om)
        Om, Z = Om[order], Z[:, order]
        return Om, Z[:N], Z[N:]
    return feig


def _famp_with(kind):
    def famp(prob, pol, X, Y):
        pol = np.atleast_2d(pol)
        nv, nc = prob.nv, prob.nc
        eps = prob.eps_qp if kind == "quasiparticle_denominator" else prob.eps_ks
        out = np.zeros((X.shape[1], len(pol)), dtype=np.complex128)
        for b, e in enumerate(pol):
            for k in range(prob.Nk):
                for c in range(nc):
                    for v in range(nv):
                        I = (k * nc + c) * nv + v
                        d = eps[k, nv + c] - eps[k, v]
                        m = sum(e[a] * prob.vel[a, k, c, v] for a in range(3))
                        my = np.conj(m) if kind == "Y_element_conjugated" else m
                        dy = d if kind == "Y_denominator_sign" else -d
                        out[:, b] += np.conj(m) / d * X[I] + my / dy * Y[I]
        return out
    return famp


def _twosided_with(kind):
    """apply_rows_twosided with one planted slip."""
    def rows_fn(prob, W_q, X, rows, block="A", alpha=None, chunk=64):
        alpha = prob.alpha if alpha is None else alpha
        nv, nc, Nk = prob.nv, prob.nc, prob.Nk
        nt = nc * nv
        pv, pc = R._psi_sets(prob)
        Fv, Fc, two = R._F_sets(prob)
        X = np.asarray(X).reshape(Nk, nt, -1)
        nb = X.shape[2]
        allk = np.arange(Nk)
        rho = R._pairs_rows(pc, Fc, allk, pv, Fv, allk, two)
        Xr = X.reshape(Nk, nc, nv, nb)
        if block == "A" or kind == "B_exchange_with_the_A_density":
            Mvc = R._pairs_rows(pv, Fv, allk, pc, Fc, allk, two)
            t = np.einsum("knvc,kcvb->nb", Mvc, Xr, optimize=True)
        else:
            t = np.einsum("kncv,kcvb->nb", rho, Xr, optimize=True)
        u = prob.Vbar @ t
        qtab = np.array([[R.q_index(prob.nk, kp, k) if kind == "q_reversed" else R.q_index(prob.nk, k, kp)
                          for kp in range(Nk)] for k in rows])
        eps_t = R.transition_energies(prob)
        out = np.zeros((len(rows), nt, nb), dtype=np.complex128)
        for i, k in enumerate(rows):
            out[i] += (alpha / Nk) * np.einsum("mcv,mb->cvb", rho[k], u).reshape(nt, nb)
            if block == "A" or kind == "diagonal_in_B":
                out[i] += eps_t[k][:, None] * X[k]
            for k0 in range(0, Nk, chunk):
                ks = np.arange(k0, min(Nk, k0 + chunk))
                kk = np.full(len(ks), k)
                W = W_q[qtab[i, ks]]
                if kind == "W_transposed":
                    W = np.transpose(W, (0, 2, 1))
                if block == "A":
                    L = R._pairs_rows(pv, Fv, ks, pv, Fv, kk, two)
                    Rt = R._pairs_rows(pc, Fc, kk, pc, Fc, ks, two)
                    D = -(1.0 / Nk) * np.einsum("xmpv,xmn,xncd->xcvdp", L, W, Rt, optimize=True)
                else:
                    L = R._pairs_rows(pc, Fc, ks, pv, Fv, kk, two)
                    Rt = R._pairs_rows(pc, Fc, kk, pv, Fv, ks, two)
                    if kind == "B_direct_densities_swapped":
                        L, Rt = R._pairs_rows(pc, Fc, kk, pv, Fv, ks, two), R._pairs_rows(pc, Fc, ks, pv, Fv, kk, two)
                    D = -(1.0 / Nk) * np.einsum("xmdv,xmn,xncp->xcvdp", L, W, Rt, optimize=True)
                out[i] += np.einsum("xcvdp,xdpb->cvb", D, Xr[ks], optimize=True).reshape(nt, nb)
        return out.reshape(len(rows) * nt, nb)
    return rows_fn


def _pairs_rows_with(kind):
    def pr(pa, Fa, ka, pb, Fb, kb, two):
        M = np.einsum("xis,xmsj->xmij", pa[ka].conj(), Fb[kb], optimize=True)
        if two and kind != "second_centre_dropped":
            Fak = Fa[ka] if kind == "second_centre_unconjugated" else Fa[ka].conj()
            M = M + np.einsum("xmti,xjt->xmij", Fak, pb[kb], optimize=True)
        return M
    return pr


def _fsets_with(kind):
    def fs(prob):
        pv, pc = R._psi_sets(prob)
        if getattr(prob, "C_R", None) is None:
            Cm = np.transpose(prob.C, (0, 2, 1)) if kind == "C_transposed" else prob.C
            Fv = np.transpose(np.tensordot(Cm, pv, axes=([2], [2])), (2, 0, 1, 3))
            Fc = np.transpose(np.tensordot(Cm, pc, axes=([2], [2])), (2, 0, 1, 3))
            return Fv, Fc, False
        kv, kc = prob.band_k()
        RC = np.asarray(prob.RC, dtype=np.float64)
        sign = -1.0 if kind == "phase_sign" else 1.0
        out = []
        for psi_n, kn in ((pv, kv), (pc, kc)):
            F = np.zeros((prob.Nk, prob.n_aux, prob.n_ao, psi_n.shape[1]), dtype=np.complex128)
            for r in range(len(RC)):
                ph = np.exp(sign * 2j * np.pi * (kn @ RC[r]))
                G = np.tensordot(np.transpose(prob.C_R[r], (0, 2, 1)) if kind == "C_transposed" else prob.C_R[r],
                                 psi_n, axes=([2], [2]))
                F += ph[:, None, None, None] * np.transpose(G, (2, 0, 1, 3))
            out.append(F)
        return out[0], out[1], True
    return fs


def _hrows_with(kind):
    """hamiltonian_rows with one planted slip."""
    def hrows(prob, W_q, rows, alpha=None, chunk=64):
        alpha = prob.alpha if alpha is None else alpha
        nv, nc, Nk, na, no = prob.nv, prob.nc, prob.Nk, prob.n_aux, prob.n_ao
        nt = nc * nv
        val, con = R._bands(prob)
        pv, pc = R._psi_sets(prob)
        C = prob.C
        Mvc = np.empty((Nk, na, nv, nc), dtype=np.complex128)
        for k0 in range(0, Nk, chunk):
            ks = slice(k0, min(Nk, k0 + chunk))
            K = ks.stop - ks.start
            Cpc = np.transpose(np.tensordot(C, pc[ks], axes=([2], [2])), (2, 1, 0, 3)).reshape(K, no, -1)
            Mvc[ks] = np.transpose(np.matmul(pv[ks].conj(), Cpc).reshape(K, nv, na, nc), (0, 2, 1, 3))
        qtab = np.array([[R.q_index(prob.nk, kp, k) if kind == "q_reversed" else R.q_index(prob.nk, k, kp)
                          for kp in range(Nk)] for k in rows])
        eps_t = R.transition_energies(prob)
        out = np.zeros((len(rows), nt, Nk, nt), dtype=np.complex128)
        for i, k in enumerate(rows):
            Mcv = R.pair_density(prob.psi, C, k, con, k, val)
            t1 = np.einsum("mcv,mn->ncv", Mcv, prob.Vbar)
            out[i] += ((alpha / Nk) * np.einsum("ncv,knpd->cvkdp", t1, Mvc)).reshape(nt, Nk, nt)
            if kind != "diagonal_dropped":
                out[i, :, k, :] += np.diag(eps_t[k])
            Cv = np.matmul(C, pv[k].T)
            Bc = np.matmul(pc[k].conj()[None], C)
            for k0 in range(0, Nk, chunk):
                ks = slice(k0, min(Nk, k0 + chunk))
                K = ks.stop - ks.start
                Mvv = np.transpose(np.tensordot(pv[ks].conj(), Cv, axes=([2], [1])), (0, 2, 1, 3)).reshape(K, na, nv * nv)
                Mcc = np.transpose(np.tensordot(Bc, pc[ks], axes=([2], [2])), (2, 1, 3, 0)).reshape(K, nc * nc, na)
                W = W_q[qtab[i, ks]]
                t2 = np.matmul(W if kind == "W_transposed" else np.transpose(W, (0, 2, 1)), Mvv)
                D = -(1.0 / Nk) * np.matmul(Mcc, t2)
                perm = (1, 3, 0, 2, 4) if kind == "column_order_swapped" else (1, 4, 0, 2, 3)
                out[i, :, ks, :] += np.transpose(D.reshape(K, nc, nc, nv, nv), perm).reshape(nt, K, nt)
        return out.reshape(len(rows) * nt, Nk * nt)
    return hrows


def _bfull_with(kind):
    def bfull(prob, W_q, alpha=None):
        A = R.build_H(prob, W_q, alpha)
        B = R.build_B(prob, W_q, alpha)
        lower_left = B.conj() if kind == "lower_left_sign" else -B.conj()
        lower_right = -A if kind == "lower_right_unconjugated" else -A.conj()
        return np.block([[A, B], [lower_left, lower_right]])
    return bfull


def _oavg_with(kind):
    def oavg(spectra, weights):
        out = np.zeros_like(np.asarray(spectra[0], dtype=np.float64))
        for S, w in zip(spectra, weights):
            out = out + (1.0 if kind == "weights_dropped" else w) * np.asarray(S, dtype=np.float64)
        return out
    return oavg


def _lrik_with(kind):
    def lrik(C_R, RC, k):
        sign = -1.0 if kind == "phase_sign" else 1.0
        ph = np.exp(sign * 2j * np.pi * (np.asarray(RC, dtype=np.float64) @ np.asarray(k, dtype=np.float64)))
        out = np.tensordot(ph, C_R, axes=(0, 0))
        return np.transpose(out, (0, 2, 1)) if kind == "transposed" else out
    return lrik


def _bh_with(kind):
    def bh(prob, W_q, alpha=None):
        alpha = prob.alpha if alpha is None else alpha
        Nk, nt = prob.Nk, prob.nc * prob.nv
        H = np.zeros((Nk * nt, Nk * nt), dtype=np.complex128)
        for k in range(Nk):
            for kp in range(Nk):
                r, c = (kp, k) if kind == "blocks_placed_transposed" else (k, kp)
                H[r * nt:(r + 1) * nt, c * nt:(c + 1) * nt] = R.hamiltonian_block(prob, W_q, alpha, k, kp)
        return H
    return bh


def _ahr_with(kind):
    def ahr(prob, W_q, X, rows, alpha=None):
        alpha = prob.alpha if alpha is None else alpha
        nt = prob.nc * prob.nv
        X = np.asarray(X).reshape(prob.Nk * nt, -1)
        out = np.zeros((len(rows) * nt, X.shape[1]), dtype=np.complex128)
        for i, k in enumerate(rows):
            for kp in range(prob.Nk):
                blk = R.hamiltonian_block(prob, W_q, alpha, k, kp)
                xs = X[k * nt:(k + 1) * nt] if kind == "own_row_of_X" else X[kp * nt:(kp + 1) * nt]
                out[i * nt:(i + 1) * nt] += blk @ xs
        return out
    return ahr


def _hs_with(kind):
    def hs(apply, P, m, omega, eta, Nk, tol=1e-12):
        S, A, B, st = [], [], [], []
        for col in range(P.shape[1]):
            a, b, n, _ = R.haydock(apply, P[:, 0 if kind == "first_column_only" else col], m, tol)
            S.append(R.continued_fraction(a, b, n, omega, eta, Nk))
            A.append(a)
            B.append(b)
            st.append(n)
        return np.array(S), np.array(A), np.array(B), np.array(st)
    return hs


def _fspec_with(kind):
    def fspec(prob, pol, Omega, X, Y, omega, eta):
        amp = np.abs(R.full_bse_amplitudes(prob, pol, X, Y)) ** 2
        if kind == "both_branches":
            Lw = R.lorentzian(np.asarray(omega)[None, :] - np.asarray(Omega)[:, None], eta) + \
                R.lorentzian(np.asarray(omega)[None, :] + np.asarray(Omega)[:, None], eta)
        else:
            Lw = R.lorentzian(np.asarray(omega)[None, :] - np.asarray(Omega)[:, None], eta)
        return (amp.T @ Lw) / (1 if kind == "missing_1_over_Nk" else prob.Nk)
    return fspec


# ---------------------------------------------------------------------------------------------------------
# the pins each family of functions answers to (the tests of the oracle modules, called with their inputs)
# ---------------------------------------------------------------------------------------------------------
HAMILTONIAN_PINS = {
    "hand_one_k": TH.test_hand_one_k,
    "hand_three_k": TH.test_hand_three_k_phase_orientation,
    "ao_bruteforce_G1": lambda: TH.test_bruteforce_ao_kernel("G1", (2, 2, 1), False),
    "ao_bruteforce_G2": lambda: TH.test_bruteforce_ao_kernel("G2", (2, 2, 1), False),
    "ao_bruteforce_G2_q_ne_minus_q": lambda: TH.test_bruteforce_ao_kernel("G2", (3, 2, 1), False),
    "ao_bruteforce_complex_vbar": lambda: TH.test_bruteforce_ao_kernel("G1", (2, 2, 1), True),
    "hermitian_G2": lambda: TH.test_hermitian(dict(TINY), "G2"),
    "zero_kernel": lambda: TH.test_zero_kernel_is_transition_energies(dict(SMALL)),
    "exchange_psd_alpha": lambda: TH.test_exchange_psd_low_rank_and_alpha(dict(SMALL)),
}
INTERP_PINS = {
    "single_R_closed_form": TI.test_single_R_closed_form,
    "R0_constant": TI.test_R0_only_gives_constant,
    "numpy_fft": lambda: TI.test_matches_numpy_fft_of_padded_box((3, 3, 2), (6, 6, 5)),
    "coarse_round_trip": lambda: TI.test_coarse_round_trip_exact((3, 2, 2)),
    "hand_three_k": TH.test_hand_three_k_phase_orientation,
}
VELOCITY_PINS = {"velocity_hand_case": TH.test_velocity_start_hand_case}
SPECTRUM_PINS = {
    "full_krylov_vs_eigh": lambda: TY.test_full_krylov_equals_eigh(dict(TINY)),
    "diagonal_closed_form": lambda: TY.test_diagonal_closed_form_and_breakdown(dict(SMALL)),
}
GRADIENT_PINS = {
    "linear_response": lambda: TG.test_apply_gradient_is_exact_linear_response(dict(TINY)),
    "linear_response_q_ne_minus_q": lambda: TG.test_apply_gradient_linear_response_where_q_differs_from_minus_q(
        dict(SMALL)),
    "first_moment": lambda: TG.test_first_moment_identity(dict(TINY)),
    "lowest_exciton_fd": lambda: TG.test_lowest_exciton_gradient_fd(dict(SMALL)),
    "spectrum_fd": lambda: TG.test_spectrum_gradient_fd(dict(TINY)),
}
PAIR_PINS = {k: HAMILTONIAN_PINS[k] for k in ("hand_one_k", "hand_three_k", "ao_bruteforce_G1",
                                                 "ao_bruteforce_G2", "ao_bruteforce_G2_q_ne_minus_q")}
SPECTRUM_EXACT_PINS = {
    "ipa_closed_form": lambda: TH.test_zero_kernel_is_transition_energies(dict(SMALL)),
    "full_krylov_vs_eigh": lambda: TY.test_full_krylov_equals_eigh(dict(TINY)),
    "gauge_covariance": lambda: TH.test_gauge_covariance(dict(SMALL)),
}
LOWEST_PINS = {
    "zero_kernel_zero_EB": TB.test_zero_kernel_has_zero_binding_energy,
    "lowest_exciton_fd": lambda: TG.test_lowest_exciton_gradient_fd(dict(SMALL)),
    "lowest_eigenpair": lambda: TH.test_lowest_exciton_is_the_lowest_eigenpair(dict(SMALL)),
}
COARSE_PINS = {"coarse_round_trip_322": lambda: TI.test_coarse_round_trip_exact((3, 2, 2)),
               "coarse_round_trip_222": lambda: TI.test_coarse_round_trip_exact((2, 2, 2))}
DENSITY_PINS = {
    "vanishes_at_Q0": TM.test_density_start_vanishes_at_zero_momentum,
    "completeness_bound": TM.test_density_start_bounded_by_completeness,
    "long_wavelength_limit": TM.test_density_start_long_wavelength_limit_is_the_velocity_form,
}
ROW_PINS = {
    "allpairs_vs_blocks_ragged": lambda: TR.test_allpairs_rows_match_blocks("RAGGED", 7, 2.0),
    "allpairs_vs_blocks_wide_v": lambda: TR.test_allpairs_rows_match_blocks("WIDE_V", 5, 2.0),
    "allpairs_vs_explicit_H": TR.test_allpairs_rows_match_explicit_H,
}
MATMUL_PINS = {
    "matmul_vs_direct_sum": lambda: TR.test_interpolate_matmul_matches_direct_sum("RAGGED"),
    "matmul_single_R": TR.test_interpolate_matmul_single_R_closed_form,
}
GEPS_PINS = {"grad_eps_vs_grad_apply": TR.test_grad_eps_matches_grad_apply}
GWQ_PINS = {
    "grad_Wq_at_vs_grad_apply_ragged": lambda: TR.test_grad_Wq_at_matches_grad_apply("RAGGED", 7),
    "grad_Wq_at_vs_grad_apply_wide_v": lambda: TR.test_grad_Wq_at_matches_grad_apply("WIDE_V", 64),
}
LANCZOS_PINS = {
    "full_krylov_vs_eigh": lambda: TY.test_full_krylov_equals_eigh(dict(TINY)),
    "moment_identities": lambda: TY.test_moment_identities(dict(SMALL)),
    "diagonal_closed_form": lambda: TY.test_diagonal_closed_form_and_breakdown(dict(SMALL)),
    "full_krylov_indefinite": lambda: TY.test_full_krylov_indefinite_operator(dict(TINY)),
}
GSPEC_PINS = {"spectrum_fd": lambda: TG.test_spectrum_gradient_fd(dict(TINY))}
GLOW_PINS = {"lowest_exciton_fd": lambda: TG.test_lowest_exciton_gradient_fd(dict(SMALL))}
TE_PINS = {k: HAMILTONIAN_PINS[k] for k in ("hand_one_k", "hand_three_k")}
TE_PINS["ipa_closed_form"] = lambda: TH.test_zero_kernel_is_transition_energies(dict(SMALL))
TE_PINS["binding_hand_case"] = TB.test_binding_energy_hand_case
QI_PINS = {k: HAMILTONIAN_PINS[k] for k in ("hand_three_k", "ao_bruteforce_G2_q_ne_minus_q")}
QI_PINS["mesh_index_of_the_difference"] = TH.test_q_index_is_the_mesh_index_of_the_difference
COUPLING_PINS = {
    "coupling_bruteforce_G1": lambda: TF.test_coupling_block_bruteforce("G1", (2, 2, 1), False),
    "coupling_bruteforce_G2": lambda: TF.test_coupling_block_bruteforce("G2", (2, 2, 1), False),
    "coupling_bruteforce_G2_q_ne_minus_q": lambda: TF.test_coupling_block_bruteforce("G2", (3, 2, 1), False),
    "coupling_bruteforce_complex_vbar": lambda: TF.test_coupling_block_bruteforce("G1", (2, 2, 1), True),
    "coupling_symmetric_G2": lambda: TF.test_coupling_block_is_symmetric("G2", False),
    "paired_eigenproblem": TF.test_paired_eigenproblem,
}
FULL_EIG_PINS = {
    "paired_eigenproblem": TF.test_paired_eigenproblem,
    "no_coupling_is_tda": TF.test_no_coupling_is_tda,
    "two_level_closed_form": lambda: TF.test_two_level_closed_form(0.2 + 0.5j),
}
FULL_AMP_PINS = {
    "resolvent_identity": TF.test_spectrum_resolvent_identity,
    "no_coupling_is_tda": TF.test_no_coupling_is_tda,
}
TWOSIDED_PINS = {
    "twosided_A": lambda: TR.test_twosided_rows_match_blocks("A", False, {}),
    "twosided_B": lambda: TR.test_twosided_rows_match_blocks("B", False, {}),
    "twosided_A_two_centre": lambda: TR.test_twosided_rows_match_blocks("A", True, {}),
    "twosided_B_two_centre": lambda: TR.test_twosided_rows_match_blocks("B", True, {}),
    "twosided_A_two_centre_momentum": lambda: TR.test_twosided_rows_match_blocks("A", True,
                                                                                 dict(momentum=(0.5, 0.25, 0.0))),
}
HROWS_PINS = {
    "hrows_vs_blocks": lambda: TR.test_hamiltonian_rows_match_blocks("RAGGED", 7, 2.0),
    "hrows_give_build_H": TR.test_hamiltonian_rows_give_build_H,
}
BFULL_PINS = {"paired_eigenproblem": TF.test_paired_eigenproblem,
              "resolvent_identity": TF.test_spectrum_resolvent_identity}
OAVG_PINS = {"equal_spectra": TO.test_offset_average_of_equal_spectra_is_that_spectrum,
             "zero_kernel_closed_form": TO.test_zero_kernel_offset_average_closed_form}
LRIK_PINS = {"real_space_%d" % i: (lambda a=a, b=b: TC.test_two_centre_coefficient_from_real_space(a, b))
             for i, (a, b) in enumerate(TC.KPAIRS)}
BUILD_H_PINS = {k: HAMILTONIAN_PINS[k] for k in ("hand_three_k", "hermitian_G2", "ao_bruteforce_G2_q_ne_minus_q")}
APPLY_ROWS_PINS = {"rows_match_explicit": lambda: TH.test_apply_rows_match_explicit(dict(SMALL)),
                   "allpairs_vs_blocks_ragged": lambda: TR.test_allpairs_rows_match_blocks("RAGGED", 7, 2.0)}
HSPEC_PINS = {"full_krylov_vs_eigh": lambda: TY.test_full_krylov_equals_eigh(dict(TINY))}
FSPEC_PINS = {"resolvent_identity": TF.test_spectrum_resolvent_identity,
              "no_coupling_is_tda": TF.test_no_coupling_is_tda}
BINDING_PINS = {
    "binding_hand_case": TB.test_binding_energy_hand_case,
    "zero_kernel_zero_EB": TB.test_zero_kernel_has_zero_binding_energy,
}

FAMILIES = {
    "hamiltonian_block": (_block_with, HAMILTONIAN_PINS,
                          ["exchange_sign", "direct_sign", "dropped_exchange", "dropped_direct",
                           "direct_without_1_over_Nk", "W_of_minus_q", "W_transposed", "Vbar_transposed",
                           "valence_density_unconjugated", "conduction_density_reversed", "transition_order",
                           "diagonal_sign"]),
    "interpolate_W": (_interp_with, INTERP_PINS, ["fourier_sign", "missing_2pi", "weights_dropped"]),
    "velocity_start": (_velocity_with, VELOCITY_PINS, ["quasiparticle_denominator", "conjugated_amplitude"]),
    "continued_fraction": (_cf_with, SPECTRUM_PINS,
                           ["eta_sign", "coefficient_shift", "b0_unsquared", "missing_1_over_Nk"]),
    "grad_apply": (_grad_with, GRADIENT_PINS,
                   ["eps_signs_swapped", "W_gradient_transposed", "valence_conjugate_dropped", "W_gradient_sign",
                    "W_gradient_without_1_over_Nk", "W_gradient_at_minus_q"]),
    "grad_WR_from_Wq": (_gwr_with, GRADIENT_PINS, ["phase_sign", "weights_dropped"]),
    "pair_density": (_pd_with, PAIR_PINS, ["conjugate_on_the_right", "C_transposed", "k_of_the_left_band"]),
    "spectrum_exact": (_spec_with, SPECTRUM_EXACT_PINS,
                       ["eigenvectors_unconjugated", "amplitude_unsquared", "missing_1_over_Nk"]),
    "lorentzian": (_lor_with, SPECTRUM_EXACT_PINS, ["full_width_for_half_width", "missing_1_over_pi",
                                                    "eta_unsquared"]),
    "lowest_exciton": (_lowest_with, LOWEST_PINS, ["largest_eigenvalue", "eigenvector_row"]),
    "coarse_to_R": (_c2r_with, COARSE_PINS, ["phase_sign", "missing_1_over_Nc"]),
    "density_start": (_ds_with, DENSITY_PINS, ["conjugated_element", "same_band_twice"]),
    "apply_H_rows_allpairs": (_allpairs_with, ROW_PINS,
                              ["ragged_chunk_dropped", "exchange_density_unconjugated", "Vbar_transposed",
                               "q_reversed", "W_transposed", "block_transposed"]),
    "interpolate_W_matmul": (_wmm_with, MATMUL_PINS, ["phase_sign", "weights_dropped", "result_transposed"]),
    "grad_eps": (_geps_with, GEPS_PINS, ["conjugate_dropped", "signs_swapped"]),
    "grad_Wq_at": (_gwq_with, GWQ_PINS, ["pairs_at_minus_q", "X_unconjugated", "result_transposed"]),
    "haydock": (_haydock_with, LANCZOS_PINS, ["start_unnormalised", "a_modulus", "a_not_subtracted",
                                              "b_squared"]),
    "grad_spectrum": (_gspec_with, GSPEC_PINS, ["same_resolvent_both_sides", "missing_i"]),
    "grad_lowest": (_glow_with, GLOW_PINS, ["second_eigenvector", "eigenvector_conjugated"]),
    "transition_energies": (_te_with, TE_PINS, ["reversed", "kohn_sham", "valence_major"]),
    "q_index": (_qi_with, QI_PINS, ["k_minus_kprime", "axes_swapped"]),
    "coupling_block": (_cb_with, COUPLING_PINS, ["exchange_density_conjugated", "direct_densities_swapped",
                                                 "W_of_minus_q", "W_transposed", "Vbar_transposed", "direct_sign",
                                                 "exchange_sign"]),
    "full_bse_eig": (_feig_with, FULL_EIG_PINS, ["lower_block_unconjugated", "negative_branch", "normalised_in_M"]),
    "full_bse_amplitudes": (_famp_with, FULL_AMP_PINS, ["quasiparticle_denominator", "Y_element_conjugated",
                                                        "Y_denominator_sign"]),
    "apply_rows_twosided": (_twosided_with, TWOSIDED_PINS,
                            ["B_exchange_with_the_A_density", "diagonal_in_B", "W_transposed", "q_reversed",
                             "B_direct_densities_swapped"]),
    "_pairs_rows": (_pairs_rows_with, TWOSIDED_PINS, ["second_centre_dropped", "second_centre_unconjugated"]),
    "_F_sets": (_fsets_with, TWOSIDED_PINS, ["phase_sign", "C_transposed"]),
    "hamiltonian_rows": (_hrows_with, HROWS_PINS, ["q_reversed", "diagonal_dropped", "W_transposed",
                                                   "column_order_swapped"]),
    "build_full": (_bfull_with, BFULL_PINS, ["lower_left_sign", "lower_right_unconjugated"]),
    "offset_average": (_oavg_with, OAVG_PINS, ["weights_dropped"]),
    "lri_coeff_k": (_lrik_with, LRIK_PINS, ["phase_sign", "transposed"]),
    "build_H": (_bh_with, BUILD_H_PINS, ["blocks_placed_transposed"]),
    "apply_H_rows": (_ahr_with, APPLY_ROWS_PINS, ["own_row_of_X"]),
    "haydock_spectrum": (_hs_with, HSPEC_PINS, ["first_column_only"]),
    "full_bse_spectrum": (_fspec_with, FSPEC_PINS, ["both_branches", "missing_1_over_Nk"]),
    "binding_energy": (_eb_with, BINDING_PINS,
                       ["kohn_sham_energies", "indirect_gap", "max_for_min", "wrong_bands", "wrong_sign"]),
}

CASES = [(fam, kind) for fam, (_, _, kinds) in FAMILIES.items() for kind in ["none"] + kinds]


def _run_pins(pins):
    failed = []
    for name, pin in pins.items():
        try:
            pin()
        except AssertionError:
            failed.append(name)
    return failed


@pytest.mark.filterwarnings("ignore::RuntimeWarning")   # some slips overflow or divide by zero, as slips do
@pytest.mark.parametrize("fam,kind", CASES, ids=["%s-%s" % c for c in CASES])
def test_planted_mistake_fails_a_pin(monkeypatch, fam, kind):
    make, pins, _ = FAMILIES[fam]
    fn = make(kind)
    # the oracle's own calls resolve through its module, the pins' calls through the package
    monkeypatch.setattr(R, fam, fn)
    if hasattr(oracle, fam):      # private helpers are not re-exported by the package
        monkeypatch.setattr(oracle, fam, fn)
    failed = _run_pins(pins)
    print("[planted %s / %s] pins failing: %s" % (fam, kind, ", ".join(failed) or "none"))
    if kind == "none":
        assert failed == []      # the copy without a slip is the oracle: every pin holds
    else:
        assert failed, "planted mistake %s in %s passes every pin" % (kind, fam)


def test_the_copies_without_a_slip_match_the_oracle():
    # the mutated copies differ from the oracle only by the slip: without one they give the oracle's values
    p = make_problem(dict(TINY), 0, "G2", coarse=(3, 3, 2))
    s3 = make_problem(dict(SMALL), 0, "G2", coarse=(3, 3, 2))
    kq = dense_kmesh(p.nk)
    Wq = R.interpolate_W(p.W_R, p.R, p.w_R, kq)
    P = R.velocity_start(p, np.eye(3))
    H = R.build_H(p, Wq)
    a, b, st, _ = R.haydock(lambda x: H @ x, P[:, 0], 12)
    rng = np.random.default_rng(0)
    Yb = rng.standard_normal((p.N, 2)) + 1j * rng.standard_normal((p.N, 2))
    X = rng.standard_normal((p.N, 2)) + 1j * rng.standard_normal((p.N, 2))
    w = np.linspace(1.0, 5.0, 31)
    Om, Z = np.linalg.eigh(H)
    gq = R.grad_apply(p, Wq, Yb, X)[1]
    t2 = make_problem(dict(SMALL), 0, "G2", coarse=(3, 3, 2), two_centre=True)
    pv2, pc2 = R._psi_sets(t2)
    Fv2, Fc2, _ = R._F_sets(t2)
    calls = {
        "hamiltonian_block": [(p, Wq, p.alpha, k, kp) for k, kp in [(0, 0), (1, 5), (6, 2)]],
        "interpolate_W": [(p.W_R, p.R, p.w_R, kq)],
        "velocity_start": [(p, np.eye(3))],
        "continued_fraction": [(a, b, st, w, 0.1, p.Nk)],
        "binding_energy": [(p, 1.5)],
        "grad_apply": [(p, Wq, Yb, X)],
        "grad_WR_from_Wq": [(gq, p.R, p.w_R, kq)],
        "pair_density": [(p.psi, p.C, 1, [0, 1], 3, [2, 3])],
        "spectrum_exact": [(Om, Z, P, w, 0.1, p.Nk)],
        "lorentzian": [(w - 2.5, 0.1)],
        "lowest_exciton": [(H,)],
        "coarse_to_R": [(Wq[:8], (2, 2, 2), p.R)],
        "density_start": [(p,)],
        "apply_H_rows_allpairs": [(s3, R.interpolate_W(s3.W_R, s3.R, s3.w_R, dense_kmesh(s3.nk)),
                                   rng.standard_normal((s3.N, 2)) + 0j, [0, 7], 2.0, 5)],
        "interpolate_W_matmul": [(p.W_R, p.R, p.w_R, kq)],
        "grad_eps": [(p, Yb, X)],
        "grad_Wq_at": [(p, Yb, X, [0, 3, 5], 3)],
        "haydock": [(lambda x: H @ x, P[:, 0], 12)],
        "grad_spectrum": [(p, Wq, P[:, :1], w[:4], 0.1, rng.standard_normal((1, 4)))],
        "grad_lowest": [(p, Wq)],
        "transition_energies": [(s3,)],
        "q_index": [((3, 2, 5), i, j) for i, j in [(0, 29), (7, 11), (13, 2)]],
        "coupling_block": [(p, Wq, p.alpha, k, kp) for k, kp in [(0, 0), (1, 5), (6, 2)]],
        "full_bse_eig": [(H, R.build_B(p, Wq))],
        "full_bse_amplitudes": [(p, np.eye(3), Z[:, :5], 0.1 * Z[:, 5:10])],
        "apply_rows_twosided": [(t2, R.interpolate_W(t2.W_R, t2.R, t2.w_R, dense_kmesh(t2.nk)),
                                 rng.standard_normal((t2.N, 2)) + 0j, [0, 5], blk, None, 4) for blk in "AB"],
        "_pairs_rows": [(pv2, Fv2, np.arange(t2.Nk), pc2, Fc2, np.arange(t2.Nk)[::-1], True)],
        "_F_sets": [(t2,), (p,)],
        "hamiltonian_rows": [(s3, R.interpolate_W(s3.W_R, s3.R, s3.w_R, dense_kmesh(s3.nk)), [0, 7], 2.0, 5)],
        "build_full": [(p, Wq)],
        "offset_average": [([w, 2 * w, 3 * w, 4 * w], R.PAPER_OFFSET_WEIGHTS)],
        "lri_coeff_k": [(t2.C_R, t2.RC, [0.25, -0.5, 1.0 / 3])],
        "build_H": [(p, Wq)],
        "apply_H_rows": [(p, Wq, X, [0, 5])],
        "haydock_spectrum": [(lambda x: H @ x, P, 10, w, 0.1, p.Nk)],
        "full_bse_spectrum": [(p, np.eye(3), Om[:5], Z[:, :5], 0.1 * Z[:, 5:10], w, 0.1)],
    }
    assert set(calls) == set(FAMILIES)
    for fam, arglists in calls.items():
        make = FAMILIES[fam][0]
        for args in arglists:
            got, ref = make("none")(*args), getattr(R, fam)(*args)
            got, ref = (got if isinstance(got, tuple) else (got,)), (ref if isinstance(ref, tuple) else (ref,))
            assert len(got) == len(ref), fam
            for g, r in zip(got, ref):
                assert np.array_equal(np.asarray(g), np.asarray(r)), fam
