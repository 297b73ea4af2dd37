"""Plain FP64 reference of the dual-k-mesh TDA-BSE path (test infrastructure only).

Conventions (shared with the paper):
* simple cubic lattice, a = 1, V = 1; R integer triples; k, q fractional;
  Fourier phases exp(+2 pi i k.R) as in the definition of C^mu(k) (Sec. III.A);
* dense Gamma-centred mesh, k index (i1*n2 + i2)*n3 + i3;
* q(k, k') = k' - k reduced into the mesh (the phase exp(i(k2 - k1).R) of
  Eq. (W_LRI), with k1 the row and k2 the column of A);
* bands per k: nv valence (ascending) then nc conduction (ascending);
* transition index I = (k*nc + c)*nv + v; blocks of vectors X[I][b].

Every function restates a definition and is deliberately unoptimised.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "kmesh", "q_index", "q_index_table", "interpolate_W", "coarse_to_R", "coarse_mesh",
    "pair_density", "lri_coeff_k", "pair_density_2c", "hamiltonian_block", "build_H", "apply_H", "apply_H_rows",
    "transition_energies", "velocity_start", "density_start", "spectrum_exact", "eig_spectrum",
    "haydock", "continued_fraction", "haydock_spectrum", "lowest_exciton",
    "binding_energy", "grad_apply", "grad_WR_from_Wq", "grad_lowest", "grad_spectrum",
    "interpolate_W_matmul", "apply_H_rows_allpairs", "hamiltonian_rows", "grad_Wq_at", "grad_eps",
    "PAPER_OFFSETS", "PAPER_OFFSET_WEIGHTS", "offset_average",
    "lorentzian", "coupling_block", "apply_B_rows", "apply_rows_twosided", "build_B", "build_full", "full_bse_eig", "full_bse_amplitudes", "full_bse_spectrum",
]


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------
def kmesh(nk):
    """Gamma-centred mesh of fractional k (Sec. IV.A.3 uses Gamma-centred meshes)."""
    n1, n2, n3 = nk
    out = np.empty((n1 * n2 * n3, 3))
    i = 0
    for a in range(n1):
        for b in range(n2):
            for c in range(n3):
                out[i] = (a / n1, b / n2, c / n3)
                i += 1
    return out


def coarse_mesh(nc3):
    return kmesh(nc3)


def q_index(nk, ik, jk):
    """Mesh index of k_j - k_i (mod the mesh): the momentum transfer of the pair (k_i, k_j)."""
    n1, n2, n3 = nk
    a1, a2, a3 = ik // (n2 * n3), (ik // n3) % n2, ik % n3
    b1, b2, b3 = jk // (n2 * n3), (jk // n3) % n2, jk % n3
    return (((b1 - a1) % n1) * n2 + (b2 - a2) % n2) * n3 + (b3 - a3) % n3


def q_index_table(nk):
    Nk = int(np.prod(nk))
    return np.array([[q_index(nk, i, j) for j in range(Nk)] for i in range(Nk)], dtype=np.int64)


# ----------------------------------------------------------------------------
# dual-k-mesh interpolation of W (Sec. III.B)
# ----------------------------------------------------------------------------
def interpolate_W(W_R, R, w_R, q_frac):
    """W_munu(q) = sum_R w_R W_munu(R) exp(+2 pi i q.R)   (Sec. III.B, Eq. (W_LRI)).

    Direct discrete Fourier sum over the (weighted, possibly truncated)
    R set of the coarse Born-von-Karman supercell, evaluated at any list
    of fractional q.
    """
    W_R = np.asarray(W_R, dtype=np.complex128)
    q_frac = np.atleast_2d(np.asarray(q_frac, dtype=np.float64))
    out = np.zeros((len(q_frac),) + W_R.shape[1:], dtype=np.complex128)
    for iq, q in enumerate(q_frac):
        for r in range(len(R)):
            out[iq] += w_R[r] * np.exp(2j * np.pi * np.dot(q, R[r])) * W_R[r]
    return out


def coarse_to_R(W_qc, coarse, R):
    """W(R) = (1/N_c) sum_{q_c} W(q_c) exp(-2 pi i q_c.R): inverse transform of the coarse-mesh W (Sec. III.B)."""
    qc = coarse_mesh(coarse)
    Nc = len(qc)
    out = np.zeros((len(R),) + W_qc.shape[1:], dtype=np.complex128)
    for r in range(len(R)):
        for iq in range(Nc):
            out[r] += np.exp(-2j * np.pi * np.dot(qc[iq], R[r])) * W_qc[iq]
    return out / Nc


# ----------------------------------------------------------------------------
# LRI pair densities (Sec. III.A, definition of C-tilde)
# ----------------------------------------------------------------------------
def pair_density(psi, C, ki, bi, kj, bj):
    """M^mu_{ij}(k_i, k_j) = sum_st conj(c^{k_i}_{s i}) C^mu_{st} c^{k_j}_{t j}.

    This is the paper's C-tilde^mu_{i k_i, j k_j} for k-independent LRI
    coefficients.  Returns [n_aux][len(bi)][len(bj)].
    """
    a = psi[ki][list(bi)]          # [ni][nao]
    b = psi[kj][list(bj)]          # [nj][nao]
    Cb = np.matmul(C, b.T)         # [mu][s][j] = sum_t C^mu_st b_jt
    return np.matmul(a.conj()[None], Cb)   # [mu][i][j]


def lri_coeff_k(C_R, RC, k):
    """C^mu_st(k) = sum_R C^mu_st(R) exp(+2 pi i k.R): Fourier transform of the two-centre LRI
    coefficients over their single lattice vector (Sec. III.A).  Returns [n_aux][n_ao][n_ao]."""
    ph = np.exp(2j * np.pi * (np.asarray(RC, dtype=np.float64) @ np.asarray(k, dtype=np.float64)))
    return np.tensordot(ph, C_R, axes=(0, 0))


def pair_density_2c(psi, C_R, RC, ka, k_a, bi, kb, k_b, bj):
    """M^mu_{ij}(k_a, k_b) = C-tilde^mu_{i k_a, j k_b}
         = sum_st conj(c^{k_a}_{s i}) c^{k_b}_{t j} [C^mu_st(k_b) + C^mu_ts(-k_a)]
    with the k-dependent two-centre coefficients of Sec. III.A (the Bloch-summed AO product expanded
    over the ABFs of both centres).  ka, kb are the psi indices, k_a, k_b the fractional k of those
    bands.  Returns [n_aux][len(bi)][len(bj)]."""
    Ceff = lri_coeff_k(C_R, RC, k_b) + np.transpose(lri_coeff_k(C_R, RC, -np.asarray(k_a)), (0, 2, 1))
    a = psi[ka][list(bi)]
    b = psi[kb][list(bj)]
    return np.matmul(a.conj()[None], np.matmul(Ceff, b.T))


def _pairs(prob, ka, bi, kb, bj):
    """The pair densities M^mu_{ij}(k_a, k_b) of a problem: k-independent C (pair_density) or two-centre
    C(R) (pair_density_2c, each band at the k of its band set)."""
    if getattr(prob, "C_R", None) is None:
        return pair_density(prob.psi, prob.C, ka, bi, kb, bj)
    kv, kc = prob.band_k()
    k_a = (kv if bi[0] < prob.nv else kc)[ka]
    k_b = (kv if bj[0] < prob.nv else kc)[kb]
    return pair_density_2c(prob.psi, prob.C_R, prob.RC, ka, k_a, bi, kb, k_b, bj)


def _bands(prob):
    return list(range(prob.nv)), list(range(prob.nv, prob.nv + prob.nc))


def hamiltonian_block(prob, W_q, alpha, k, kp, cache=None):
    """Block A[(k, c, v), (k', c', v')] of the TDA Hamiltonian (Eq. (Hamiltonian)).

    diagonal : (E^GW_{c k} - E^GW_{v k}) delta
    exchange : + alpha (c k*, v k | V | v' k'*, c' k')
             = + (alpha/N_k) sum_munu M^mu_{cv}(k,k) Vbar_munu M^nu_{v'c'}(k',k')
    direct   : - (v' k'*, v k | W | c k*, c' k')
             = - (1/N_k) sum_munu M^mu_{v'v}(k',k) W_munu(k'-k) M^nu_{cc'}(k,k')
    (kernel integrals of Eq. (W_LRI) and the exchange line below it,
    with a = c, i = v, k1 = k, b = c', j = v', k2 = k').
    Returned as [nc*nv][nc*nv] with row (c, v) and column (c', v').
    """
    val, con = _bands(prob)
    Nk = prob.Nk
    nc, nv = prob.nc, prob.nv
    Mcv = _pairs(prob, k, con, k, val)        # [mu][c][v]
    Mvc = _pairs(prob, kp, val, kp, con)      # [nu][v'][c']
    Mvv = _pairs(prob, kp, val, k, val)       # [mu][v'][v]
    Mcc = _pairs(prob, k, con, kp, con)       # [nu][c][c']
    Wq = W_q[q_index(prob.nk, k, kp)]
    # exchange: sum_mu sum_nu Mcv[mu,c,v] Vbar[mu,nu] Mvc[nu,v',c']
    t1 = np.einsum("mcv,mn->ncv", Mcv, prob.Vbar)
    Xb = (alpha / Nk) * np.einsum("ncv,npd->cvdp", t1, Mvc)
    # direct: sum_mu sum_nu Mvv[mu,v',v] W[mu,nu] Mcc[nu,c,c']
    t2 = np.einsum("mpv,mn->npv", Mvv, Wq)
    Db = -(1.0 / Nk) * np.einsum("npv,ncd->cvdp", t2, Mcc)
    blk = (Xb + Db).reshape(nc * nv, nc * nv)
    if k == kp:
        blk = blk + np.diag(transition_energies(prob)[k])
    return blk


def transition_energies(prob, eps=None):
    """(E_{c k} - E_{v k}) per k as [Nk][nc*nv] with (c, v) order (diagonal of Eq. (Hamiltonian))."""
    e = prob.eps_qp if eps is None else eps
    nv, nc = prob.nv, prob.nc
    out = np.empty((len(e), nc * nv))
    for k in range(len(e)):
        for c in range(nc):
            for v in range(nv):
                out[k, c * nv + v] = e[k, nv + c] - e[k, v]
    return out


def build_H(prob, W_q, alpha=None):
    """Explicit TDA Hamiltonian A [N][N] (Eq. (Hamiltonian), TDA as in Sec. II.C)."""
    alpha = prob.alpha if alpha is None else alpha
    Nk, nt = prob.Nk, prob.nc * prob.nv
    H = np.zeros((Nk * nt, Nk * nt), dtype=np.complex128)
    for k in range(Nk):
        for kp in range(Nk):
            H[k * nt:(k + 1) * nt, kp * nt:(kp + 1) * nt] = hamiltonian_block(prob, W_q, alpha, k, kp)
    return H


def coupling_block(prob, W_q, alpha, k, kp):
    """Block B[(k, c, v), (k', c', v')] of the coupling block of Eq. (Hamiltonian).

    exchange : + alpha (c k*, v k | V | c' k'*, v' k')
             = + (alpha/N_k) sum_munu M^mu_{cv}(k,k) Vbar_munu M^nu_{c'v'}(k',k')
    direct   : - (c' k'*, v k | W | c k*, v' k')
             = - (1/N_k) sum_munu M^mu_{c'v}(k',k) W_munu(k'-k) M^nu_{cv'}(k,k')
    (a = c, i = v, k1 = k, b = c', j = v', k2 = k'; the first density of the direct integral
    carries k' -> k as in the resonant block, hence the same W(k' - k)).
    Returned as [nc*nv][nc*nv] with row (c, v) and column (c', v').
    """
    val, con = _bands(prob)
    nc, nv = prob.nc, prob.nv
    Mcv = _pairs(prob, k, con, k, val)        # [mu][c][v]
    Mcv2 = _pairs(prob, kp, con, kp, val)     # [nu][c'][v']
    Mcpv = _pairs(prob, kp, con, k, val)      # [mu][c'][v]
    Mcvp = _pairs(prob, k, con, kp, val)      # [nu][c][v']
    Wq = W_q[q_index(prob.nk, k, kp)]
    Xb = (alpha / prob.Nk) * np.einsum("mcv,mn,ndp->cvdp", Mcv, prob.Vbar, Mcv2)
    Db = -(1.0 / prob.Nk) * np.einsum("mdv,mn,ncp->cvdp", Mcpv, Wq, Mcvp)
    return (Xb + Db).reshape(nc * nv, nc * nv)


def apply_B_rows(prob, W_q, X, rows, alpha=None):
    """Rows k in `rows` of B X, each row block of the coupling block built by coupling_block and
    multiplied by X.  Returns [len(rows)*nc*nv][nb]."""
    alpha = prob.alpha if alpha is None else alpha
    nt = prob.nc * prob.nv
    X = np.asarray(X).reshape(prob.Nk * nt, -1)
    out = np.zeros((len(rows) * nt, X.shape[1]), dtype=np.complex128)
    for i, k in enumerate(rows):
        for kp in range(prob.Nk):
            out[i * nt:(i + 1) * nt] += coupling_block(prob, W_q, alpha, k, kp) @ X[kp * nt:(kp + 1) * nt]
    return out


def _F_sets(prob):
    """F[k][mu][s][n] = sum_t C^mu_st(k_n) c^k_{tn} for the valence and the conduction bands, with which
    every pair density is M^mu_ij(k_a, k_b) = sum_s conj(c^{k_a}_{si}) F[k_b][mu][s][j]
                                           + sum_t conj(F[k_a][mu][t][i]) c^{k_b}_{tj}   (two-centre C(R))
    or the first term alone (k-independent C).  The second term is sum_st conj(c_si) c_tj C^mu_ts(-k_a) for
    real C(R) (C^mu(-k) = conj C^mu(k)).  Returns (Fv, Fc, two_sided)."""
    pv, pc = _psi_sets(prob)
    if getattr(prob, "C_R", None) is None:
        Fv = np.transpose(np.tensordot(prob.C, pv, axes=([2], [2])), (2, 0, 1, 3))        # [k][mu][s][v]
        Fc = np.transpose(np.tensordot(prob.C, pc, axes=([2], [2])), (2, 0, 1, 3))
        return Fv, Fc, False
    if np.iscomplexobj(prob.C_R):
        raise ValueError("the row-at-a-time two-centre form takes real C(R)")
    kv, kc = prob.band_k()
    RC = np.asarray(prob.RC, dtype=np.float64)
    out = []
    for psi_n, kn in ((pv, kv), (pc, kc)):
        F = np.zeros((prob.Nk, prob.n_aux, prob.n_ao, psi_n.shape[1]), dtype=np.complex128)
        for r in range(len(RC)):
            ph = np.exp(2j * np.pi * (kn @ RC[r]))                                          # [k]
            G = np.tensordot(prob.C_R[r], psi_n, axes=([2], [2]))                           # [mu][s][k][n]
            F += ph[:, None, None, None] * np.transpose(G, (2, 0, 1, 3))
        out.append(F)
    return out[0], out[1], True


def _pairs_rows(pa, Fa, ka, pb, Fb, kb, two):
    """M^mu_ij(k_a, k_b) for the pairs (ka[x], kb[x]) at once from psi sets and F sets: [x][mu][i][j]."""
    M = np.einsum("xis,xmsj->xmij", pa[ka].conj(), Fb[kb], optimize=True)
    if two:
        M = M + np.einsum("xmti,xjt->xmij", Fa[ka].conj(), pb[kb], optimize=True)
    return M


def apply_rows_twosided(prob, W_q, X, rows, block="A", alpha=None, chunk=64):
    """Rows k in `rows` of A X (block "A", Eq. (Hamiltonian)) or of B X (block "B", coupling block), every
    k' of a row at once, for k-independent or real two-centre coefficients (pair densities from _F_sets).
    The same sums as hamiltonian_block / coupling_block in another evaluation order.  [len(rows)*nt][nb]."""
    alpha = prob.alpha if alpha is None else alpha
    nv, nc, Nk, na = prob.nv, prob.nc, prob.Nk, prob.n_aux
    nt = nc * nv
    pv, pc = _psi_sets(prob)
    Fv, Fc, two = _F_sets(prob)
    X = np.asarray(X).reshape(Nk, nt, -1)
    nb = X.shape[2]
    allk = np.arange(Nk)
    rho = _pairs_rows(pc, Fc, allk, pv, Fv, allk, two)                     # [k][mu][c][v] = M^mu_cv(k,k)
    Xr = X.reshape(Nk, nc, nv, nb)
    # exchange: t[nu][b] = sum_k' sum_{c'v'} M^nu_{v'c'}(k',k') X  (A) or M^nu_{c'v'}(k',k') X  (B)
    if block == "A":
        Mvc = _pairs_rows(pv, Fv, allk, pc, Fc, allk, two)                 # [k][nu][v'][c'] = M^nu_v'c'(k,k)
        t = np.einsum("knvc,kcvb->nb", Mvc, Xr, optimize=True)
    else:
        t = np.einsum("kncv,kcvb->nb", rho, Xr, optimize=True)
    u = prob.Vbar @ t
    qtab = np.array([[q_index(prob.nk, k, kp) for kp in range(Nk)] for k in rows])
    eps_t = transition_energies(prob)
    out = np.zeros((len(rows), nt, nb), dtype=np.complex128)
    for i, k in enumerate(rows):
        out[i] += (alpha / Nk) * np.einsum("mcv,mb->cvb", rho[k], u).reshape(nt, nb)
        if block == "A":
            out[i] += eps_t[k][:, None] * X[k]
        for k0 in range(0, Nk, chunk):
            ks = np.arange(k0, min(Nk, k0 + chunk))
            K = len(ks)
            kk = np.full(K, k)
            W = W_q[qtab[i, ks]]                                              # [K][mu][nu]
            if block == "A":
                L = _pairs_rows(pv, Fv, ks, pv, Fv, kk, two)                  # [K][mu][v'][v] = M_v'v(k',k)
                Rt = _pairs_rows(pc, Fc, kk, pc, Fc, ks, two)                 # [K][nu][c][c'] = M_cc'(k,k')
                D = -(1.0 / Nk) * np.einsum("xmpv,xmn,xncd->xcvdp", L, W, Rt, optimize=True)   # [(c v)][(c' v')]
            else:
                L = _pairs_rows(pc, Fc, ks, pv, Fv, kk, two)                  # [K][mu][c'][v] = M_c'v(k',k)
                Rt = _pairs_rows(pc, Fc, kk, pv, Fv, ks, two)                 # [K][nu][c][v'] = M_cv'(k,k')
                D = -(1.0 / Nk) * np.einsum("xmdv,xmn,xncp->xcvdp", L, W, Rt, optimize=True)
            out[i] += np.einsum("xcvdp,xdpb->cvb", D, Xr[ks], optimize=True).reshape(nt, nb)
    return out.reshape(len(rows) * nt, nb)


def build_B(prob, W_q, alpha=None):
    """Explicit coupling block B [N][N] of Eq. (Hamiltonian)."""
    alpha = prob.alpha if alpha is None else alpha
    Nk, nt = prob.Nk, prob.nc * prob.nv
    B = np.zeros((Nk * nt, Nk * nt), dtype=np.complex128)
    for k in range(Nk):
        for kp in range(Nk):
            B[k * nt:(k + 1) * nt, kp * nt:(kp + 1) * nt] = coupling_block(prob, W_q, alpha, k, kp)
    return B


def build_full(prob, W_q, alpha=None):
    """The full BSE Hamiltonian [[A, B], [-B*, -A*]] [2N][2N] (matrix form above Eq. (Hamiltonian))."""
    A = build_H(prob, W_q, alpha)
    B = build_B(prob, W_q, alpha)
    return np.block([[A, B], [-B.conj(), -A.conj()]])


def full_bse_eig(A, B):
    """Positive eigenvalues Omega_S (ascending) of [[A, B], [-B*, -A*]] with right eigenvectors (X, Y)
    normalised as X^H X - Y^H Y = 1 (the convention of Eqs. (right)/(left)).

    Paired formulation: with J = diag(I, -I) the Hamiltonian is J M, M = [[A, B], [B*, A*]] Hermitian
    and (for a stable ground state) positive definite, so H z = Omega z is the Hermitian-definite
    problem J z = (1/Omega) M z; its M-orthonormal solutions with 1/Omega > 0 are the positive branch,
    rescaled so that z^H J z = 1.  Returns Omega [N], X [N][N], Y [N][N] (column S)."""
    import scipy.linalg
    N = A.shape[0]
    M = np.block([[A, B], [B.conj(), A.conj()]])
    J = np.diag(np.r_[np.ones(N), -np.ones(N)]).astype(np.complex128)
    lam, Z = scipy.linalg.eigh(J, M)          # J z = lam M z, z^H M z = 1
    pos = lam > 0
    Om = 1.0 / lam[pos]
    Z = Z[:, pos] * np.sqrt(Om)[None, :]      # z^H J z = lam z^H M z = 1/Omega -> 1
    order = np.argsort(Om)
    Om, Z = Om[order], Z[:, order]
    return Om, Z[:N], Z[N:]


def full_bse_amplitudes(prob, pol, X, Y):
    """Oscillator amplitudes of Eq. (full_BSE_epsilon2): for each exciton S and polarisation e
    a_S = sum_{cvk} [e.<v k|v|c k> / (E_ck - E_vk)] X_{cvk} + [e.<c k|v|v k> / (E_vk - E_ck)] Y_{cvk}
    with <v|v|c> = conj <c|v|v> and Kohn-Sham energies.  Returns [n_S][n_pol]."""
    pol = np.atleast_2d(pol)
    nv, nc = prob.nv, prob.nc
    out = np.zeros((X.shape[1], len(pol)), dtype=np.complex128)
    for b, e in enumerate(pol):
        for k in range(prob.Nk):
            for c in range(nc):
                for v in range(nv):
                    I = (k * nc + c) * nv + v
                    d = prob.eps_ks[k, nv + c] - prob.eps_ks[k, v]
                    m = sum(e[a] * prob.vel[a, k, c, v] for a in range(3))
                    out[:, b] += np.conj(m) / d * X[I] + m / (-d) * Y[I]
    return out


def full_bse_spectrum(prob, pol, Omega, X, Y, omega, eta):
    """S_e(omega) = (1/N_k) sum_S |a_S|^2 L_eta(omega - Omega_S) over the positive solutions
    (Eq. (full_BSE_epsilon2) without 4 pi^2/(3V)).  Returns [n_pol][n_omega]."""
    amp = np.abs(full_bse_amplitudes(prob, pol, X, Y)) ** 2
    L = lorentzian(np.asarray(omega)[None, :] - np.asarray(Omega)[:, None], eta)
    return (amp.T @ L) / prob.Nk


def apply_H_rows(prob, W_q, X, rows, alpha=None):
    """Rows k in `rows` of H X, each row block built from Eq. (Hamiltonian) and multiplied by X.

    Returns [len(rows)*nc*nv][nb].  Used where the full H does not fit.
    """
    alpha = prob.alpha if alpha is None else alpha
    nt = prob.nc * prob.nv
    X = np.asarray(X).reshape(prob.Nk * nt, -1)
    out = np.zeros((len(rows) * nt, X.shape[1]), dtype=np.complex128)
    for i, k in enumerate(rows):
        for kp in range(prob.Nk):
            out[i * nt:(i + 1) * nt] += hamiltonian_block(prob, W_q, alpha, k, kp) @ X[kp * nt:(kp + 1) * nt]
    return out


def apply_H(prob, W_q, X, alpha=None):
    return apply_H_rows(prob, W_q, X, list(range(prob.Nk)), alpha)


# ----------------------------------------------------------------------------
# spectrum (Eq. (abs_vel)) and lowest exciton (E_B, Sec. IV.B.3)
# ----------------------------------------------------------------------------
def velocity_start(prob, pol):
    """p_{cvk} = e.<c k| v |v k> / (E^KS_{ck} - E^KS_{vk})  for each polarisation e (rows of pol).

    The velocity-form oscillator strength of Eq. (abs_vel): for an exciton
    X^S the amplitude is |sum_I conj(p_I) X^S_I|^2.  Returns [N][n_pol].
    """
    pol = np.atleast_2d(pol)
    nv, nc = prob.nv, prob.nc
    out = np.zeros((prob.N, len(pol)), dtype=np.complex128)
    for b, e in enumerate(pol):
        for k in range(prob.Nk):
            for c in range(nc):
                for v in range(nv):
                    d = prob.eps_ks[k, nv + c] - prob.eps_ks[k, v]
                    amp = sum(e[a] * prob.vel[a, k, c, v] for a in range(3))
                    out[(k * nc + c) * nv + v, b] = amp / d
    return out


def density_start(prob):
    """p_{cvk}(Q) = <c k+Q| e^{iQ.r} |v k> = <u_c^{k+Q}|u_v^k>: the transition density of a finite exciton
    momentum Q, the matrix element the long-wavelength appendix writes as <u_i^k|u_a^{k+q}> (here
    conjugated, so that the amplitude of an exciton X^S is |sum_I conj(p_I) X^S_I|^2 as for the velocity
    form).  With the NAO Bloch sums orthonormal and each orbital's factor e^{iQ.(r - R)} taken at its centre,
    <u_c^{k+Q}|u_v^k> = sum_s conj(c^{k+Q}_{s c}) c^k_{s v}; the conduction bands of a finite-momentum
    problem are those at k + Q.  Its Q -> 0 limit is Q . <c|v|v>/(E_c - E_v), the velocity form of
    Eq. (abs_vel) along Q (the perturbation expansion of the same appendix).  Returns [N][1]."""
    nv, nc = prob.nv, prob.nc
    out = np.zeros((prob.N, 1), dtype=np.complex128)
    for k in range(prob.Nk):
        for c in range(nc):
            for v in range(nv):
                out[(k * nc + c) * nv + v, 0] = np.vdot(prob.psi[k, nv + c], prob.psi[k, v])
    return out


def lorentzian(x, eta):
    """L_eta(x) = (eta/pi) / (x^2 + eta^2): eta is the half width at half maximum."""
    return (eta / np.pi) / (x * x + eta * eta)


def spectrum_exact(Omega, Z, P, omega, eta, Nk):
    """S_e(omega) = (1/N_k) sum_S |<X^S|p_e>|^2 L_eta(omega - Omega_S) (Eq. (abs_vel) without 4 pi^2/(3V)).

    Omega [n_S], Z [N][n_S] eigenvectors, P [N][n_pol]; returns [n_pol][n_omega].
    """
    amp = np.abs(Z.conj().T @ P) ** 2      # [S][pol]
    L = lorentzian(np.asarray(omega)[None, :] - np.asarray(Omega)[:, None], eta)   # [S][w]
    return (amp.T @ L) / Nk


def eig_spectrum(H, P, omega, eta, Nk):
    Om, Z = np.linalg.eigh(H)
    return spectrum_exact(Om, Z, P, omega, eta, Nk), Om, Z


def lowest_exciton(H):
    Om, Z = np.linalg.eigh(H)
    return Om[0], Z[:, 0]


def binding_energy(prob, Omega1):
    """E_B = min_k [E_{c1 k} - E_{v_top k}] - Omega_1 (Sec. IV.B.3: the smallest direct quasiparticle gap over the mesh minus the lowest excitation)."""
    return (prob.eps_qp[:, prob.nv] - prob.eps_qp[:, prob.nv - 1]).min() - Omega1


# ----------------------------------------------------------------------------
# k-offset averaging (Sec. IV.A, k-point convergence; the averaging scheme of Sander et al. 2015)
# ----------------------------------------------------------------------------
# The four classes of a 3x3x3 grid of mesh offsets that the paper uses, in units of the dense-mesh spacing,
# with their weights (the class sizes over 27).
PAPER_OFFSETS = ((0.0, 0.0, 0.0), (1.0 / 3, 0.0, 0.0), (1.0 / 3, 1.0 / 3, 0.0), (2.0 / 3, 1.0 / 3, 0.0))
PAPER_OFFSET_WEIGHTS = (1.0 / 27, 8.0 / 27, 6.0 / 27, 12.0 / 27)


def offset_average(spectra, weights):
    """Offset-averaged spectrum sum_j w_j S_j, S_j computed independently on the dense mesh shifted by the
    j-th offset (same W(q): q = k' - k does not move when k and k' shift together)."""
    out = np.zeros_like(np.asarray(spectra[0], dtype=np.float64))
    for S, w in zip(spectra, weights):
        out = out + w * np.asarray(S, dtype=np.float64)
    return out


# ----------------------------------------------------------------------------
# Haydock recurrence (not in the paper; Haydock-Heine-Kelly, Benedict-Shirley)
# ----------------------------------------------------------------------------
def haydock(apply, p, m, tol=1e-12):
    """Lanczos tridiagonalisation of a Hermitian operator from start vector p.

    b_0 = |p|, q_1 = p / b_0, q_0 = 0.  For j = 1..m:
      w = H q_j;  a_j = Re q_j^H w;  w -= a_j q_j + b_{j-1} q_{j-1};
      full re-orthogonalisation against q_1..q_j, done twice (classical Gram-Schmidt);
      b_j = |w|;  stop (breakdown) if b_j <= tol * s_j;  q_{j+1} = w / b_j,
    s_j = max(|a_1|, .., |a_j|, b_1, .., b_{j-1}): the largest recurrence coefficient so far.  b_j has the
    units of H (the q_j are unit vectors), so the test compares it with H's own scale as the chain has seen
    it; b_0 = |p| carries the start vector's scale and does not enter.
    Returns a [m] (a_1..a_m), b [m+1] (b_0..b_m), steps done, basis [steps][N].
    """
    p = np.asarray(p, dtype=np.complex128)
    b0 = np.linalg.norm(p)
    a = np.zeros(m)
    b = np.zeros(m + 1)
    b[0] = b0
    Q = [p / b0]
    qprev = np.zeros_like(p)
    steps = m
    for j in range(1, m + 1):
        qj = Q[-1]
        w = apply(qj)
        a[j - 1] = np.real(np.vdot(qj, w))
        w = w - a[j - 1] * qj - (b[j - 1] if j > 1 else 0.0) * qprev
        Qm = np.array(Q)
        for _ in range(2):
            w = w - Qm.T @ (Qm.conj() @ w)
        b[j] = np.linalg.norm(w)
        scale = max(np.abs(a[:j]).max(), b[1:j].max(initial=0.0))
        if b[j] <= tol * scale:
            steps = j
            break
        qprev = qj
        if j < m:
            Q.append(w / b[j])
    return a, b, steps, np.array(Q[:steps])


def continued_fraction(a, b, steps, omega, eta, Nk):
    """S(omega) = -(1/(pi N_k)) Im f(omega + i eta),
    f(z) = b_0^2 / (z - a_1 - b_1^2 / (z - a_2 - ... - b_{m-1}^2 / (z - a_m))), no terminator.
    """
    z = np.asarray(omega, dtype=np.float64) + 1j * eta
    g = z - a[steps - 1]
    for j in range(steps - 1, 0, -1):
        g = z - a[j - 1] - b[j] ** 2 / g
    f = b[0] ** 2 / g
    return -np.imag(f) / (np.pi * Nk)


def haydock_spectrum(apply, P, m, omega, eta, Nk, tol=1e-12):
    """Independent chains for the columns of P; returns S [n_pol][n_omega], a, b, steps."""
    S, A, B, st = [], [], [], []
    for col in range(P.shape[1]):
        a, b, s, _ = haydock(apply, P[:, col], m, tol)
        S.append(continued_fraction(a, b, s, omega, eta, Nk))
        A.append(a)
        B.append(b)
        st.append(s)
    return np.array(S), np.array(A), np.array(B), np.array(st)


# ----------------------------------------------------------------------------
# gradients (PyTorch convention: dL = Re sum conj(g) d theta)
# ----------------------------------------------------------------------------
def grad_apply(prob, W_q, Ybar, X, alpha=None):
    """Gradients of L = Re sum_{I,b} conj(Ybar_Ib) (H X)_Ib.

    g_eps[k][v]   = -Re sum_{c,b} conj(Ybar_{cvk,b}) X_{cvk,b}
    g_eps[k][nv+c]=  Re sum_{v,b} conj(Ybar_{cvk,b}) X_{cvk,b}
    g_Wq[q]_munu  = -(1/N_k) sum_{k, k' = k+q} sum_b sum_{cvc'v'}
                     Ybar_{cvk,b} conj(M^mu_{v'v}(k',k) M^nu_{cc'}(k,k') X_{c'v'k',b})
    (derivative of the direct term of Eq. (Hamiltonian) through Eq. (W_LRI)).
    """
    nv, nc, Nk = prob.nv, prob.nc, prob.Nk
    nt = nc * nv
    val, con = _bands(prob)
    Ybar = np.asarray(Ybar).reshape(prob.N, -1)
    X = np.asarray(X).reshape(prob.N, -1)
    g_eps = np.zeros((Nk, nv + nc))
    for k in range(Nk):
        for c in range(nc):
            for v in range(nv):
                I = (k * nc + c) * nv + v
                s = np.real(np.vdot(Ybar[I], X[I]))
                g_eps[k, nv + c] += s
                g_eps[k, v] -= s
    g_Wq = np.zeros((Nk, prob.n_aux, prob.n_aux), dtype=np.complex128)
    for k in range(Nk):
        for kp in range(Nk):
            Mvv = _pairs(prob, kp, val, k, val)   # [mu][v'][v]
            Mcc = _pairs(prob, k, con, kp, con)   # [nu][c][c']
            G = Ybar[k * nt:(k + 1) * nt] @ X[kp * nt:(kp + 1) * nt].conj().T   # [(c v)][(c' v')]
            G = G.reshape(nc, nv, nc, nv)
            g_Wq[q_index(prob.nk, k, kp)] += -(1.0 / Nk) * np.einsum(
                "mpv,ncd,cvdp->mn", Mvv.conj(), Mcc.conj(), G)
    return g_eps, g_Wq


def grad_WR_from_Wq(g_Wq, R, w_R, q_frac):
    """g_WR[R] = w_R sum_q exp(-2 pi i q.R) g_Wq[q]: the adjoint of interpolate_W."""
    out = np.zeros((len(R),) + g_Wq.shape[1:], dtype=np.complex128)
    for r in range(len(R)):
        for iq, q in enumerate(q_frac):
            out[r] += np.exp(-2j * np.pi * np.dot(q, R[r])) * g_Wq[iq]
        out[r] *= w_R[r]
    return out


# ----------------------------------------------------------------------------
# the same definitions evaluated a whole row of pairs at a time (large meshes)
#
# These functions compute exactly the quantities of interpolate_W, apply_H_rows
# and grad_apply; the sums over k' (or k) are evaluated for all pairs of a row
# at once with matrix products instead of one (k, k') block after another, so
# that sampled rows stay affordable on a 16x16x16 mesh.  Nothing else changes:
# the same pair densities, the same W(k' - k), the same terms.
# ----------------------------------------------------------------------------
def interpolate_W_matmul(W_R, R, w_R, q_frac):
    """W_munu(q) = sum_R w_R W_munu(R) exp(+2 pi i q.R) (Sec. III.B) as one matrix product
    [n_q x n_R] x [n_R x n_aux^2] of the phase table with the stacked W(R)."""
    W_R = np.asarray(W_R, dtype=np.complex128)
    q_frac = np.atleast_2d(np.asarray(q_frac, dtype=np.float64))
    ph = np.asarray(w_R)[None, :] * np.exp(2j * np.pi * (q_frac @ np.asarray(R, dtype=np.float64).T))
    return (ph @ W_R.reshape(len(R), -1)).reshape((len(q_frac),) + W_R.shape[1:])


def _psi_sets(prob):
    val, con = _bands(prob)
    return prob.psi[:, val, :], prob.psi[:, con, :]      # [Nk][nv][nao], [Nk][nc][nao]


def apply_H_rows_allpairs(prob, W_q, X, rows, alpha=None, chunk=64):
    """Rows k in `rows` of H X (Eq. (Hamiltonian), kernel of Eq. (W_LRI)), as apply_H_rows.

    For a row k and every k' of a chunk at once:
      Mvv[k'][mu][v'][v] = M^mu_{v'v}(k', k),  Mcc[k'][nu][c][c'] = M^nu_{cc'}(k, k'),
      direct block  -(1/N_k) sum_munu Mvv[k'][mu][v'][v] W_munu(k' - k) Mcc[k'][nu][c][c'];
    the exchange sum over k' is taken inside, (alpha/N_k) M_cv(k,k) Vbar (sum_k' M_v'c'(k',k') X(k')).
    Returns [len(rows)*nc*nv][nb]."""
    alpha = prob.alpha if alpha is None else alpha
    nv, nc, Nk = prob.nv, prob.nc, prob.Nk
    nt = nc * nv
    val, con = _bands(prob)
    pv, pc = _psi_sets(prob)
    if getattr(prob, "C_R", None) is not None:
        raise NotImplementedError("row-at-a-time forms take k-independent LRI coefficients")
    C = prob.C
    X = np.asarray(X).reshape(Nk, nt, -1)           # [k][(c v)][b]
    nb = X.shape[2]
    Xr = X.reshape(Nk, nc, nv, nb)
    # exchange: t[nu][b] = sum_k' sum_{v'c'} M^nu_{v'c'}(k',k') X[(c' v' k')][b]
    t = np.zeros((prob.n_aux, nb), dtype=np.complex128)
    for k0 in range(0, Nk, chunk):
        ks = slice(k0, min(Nk, k0 + chunk))
        K = ks.stop - ks.start
        Cpc = np.tensordot(C, pc[ks], axes=([2], [2]))                            # [nu][s][K][c']  C^nu psi_c'(k')
        Cpc = np.transpose(Cpc, (2, 1, 0, 3)).reshape(K, prob.n_ao, -1)           # [K][s][(nu c')]
        Mvc = np.matmul(pv[ks].conj(), Cpc).reshape(K, nv, prob.n_aux, nc)        # [K][v'][nu][c']
        Mvc = np.transpose(Mvc, (0, 2, 1, 3))                                     # [K][nu][v'][c'] = M^nu_{v'c'}(k',k')
        # t[nu][b] += sum over (k', v', c') of Mvc[k'][nu][v'][c'] X[k'][c'][v'][b]
        t += np.transpose(Mvc, (1, 0, 2, 3)).reshape(prob.n_aux, -1) @ \
            np.transpose(Xr[ks], (0, 2, 1, 3)).reshape(-1, nb)
    u = prob.Vbar @ t                                                             # u[mu] = sum_nu Vbar[mu][nu] t[nu]
    qtab = np.array([[q_index(prob.nk, k, kp) for kp in range(Nk)] for k in rows])
    eps_t = transition_energies(prob)
    out = np.zeros((len(rows), nt, nb), dtype=np.complex128)
    for i, k in enumerate(rows):
        Mcv = pair_density(prob.psi, C, k, con, k, val)                           # [mu][c][v]
        out[i] += (alpha / Nk) * np.einsum("mcv,mb->cvb", Mcv, u).reshape(nt, nb)
        out[i] += eps_t[k][:, None] * X[k]
        Cv = np.matmul(C, pv[k].T)                                                # [mu][s][v]  (C^mu psi_v(k))
        Bc = np.matmul(pc[k].conj()[None], C)                                     # [nu][c][t]  (psi_c(k)^H C^nu)
        for k0 in range(0, Nk, chunk):
            ks = slice(k0, min(Nk, k0 + chunk))
            K = ks.stop - ks.start
            Mvv = np.tensordot(pv[ks].conj(), Cv, axes=([2], [1]))                # [K][v'][mu][v]
            Mvv = np.transpose(Mvv, (0, 2, 1, 3)).reshape(K, prob.n_aux, nv * nv)  # [K][mu][(v' v)]
            Mcc = np.tensordot(Bc, pc[ks], axes=([2], [2]))                       # [nu][c][K][c']
            Mcc = np.transpose(Mcc, (2, 1, 3, 0)).reshape(K, nc * nc, prob.n_aux)  # [K][(c c')][nu]
            W = W_q[qtab[i, ks]]                                                  # [K][mu][nu]
            t2 = np.matmul(np.transpose(W, (0, 2, 1)), Mvv)                       # [K][nu][(v' v)]
            D = -(1.0 / Nk) * np.matmul(Mcc, t2)                                  # [K][(c c')][(v' v)]
            D = np.transpose(D.reshape(K, nc, nc, nv, nv), (0, 1, 4, 2, 3)).reshape(K, nt, nt)  # [(c v)][(c' v')]
            out[i] += np.transpose(D, (1, 0, 2)).reshape(nt, K * nt) @ X[ks].reshape(K * nt, nb)   # sum_k' D X(k')
    return out.reshape(len(rows) * nt, nb)


def hamiltonian_rows(prob, W_q, rows, alpha=None, chunk=64):
    """Rows k in `rows` of the explicit TDA Hamiltonian A (Eq. (Hamiltonian), kernels of Eq. (W_LRI)),
    every column block k' of a row at once: the same blocks hamiltonian_block gives one (k, k') at a time.

      exchange  (alpha/N_k) sum_munu M^mu_{cv}(k,k) Vbar_munu M^nu_{v'c'}(k',k')
      direct   -(1/N_k)     sum_munu M^mu_{v'v}(k',k) W_munu(k'-k) M^nu_{cc'}(k,k')
      diagonal  (E_ck - E_vk) on the block k' = k.
    Returns [len(rows)*nc*nv][N] with row (k, c, v) and column (k', c', v')."""
    alpha = prob.alpha if alpha is None else alpha
    nv, nc, Nk, na = prob.nv, prob.nc, prob.Nk, prob.n_aux
    nt = nc * nv
    val, con = _bands(prob)
    pv, pc = _psi_sets(prob)
    if getattr(prob, "C_R", None) is not None:
        raise NotImplementedError("row-at-a-time forms take k-independent LRI coefficients")
    C = prob.C
    # M^nu_{v'c'}(k',k') for every k': [Nk][nu][v'][c']
    Mvc = np.empty((Nk, na, nv, nc), dtype=np.complex128)
    for k0 in range(0, Nk, chunk):
        ks = slice(k0, min(Nk, k0 + chunk))
        K = ks.stop - ks.start
        Cpc = np.tensordot(C, pc[ks], axes=([2], [2]))                            # [nu][s][K][c']
        Cpc = np.transpose(Cpc, (2, 1, 0, 3)).reshape(K, prob.n_ao, -1)           # [K][s][(nu c')]
        M = np.matmul(pv[ks].conj(), Cpc).reshape(K, nv, na, nc)                  # [K][v'][nu][c']
        Mvc[ks] = np.transpose(M, (0, 2, 1, 3))
    qtab = np.array([[q_index(prob.nk, k, kp) for kp in range(Nk)] for k in rows])
    eps_t = transition_energies(prob)
    out = np.zeros((len(rows), nt, Nk, nt), dtype=np.complex128)
    for i, k in enumerate(rows):
        Mcv = pair_density(prob.psi, C, k, con, k, val)                           # [mu][c][v]
        t1 = np.einsum("mcv,mn->ncv", Mcv, prob.Vbar)                             # [nu][c][v]
        Xb = (alpha / Nk) * np.einsum("ncv,knpd->cvkdp", t1, Mvc)                 # [c][v][k'][c'][v']
        out[i] += Xb.reshape(nt, Nk, nt)
        out[i, :, k, :] += np.diag(eps_t[k])
        Cv = np.matmul(C, pv[k].T)                                                # [mu][s][v]
        Bc = np.matmul(pc[k].conj()[None], C)                                     # [nu][c][t]
        for k0 in range(0, Nk, chunk):
            ks = slice(k0, min(Nk, k0 + chunk))
            K = ks.stop - ks.start
            Mvv = np.tensordot(pv[ks].conj(), Cv, axes=([2], [1]))                # [K][v'][mu][v]
            Mvv = np.transpose(Mvv, (0, 2, 1, 3)).reshape(K, na, nv * nv)         # [K][mu][(v' v)]
            Mcc = np.tensordot(Bc, pc[ks], axes=([2], [2]))                       # [nu][c][K][c']
            Mcc = np.transpose(Mcc, (2, 1, 3, 0)).reshape(K, nc * nc, na)         # [K][(c c')][nu]
            W = W_q[qtab[i, ks]]                                                  # [K][mu][nu]
            t2 = np.matmul(np.transpose(W, (0, 2, 1)), Mvv)                       # [K][nu][(v' v)]
            D = -(1.0 / Nk) * np.matmul(Mcc, t2)                                  # [K][(c c')][(v' v)]
            D = np.transpose(D.reshape(K, nc, nc, nv, nv), (1, 4, 0, 2, 3))       # [c][v][K][c'][v']
            out[i, :, ks, :] += D.reshape(nt, K, nt)
    return out.reshape(len(rows) * nt, Nk * nt)


def grad_Wq_at(prob, Ybar, X, qs, chunk=64):
    """g_Wq[q] of L = Re sum conj(Ybar) (H X) for the q in `qs` (the W part of grad_apply), every k of a q
    at once:  g_Wq[q]_munu = -(1/N_k) sum_{k, k' = k + q} sum_{cvc'v'} conj(M^mu_{v'v}(k',k)) conj(M^nu_{cc'}(k,k'))
    G[(c v)][(c' v')],  G = Ybar(k) X(k')^H.  Returns [len(qs)][n_aux][n_aux]."""
    nv, nc, Nk, na = prob.nv, prob.nc, prob.Nk, prob.n_aux
    nt = nc * nv
    pv, pc = _psi_sets(prob)
    if getattr(prob, "C_R", None) is not None:
        raise NotImplementedError("row-at-a-time forms take k-independent LRI coefficients")
    C = prob.C
    Ybar = np.asarray(Ybar).reshape(Nk, nt, -1)
    X = np.asarray(X).reshape(Nk, nt, -1)
    out = np.zeros((len(qs), na, na), dtype=np.complex128)
    n = np.array(prob.nk)
    kidx = np.array(np.unravel_index(np.arange(Nk), prob.nk)).T                  # [Nk][3] mesh coordinates
    for i, q in enumerate(qs):
        # k' = k + q on the mesh, i.e. q_index(k, k') = q
        kps = np.ravel_multi_index(tuple(((kidx + np.array(np.unravel_index(q, prob.nk))) % n).T), prob.nk)
        for k0 in range(0, Nk, chunk):
            ks = np.arange(k0, min(Nk, k0 + chunk))
            kp = kps[ks]
            K = len(ks)
            Cv = np.tensordot(C, pv[ks], axes=([2], [2]))                         # [mu][s][K][v]  C^mu psi_v(k)
            Cv = np.transpose(Cv, (2, 1, 0, 3)).reshape(K, prob.n_ao, -1)         # [K][s][(mu v)]
            Mvv = np.matmul(pv[kp].conj(), Cv).reshape(K, nv, na, nv)             # [K][v'][mu][v]
            Mvv = np.transpose(Mvv, (0, 2, 1, 3))                                 # [K][mu][v'][v]  M^mu_{v'v}(k',k)
            Cc = np.tensordot(C, pc[kp], axes=([2], [2]))                         # [nu][s][K][c']  C^nu psi_c'(k')
            Cc = np.transpose(Cc, (2, 1, 0, 3)).reshape(K, prob.n_ao, -1)         # [K][s][(nu c')]
            Mcc = np.matmul(pc[ks].conj(), Cc).reshape(K, nc, na, nc)             # [K][c][nu][c']
            Mcc = np.transpose(Mcc, (0, 2, 1, 3))                                 # [K][nu][c][c']  M^nu_{cc'}(k,k')
            G = np.matmul(Ybar[ks], np.transpose(X[kp].conj(), (0, 2, 1)))        # [K][(c v)][(c' v')]
            G = np.transpose(G.reshape(K, nc, nv, nc, nv), (0, 1, 3, 4, 2)).reshape(K, nc * nc, nv * nv)  # [(c c')][(v' v)]
            Z = np.matmul(Mcc.conj().reshape(K, na, nc * nc), G)                  # [K][nu][(v' v)]
            # sum over (k, v', v) of conj(Mvv[k][mu][(v' v)]) Z[k][nu][(v' v)]
            A = np.transpose(Mvv.conj().reshape(K, na, nv * nv), (1, 0, 2)).reshape(na, -1)
            Bz = np.transpose(Z, (1, 0, 2)).reshape(na, -1)
            out[i] += -(1.0 / Nk) * (A @ Bz.T)
    return out



def grad_eps(prob, Ybar, X):
    """The energy part of grad_apply alone: d/d eps of L = Re sum conj(Ybar) (H X) through the diagonal
    (E_ck - E_vk) of Eq. (Hamiltonian):  g[k][nv+c] = sum_v s_cvk,  g[k][v] = -sum_c s_cvk,
    s_cvk = Re sum_b conj(Ybar_{cvk,b}) X_{cvk,b}."""
    nv, nc, Nk = prob.nv, prob.nc, prob.Nk
    s = np.real(np.sum(np.conj(np.asarray(Ybar)) * np.asarray(X), axis=1)).reshape(Nk, nc, nv)
    g = np.zeros((Nk, nv + nc))
    g[:, nv:] = s.sum(axis=2)
    g[:, :nv] = -s.sum(axis=1)
    return g

def grad_lowest(prob, W_q, H=None, alpha=None):
    """dOmega_1/d(eps, W_q): Hellmann-Feynman, dOmega_1 = x^H dH x with x the lowest eigenvector."""
    if H is None:
        H = build_H(prob, W_q, alpha)
    Om, Z = np.linalg.eigh(H)
    x = Z[:, :1]
    g_eps, g_Wq = grad_apply(prob, W_q, x, x, alpha)
    return Om[0], g_eps, g_Wq


def grad_spectrum(prob, W_q, P, omega, eta, gamma, H=None, alpha=None):
    """Gradient of L = sum_{e, w} gamma[e][w] S_e(w) through the exact resolvent.

    dS_e(w) = -(1/(pi N_k)) Im( yt^H dH y ), y = (z - H)^-1 p_e, yt = (conj z - H)^-1 p_e,
    z = w + i eta, so L's gradient is grad_apply with the pairs
    Ybar = -(i gamma / (pi N_k)) yt and X = y, summed over (e, w).
    """
    if H is None:
        H = build_H(prob, W_q, alpha)
    Om, U = np.linalg.eigh(H)
    Nk = prob.Nk
    Ys, Xs = [], []
    for e in range(P.shape[1]):
        c = U.conj().T @ P[:, e]
        for iw, w in enumerate(omega):
            z = w + 1j * eta
            y = U @ (c / (z - Om))
            yt = U @ (c / (np.conj(z) - Om))
            Ys.append(-(1j * gamma[e][iw] / (np.pi * Nk)) * yt)
            Xs.append(y)
    return grad_apply(prob, W_q, np.array(Ys).T, np.array(Xs).T, alpha)
