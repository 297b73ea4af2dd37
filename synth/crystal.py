"""Synthetic crystals standing in for the paper's DFT + G0W0 front end.

The paper feeds its BSE step with Kohn-Sham/GW band energies and NAO
coefficients (Sec. II.A and the workflow of Sec. III.B), LRI coefficients
C^mu (Sec. III.A), the truncated bare Coulomb matrix (Sec. III.A) and the
static screened interaction W_munu(R) on a small Born-von-Karman R set
(Sec. III.B).  None of the real-material data ship with the paper, so
this module draws seeded synthetic stand-ins with the same shapes, band
counts and structure:

* bands: a random short-range tight-binding H(R) on a simple cubic lattice
  (a = 1, V = 1), hoppings to the 6 nearest cells, half filling, a
  scissor on the conduction bands standing in for E^GW vs E^KS;
* C^mu: random complex Gaussian matrices, made Hermitian (the k-independent
  form of the paper's two-centre relation for real ABFs), or (two_centre=True)
  real two-centre coefficients C^mu_st(R) on R = 0 and the six nearest cells,
  nonzero only when the auxiliary function mu sits on the atom of the first
  AO s (the support of the paper's LRI coefficients, Sec. III.A);
* Vbar: a real symmetric positive semi-definite matrix;
* W(R): generator "G1" (real PSD L L^T times exp(-|R|/1.5), as quoted for
  the benchmark workloads) or "G2" (real, W(-R) = W(R)^T but not
  symmetric, so that W(q) is complex Hermitian and W(q) != W(-q));
* velocity matrix elements <c k| dH/dk_alpha |v k> of the tight-binding
  model (the front end's dipoles; the BSE step divides them by the
  transition energy itself).

Energies are in eV, lengths in lattice units, k in fractional units with
phases exp(2 pi i k.R).  Nothing here evaluates the BSE method itself.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_BASE = 260705853

# Constants of the generators (frozen after calibration at the tiny
# workload so that the exciton kernel is a moderate perturbation of the
# transition energies).
DELTA_ONSITE = 4.0      # eV, on-site splitting between the two halves of the AOs
HOP_SCALE = 0.3         # eV, hopping amplitude t = HOP_SCALE / sqrt(n_ao)
GAP_TARGET = 2.0        # eV, min_k (e_c - e_v) after the scissor
DECAY_LEN = 1.5         # lattice units, W(R) ~ exp(-|R| / DECAY_LEN)
V_KERNEL = 0.3          # eV, target spectral norm of the exchange block (random-matrix estimate)
W_KERNEL = 0.4          # eV, target spectral norm of the direct block (random-matrix estimate)
TC_ATOMS = 2            # atoms per cell carrying the AOs and auxiliary functions of two-centre inputs
TC_NEIGHBOUR = 0.5      # amplitude of the nearest-cell two-centre coefficients relative to R = 0

CONFIGS = {
    # tiny: full diagonalisation + Haydock 200
    "mesh4_ao16": dict(cfg_id=0, coarse=(2, 2, 2), dense=(4, 4, 4), n_ao=16, nv=4, nc=4,
               n_aux=64, r_cut=None, nb=3, haydock_steps=200),
    # plain FP64 on the GPU: matrix-free apply on blocks of 8, Haydock 300
    "mesh8_ao64": dict(cfg_id=1, coarse=(4, 4, 4), dense=(8, 8, 8), n_ao=64, nv=4, nc=8,
               n_aux=256, r_cut=None, nb=8, haydock_steps=300),
    # precision form
    "mesh12_ao96": dict(cfg_id=2, coarse=(4, 4, 4), dense=(12, 12, 12), n_ao=96, nv=6, nc=10,
               n_aux=384, r_cut=None, nb=8, haydock_steps=300),
    # differentiation form
    "mesh8_ao64_grad": dict(cfg_id=3, coarse=(4, 4, 4), dense=(8, 8, 8), n_ao=64, nv=4, nc=8,
               n_aux=256, r_cut=None, nb=4, haydock_steps=300),
    # largest
    "mesh16_ao128": dict(cfg_id=4, coarse=(6, 6, 6), dense=(16, 16, 16), n_ao=128, nv=8, nc=8,
               n_aux=512, r_cut=3.0, nb=16, haydock_steps=100),
}


def dense_kmesh(nk, offset=(0.0, 0.0, 0.0)):
    """Mesh k = ((i1 + o1)/n1, (i2 + o2)/n2, (i3 + o3)/n3), index (i1*n2 + i2)*n3 + i3: Gamma-centred for
    a zero offset o, shifted by o mesh spacings otherwise."""
    n1, n2, n3 = nk
    o1, o2, o3 = (float(x) for x in offset)
    i1, i2, i3 = np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij")
    k = np.stack([(i1.ravel() + o1) / n1, (i2.ravel() + o2) / n2, (i3.ravel() + o3) / n3], axis=1)
    return k.astype(np.float64)


def ws_rset(coarse, r_cut: Optional[float] = None):
    """Wigner-Seitz style R set of the coarse Born-von-Karman supercell.

    Cube of integer vectors |R_i| <= N_i/2 (even N_i) or (N_i-1)/2 (odd).
    Points on a face (|R_i| = N_i/2) are shared between images, so each
    carries the weight prod_i (1/2 if on that face else 1); the weights
    of one class (R mod N) add to 1.  With r_cut, points with
    |R| > r_cut (Euclidean, lattice units) are dropped.
    """
    axes = []
    for n in coarse:
        h = n // 2
        axes.append(np.arange(-h, h + 1) if n % 2 == 0 else np.arange(-(n - 1) // 2, (n - 1) // 2 + 1))
    R = np.array([(a, b, c) for a in axes[0] for b in axes[1] for c in axes[2]], dtype=np.int32)
    w = np.ones(len(R))
    for i, n in enumerate(coarse):
        if n % 2 == 0:
            w = w * np.where(np.abs(R[:, i]) == n // 2, 0.5, 1.0)
    if r_cut is not None:
        keep = np.sqrt((R.astype(np.float64) ** 2).sum(1)) <= r_cut + 1e-12
        R, w = R[keep], w[keep]
    return np.ascontiguousarray(R), np.ascontiguousarray(w)


def polarisations(n):
    """First n polarisation vectors: x, y, z, (x+y), (y+z), (x+z) /sqrt2, (x+y+z)/sqrt3, then (x-y)/sqrt2."""
    s2, s3 = np.sqrt(0.5), np.sqrt(1.0 / 3.0)
    base = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (s2, s2, 0), (0, s2, s2), (s2, 0, s2),
            (s3, s3, s3), (s2, -s2, 0)]
    out = []
    for i in range(n):
        b = base[i % len(base)]
        out.append(b)
    return np.array(out, dtype=np.float64)


def _cn(rng, shape):
    """Complex normal CN(0, 1): real and imaginary parts N(0, 1/2)."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * np.sqrt(0.5)


@dataclass
class Problem:
    name: str
    nk: tuple
    coarse: tuple
    n_ao: int
    nv: int
    nc: int
    n_aux: int
    alpha: float
    eps_ks: np.ndarray      # f64 [Nk][nv+nc]  valence (ascending) then conduction (ascending)
    eps_qp: np.ndarray      # f64 [Nk][nv+nc]  eps_ks + scissor on the conduction bands
    psi: np.ndarray         # c128 [Nk][nv+nc][n_ao]  row n = coefficients c_{s n}^k
    vel: np.ndarray         # c128 [3][Nk][nc][nv]  <c k| dH/dk_alpha |v k>
    C: np.ndarray           # c128 [n_aux][n_ao][n_ao]  each Hermitian
    Vbar: np.ndarray        # c128 [n_aux][n_aux]  real symmetric PSD
    R: np.ndarray           # int32 [NR][3]
    w_R: np.ndarray         # f64 [NR]
    W_R: np.ndarray         # c128 [NR][n_aux][n_aux]  real entries
    H_R: dict = field(default_factory=dict)   # tight-binding hoppings {R tuple: [n_ao][n_ao]}
    wgen: str = "G1"
    seed: int = 0
    offset: tuple = (0.0, 0.0, 0.0)            # mesh offset in units of the dense-mesh spacing
    momentum: tuple = (0.0, 0.0, 0.0)          # exciton momentum Q in units of the dense-mesh spacing
    C_R: Optional[np.ndarray] = None           # f64 [NRC][n_aux][n_ao][n_ao] two-centre C^mu_st(R) (C is None then)
    RC: Optional[np.ndarray] = None            # int32 [NRC][3] the R of C_R

    @property
    def Nk(self):
        return int(np.prod(self.nk))

    @property
    def N(self):
        return self.Nk * self.nv * self.nc

    @property
    def kfrac(self):
        return dense_kmesh(self.nk, self.offset)

    def band_k(self):
        """(k of the valence bands, k of the conduction bands) per mesh point, fractional [Nk][3] each:
        the shifted mesh, and for the conduction bands that mesh moved by the exciton momentum."""
        shifted = tuple(o + m for o, m in zip(self.offset, self.momentum))
        return dense_kmesh(self.nk, self.offset), dense_kmesh(self.nk, shifted)


def _tb_hoppings(rng, n_ao):
    t = HOP_SCALE / np.sqrt(n_ao)
    h = n_ao // 2
    G0 = _cn(rng, (n_ao, n_ao))
    H0 = np.diag(np.r_[-0.5 * DELTA_ONSITE * np.ones(h), 0.5 * DELTA_ONSITE * np.ones(n_ao - h)]).astype(np.complex128)
    H0 = H0 + t * (G0 + G0.conj().T) / 2
    HR = {(0, 0, 0): H0}
    for ax in range(3):
        e = [0, 0, 0]
        e[ax] = 1
        G = t * _cn(rng, (n_ao, n_ao))
        HR[tuple(e)] = G
        HR[tuple(-x for x in e)] = G.conj().T
    return HR


def _bands(HR, kfrac, n_ao, nv, nc):
    Nk = len(kfrac)
    h = n_ao // 2
    sel = np.r_[np.arange(h - nv, h), np.arange(h, h + nc)]
    eps = np.empty((Nk, nv + nc))
    psi = np.empty((Nk, nv + nc, n_ao), dtype=np.complex128)
    vel = np.empty((3, Nk, nc, nv), dtype=np.complex128)
    for ik, k in enumerate(kfrac):
        Hk = np.zeros((n_ao, n_ao), dtype=np.complex128)
        dH = np.zeros((3, n_ao, n_ao), dtype=np.complex128)
        for R, M in HR.items():
            ph = np.exp(2j * np.pi * np.dot(k, R))
            Hk += M * ph
            for a in range(3):
                if R[a] != 0:
                    dH[a] += 1j * R[a] * M * ph
        Hk = 0.5 * (Hk + Hk.conj().T)
        e, U = np.linalg.eigh(Hk)
        U = U[:, sel]
        # deterministic gauge: largest component of each band real and positive
        idx = np.argmax(np.abs(U), axis=0)
        ph = U[idx, np.arange(U.shape[1])]
        U = U * (np.abs(ph) / ph)[None, :]
        eps[ik] = e[sel]
        psi[ik] = U.T
        Uv, Uc = U[:, :nv], U[:, nv:]
        for a in range(3):
            vel[a, ik] = Uc.conj().T @ dH[a] @ Uv
    return eps, psi, vel


def make_problem(cfg="mesh4_ao16", seed=0, wgen="G1", **over) -> Problem:
    """Draw the synthetic crystal of a named workload (or a dict), with overrides.

    Overrides: dense, coarse, n_ao, nv, nc, n_aux, r_cut, alpha, two_centre (real two-centre LRI
    coefficients C^mu_st(R) in C_R / RC instead of the k-independent Hermitian C, which is then None),
    momentum (finite exciton momentum Q:
    transitions (v k, c k+Q), i.e. the conduction bands of the band arrays taken at k + Q / n while the
    valence bands stay at k; the velocity elements are then zero, the optical start vectors being a
    Q = 0 notion), offset (the dense mesh shifted by
    offset mesh spacings: bands, start vectors and the velocity elements at the shifted k; C, Vbar, W and
    the quasiparticle scissor are those of the unshifted mesh, so the problems of several offsets share
    everything but the bands).
    Independent child streams (SeedSequence([SEED_BASE, cfg_id, seed]))
    feed the bands, C, Vbar and W so that changing one size leaves the
    other draws' structure intact.
    """
    if isinstance(cfg, str):
        name = cfg
        c = dict(CONFIGS[cfg])
    else:
        name = cfg.get("name", "custom")
        c = dict(cfg)
    c.update(over)
    cfg_id = int(c.get("cfg_id", 99))
    nk = tuple(int(x) for x in c["dense"])
    coarse = tuple(int(x) for x in c["coarse"])
    n_ao, nv, nc, n_aux = int(c["n_ao"]), int(c["nv"]), int(c["nc"]), int(c["n_aux"])
    if nv > n_ao // 2 or nc > n_ao - n_ao // 2:
        raise ValueError("band window exceeds the tight-binding model")
    alpha = float(c.get("alpha", 2.0))
    ss = np.random.SeedSequence([SEED_BASE, cfg_id, int(seed)])
    r_tb, r_c, r_v, r_w, r_2c = (np.random.default_rng(s) for s in ss.spawn(5))

    HR = _tb_hoppings(r_tb, n_ao)
    offset = tuple(float(x) for x in c.get("offset", (0.0, 0.0, 0.0)))
    kf = dense_kmesh(nk, offset)
    eps_ks, psi, vel = _bands(HR, kf, n_ao, nv, nc)
    e0 = eps_ks if offset == (0.0, 0.0, 0.0) else _bands(HR, dense_kmesh(nk), n_ao, nv, nc)[0]
    gap = (e0[:, nv] - e0[:, nv - 1]).min()
    momentum = tuple(float(x) for x in c.get("momentum", (0.0, 0.0, 0.0)))
    if momentum != (0.0, 0.0, 0.0):
        shifted = tuple(o + m for o, m in zip(offset, momentum))
        e_q, psi_q, _ = _bands(HR, dense_kmesh(nk, shifted), n_ao, nv, nc)
        eps_ks[:, nv:], psi[:, nv:] = e_q[:, nv:], psi_q[:, nv:]
        vel = np.zeros_like(vel)
    eps_qp = eps_ks.copy()
    eps_qp[:, nv:] += GAP_TARGET - gap

    sigma_c = 1.0 / np.sqrt(n_ao)
    G = _cn(r_c, (n_aux, n_ao, n_ao))
    C = sigma_c * 0.5 * (G + np.conj(np.transpose(G, (0, 2, 1))))
    C_R = RC = None
    if c.get("two_centre", False):
        C_R, RC = _two_centre(r_2c, n_ao, n_aux, sigma_c)
        C = None

    # Scales chosen so that the exchange and direct blocks have roughly
    # config-independent spectral norms (random-matrix estimates with
    # |M| ~ 1/sqrt(n_ao)); the values are conventions, not physics.
    Nk = int(np.prod(nk))
    Q = r_v.standard_normal((n_aux, n_aux))
    b_v = V_KERNEL * n_ao / (8.0 * nc * nv)
    Vbar = (b_v * (Q @ Q.T) / n_aux).astype(np.complex128)

    R, w_R = ws_rset(coarse, c.get("r_cut"))
    rn = np.sqrt((R.astype(np.float64) ** 2).sum(1))
    f_r = float((w_R * np.exp(-rn / DECAY_LEN)).sum())
    a_w = W_KERNEL * Nk * n_ao / (2.0 * np.sqrt(2.0 * Nk * nc * nv * n_aux) * f_r)
    if wgen == "G1":
        L = r_w.standard_normal((n_aux, n_aux))
        base = a_w * (L @ L.T) / n_aux
        W_R = (np.exp(-rn / DECAY_LEN)[:, None, None] * base[None]).astype(np.complex128)
    elif wgen == "G2":
        W_R = _w_g2(r_w, R, coarse, n_aux, a_w)
    else:
        raise ValueError(wgen)
    return Problem(name=name, nk=nk, coarse=coarse, n_ao=n_ao, nv=nv, nc=nc, n_aux=n_aux,
                   alpha=alpha, eps_ks=eps_ks, eps_qp=eps_qp, psi=psi, vel=vel, C=C,
                   Vbar=Vbar, R=R, w_R=w_R, W_R=W_R, H_R=HR, wgen=wgen, seed=seed, offset=offset,
                   momentum=momentum, C_R=C_R, RC=RC)


def _two_centre(rng, n_ao, n_aux, sigma_c):
    """Real C^mu_st(R) on R = 0 and the six nearest cells.

    AO s sits on atom s * TC_ATOMS // n_ao and auxiliary function mu on atom mu * TC_ATOMS // n_aux; a
    coefficient is nonzero only when mu sits on the atom of s.  Entries are N(0, a^2 d_R^2) with d_0 = 1,
    d_R = TC_NEIGHBOUR for the neighbours, and a chosen so that the mean square of an entry of
    C^mu_st(k1) + C^mu_ts(-k2) equals that of the k-independent draw (sigma_c^2 / 2).
    """
    RC = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)],
                  dtype=np.int32)
    d = np.r_[1.0, TC_NEIGHBOUR * np.ones(len(RC) - 1)]
    a = sigma_c * np.sqrt(TC_ATOMS / (4.0 * (d ** 2).sum()))
    atom_s = np.arange(n_ao) * TC_ATOMS // n_ao
    atom_mu = np.arange(n_aux) * TC_ATOMS // n_aux
    mask = (atom_mu[:, None] == atom_s[None, :]).astype(np.float64)          # [mu][s]
    C_R = rng.standard_normal((len(RC), n_aux, n_ao, n_ao)) * (a * d)[:, None, None, None]
    C_R *= mask[None, :, :, None]
    return np.ascontiguousarray(C_R), RC


def _w_g2(rng, R, coarse, n_aux, amp):
    """Real W(R) with W(-R) = W(R)^T, shared by all images of a class R mod N.

    Each class gets an independent real Gaussian matrix; the class of -R
    gets its transpose, and a class equal to its own negative gets the
    symmetric part.  Amplitude exp(-|R_min|/1.5) with R_min the shortest
    image of the class.
    """
    N = np.array(coarse)
    cls = [tuple(int(x) for x in np.mod(r, N)) for r in R]
    rn = np.sqrt((R.astype(np.float64) ** 2).sum(1))
    rmin = {}
    for cl, d in zip(cls, rn):
        rmin[cl] = min(rmin.get(cl, np.inf), d)
    mats = {}
    for cl in sorted(set(cls)):
        if cl in mats:
            continue
        neg = tuple(int(x) for x in np.mod(-np.array(cl), N))
        A = rng.standard_normal((n_aux, n_aux)) * amp * np.exp(-rmin[cl] / DECAY_LEN) / np.sqrt(n_aux)
        if neg == cl:
            mats[cl] = 0.5 * (A + A.T)
        else:
            mats[cl] = A
            mats[neg] = A.T
    return np.stack([mats[c] for c in cls]).astype(np.complex128)


def random_block(N, nb, seed=0, tag=0):
    """Complex Gaussian block X [N][nb], each column normalised to 1."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 1000 + int(tag), int(seed)]))
    X = _cn(rng, (N, nb))
    return X / np.linalg.norm(X, axis=0, keepdims=True)
