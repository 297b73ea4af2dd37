"""Writes the oracle's reference values for the two 8x8x8 workloads (FP64 on the CPU, oracle only).

Nothing here comes from the HIP path: the inputs are drawn by `synth` from their seeds, and every stored
number is computed by `oracle/` from them.  The GPU tests regenerate the same inputs from the same seeds
and compare their results with these values.

mesh8_ao64_spectrum.json   dense 8x8x8 mesh from coarse 4x4x4, N_ao 64, 4 + 8 bands, N_aux 256, generator
                           G1, seed 0 (BSE dim 16384): the oracle's own Haydock recurrence (Lanczos with CGS2,
                           300 steps, 8 polarisations) on the explicit A of Eq. (Hamiltonian), its
                           coefficients a, b (the spectrum of Eq. (abs_vel) follows from them by the continued
                           fraction), the four lowest eigenvalues of A from eigh, the binding energy of
                           Sec. IV.B.3, and the largest difference between the Haydock spectrum and the
                           eigh spectrum on the 2001-point grid.
mesh8_ao64_grad.json       the differentiation workload (same sizes, generator G2, seed 0): from eigh of A,
                           the lowest exciton energy and its exact gradients (Hellmann-Feynman) with respect to
                           the energies (every k) and to W(q) (sampled entries at a few q), and the exact
                           resolvent gradient of L = sum gamma S(omega) over 4 polarisations and 64
                           frequencies on [Omega_1 - 0.5, Omega_1 + 2.5] eV.

Usage: python tests/golden/make_mesh8_golden.py [spectrum] [grad] [spectrum-values]
Runs for about 30-60 minutes on 8 cores and needs about 20 GB of memory.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from synth import dense_kmesh, make_problem, polarisations  # noqa: E402

ETA = 0.1
# q of the sampled W(q) gradients: q = 0 (its own negative), a pair {q, -q} and a generic q
GRAD_Q = [0, 9, 503, 300]
N_ENTRIES = 256


def log(msg):
    print("[golden %s] %s" % (time.strftime("%H:%M:%S"), msg), flush=True)


def explicit_A(p, Wq):
    rows = []
    for k0 in range(0, p.Nk, 64):
        rows.append(O.hamiltonian_rows(p, Wq, list(range(k0, min(p.Nk, k0 + 64)))))
        log("A rows %d / %d" % (min(p.Nk, k0 + 64), p.Nk))
    H = np.vstack(rows)
    return H


def sampled_entries(g, seed):
    """A seeded set of (mu, nu) entries of each matrix g[i], with the largest modulus of each."""
    rng = np.random.default_rng(seed)
    na = g.shape[1]
    mu = rng.integers(0, na, N_ENTRIES)
    nu = rng.integers(0, na, N_ENTRIES)
    return {"mu": mu.tolist(), "nu": nu.tolist(),
            "re": [g[i][mu, nu].real.tolist() for i in range(len(g))],
            "im": [g[i][mu, nu].imag.tolist() for i in range(len(g))],
            "absmax": [float(np.abs(g[i]).max()) for i in range(len(g))]}


def spectrum_golden():
    cfg, seed, wgen, nb, m = "mesh8_ao64", 0, "G1", 8, 300
    p = make_problem(cfg, seed, wgen)
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))
    log("W(q) done")
    H = explicit_A(p, Wq)
    pol = polarisations(nb)
    P = O.velocity_start(p, pol)
    te = O.transition_energies(p)
    lo, hi, n_w = float(te.min() - 1.0), float(te.max() + 1.0), 2001
    w = np.linspace(lo, hi, n_w)
    S_h, a, b, st = O.haydock_spectrum(lambda x: H @ x, P, m, w, ETA, p.Nk)
    log("Haydock done")
    S_e, Om, _ = O.eig_spectrum(H, P, w, ETA, p.Nk)
    log("eigh done")
    gap = float(np.abs(S_h - S_e).max() / np.abs(S_e).max())
    out = {
        "_about": "Oracle values for the 8x8x8 / N_ao 64 / N_aux 256 workload (generator G1, seed 0), written by "
                  "tests/golden/make_mesh8_golden.py from oracle/ only.  Spectrum of Eq. (abs_vel) through the "
                  "oracle's Haydock recurrence on the explicit A of Eq. (Hamiltonian); binding energy of "
                  "Sec. IV.B.3.",
        "config": cfg, "seed": seed, "wgen": wgen, "nb": nb, "n_steps": m, "eta": ETA,
        "omega": {"lo": lo, "hi": hi, "n": n_w},
        "polarisations": pol.tolist(),
        "a": a.tolist(), "b": b.tolist(), "steps": st.tolist(), "S": S_h.tolist(),
        "haydock_vs_eigh_max_rel": gap,
        "omega_lowest": Om[:4].tolist(),
        "binding_energy": float(O.binding_energy(p, Om[0])),
    }
    with open(os.path.join(HERE, "mesh8_ao64_spectrum.json"), "w") as f:
        json.dump(out, f)
    log("spectrum golden written, Haydock vs eigh %.3e" % gap)


def spectrum_values():
    """Adds the spectrum S [nb][n_omega] (the continued fraction of the stored a, b) to an existing
    mesh8_ao64_spectrum.json, for readers that do not evaluate it themselves."""
    path = os.path.join(HERE, "mesh8_ao64_spectrum.json")
    g = json.load(open(path))
    Nk = int(np.prod(make_problem(g["config"], g["seed"], g["wgen"]).nk))
    w = np.linspace(g["omega"]["lo"], g["omega"]["hi"], g["omega"]["n"])
    g["S"] = [O.continued_fraction(np.array(g["a"][i]), np.array(g["b"][i]), g["steps"][i], w, g["eta"], Nk).tolist()
              for i in range(g["nb"])]
    with open(path, "w") as f:
        json.dump(g, f)
    log("spectrum values added")


def grad_golden():
    cfg, seed, wgen, nb = "mesh8_ao64_grad", 0, "G2", 4
    p = make_problem(cfg, seed, wgen)
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, dense_kmesh(p.nk))
    log("W(q) done")
    H = explicit_A(p, Wq)
    Om, U = np.linalg.eigh(H)
    del H
    log("eigh done")
    x = U[:, :1]
    ge_low = O.grad_eps(p, x, x)
    gq_low = O.grad_Wq_at(p, x, x, GRAD_Q)
    log("lowest-exciton gradients done")
    pol = polarisations(nb)
    P = O.velocity_start(p, pol)
    n_w = 64
    w = np.linspace(Om[0] - 0.5, Om[0] + 2.5, n_w)
    gamma = np.random.default_rng(np.random.SeedSequence([260705853, 3, 64])).standard_normal((nb, n_w))
    # exact resolvent: y = (z - A)^-1 p, yt = (conj z - A)^-1 p, dS = -(1/(pi Nk)) Im(yt^H dA y)
    c = U.conj().T @ P                                    # [S][pol]
    Ys, Xs = [], []
    S = np.zeros((nb, n_w))
    for e in range(nb):
        z = w + 1j * ETA
        Y = U @ (c[:, e][:, None] / (z[None, :] - Om[:, None]))           # [N][w]
        Yt = U @ (c[:, e][:, None] / (np.conj(z)[None, :] - Om[:, None]))
        S[e] = -np.imag(P[:, e].conj() @ Y) / (np.pi * p.Nk)
        Ys.append(-(1j * gamma[e][None, :] / (np.pi * p.Nk)) * Yt)
        Xs.append(Y)
    Ybar, X = np.hstack(Ys), np.hstack(Xs)
    ge_spec = O.grad_eps(p, Ybar, X)
    gq_spec = O.grad_Wq_at(p, Ybar, X, GRAD_Q)
    log("spectrum gradients done")
    S_ref = O.spectrum_exact(Om, U, P, w, ETA, p.Nk)
    out = {
        "_about": "Oracle values for the differentiation workload 8x8x8 / N_ao 64 / N_aux 256 (generator G2, "
                  "seed 0), written by tests/golden/make_mesh8_golden.py from oracle/ only: the lowest "
                  "eigenvalues of the explicit A of Eq. (Hamiltonian) (eigh), the Hellmann-Feynman gradient of "
                  "Omega_1 and the exact-resolvent gradient of L = sum gamma S(omega) (Eq. (abs_vel)) with "
                  "respect to eps (all) and W(q) (sampled entries at the q listed).",
        "config": cfg, "seed": seed, "wgen": wgen, "nb": nb, "eta": ETA,
        "omega_lowest": Om[:4].tolist(),
        "binding_energy": float(O.binding_energy(p, Om[0])),
        "grad_q": GRAD_Q,
        "lowest": {"g_eps": ge_low.tolist(), "g_Wq": sampled_entries(gq_low, 1)},
        "spectrum": {"omega": w.tolist(), "polarisations": pol.tolist(),
                     "gamma": gamma.tolist(), "S": S.tolist(),
                     "S_check": float(np.abs(S - S_ref).max() / np.abs(S_ref).max()),
                     "g_eps": ge_spec.tolist(), "g_Wq": sampled_entries(gq_spec, 2)},
    }
    with open(os.path.join(HERE, "mesh8_ao64_grad.json"), "w") as f:
        json.dump(out, f)
    log("gradient golden written")


if __name__ == "__main__":
    what = sys.argv[1:] or ["spectrum", "grad"]
    if "spectrum" in what:
        spectrum_golden()
    if "grad" in what:
        grad_golden()
    if "spectrum-values" in what:
        spectrum_values()
