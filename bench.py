"""Benchmark of the dual-k-mesh TDA-BSE hot path on one MI355X.

One step is one pass of the whole path over one synthetic crystal whose
inputs are already resident in HBM:
  interpolate W(R) -> W(q) on the dense mesh (FP64 on the matrix cores),
  build the plan (pair-density halves, rho, precision conversion),
  velocity-form start vectors for nb polarisations,
  Haydock: n_steps block applies of A (pair densities formed on the fly)
           with the FP64 Lanczos recurrence, CGS2 and the continued fraction,
  one adjoint apply (gradient of the first spectral moment p^H A p with
  respect to W(R) and the energies).
Reported value: algorithmic H.X flops of the step (n_steps x F_apply) divided
by the wall time of the whole step (GFLOP/s), so everything else in the
step counts as overhead.  Before the timed region the FP64 path is run once
as the reference: the headline precision is the fastest one whose spectrum
stays within 1e-5 (relative, max norm over polarisations and frequencies)
of the FP64 spectrum.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec auto|f64|f32|bf16x3]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONDUCTION = None  # BF16x3 conduction route ("mc", "u" or the plan's choice)
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16x3": 2516.6 / 3.0}
METRIC = "BSE H\u00b7X GFLOP/s & %MFMA peak, mixed vs FP64 at \u22641e-5 rel. spectrum error"
# default workload of each mode
MODE_CONFIG = {"apply": "mesh16_ao128", "spectrum": "mesh8_ao64", "precision": "mesh12_ao96",
               "gradients": "mesh8_ao64_grad", "largest": "mesh16_ao128", "offsets": "mesh8_ao64",
               "two_centre": "mesh8_ao64", "full_bse": "mesh8_ao64"}
HBM_PEAK_GBS = 8000.0


def f_apply(Nk, n_ao, nv, nc, n_aux, nb, q_formed=None):
    """Algorithmic flops of one block apply (8 real flops per complex MAC).

    With q_formed, the pair-density and W terms count only the Nk x q_formed pairs whose blocks
    are formed (the pair symmetry); the X term still counts every pair."""
    N = Nk * nv * nc
    formed = Nk if q_formed is None else q_formed
    return (8 * (Nk * formed * (n_aux * n_ao * (nc ** 2 + nv ** 2) + n_aux ** 2 * min(nc, nv) ** 2)
                 + Nk ** 2 * n_aux * nc * nv * nb * (nc + nv)
                 + 2 * Nk * nc * nv * n_aux * nb + n_aux ** 2 * nb) + 2 * N * nb)


def kernel_flops_per_pair(p, prec, route="mc"):
    """Algorithmic flops per (k, k') pair of each single-kernel stage of the direct term.

    wstep      P = conj(M_v) W(q)              8 n_aux^2 nv^2
               route "fused" (BF16x3): P and T = M_c P^T in one kernel, P kept on chip
                                                8 n_aux^2 nv^2 + 8 n_aux nc^2 nv^2
    pairdens_v M_vv' from the halves            8 n_aux n_ao nv^2
    pairdens_c M_cc' from the halves            8 n_aux n_ao nc^2      (routes "mc", "fused")
    dblock     route "mc": T = M_c P^T          8 n_aux nc^2 nv^2
               route "u" (BF16x3): U = B_c^T P^T and T = psi U (conduction pair densities never formed)
                                                8 nc n_ao n_aux nv^2 + 8 nc^2 n_ao nv^2
    """
    na, no, nv, nc = p.n_aux, p.n_ao, p.nv, p.nc
    d = {"wstep": 8 * na * na * nv * nv, "pairdens_c": 8 * na * no * nc * nc,
         "pairdens_v": 8 * na * no * nv * nv, "dblock": 8 * na * nc * nc * nv * nv}
    if route == "u":
        d["dblock"] = 8 * nc * no * na * nv * nv + 8 * nc * nc * no * nv * nv
    if route == "fused":
        d["wstep"] += d.pop("dblock")
    return d


def kernel_bytes_per_pair(p, prec, route="mc"):
    """Algorithmic HBM bytes per (k, k') pair of the single-kernel stages (each operand once)."""
    na, no, nv, nc, Nk = p.n_aux, p.n_ao, p.nv, p.nc, p.Nk
    e = 16 if prec == "f64" else 8
    d = {"wstep": e * (2 * nv * nv * na) + e * na * na / Nk,
         "pairdens_v": e * nv * nv * na + e * (nv * na * no) / Nk,
         "pairdens_c": e * nc * nc * na + e * (nc * na * no) / Nk,
         "dblock": (e * nv * nv * na + 8 * nc * nc * nv * nv + e * nc * no * na / Nk) if route == "u"
         else e * (nc * nc * na + nv * nv * na) + e * nc * nc * nv * nv}
    if route == "fused":  # reads M_v, M_c and W(q), writes T (c64); P stays on chip
        del d["dblock"]
        d["wstep"] = e * (nv * nv * na + nc * nc * na) + e * na * na / Nk + 8 * nc * nc * nv * nv
    return d


def copy_calibration(nbytes=1 << 30):
    """One plain device copy of a known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (apply mode: block applies; default 5)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps before the timed ones (default 1)")
    ap.add_argument("--prec", default=None, choices=["auto", "f64", "f32", "bf16x3"],
                    help="apply mode: arithmetic of the timed apply (default bf16x3); spectrum mode: auto picks "
                         "the fastest precision within 1e-5 of the FP64 spectrum")
    ap.add_argument("--config", default=None, help="workload (synth.CONFIGS); each mode has its own default")
    ap.add_argument("--haydock-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64", action="store_true", help="apply mode: skip the FP64 reference apply")
    ap.add_argument("--no-gate", action="store_true", help="apply mode: skip the 8x8x8 spectrum gate")
    ap.add_argument("--no-adjoint", action="store_true", help="apply mode: skip the adjoint apply")
    ap.add_argument("--cpu-rows", type=int, default=2)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run one 1 GiB device copy (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--conduction", default="auto", choices=["auto", "mc", "u"],
                    help="BF16x3 conduction side of the direct term: the plan's choice (auto), forming the "
                         "conduction pair densities (mc) or the B_c(k) contraction (u)")
    ap.add_argument("--mode", default="apply",
                    choices=["apply", "spectrum", "precision", "gradients", "largest", "offsets", "two_centre",
                             "full_bse"],
                    help="apply (default): block applies of A on the largest workload, with the FP64 apply, "
                         "the oracle's sampled rows and the adjoint beside them and the 8x8x8 spectrum gate; "
                         "spectrum: the 8x8x8 Haydock pipeline timed per precision; precision: per-precision "
                         "apply and short-Haydock errors on the 12x12x12 workload; gradients: LOBPCG and "
                         "spectrum gradients checked by central finite differences; largest: one BF16x3 apply "
                         "and adjoint on the 16x16x16 / N_ao = 128 workload; offsets: the spectrum averaged over "
                         "the four shifted dense meshes of the k-offset scheme; two_centre: the BF16x3 apply "
                         "and Haydock run with k-dependent two-centre LRI coefficients beside the "
                         "k-independent ones; full_bse: the spectrum of the full BSE (coupling block B) by the "
                         "structure-preserving Lanczos recurrence beside the TDA Haydock spectrum")
    args = ap.parse_args()
    args.config = args.config or MODE_CONFIG[args.mode]
    if args.steps is None:
        args.steps = 5 if args.mode == "apply" else 1
    if args.warmup is None:
        args.warmup = 1
    if args.prec is None:
        args.prec = "bf16x3" if args.mode == "apply" else "auto"
    global CONDUCTION
    CONDUCTION = None if args.conduction == "auto" else args.conduction
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.mode == "precision":
        precision_mode(args.config, args.haydock_steps or 10)
        return
    if args.mode == "offsets":
        from synth import CONFIGS
        offsets_mode(args.config, args.haydock_steps or CONFIGS[args.config]["haydock_steps"])
        return
    if args.mode == "full_bse":
        from synth import CONFIGS
        full_bse_mode(args.config, args.haydock_steps or CONFIGS[args.config]["haydock_steps"])
        return
    if args.mode == "two_centre":
        from synth import CONFIGS
        two_centre_mode(args.config, args.haydock_steps or CONFIGS[args.config]["haydock_steps"])
        return
    if args.mode == "largest":
        largest_mode(args.config)
        return
    if args.mode == "gradients":
        from synth import CONFIGS
        gradients_mode(args.config, args.haydock_steps or CONFIGS[args.config]["haydock_steps"])
        return

    if args.mode == "spectrum":
        spectrum_mode(args)
        return
    apply_mode(args)


def spectrum_mode(args):
    """The 8x8x8 pipeline: interpolation, plan, start vectors, a Haydock run and one adjoint per step, each
    precision timed, the fastest one within 1e-5 of the FP64 spectrum timed over the steps."""
    import torch
    from paper_2607_05853_amd import bse as B
    from synth import CONFIGS, dense_kmesh, make_problem, polarisations

    cfg = CONFIGS[args.config]
    m = args.haydock_steps or cfg["haydock_steps"]
    nb = cfg["nb"]
    eta = 0.1
    dev = torch.device("cuda:0")
    T = lambda a, dt=torch.complex128: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)
    sync = torch.cuda.synchronize

    p = make_problem(args.config, 0, "G1")
    kq = dense_kmesh(p.nk)
    te = p.eps_qp[:, p.nv:][:, :, None] - p.eps_qp[:, :p.nv][:, None, :]
    omega = np.linspace(te.min() - 1.0, te.max() + 1.0, 2001)
    pol = polarisations(nb)
    # inputs resident in HBM before any timed region
    d_WR, d_psi, d_C = T(p.W_R), T(p.psi), T(p.C)
    d_V, d_eps, d_vel, d_eks = T(p.Vbar), T(p.eps_qp, torch.float64), T(p.vel), T(p.eps_ks, torch.float64)
    Fa = f_apply(p.Nk, p.n_ao, p.nv, p.nc, p.n_aux, nb)
    print("[bench] workload %s: N=%d, nb=%d, Haydock %d steps, F_apply=%.3f TFLOP" %
          (args.config, p.N, nb, m, Fa / 1e12), file=sys.stderr, flush=True)

    def step(prec, timing=False):
        Wq = B.interpolate_W(d_WR, p.R, p.w_R, kq)
        plan = B.Plan(p.nk, p.n_ao, p.nv, p.nc, p.n_aux, d_eps, d_psi, d_C, d_V, Wq, alpha=p.alpha,
                      prec=prec, max_nb=nb, conduction=CONDUCTION if prec == "bf16x3" else None)
        plan.set_R(p.R, p.w_R)
        if timing:
            plan.set_timing(True)
        P = plan.velocity_start(d_vel, d_eks, pol)
        out = plan.haydock(P, m, omega, eta)
        g = plan.apply_adjoint(P, P, want_WR=True, want_eps=True)
        st = plan.stage_times() if timing else None
        pairs[prec] = plan.pairs
        routes[prec] = plan.conduction
        plan.close()
        del Wq, P, g
        return out, st

    pairs, routes = {}, {}

    # FP64 reference (untimed): spectrum and step time
    sync()
    t0 = time.time()
    ref, st64 = step("f64", timing=True)
    sync()
    t_f64 = time.time() - t0
    print("[bench] f64 step %.2f s (%.1f GFLOP/s)" % (t_f64, m * Fa / t_f64 / 1e9), file=sys.stderr, flush=True)
    S_ref = ref["S"]
    errs, times = {"f64": 0.0}, {"f64": t_f64}
    cands = ["bf16x3", "f32"] if args.prec == "auto" else ([args.prec] if args.prec != "f64" else [])
    chosen = "f64" if args.prec in ("auto", "f64") else None
    for prec in cands:
        sync()
        t0 = time.time()
        out, _ = step(prec)
        sync()
        times[prec] = time.time() - t0
        errs[prec] = float(np.abs(out["S"] - S_ref).max() / np.abs(S_ref).max())
        print("[bench] %s step %.2f s, spectrum error vs f64 %.2e" % (prec, times[prec], errs[prec]),
              file=sys.stderr, flush=True)
        if args.prec == "auto" and errs[prec] <= 1e-5 and (chosen == "f64" or times[prec] < times[chosen]):
            chosen = prec
        if args.prec == prec:
            chosen = prec
    prec = chosen

    for _ in range(args.warmup):
        step(prec)
    sync()
    t0 = time.time()
    st_all = None
    for i in range(args.steps):
        out, st = step(prec, timing=(i == args.steps - 1))
        st_all = st
    sync()
    dt = (time.time() - t0) / args.steps
    value = m * Fa / dt / 1e9
    print("[bench] timed: %s %.3f s/step -> %.1f GFLOP/s" % (prec, dt, value), file=sys.stderr, flush=True)

    # roofline of the dominant single kernel (event-timed on the library's stream)
    fpp = kernel_flops_per_pair(p, prec, routes[prec])
    cand = {k: v for k, v in st_all.items() if k in fpp and v[1] > 0}
    dom = max(cand, key=lambda k: cand[k][0])
    ms, n = cand[dom]
    # every Haydock apply runs the direct-term kernels over Nk x (q formed) pairs (about half of Nk^2
    # under the pair symmetry); the adjoint pass runs the two pair-density kernels over all Nk^2 pairs
    q_formed, q_total = pairs[prec]
    pairs_run = m * p.Nk * q_formed + (p.Nk * p.Nk if dom.startswith("pairdens") else 0)
    pairs_per_launch = pairs_run / n
    achieved = fpp[dom] * pairs_per_launch / (ms / n * 1e-3) / 1e12
    traffic = measured_traffic(dom, args.config, prec)
    roof = {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[prec],
            "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[prec],
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "algorithmic_bytes_per_launch": kernel_bytes_per_pair(p, prec, routes[prec])[dom] * pairs_per_launch,
            "avg_launch_ms": ms / n, "launches": n, "pairs_per_launch": pairs_per_launch}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(p, kq, nb, Fa, args.cpu_rows)

    stages = {k: round(v[0], 3) for k, v in st_all.items() if v[1] > 0}
    Fx = f_apply(p.Nk, p.n_ao, p.nv, p.nc, p.n_aux, nb, q_formed=q_formed)
    rec = {
        "metric": "BSE H\u00b7X GFLOP/s & %MFMA peak, mixed vs FP64 at \u22641e-5 rel. spectrum error",
        "value": value, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": "%s: dense %s k-mesh from coarse %s, N_ao=%d, nv=%d, nc=%d, N_aux=%d, BSE dim %d, "
                               "blocks of %d, Haydock %d steps, eta=%.2f eV" %
                               (args.config, "x".join(map(str, p.nk)), "x".join(map(str, p.coarse)), p.n_ao, p.nv,
                                p.nc, p.n_aux, p.N, nb, m, eta),
                   "F_apply_TFLOP": Fa / 1e12, "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "precision": {k: {"s_per_step": times[k], "spectrum_rel_err_vs_f64": errs[k],
                          "GFLOP_s": m * Fa / times[k] / 1e9} for k in times},
        "speedup_vs_f64_gpu": t_f64 / dt,
        # D(k, k-q) = D(k-q, k)^dagger: the apply forms the direct blocks of q_formed of the q_total
        # differences; F_apply counts all of them, the executed count scales its pair term
        "direct_pairs": {"q_formed": q_formed, "q_total": q_total,
                         "F_apply_executed_TFLOP": Fx / 1e12},
        "pct_mfma_peak_apply": m * Fx / dt / 1e12 / PEAK_TFLOPS[prec],
        "pct_mfma_peak_apply_F_apply": value / 1e3 / PEAK_TFLOPS[prec],
        "stage_ms_last_step": stages,
        "conduction": routes[prec],
    }
    print(json.dumps(rec), flush=True)


def log(msg):
    print("[bench %s] %s" % (time.strftime("%H:%M:%S"), msg), file=sys.stderr, flush=True)


def workload_text(p, config, nb, r_cut=None):
    cut = ", W(R) within |R|<=%g (%d R)" % (r_cut, len(p.R)) if r_cut else ", %d R" % len(p.R)
    return ("%s: dense %s k-mesh from coarse %s%s, N_ao=%d, nv=%d, nc=%d, N_aux=%d, BSE dim %d, blocks of %d" %
            (config, "x".join(map(str, p.nk)), "x".join(map(str, p.coarse)), cut, p.n_ao, p.nv, p.nc, p.n_aux,
             p.N, nb))


def dominant_roofline(p, prec, route, stages, pairs_run, config):
    """Roofline of the single-kernel stage that takes the most time: its algorithmic flops per launch
    (per-pair figure of kernel_flops_per_pair x the pairs one launch covers) over its average launch time
    (HIP events on the library's stream over the timed steps)."""
    fpp = kernel_flops_per_pair(p, prec, route)
    cand = {k: v for k, v in stages.items() if k in fpp and v[1] > 0}
    dom = max(cand, key=lambda k: cand[k][0])
    ms, n = cand[dom]
    pairs_per_launch = pairs_run / n
    achieved = fpp[dom] * pairs_per_launch / (ms / n * 1e-3) / 1e12
    traffic = measured_traffic(dom, config, prec)
    roof = {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS[prec],
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "algorithmic_flops_per_pair": fpp[dom],
            "algorithmic_bytes_per_launch": kernel_bytes_per_pair(p, prec, route)[dom] * pairs_per_launch,
            "avg_launch_ms": ms / n, "launches": n, "pairs_per_launch": pairs_per_launch}
    if traffic and traffic.get("mfma_issue_frac") is not None:
        roof["mfma_issue_frac"] = traffic["mfma_issue_frac"]
    return roof


def apply_mode(args):
    """Block applies of A (Eq. (Hamiltonian), pair densities formed on the fly) on one workload.

    One step is one apply of A to a block of nb vectors resident in HBM.  Around the timed steps: the FP64
    apply of the same block on the GPU (speedup and error of the timed precision against it), the oracle's
    FP64 apply on sampled k rows (the CPU baseline, and the error of both GPU results against it), one
    adjoint apply, and the 8x8x8 spectrum gate (the timed precision's 300-step Haydock spectrum against the
    oracle's, stored by tests/golden/make_mesh8_golden.py)."""
    import torch
    from paper_2607_05853_amd import bse as B
    from synth import CONFIGS, dense_kmesh, make_problem, random_block

    config, prec = args.config, args.prec
    if prec == "auto":
        prec = "bf16x3"
    cfg = CONFIGS[config]
    nb = cfg["nb"]
    dev = torch.device("cuda:0")
    T = lambda a, dt=torch.complex128: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)
    sync = torch.cuda.synchronize
    t0 = time.time()
    p = make_problem(config, 0, "G1")
    kq = dense_kmesh(p.nk)
    Fa = f_apply(p.Nk, p.n_ao, p.nv, p.nc, p.n_aux, nb)
    log("workload %s: N=%d, nb=%d, F_apply=%.1f TFLOP, inputs drawn in %.1f s" %
        (config, p.N, nb, Fa / 1e12, time.time() - t0))
    # inputs resident in HBM before any timed region
    d_WR, d_psi, d_C, d_V = T(p.W_R), T(p.psi), T(p.C), T(p.Vbar)
    d_eps = T(p.eps_qp, torch.float64)
    Xh = random_block(p.N, nb, seed=1)
    X = T(Xh)
    Y = torch.empty_like(X)

    def make_plan(pr):
        t = time.time()
        Wq = B.interpolate_W(d_WR, p.R, p.w_R, kq)
        plan = B.Plan(p.nk, p.n_ao, p.nv, p.nc, p.n_aux, d_eps, d_psi, d_C, d_V, Wq, alpha=p.alpha, prec=pr,
                      max_nb=nb, conduction=CONDUCTION if pr == "bf16x3" else None)
        plan.set_R(p.R, p.w_R)
        del Wq
        sync()
        torch.cuda.empty_cache()
        log("%s plan %.2f s (%.1f GB), pairs %s, conduction %s" %
            (pr, time.time() - t, plan.bytes / 2**30, plan.pairs, plan.conduction))
        return plan

    plan = make_plan(prec)
    for _ in range(args.warmup):
        plan.apply(X, out=Y)
    sync()
    log("%d warmup applies done" % args.warmup)
    plan.set_timing(True)
    plan.stage_times()
    sync()
    t0 = time.time()
    for i in range(args.steps):
        plan.apply(X, out=Y)
    sync()
    dt = (time.time() - t0) / args.steps
    stages = plan.stage_times()
    plan.set_timing(False)
    value = Fa / dt / 1e9
    log("timed: %d %s applies, %.3f s per apply -> %.1f GFLOP/s" % (args.steps, prec, dt, value))
    q_formed, q_total = plan.pairs
    route = "fused" if plan.fused else plan.conduction
    roof = dominant_roofline(p, prec, route, stages, args.steps * p.Nk * q_formed, config)
    Fx = f_apply(p.Nk, p.n_ao, p.nv, p.nc, p.n_aux, nb, q_formed=q_formed)
    stage_ms = {k: round(v[0] / args.steps, 2) for k, v in stages.items() if v[1] > 0}

    adj = None
    if not args.no_adjoint:
        Yb = T(random_block(p.N, nb, seed=2))
        plan.set_timing(True)
        plan.stage_times()
        sync()
        t0 = time.time()
        g = plan.apply_adjoint(Yb, X, want_WR=True, want_eps=True)
        sync()
        ta = time.time() - t0
        st = {k: round(v[0], 1) for k, v in plan.stage_times().items() if v[1] > 0}
        plan.set_timing(False)
        na, no, nv, nc = p.n_aux, p.n_ao, p.nv, p.nc
        Fg = 8 * p.Nk ** 2 * (na * no * (nv ** 2 + nc ** 2) + nv ** 2 * nc ** 2 * na + na ** 2 * nv ** 2
                              + nv ** 2 * nc ** 2 * nb)
        adj = {"s": ta, "F_TFLOP": Fg / 1e12, "GFLOP_s": Fg / ta / 1e9, "stage_ms": st}
        log("adjoint %.2f s" % ta)
        del g, Yb
    plan.close()
    del plan
    torch.cuda.empty_cache()

    rows = list(np.linspace(0, p.Nk - 1, args.cpu_rows).astype(int)) if args.cpu_rows > 0 else []
    cpu = orc = None
    if not args.no_cpu_baseline and rows:
        cpu, orc = cpu_baseline_rows(p, kq, Xh, rows, Fa)
        log("oracle rows %s: %.1f s (%.2f GFLOP/s on %d threads)" % (rows, cpu["_t"], cpu["value"], cpu["cores"]))
        del cpu["_t"]

    # kernel part of the result: Y - D X with D the FP64 diagonal of transition energies
    te = (d_eps[:, p.nv:][:, :, None] - d_eps[:, :p.nv][:, None, :]).reshape(-1, 1)
    DX = te * X
    nt = p.nc * p.nv

    def rows_of(Z):
        return np.vstack([Z[k * nt:(k + 1) * nt].cpu().numpy() for k in rows])

    acc = {}
    if orc is not None:
        ref, DXr = orc
        acc["kernel_rel_err_vs_oracle_rows"] = float(np.abs(rows_of(Y) - ref).max() / np.abs(ref - DXr).max())
        acc["oracle_rows"] = [int(k) for k in rows]
    prec_rec = {prec: {"apply_s": dt, "GFLOP_s": value}}
    speedup = None
    if not args.no_f64 and prec != "f64":
        plan = make_plan("f64")
        Y64 = torch.empty_like(X)
        plan.set_timing(True)
        plan.stage_times()
        sync()
        t0 = time.time()
        plan.apply(X, out=Y64)
        sync()
        t64 = time.time() - t0
        st64 = {k: round(v[0], 1) for k, v in plan.stage_times().items() if v[1] > 0}
        plan.close()
        del plan
        torch.cuda.empty_cache()
        log("f64 apply %.2f s" % t64)
        prec_rec["f64"] = {"apply_s": t64, "GFLOP_s": Fa / t64 / 1e9, "stage_ms": st64}
        speedup = t64 / dt
        acc["kernel_rel_err_vs_f64_gpu"] = ((Y - Y64).abs().max() / (Y64 - DX).abs().max()).item()
        if orc is not None:
            acc["f64_gpu_kernel_rel_err_vs_oracle_rows"] = float(np.abs(rows_of(Y64) - orc[0]).max() /
                                                                 np.abs(orc[0] - orc[1]).max())
        del Y64
    gate = None
    if not args.no_gate:
        gate = spectrum_gate(prec)

    rec = {
        "metric": METRIC,
        "value": value, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": workload_text(p, config, nb, cfg.get("r_cut")) +
                   "; one step = one apply of A to the block", "F_apply_TFLOP": Fa / 1e12,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "accuracy": acc,
        "precision": prec_rec,
        "speedup_vs_f64_gpu": speedup,
        # D(k, k-q) = D(k-q, k)^dagger: the apply forms the direct blocks of q_formed of the q_total
        # differences; F_apply counts all of them, the executed count scales its pair terms
        "direct_pairs": {"q_formed": q_formed, "q_total": q_total, "F_apply_executed_TFLOP": Fx / 1e12},
        "pct_mfma_peak_apply": Fx / dt / 1e12 / PEAK_TFLOPS[prec],
        "pct_mfma_peak_apply_F_apply": Fa / dt / 1e12 / PEAK_TFLOPS[prec],
        "stage_ms_per_apply": stage_ms,
        "conduction": route,
        "adjoint": adj,
        "spectrum_gate": gate,
    }
    print(json.dumps(rec), flush=True)


def spectrum_gate(prec):
    """The timed precision's 300-step Haydock spectrum at the 8x8x8 workload (generator G1, seed 0, 8
    polarisations, 2001 frequencies) against the oracle's Haydock spectrum of the explicit A stored by
    tests/golden/make_mesh8_golden.py."""
    import torch
    from paper_2607_05853_amd import bse as B
    from synth import dense_kmesh, make_problem
    path = os.path.join(ROOT, "tests", "golden", "mesh8_ao64_spectrum.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    p = make_problem(g["config"], g["seed"], g["wgen"])
    dev = torch.device("cuda:0")
    T = lambda a, dt=torch.complex128: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)
    w = np.linspace(g["omega"]["lo"], g["omega"]["hi"], g["omega"]["n"])
    t0 = time.time()
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
    plan = B.plan_from_problem(p, Wq, prec=prec, max_nb=g["nb"])
    del Wq
    P = plan.velocity_start(T(p.vel), T(p.eps_ks, torch.float64), np.array(g["polarisations"]))
    out = plan.haydock(P, g["n_steps"], w, g["eta"])
    torch.cuda.synchronize()
    t = time.time() - t0
    plan.close()
    S_or = np.array(g["S"])
    err = float(np.abs(out["S"] - S_or).max() / np.abs(S_or).max())
    log("spectrum gate: %s 300-step Haydock at %s in %.1f s, error vs oracle %.2e" % (prec, g["config"], t, err))
    return {"workload": "%s (generator %s, seed %d): %d polarisations, %d Haydock steps, %d frequencies, eta=%g eV"
                        % (g["config"], g["wgen"], g["seed"], g["nb"], g["n_steps"], g["omega"]["n"], g["eta"]),
            "prec": prec, "s": t, "spectrum_rel_err_vs_oracle": err, "target": 1e-5, "pass": err <= 1e-5,
            "oracle_haydock_vs_eigh": g["haydock_vs_eigh_max_rel"]}


def _setup(config, wgen="G1"):
    import torch
    from paper_2607_05853_amd import bse as B
    from synth import dense_kmesh, make_problem
    dev = torch.device("cuda:0")
    T = lambda a, dt=torch.complex128: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)
    p = make_problem(config, 0, wgen)
    return B, T, p, dense_kmesh(p.nk), torch


def precision_mode(config, m):
    """Apply and short-Haydock spectrum of each precision against the FP64 GPU path on one seed."""
    from synth import CONFIGS, polarisations, random_block
    B, T, p, kq, torch = _setup(config)
    nb = CONFIGS[config]["nb"]
    Fa = f_apply(p.Nk, p.n_ao, p.nv, p.nc, p.n_aux, nb)
    W_R, eps = T(p.W_R), T(p.eps_qp, torch.float64)
    X = T(random_block(p.N, nb, seed=1))
    te = p.eps_qp[:, p.nv:][:, :, None] - p.eps_qp[:, :p.nv][:, None, :]
    omega = np.linspace(te.min() - 1.0, te.max() + 1.0, 2001)
    out = {}
    Yref = Sref = None
    for prec in ["f64", "bf16x3", "f32"]:
        Wq = B.interpolate_W(W_R, p.R, p.w_R, kq)
        plan = B.Plan(p.nk, p.n_ao, p.nv, p.nc, p.n_aux, eps, T(p.psi), T(p.C), T(p.Vbar), Wq, alpha=p.alpha,
                      prec=prec, max_nb=nb, conduction=CONDUCTION if prec == "bf16x3" else None)
        del Wq
        torch.cuda.synchronize()
        t0 = time.time()
        Y = plan.apply(X)
        torch.cuda.synchronize()
        ta = time.time() - t0
        print("[precision] %s apply %.3f s" % (prec, ta), file=sys.stderr, flush=True)
        P = plan.velocity_start(T(p.vel), T(p.eps_ks, torch.float64), polarisations(nb))
        t0 = time.time()
        S = plan.haydock(P, m, omega, 0.1)["S"]
        th = time.time() - t0
        if Yref is None:
            Yref, Sref = Y.clone(), S
        rec = {"apply_s": ta, "apply_GFLOP_s": Fa / ta / 1e9,
               "apply_rel_err_vs_f64": float((Y - Yref).abs().max() / Yref.abs().max()),
               "haydock_s": th, "spectrum_rel_err_vs_f64": float(np.abs(S - Sref).max() / np.abs(Sref).max())}
        out[prec] = rec
        print("[precision] %s %s" % (prec, json.dumps(rec)), file=sys.stderr, flush=True)
        plan.close()
        del plan, Y, P
        torch.cuda.empty_cache()
    print(json.dumps({"mode": "precision", "workload": "%s: dense %s, N_ao=%d, nv=%d, nc=%d, N_aux=%d, BSE dim %d, "
                                                  "blocks of %d, Haydock %d steps" %
                      (config, "x".join(map(str, p.nk)), p.n_ao, p.nv, p.nc, p.n_aux, p.N, nb, m),
                      "F_apply_TFLOP": Fa / 1e12, "results": out}), flush=True)


def largest_mode(config):
    """One BF16x3 apply and one adjoint (W(R) and energy gradients) at the largest workload, timed with the
    stage breakdown; the apply is run once untimed first."""
    from synth import CONFIGS, random_block
    B, T, p, kq, torch = _setup(config)
    nb = CONFIGS[config]["nb"]
    t0 = time.time()
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, kq)
    torch.cuda.synchronize()
    t_interp = time.time() - t0
    t0 = time.time()
    plan = B.Plan(p.nk, p.n_ao, p.nv, p.nc, p.n_aux, T(p.eps_qp, torch.float64), T(p.psi), T(p.C), T(p.Vbar), Wq,
                  alpha=p.alpha, prec="bf16x3", max_nb=nb, conduction=CONDUCTION)
    plan.set_R(p.R, p.w_R)
    del Wq
    torch.cuda.synchronize()
    t_plan = time.time() - t0
    print("[largest] interpolation %.2f s, plan %.2f s (%.1f GB)" % (t_interp, t_plan, plan.bytes / 2**30),
          file=sys.stderr, flush=True)
    X, Yb = T(random_block(p.N, nb, seed=1)), T(random_block(p.N, nb, seed=2))
    plan.apply(X)
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.stage_times()
    t0 = time.time()
    plan.apply(X)
    torch.cuda.synchronize()
    ta = time.time() - t0
    st_apply = {k: round(v[0], 1) for k, v in plan.stage_times().items() if v[1]}
    print("[largest] apply %.2f s %s" % (ta, st_apply), file=sys.stderr, flush=True)
    t0 = time.time()
    plan.apply_adjoint(Yb, X, want_WR=True, want_eps=True)
    torch.cuda.synchronize()
    tg = time.time() - t0
    st_adj = {k: round(v[0], 1) for k, v in plan.stage_times().items() if v[1]}
    print("[largest] adjoint %.2f s %s" % (tg, st_adj), file=sys.stderr, flush=True)
    qf, qt = plan.pairs
    Fa = f_apply(p.Nk, p.n_ao, p.nv, p.nc, p.n_aux, nb)
    Fx = f_apply(p.Nk, p.n_ao, p.nv, p.nc, p.n_aux, nb, q_formed=qf)
    # adjoint flops: pair densities (both sides), Z = Gm conj(M_c), g_W = Gv^T Z over every pair, Gm
    na, no, nv, nc = p.n_aux, p.n_ao, p.nv, p.nc
    Fg = 8 * p.Nk ** 2 * (na * no * (nv ** 2 + nc ** 2) + nv ** 2 * nc ** 2 * na + na ** 2 * nv ** 2
                          + nv ** 2 * nc ** 2 * nb)
    print(json.dumps({
        "mode": "largest", "workload": "%s: dense %s from coarse %s, N_ao=%d, nv=%d, nc=%d, N_aux=%d, |R|<=%g, "
                                       "BSE dim %d, blocks of %d" %
        (config, "x".join(map(str, p.nk)), "x".join(map(str, p.coarse)), p.n_ao, p.nv, p.nc, p.n_aux,
         CONFIGS[config]["r_cut"], p.N, nb),
        "prec": "bf16x3", "conduction": plan.conduction, "plan_GB": plan.bytes / 2**30, "interpolate_s": t_interp, "plan_s": t_plan,
        "apply_s": ta, "F_apply_TFLOP": Fa / 1e12, "apply_GFLOP_s": Fa / ta / 1e9,
        "pct_mfma_peak_apply_F_apply": Fa / ta / 1e12 / PEAK_TFLOPS["bf16x3"],
        "direct_pairs": {"q_formed": qf, "q_total": qt, "F_apply_executed_TFLOP": Fx / 1e12},
        "pct_mfma_peak_apply": Fx / ta / 1e12 / PEAK_TFLOPS["bf16x3"],
        "apply_stage_ms": st_apply, "adjoint_s": tg, "F_adjoint_TFLOP": Fg / 1e12,
        "adjoint_GFLOP_s": Fg / tg / 1e9, "adjoint_stage_ms": st_adj}), flush=True)
    plan.close()


def full_bse_mode(config, m):
    """Full BSE: the BF16x3 spectrum of Eq. (full_BSE_epsilon2) from m steps of the structure-preserving
    Lanczos recurrence (one full apply = A on [X | conj Y] and B on [Y | conj X] per step), timed, beside
    the BF16x3 TDA Haydock spectrum of the same m; the BF16x3 error against FP64 on a shorter run of both."""
    from synth import CONFIGS, polarisations, random_block
    B, T, p, kq, torch = _setup(config)
    nb = CONFIGS[config]["nb"]
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, kq)
    te = p.eps_qp[:, p.nv:][:, :, None] - p.eps_qp[:, :p.nv][:, None, :]
    omega = np.linspace(te.min() - 1.0, te.max() + 1.0, 2001)
    res = {}
    m_short = 40
    spec = {}
    for prec in ["bf16x3", "f64"]:
        plan = B.plan_from_problem(p, Wq, prec=prec, max_nb=2 * nb)
        P = plan.velocity_start(T(p.vel), T(p.eps_ks, torch.float64), polarisations(nb))
        r = {"q_formed_A": plan.pairs[0], "conduction": plan.conduction}
        X = T(random_block(p.N, nb, seed=1))
        XY = T(random_block(2 * p.N, nb, seed=2))
        plan.apply_full(XY)
        torch.cuda.synchronize()
        for name, fn in [("apply_A_ms", lambda: plan.apply(X)), ("apply_B_ms", lambda: plan.apply_coupling(X)),
                         ("apply_full_ms", lambda: plan.apply_full(XY))]:
            plan.set_timing(True)
            torch.cuda.synchronize()
            t0 = time.time()
            fn()
            torch.cuda.synchronize()
            r[name] = (time.time() - t0) * 1e3
            r[name.replace("_ms", "_stage_ms")] = {k: round(v[0], 2) for k, v in plan.stage_times().items() if v[1]}
            plan.set_timing(False)
        spec[prec] = plan.full_spectrum(P, m_short, omega, 0.1)["S"]
        if prec == "bf16x3":
            torch.cuda.synchronize()
            t0 = time.time()
            out = plan.full_spectrum(P, m, omega, 0.1)
            torch.cuda.synchronize()
            r["full_spectrum_s"] = time.time() - t0
            r["full_steps"] = int(out["steps"].min())
            r["max_abs_diagonal_over_max_offdiagonal"] = float(np.abs(out["a"]).max() / np.abs(out["b"][:, 1:]).max())
            torch.cuda.synchronize()
            t0 = time.time()
            hay = plan.haydock(P, m, omega, 0.1)
            torch.cuda.synchronize()
            r["tda_haydock_s"] = time.time() - t0
            r["max_rel_diff_full_vs_tda"] = float(np.abs(out["S"] - hay["S"]).max() / np.abs(hay["S"]).max())
            r["peak_shift_eV (full - tda, first polarisation)"] = float(omega[np.argmax(out["S"][0])] -
                                                                       omega[np.argmax(hay["S"][0])])
            torch.cuda.synchronize()
            t0 = time.time()
            omf, _, itf = plan.full_lowest(n_block=4, max_iter=200, tol=1e-6, want_vectors=False,
                                           allow_unconverged=True)
            torch.cuda.synchronize()
            r["full_lowest"] = {"omega_eV": [float(x) for x in omf], "iterations": itf, "s": time.time() - t0,
                                "tol": 1e-6}
            omt, _, itt = plan.lowest_excitons(n_block=4, max_iter=200, tol=1e-6, want_vectors=False,
                                               allow_unconverged=True)
            r["tda_lowest"] = {"omega_eV": [float(x) for x in omt], "iterations": itt}
            r["omega1_shift_meV (full - tda)"] = float(1e3 * (omf[0] - omt[0]))
        res[prec] = r
        plan.close()
        print("[full_bse mode] %s done" % prec, file=sys.stderr, flush=True)
    err = float(np.abs(spec["bf16x3"] - spec["f64"]).max() / np.abs(spec["f64"]).max())
    # the coupling block's direct term on BF16x3 (one B apply of the 2 n_b packed columns is what the full
    # apply runs; here the stage of a B apply on n_b columns): algorithmic bytes of its per-pair
    # intermediates G_B, M2, P_B (each written once and read once, G_B read by both W-step column tiles
    # counted once) and its MFMA flops, against the stage time
    rb = res["bf16x3"]
    pairs = p.Nk * rb["q_formed_A"]  # the coupling block forms the same q (W(q) Hermitian here)
    ntv = p.nc * p.nv
    by = 6 * 8.0 * ntv * p.n_aux * pairs
    fl = 8.0 * pairs * (2 * p.n_aux * p.n_ao * ntv + p.n_aux ** 2 * ntv + p.n_aux * ntv ** 2)
    tst = rb["apply_B_stage_ms"].get("coupling", float("nan")) / 1e3
    stage_roof = {"stage": "coupling (B direct term)", "bound": "hbm", "achieved": by / tst / 1e9, "peak": 8000.0,
                  "unit": "GB/s", "frac": by / tst / 8e12, "mfma_TFLOP_s": fl / tst / 1e12,
                  "mfma_frac": fl / tst / 1e12 / PEAK_TFLOPS["bf16x3"]}
    cpu = None
    if not os.environ.get("BENCH_NO_CPU"):
        import oracle as O
        Wq_o = O.interpolate_W_matmul(p.W_R, p.R, p.w_R, kq)
        sel = [0, p.Nk // 2]
        t0 = time.time()
        O.apply_rows_twosided(p, Wq_o, random_block(p.N, nb, seed=3), sel, "B")
        tc_ = time.time() - t0
        cpu = {"value": tc_ * p.Nk / len(sel), "unit": "s per B apply", "kind": "oracle",
               "sample": "%d of %d k rows of one FP64 coupling apply (row-at-a-time form), %.1f s, extrapolated x%d"
                         % (len(sel), p.Nk, tc_, p.Nk // len(sel)),
               "gpu_bf16x3_B_apply_s": rb["apply_B_ms"] / 1e3}
    print(json.dumps({"mode": "full_bse", "workload": "%s, %d chains, %d Lanczos steps (error check %d steps)" %
                      (config, nb, m, m_short), "stage_roofline": stage_roof, "cpu_baseline": cpu, "runs": res,
                      "spectrum_rel_err_bf16x3_vs_f64_%d_steps" % m_short: err}), flush=True)


def two_centre_mode(config, m):
    """k-dependent two-centre LRI coefficients: one apply per precision (BF16x3 error against FP64) and the
    BF16x3 Haydock spectrum, each beside the same run with the k-independent coefficients of the workload."""
    from synth import CONFIGS, make_problem, polarisations, random_block
    import torch
    from paper_2607_05853_amd import bse as B
    from synth import dense_kmesh
    dev = torch.device("cuda:0")
    T = lambda a, dt=torch.complex128: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)
    nb = CONFIGS[config]["nb"]
    res = {}
    for kind in ["k_independent", "two_centre"]:
        p = make_problem(config, 0, "G1", two_centre=(kind == "two_centre"))
        Fa = f_apply(p.Nk, p.n_ao, p.nv, p.nc, p.n_aux, nb)
        Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, dense_kmesh(p.nk))
        X = T(random_block(p.N, nb, seed=1))
        te = p.eps_qp[:, p.nv:][:, :, None] - p.eps_qp[:, :p.nv][:, None, :]
        omega = np.linspace(te.min() - 1.0, te.max() + 1.0, 2001)
        r = {}
        Y64 = None
        for prec in ["f64", "bf16x3"]:
            torch.cuda.synchronize()
            t0 = time.time()
            plan = B.plan_from_problem(p, Wq, prec=prec, max_nb=nb)
            torch.cuda.synchronize()
            t_plan = time.time() - t0
            plan.apply(X)
            torch.cuda.synchronize()
            plan.set_timing(True)
            t0 = time.time()
            Y = plan.apply(X)
            torch.cuda.synchronize()
            ta = time.time() - t0
            st = {k: round(v[0], 2) for k, v in plan.stage_times().items() if v[1]}
            plan.set_timing(False)
            e = {"plan_s": t_plan, "apply_ms": ta * 1e3, "apply_stage_ms": st, "q_formed": plan.pairs[0],
                 "conduction": plan.conduction}
            if prec == "f64":
                Y64 = Y
            else:
                e["apply_rel_err_vs_f64"] = float((Y - Y64).abs().max() / Y64.abs().max())
                P = plan.velocity_start(T(p.vel), T(p.eps_ks, torch.float64), polarisations(nb))
                torch.cuda.synchronize()
                t0 = time.time()
                out = plan.haydock(P, m, omega, 0.1)
                torch.cuda.synchronize()
                th = time.time() - t0
                e.update({"haydock_steps": m, "haydock_s": th, "GFLOP_s": m * Fa / th / 1e9})
            r[prec] = e
            plan.close()
            print("[two_centre mode] %s %s done" % (kind, prec), file=sys.stderr, flush=True)
        res[kind] = r
    # the conduction pair densities of the two-centre BF16x3 apply (two one-sided GEMMs per q batch): their
    # algorithmic flops and the bytes of their two c64 results, against the stage time
    p2 = make_problem(config, 0, "G1", two_centre=True)
    r2 = res["two_centre"]["bf16x3"]
    qf = r2["q_formed"]
    pairs = p2.Nk * qf
    fl = 2 * 8.0 * p2.n_aux * p2.n_ao * p2.nc ** 2 * pairs
    by = 2 * 8.0 * p2.nc ** 2 * p2.n_aux * pairs
    tst = r2["apply_stage_ms"].get("pairdens_c", float("nan")) / 1e3
    stage_roof = {"stage": "pairdens_c (two one-sided GEMMs per batch)", "bound": "hbm",
                  "achieved": by / tst / 1e9, "peak": 8000.0, "unit": "GB/s", "frac": by / tst / 8e12,
                  "mfma_TFLOP_s": fl / tst / 1e12, "mfma_frac": fl / tst / 1e12 / PEAK_TFLOPS["bf16x3"]}
    cpu = None
    if not os.environ.get("BENCH_NO_CPU"):
        import oracle as O
        Wq_o = O.interpolate_W_matmul(p2.W_R, p2.R, p2.w_R, dense_kmesh(p2.nk))
        sel = [0, p2.Nk // 2]
        t0 = time.time()
        O.apply_rows_twosided(p2, Wq_o, random_block(p2.N, nb, seed=3), sel, "A")
        tc_ = time.time() - t0
        t_apply = tc_ * p2.Nk / len(sel)
        cpu = {"value": f_apply(p2.Nk, p2.n_ao, p2.nv, p2.nc, p2.n_aux, nb) / t_apply / 1e9, "unit": "GFLOP/s",
               "kind": "oracle", "sample": "%d of %d k rows of one FP64 two-centre apply (row-at-a-time form), "
               "%.1f s, extrapolated x%d" % (len(sel), p2.Nk, tc_, p2.Nk // len(sel)),
               "gpu_bf16x3_apply_GFLOP_s": f_apply(p2.Nk, p2.n_ao, p2.nv, p2.nc, p2.n_aux, nb) /
               (r2["apply_ms"] / 1e3) / 1e9}
    print(json.dumps({"mode": "two_centre", "workload": "%s, %d Haydock steps, blocks of %d" % (config, m, nb),
                      "coefficients": "real C^mu_st(R) on R = 0 and the 6 nearest cells, mu on the atom of s",
                      "stage_roofline": stage_roof, "cpu_baseline": cpu,
                      "runs": res,
                      "haydock_ratio_two_centre_over_k_independent":
                          res["two_centre"]["bf16x3"]["haydock_s"] / res["k_independent"]["bf16x3"]["haydock_s"]}),
          flush=True)


def offsets_mode(config, m):
    """k-offset averaging: the BF16x3 Haydock spectrum on each of the paper's four shifted dense meshes (one
    W(q) interpolation shared by all), averaged with the paper's weights."""
    from synth import CONFIGS, polarisations
    B, T, p, kq, torch = _setup(config)
    nb = CONFIGS[config]["nb"]
    Fa = f_apply(p.Nk, p.n_ao, p.nv, p.nc, p.n_aux, nb)
    offs, wts = B.offset_set()
    te = p.eps_qp[:, p.nv:][:, :, None] - p.eps_qp[:, :p.nv][:, None, :]
    omega = np.linspace(te.min() - 1.0, te.max() + 1.0, 2001)
    torch.cuda.synchronize()
    t0 = time.time()
    Wq = B.interpolate_W(T(p.W_R), p.R, p.w_R, kq)
    plans, Ps, per = [], [], []
    from synth import make_problem
    for o in offs:
        ta = time.time()
        po = make_problem(config, 0, "G1", offset=tuple(o))
        t_gen = time.time() - ta
        ta = time.time()
        pl = B.Plan(po.nk, po.n_ao, po.nv, po.nc, po.n_aux, T(po.eps_qp, torch.float64), T(po.psi), T(po.C),
                    T(po.Vbar), Wq, alpha=po.alpha, prec="bf16x3", max_nb=nb, conduction=CONDUCTION)
        Ps.append(pl.velocity_start(T(po.vel), T(po.eps_ks, torch.float64), polarisations(nb)))
        plans.append(pl)
        torch.cuda.synchronize()
        per.append({"offset": [float(x) for x in o], "bands_s (host, input generation)": t_gen,
                    "plan_s": time.time() - ta})
    torch.cuda.synchronize()
    t_setup = time.time() - t0
    t0 = time.time()
    out = B.offset_spectrum(plans, Ps, wts, m, omega, 0.1)
    torch.cuda.synchronize()
    t_spec = time.time() - t0
    S0 = plans[0].haydock(Ps[0], m, omega, 0.1)["S"]
    diff = float(np.abs(out["S"] - S0).max() / np.abs(out["S"]).max())
    for pl in plans:
        pl.close()
    print(json.dumps({"mode": "offsets", "workload": "%s, %d offsets x %d Haydock steps, blocks of %d, BF16x3" %
                      (config, len(offs), m, nb), "weights": [float(x) for x in wts],
                      "setup_s (interpolation once + plans + start vectors, GPU)": t_setup - sum(
                          x["bands_s (host, input generation)"] for x in per),
                      "averaged_spectrum_s": t_spec, "GFLOP_s": len(offs) * m * Fa / t_spec / 1e9,
                      "max_rel_diff_average_vs_unshifted": diff, "per_offset": per}), flush=True)


def gradients_mode(config, m):
    """Gradients of Omega_1 (LOBPCG) and of the Haydock spectrum at 64 frequencies w.r.t. W(R) and eps,
    against central finite differences of the same GPU path (FP64, h = 1e-6)."""
    from synth import CONFIGS, polarisations
    from paper_2607_05853_amd import autograd as AG
    B, T, p, kq, torch = _setup(config, "G2")
    nb = CONFIGS[config]["nb"]
    eta, h = 0.1, 1e-6
    rng = np.random.default_rng(7)
    idx = {tuple(r): i for i, r in enumerate(p.R)}
    dW = np.zeros(p.W_R.shape)
    for i, r in enumerate(p.R):
        j = idx[tuple(-r)]
        if j < i:
            continue
        A = rng.standard_normal(p.W_R.shape[1:])
        if i == j:
            A = A + A.T
        dW[i], dW[j] = A, A.T
    # scale the direction so that h * dW is a 1e-6 relative change of W(R): the directional
    # derivative is then well above the rounding noise of the difference quotient
    dW = (dW * (np.abs(p.W_R).max() / np.abs(dW).max())).astype(complex)
    de = rng.standard_normal(p.eps_qp.shape)

    def build(W_R, eps):
        Wq = B.interpolate_W(W_R, p.R, p.w_R, kq)
        pl = B.Plan(p.nk, p.n_ao, p.nv, p.nc, p.n_aux, eps, T(p.psi), T(p.C), T(p.Vbar), Wq, alpha=p.alpha,
                    prec="f64", max_nb=max(nb, 64))
        pl.set_R(p.R, p.w_R)
        return pl

    res = {}
    W_R = T(p.W_R).requires_grad_(True)
    eps = T(p.eps_qp, torch.float64).requires_grad_(True)
    plan = build(W_R.detach(), eps.detach())
    t0 = time.time()
    om_all, _, _ = plan.lowest_excitons(n_block=nb, tol=1e-12, max_iter=500)
    res["Omega2_minus_Omega1_eV"] = float(om_all[1] - om_all[0])
    om1 = AG.lowest_exciton_energy(plan, W_R, eps, n_block=nb, tol=1e-12, max_iter=500)
    om1.backward()
    torch.cuda.synchronize()
    res["lowest_s"] = time.time() - t0
    print("[gradients] Omega_1 and its gradient: %.1f s" % res["lowest_s"], file=sys.stderr, flush=True)
    gW, ge = W_R.grad.detach().cpu().numpy(), eps.grad.detach().cpu().numpy()

    def om(Wr, e):
        pl = build(T(Wr), T(e, torch.float64))
        o, _, it = pl.lowest_excitons(n_block=nb, tol=1e-13, max_iter=800, allow_unconverged=True)
        pl.close()
        print("[gradients] LOBPCG for finite differences: %d iterations" % it, file=sys.stderr, flush=True)
        return o[0]

    # Omega_1 depends on W only through the weak binding (its W derivative is ~1e-6 of its eps
    # derivative here), so the W difference quotient takes a larger step to stay above the
    # ~1e-15 relative rounding of the eigenvalue
    hW = 1e-4
    fdW = (om(p.W_R + hW * dW, p.eps_qp) - om(p.W_R - hW * dW, p.eps_qp)) / (2 * hW)
    fde = (om(p.W_R, p.eps_qp + h * de) - om(p.W_R, p.eps_qp - h * de)) / (2 * h)
    res["fd_step_W_Omega1"] = hW
    anW, ane = float(np.real(np.vdot(gW, dW))), float(np.sum(ge * de))
    res["Omega1_eV"] = float(om1.item())
    res["dOmega1_dW"] = {"adjoint": anW, "fd": fdW}
    res["dOmega1_deps"] = {"adjoint": ane, "fd": fde}
    res["dOmega1_dW_fd_rel_err"] = abs(fdW - anW) / abs(anW)
    res["dOmega1_deps_fd_rel_err"] = abs(fde - ane) / abs(ane)
    print("[gradients] lowest %s" % json.dumps(res), file=sys.stderr, flush=True)

    omega = np.linspace(res["Omega1_eV"] - 0.5, res["Omega1_eV"] + 2.5, 64)
    gamma = rng.standard_normal((nb, len(omega)))
    W_R2 = T(p.W_R).requires_grad_(True)
    eps2 = T(p.eps_qp, torch.float64).requires_grad_(True)
    P = plan.velocity_start(T(p.vel), T(p.eps_ks, torch.float64), polarisations(nb))
    t0 = time.time()
    S = AG.haydock_spectrum(plan, P, W_R2, eps2, m, omega, eta)
    torch.sum(T(gamma, torch.float64) * S).backward()
    torch.cuda.synchronize()
    res["spectrum_grad_s"] = time.time() - t0

    def spec(Wr, e):
        pl = build(T(Wr), T(e, torch.float64))
        s = pl.haydock(P, m, omega, eta)["S"]
        pl.close()
        print("[gradients] Haydock for finite differences done", file=sys.stderr, flush=True)
        return float(np.sum(gamma * s))

    fdW = (spec(p.W_R + h * dW, p.eps_qp) - spec(p.W_R - h * dW, p.eps_qp)) / (2 * h)
    fde = (spec(p.W_R, p.eps_qp + h * de) - spec(p.W_R, p.eps_qp - h * de)) / (2 * h)
    anW = float(np.real(np.vdot(W_R2.grad.detach().cpu().numpy(), dW)))
    ane = float(np.sum(eps2.grad.detach().cpu().numpy() * de))
    res["dS_dW"] = {"adjoint": anW, "fd": fdW}
    res["dS_deps"] = {"adjoint": ane, "fd": fde}
    res["dS_dW_fd_rel_err"] = abs(fdW - anW) / abs(anW)
    res["dS_deps_fd_rel_err"] = abs(fde - ane) / abs(ane)

    # the mixed-precision path: the same two gradients from a BF16x3 plan, against the FP64 adjoint ones
    def relmax(a, b):
        return float(np.abs(a - b).max() / np.abs(b).max())

    Wq3 = B.interpolate_W(T(p.W_R), p.R, p.w_R, kq)
    pl3 = B.Plan(p.nk, p.n_ao, p.nv, p.nc, p.n_aux, T(p.eps_qp, torch.float64), T(p.psi), T(p.C), T(p.Vbar), Wq3,
                 alpha=p.alpha, prec="bf16x3", max_nb=max(nb, 64))
    pl3.set_R(p.R, p.w_R)
    t0 = time.time()
    # Omega_1: Hellmann-Feynman through the BF16x3 adjoint with the FP64 eigenvector (the residual of LOBPCG
    # on the BF16x3 operator cannot fall below that operator's rounding, ~4e-8 of |A|)
    _, Xl, _ = plan.lowest_excitons(n_block=nb, tol=1e-12, max_iter=500)
    x1 = Xl[:, :1].contiguous()
    g3 = pl3.apply_adjoint(x1, x1, want_WR=True, want_eps=True)
    om3 = torch.real(torch.sum(torch.conj(x1) * pl3.apply(x1)))
    W_R4 = T(p.W_R).requires_grad_(True)
    eps4 = T(p.eps_qp, torch.float64).requires_grad_(True)
    S3 = AG.haydock_spectrum(pl3, P, W_R4, eps4, m, omega, eta)
    torch.sum(T(gamma, torch.float64) * S3).backward()
    torch.cuda.synchronize()
    res["bf16x3_vs_f64"] = {
        "time_s": time.time() - t0,
        "Omega1_rel_err": abs(om3.item() - res["Omega1_eV"]) / abs(res["Omega1_eV"]),
        "dOmega1_dW_rel_err": relmax(g3["W_R"].cpu().numpy(), gW),
        "dOmega1_deps_rel_err": relmax(g3["eps"].cpu().numpy(), ge),
        "spectrum_rel_err": relmax(S3.detach().cpu().numpy(), S.detach().cpu().numpy()),
        "dS_dW_rel_err": relmax(W_R4.grad.detach().cpu().numpy(), W_R2.grad.detach().cpu().numpy()),
        "dS_deps_rel_err": relmax(eps4.grad.detach().cpu().numpy(), eps2.grad.detach().cpu().numpy())}
    print("[gradients] bf16x3 %s" % json.dumps(res["bf16x3_vs_f64"]), file=sys.stderr, flush=True)
    pl3.close()
    print(json.dumps({"mode": "gradients", "workload": "%s: dense %s, N_ao=%d, nv=%d, nc=%d, N_aux=%d, BSE dim %d, "
                                                      "LOBPCG block %d, spectrum at 64 frequencies, Haydock %d steps"
                      % (config, "x".join(map(str, p.nk)), p.n_ao, p.nv, p.nc, p.n_aux, p.N, nb, m),
                      "fd_step": h, "results": res}), flush=True)


# the sources of everything a timed apply runs (plan dispatch, the pair-density, W-step, T and T.X kernels);
# the Lanczos, LOBPCG, full-BSE and interpolation sources do not change a counter taken on an apply
APPLY_SOURCES = ("api.hip", "apply.hip", "direct_b3.hip", "gemm.hip", "util.hip", "bse_internal.h", "mfma_common.h")


def source_digest():
    """Digest of the HIP sources of the apply: counter summaries taken on other sources are stale."""
    import hashlib
    h = hashlib.sha256()
    cdir = os.path.join(ROOT, "paper_2607_05853_amd", "csrc")
    for f in APPLY_SOURCES:
        with open(os.path.join(cdir, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, config, prec):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it matches these sources."""
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s_%s.txt" % (kernel, config, prec))
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_digest") != source_digest():
        return None
    try:
        out = {"bytes_per_launch": float(vals["hbm_bytes_per_launch"])}
    except (KeyError, ValueError):
        return None
    try:
        out["mfma_issue_frac"] = float(vals["mfma_issue_frac"])
    except (KeyError, ValueError):
        pass
    return out


def cpu_baseline(p, kq, nb, Fa, rows):
    """The FP64 oracle's matrix-free apply on a sample of k rows, extrapolated to one apply."""
    import oracle as O
    from synth import random_block
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    Wq = O.interpolate_W(p.W_R, p.R, p.w_R, kq)
    X = random_block(p.N, nb, seed=3)
    sel = list(np.linspace(0, p.Nk - 1, rows).astype(int))
    t0 = time.time()
    O.apply_H_rows(p, Wq, X, sel)
    t = time.time() - t0
    t_apply = t * p.Nk / rows
    return {"value": Fa / t_apply / 1e9, "unit": "GFLOP/s", "cores": int(cores), "kind": "oracle",
            "sample": "%d of %d k rows of one FP64 matrix-free apply (nb=%d), %.1f s, extrapolated x%d"
                      % (rows, p.Nk, nb, t, p.Nk // rows)}


def cpu_baseline_rows(p, kq, Xh, rows, Fa):
    """The FP64 oracle's row-at-a-time apply (every k' of a row at once, the form used for sampled rows on
    the large meshes) on a few k rows of the same block, extrapolated to one apply; returns the baseline
    record and (the oracle's rows, their D X) for the accuracy figures."""
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    W = O.interpolate_W_matmul(p.W_R, p.R, p.w_R, kq)
    t0 = time.time()
    ref = O.apply_H_rows_allpairs(p, W, Xh, rows)
    t = time.time() - t0
    del W
    nt = p.nc * p.nv
    te = O.transition_energies(p)
    DXr = np.vstack([te[k][:, None] * Xh[k * nt:(k + 1) * nt] for k in rows])
    t_apply = t * p.Nk / len(rows)
    rec = {"value": Fa / t_apply / 1e9, "unit": "GFLOP/s", "cores": int(cores), "kind": "oracle",
           "sample": "%d of %d k rows of one FP64 apply (row-at-a-time oracle form, nb=%d), %.1f s, extrapolated x%d"
                     % (len(rows), p.Nk, Xh.shape[1], t, p.Nk // len(rows)), "_t": t}
    return rec, (ref, DXr)


if __name__ == "__main__":
    main()
