/*
 * bse.h - C ABI of the MI355X (gfx950) dual-k-mesh Tamm-Dancoff BSE hot path.
 *
 * The operations follow the paper's statement of the problem:
 *   inputs  : quasiparticle energies E^GW_nk and Kohn-Sham coefficients c^k_sn
 *             (Sec. II.A), LRI coefficients C^mu (Sec. III.A), the truncated bare
 *             Coulomb matrix Vbar (Sec. III.A) and the static screened interaction
 *             W_munu(R) on a small Born-von-Karman R set (Sec. III.B, workflow);
 *   outputs : the action of the TDA Hamiltonian A (Eq. (Hamiltonian) with the
 *             LRI kernel of Eq. (W_LRI)), the absorption spectrum (Eq. (abs_vel))
 *             and the lowest exciton (binding energy, Sec. IV.B.3).
 *
 * Conventions shared by every call
 *   - all arrays row-major; complex = interleaved {re, im} doubles ("c128") or
 *     floats ("c64"); "device" pointers point to HIP device memory of the current
 *     device, "host" pointers to ordinary host memory;
 *   - lattice: simple cubic, a = 1, cell volume 1; R integer triples; k and q in
 *     fractional coordinates; Fourier phases exp(+2 pi i k.R);
 *   - dense Gamma-centred k mesh n1 x n2 x n3, k index (i1*n2 + i2)*n3 + i3;
 *     q(k, k') = k' - k reduced into the mesh;
 *   - bands per k: nv valence (ascending) then nc conduction (ascending);
 *   - transition index I = (k*nc + c)*nv + v, vector index b fastest: X[I][nb].
 *
 * Ownership: the caller owns every argument buffer; the library never frees or
 * keeps a caller pointer beyond the call.  A plan owns copies of what it needs.
 * Streams: every call is asynchronous on the HIP stream passed as `hip_stream`
 * (NULL = default stream); device results are valid after a stream sync.  Host
 * outputs are written before the call returns.  A plan is not thread-safe;
 * distinct plans may be used concurrently.
 * Errors: no exception or abort crosses this ABI.  Argument validation happens
 * before any HIP call.  HIP failures map to BSE_EDEVICE and the hipError text is
 * available from bse_last_error() (thread-local).
 */
#ifndef BSE_H
#define BSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BSE_OK = 0,
    BSE_EINVAL = 1,      /* null pointer, non-positive size, unknown enum        */
    BSE_ESHAPE = 2,      /* sizes inconsistent with each other or with the plan   */
    BSE_ENOMEM = 3,      /* device allocation failed; nothing was launched on the
                            missing buffer and the plan stays usable: workspaces a
                            plan allocates on first use are completed by the next
                            call (tests force it with BSE_TEST_FAIL_ALLOC=n, which
                            fails the n-th device allocation made under that value) */
    BSE_EDEVICE = 4,     /* a HIP call failed                                     */
    BSE_ENOTHERM = 5,    /* plan creation found a non-Hermitian C^mu or Vbar      */
    BSE_INFO_BREAKDOWN = 100, /* a Haydock chain stopped early (not an error)      */
    BSE_INFO_NOT_CONVERGED = 101 /* an iterative driver hit its iteration limit    */
} bse_status;

/* Arithmetic of the pair-density / screened-interaction contractions.
 * BSE_F64    : complex128 storage and FP64 MFMA.
 * BSE_F32    : complex64 storage and FP32 MFMA, FP32 accumulation inside a tile.
 * BSE_BF16X3 : complex64 storage; each operand split as hi = bf16(x),
 *              lo = bf16(x - hi) and multiplied as hi*hi + hi*lo + lo*hi on BF16
 *              MFMA with FP32 accumulation (Henry, Tang & Heinecke, ARITH 2019).
 * For every precision the diagonal, the exchange term, accumulation across k'
 * and the Lanczos recurrence run in FP64. */
typedef enum { BSE_F64 = 0, BSE_F32 = 1, BSE_BF16X3 = 2 } bse_prec;

#define BSE_CHECK_HERMITIAN 1u   /* accepted; plan creation always verifies C^mu and Vbar */
#define BSE_ALL_PAIRS 2u         /* plan_create: form every (k, k') block of the direct term */
#define BSE_CONDUCTION_MC 4u     /* plan_create, BF16X3: form the conduction pair densities M_cc' */
#define BSE_CONDUCTION_U 8u      /* plan_create, BF16X3: contract B_c(k) with the W step instead  */

typedef struct {
    int32_t nk[3];       /* dense Gamma-centred mesh n1, n2, n3 (Sec. IV.A.3)                */
    int32_t n_ao;        /* NAO basis functions per cell                                    */
    int32_t nv, nc;      /* valence / conduction bands in the transition space              */
    int32_t n_aux;       /* auxiliary basis functions per cell                              */
    double alpha;        /* exchange factor: 2 singlet, 0 triplet (Eq. (Hamiltonian))       */
} bse_dims;

typedef struct bse_plan bse_plan;  /* opaque */

/* ---------------------------------------------------------------------------
 * Dual-k-mesh interpolation of the screened interaction (Sec. III.B: W(k) on
 * the coarse mesh -> W(R) on the BvK supercell, truncated -> W(q) on the dense
 * mesh; phase of Eq. (W_LRI)):
 *     W_q[q] = sum_R w_R W_R[R] exp(+2 pi i q.R)
 * W_R     device c128 [n_R][n_aux][n_aux]
 * R       host int32 [n_R][3]; w_R host f64 [n_R] (Wigner-Seitz face weights)
 * q_frac  host f64 [n_q][3] (any list of fractional q)
 * W_q     device [n_q][n_aux][n_aux], c128 if out_prec == BSE_F64 else c64
 * The sum is evaluated in FP64 on the matrix cores whatever out_prec is.
 * ------------------------------------------------------------------------- */
bse_status bse_interpolate_W(int32_t n_aux, int32_t n_R, const void* W_R,
                             const int32_t* R, const double* w_R,
                             int32_t n_q, const double* q_frac,
                             void* W_q, bse_prec out_prec, void* hip_stream);

/* The same interpolation for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): arguments, results and errors as bse_interpolate_W, but the
 * workspace (the q, R and weight tables and the [n_q][n_R] phase table) lives
 * in a static device array of 16 MiB per GPU, held until the process ends,
 * and no device memory is allocated or freed.  Sizes whose workspace exceeds
 * it (about n_q * n_R > 10^6: 16 bytes per phase plus 36 per q and R) return
 * BSE_ESHAPE before any HIP call.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams or host threads) race; calls
 * on one stream are ordered.  The host tables are copied with
 * hipMemcpyAsync from the caller's host memory. */
bse_status bse_interpolate_W_noalloc(int32_t n_aux, int32_t n_R, const void* W_R,
                                     const int32_t* R, const double* w_R,
                                     int32_t n_q, const double* q_frac,
                                     void* W_q, bse_prec out_prec, void* hip_stream);

/* Conjugate transpose of the map above (the adjoint used for gradients):
 *     g_WR[R] = w_R sum_q exp(-2 pi i q.R) g_Wq[q]
 * With q the coarse mesh and w_R = 1/N_coarse this is also the coarse -> R
 * inverse transform of the workflow.  g_Wq, g_WR device c128. */
bse_status bse_interpolate_W_adjoint(int32_t n_aux, int32_t n_R, const int32_t* R,
                                     const double* w_R, int32_t n_q, const double* q_frac,
                                     const void* g_Wq, void* g_WR, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Plan: copies the inputs of Eq. (Hamiltonian) and precomputes the halves of
 * the LRI pair densities (Sec. III.A, C-tilde in the Kohn-Sham basis):
 *     B^mu_n(k) = psi_n(k)^dagger C^mu            (n valence or conduction)
 *     rho^mu_{cvk} = B^mu_c(k) psi_v(k) = M^mu_cv(k, k)
 * so that M^mu_ij(k, k') = psi_i(k)^dagger C^mu psi_j(k') = B^mu_i(k) psi_j(k').
 * eps_qp  device f64 [Nk][nv+nc]   E^GW (valence first)
 * psi     device c128 [Nk][nv+nc][n_ao]   row n = c^k_{s n}
 * C       device c128 [n_aux][n_ao][n_ao], each C^mu Hermitian (the k-independent
 *         form of the two-centre relation of Sec. III.A); the direct term uses
 *         conj M^mu_ij(k,k') = M^mu_ji(k',k) and the exchange term
 *         M^nu_v'c'(k',k') = conj rho^nu_c'v'k', which hold only then
 * Vbar    device c128 [n_aux][n_aux], Hermitian (V_munu(0) of Sec. III.A)
 * Plan creation checks on the device, before anything else is allocated, that
 * max |C^mu - C^mu^H| <= 1e-12 max |C| over all mu and max |Vbar - Vbar^H| <=
 * 1e-12 max |Vbar|, and returns BSE_ENOTHERM (nothing created) otherwise: for
 * other inputs the plan would apply an operator different from Eq.
 * (Hamiltonian).  This synchronises the stream once.
 * W_q     device c128 [Nk][n_aux][n_aux], q = dense-mesh index
 * prec    arithmetic of the direct term; max_nb the largest block size later used
 * flags   BSE_ALL_PAIRS (BSE_CHECK_HERMITIAN is accepted and changes nothing)
 * Pair symmetry: with Hermitian C^mu the direct block of Eq. (Hamiltonian)
 * obeys D(k, k-q) = D(k-q, k)^dagger as soon as W_q(-q) = conj W_q(q)
 * elementwise (true for any real W(R) interpolated with Sec. III.B).  Plan
 * creation tests that relation on the given W_q (to 1e-12 of max |W_q|); when
 * it holds, bse_apply forms the blocks of one q of each pair {q, -q} (and of
 * the q equal to their own negative) and takes the others from the relation,
 * about half of the direct-term work.  BSE_ALL_PAIRS forms every block.
 * bse_plan_pairs reports which mode a plan uses.
 * Conduction side of the direct term on BF16X3 (FP64 / FP32 always form M_cc'):
 * either the pair densities M^nu_cc'(k,k') = B^nu_c(k) psi_c'(k') are formed and
 * the block taken as sum_nu M_cc' P (BSE_CONDUCTION_MC), or B_c(k) is contracted
 * with P first and psi_c'(k') applied last, so M_cc' never exists
 * (BSE_CONDUCTION_U; needs n_v^2 <= 128 and n_ao <= 128).  Both compute the same
 * sums; without either flag the plan takes the one with the smaller estimated
 * time (matrix-core work against the M_cc' traffic), bse_plan_conduction tells
 * which.  Giving both flags is BSE_EINVAL.
 * On success *out receives the plan (destroy with bse_plan_destroy).
 * ------------------------------------------------------------------------- */
bse_status bse_plan_create(const bse_dims* d, const double* eps_qp, const void* psi,
                           const void* C, const void* Vbar, const void* W_q,
                           bse_prec prec, int32_t max_nb, uint32_t flags,
                           void* hip_stream, bse_plan** out);

/* ---------------------------------------------------------------------------
 * Plan with k-dependent two-centre LRI coefficients (Sec. III.A).  In place of
 * the k-independent C^mu the plan takes the real coefficients C^mu_st(R) of the
 * AO pair (s at cell 0, t at cell R) for the ABF mu on the atom of s, with
 *     C^mu_st(k) = sum_R C^mu_st(R) exp(+2 pi i k.R)
 * and forms the Kohn-Sham coefficients of the paper's C-tilde,
 *     M^mu_ij(k_a, k_b) = sum_st conj(c^{k_a}_{s i}) c^{k_b}_{t j} [C^mu_st(k_b) + C^mu_ts(-k_a)],
 * the first term for the ABFs on the centre of s, the second for those on the
 * centre of t.  Every operation of bse_plan_create's plans (apply, adjoint,
 * Haydock, LOBPCG, offsets, full BSE) runs on such a plan unchanged.
 * n_RC    number of lattice vectors of the coefficients (> 0)
 * RC      host int32 [n_RC][3]
 * C_R     device f64 [n_RC][n_aux][n_ao][n_ao], C_R[r][mu][s][t] = C^mu_st(R_r)
 *         (real: the relation conj M_ij(k_a, k_b) = M_ji(k_b, k_a), on which the
 *         pair symmetry and the Hermiticity of A rest, holds for real C only)
 * k_frac  host f64 [2][Nk][3]: fractional k of the valence bands of each mesh
 *         point, then of its conduction bands (the mesh itself, shifted by an
 *         offset, and for the conduction bands moved by an exciton momentum)
 * Other arguments as bse_plan_create.  Per pair the direct term forms the
 * one-sided products for both orders of the pair (twice the pair-density GEMM
 * work) and adds them; on BF16X3 the conduction side always forms M_cc'
 * (BSE_CONDUCTION_U is BSE_EINVAL); the Hermiticity check covers Vbar only
 * (real C_R guarantees the relation).
 * ------------------------------------------------------------------------- */
bse_status bse_plan_create_2c(const bse_dims* d, const double* eps_qp, const void* psi, int32_t n_RC,
                              const int32_t* RC, const double* C_R, const double* k_frac,
                              const void* Vbar, const void* W_q, bse_prec prec, int32_t max_nb,
                              uint32_t flags, void* hip_stream, bse_plan** out);

bse_status bse_plan_destroy(bse_plan* plan);

/* Register the R set (host int32 [n_R][3], host f64 weights) used by
 * bse_apply_adjoint to return g_WR. */
bse_status bse_plan_set_R(bse_plan* plan, int32_t n_R, const int32_t* R, const double* w_R);

/* Replace the quasiparticle energies (device f64 [Nk][nv+nc]) of a plan. */
bse_status bse_plan_set_eps(bse_plan* plan, const double* eps_qp, void* hip_stream);

/* Number of q (dense-mesh differences k' - k) whose direct blocks bse_apply
 * forms (*formed) out of *total = N_k: N_k with BSE_ALL_PAIRS or when the
 * pair symmetry does not hold, about N_k / 2 otherwise.  Host pointers. */
bse_status bse_plan_pairs(const bse_plan* plan, int64_t* formed, int64_t* total);

/* *forms_mc = 1 when the plan's direct term forms the conduction pair densities
 * M_cc' (always on FP64 / FP32), 0 when it uses the B_c(k) contraction (BF16X3).
 * Host pointer. */
bse_status bse_plan_conduction(const bse_plan* plan, int32_t* forms_mc);

/* *fused = 1 when bse_apply forms the W step P = conj(M_v) W(q) and the direct
 * block T = M_c P^T in one kernel, so that P never leaves the chip (BF16X3 plans
 * on the M_cc' route with n_v = n_c = 8, N_aux a multiple of 256 and an even
 * N_k; the same sums as the two GEMMs, summed in another order), 0 otherwise.
 * The environment variable BSE_FUSED_WSTEP=0, read at every apply, selects the
 * two GEMMs instead.  Host pointer. */
bse_status bse_plan_fused(const bse_plan* plan, int32_t* fused);

/* *frag = 1 when the plan stores its BF16X3 halves B^mu_n(k) in the fragment
 * order of the pair-density kernel (BF16X3 with k-independent coefficients,
 * N_ao of 64 or 128, N_aux a multiple of 32, n_v^2 a multiple of 8): per k and band
 * side the [n_band N_aux][N_ao] matrix is laid out as 32-column by 16-k blocks
 * of 1 KiB, each the operand of one matrix-core step, so that the streaming
 * kernel reads whole KiB instead of 32-byte pieces of 32 rows.  The results are
 * identical to those of the row layout.  BSE_FRAG_HALVES=0 in the environment
 * at plan creation keeps the row layout.  Host pointer. */
bse_status bse_plan_frag(const bse_plan* plan, int32_t* frag);

/* Device bytes held by the plan (copies, halves and workspaces). */
bse_status bse_plan_bytes(const bse_plan* plan, uint64_t* bytes);

/* ---------------------------------------------------------------------------
 * Y = A X with A the TDA block of Eq. (Hamiltonian):
 *   A_{cvk,c'v'k'} = (E_ck - E_vk) delta
 *                  + (alpha/N_k) sum_munu M^mu_cv(k,k) Vbar_munu M^nu_v'c'(k',k')
 *                  - (1/N_k) sum_munu M^mu_v'v(k',k) W_munu(k'-k) M^nu_cc'(k,k')
 * applied matrix-free: pair densities are formed on the fly every call.
 * X, Y device c128 [N][nb], N = Nk*nc*nv, 1 <= nb <= max_nb; X and Y must not
 * overlap.
 * ------------------------------------------------------------------------- */
bse_status bse_apply(bse_plan* plan, const void* X, void* Y, int32_t nb, void* hip_stream);

/* Vector-Jacobian product of L = Re sum_{I,b} conj(Ybar_Ib) (A X)_Ib with
 * respect to the screened interaction and the energies (PyTorch convention
 * dL = Re sum conj(g) d theta):
 *   g_Wq[q]_munu = -(1/N_k) sum_{k, k'=k+q} sum_b sum_{cvc'v'}
 *                  Ybar_{cvk,b} conj(M^mu_v'v(k',k) M^nu_cc'(k,k') X_{c'v'k',b})
 *   g_WR[R]      = w_R sum_q exp(-2 pi i q.R) g_Wq[q]     (needs bse_plan_set_R)
 *   g_eps[k][nv+c] = Re sum_{v,b} conj(Ybar) X,  g_eps[k][v] = -Re sum_{c,b} conj(Ybar) X
 * Ybar, X device c128 [N][nb]; g_WR device c128 [n_R][n_aux][n_aux];
 * g_Wq device c128 [Nk][n_aux][n_aux]; g_eps device f64 [Nk][nv+nc].
 * Each output pointer may be NULL (not computed); outputs are overwritten.
 * The gradient with respect to X is A Ybar (A is Hermitian): use bse_apply.
 * ------------------------------------------------------------------------- */
bse_status bse_apply_adjoint(bse_plan* plan, const void* Ybar, const void* X, int32_t nb,
                             void* g_WR, void* g_Wq, double* g_eps, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Velocity-form start vectors of Eq. (abs_vel):
 *   P[I][b] = sum_alpha e_b[alpha] vel[alpha][k][c][v] / (E^KS_ck - E^KS_vk)
 * vel     device c128 [3][Nk][nc][nv]  (<c k| dH/dk_alpha |v k>)
 * eps_ks  device f64 [Nk][nv+nc]
 * pol     host f64 [nb][3] polarisation vectors
 * P       device c128 [N][nb]
 * ------------------------------------------------------------------------- */
bse_status bse_velocity_start(const bse_plan* plan, const void* vel, const double* eps_ks,
                              int32_t nb, const double* pol, void* P, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Start vector of a momentum-resolved spectrum (finite exciton momentum Q, the
 * extension of the conclusion; matrix element of the long-wavelength appendix
 * at finite q):
 *   P[I] = <c k+Q| e^{iQ.r} |v k> = <u_c^{k+Q}|u_v^k> = sum_s conj(psi[k][nv+c][s]) psi[k][v][s]
 * for orthonormal NAO Bloch sums with each orbital's e^{iQ.(r-R)} taken at its
 * centre.  psi is the band array of the plan (device c128 [Nk][nv+nc][n_ao],
 * valence rows at k, conduction rows at k + Q); P device c128 [N] (one column).
 * Haydock on a plan built at momentum Q from this vector gives
 * S(Q, w) = -(1/(pi N_k)) Im <P|(w + i eta - A_Q)^-1|P>; as Q -> 0, P / |Q|
 * tends to the velocity-form vector along Q.
 * ------------------------------------------------------------------------- */
bse_status bse_density_start(const bse_plan* plan, const void* psi, void* P, void* hip_stream);

/* ---------------------------------------------------------------------------
 * nb independent Haydock chains (Lanczos with full re-orthogonalisation by
 * classical Gram-Schmidt done twice) from the start vectors P, in FP64:
 *   b_0 = |p|, q_1 = p / b_0;  w = A q_j;  a_j = Re q_j^H w;
 *   w -= a_j q_j + b_{j-1} q_{j-1};  w -= Q (Q^H w) twice;  b_j = |w|;
 *   breakdown when b_j <= 1e-12 max(|a_1|, .., |a_j|, b_1, .., b_{j-1}) (the
 *   chain's own scale of A, so the test does not depend on |p|; the chain
 *   stops, steps_done = j);
 * then the continued fraction
 *   S_b(w) = -(1/(pi N_k)) Im  b_0^2 / (z - a_1 - b_1^2 / (z - a_2 - ... - b_{m-1}^2/(z - a_m))),
 *   z = w + i eta
 * (the velocity-form spectrum of Eq. (abs_vel) per polarisation, without the
 * constant 4 pi^2 / (3 V), Lorentzian half width eta).
 * P device c128 [N][nb]; omega host f64 [n_w]; S host f64 [nb][n_w];
 * a host f64 [nb][n_steps] (a_1..a_m); b host f64 [nb][n_steps+1] (b_0..b_m);
 * steps_done host int32 [nb]; basis_out NULL or device c128 [nb][n_steps][N]
 * (the Lanczos vectors q_1..q_m, e.g. for the spectrum's VJP).  Synchronises
 * the stream once at the end.  Returns BSE_INFO_BREAKDOWN if any chain broke
 * down (its results are still valid).
 * ------------------------------------------------------------------------- */
bse_status bse_haydock_spectrum(bse_plan* plan, const void* P, int32_t nb, int32_t n_steps,
                                const double* omega, int32_t n_w, double eta,
                                double* S, double* a, double* b, int32_t* steps_done,
                                void* basis_out, void* hip_stream);

/* ---------------------------------------------------------------------------
 * k-offset averaging (Sec. IV.A, the k-point convergence study): the spectrum
 * averaged over dense meshes shifted by offsets o_j (fractions of the mesh
 * spacing, k_i + o_j / n) with weights w_j,
 *     S(w) = sum_j w_j S_j(w),
 * S_j the Haydock spectrum of plans[j], a plan built from the bands (psi, E)
 * of the j-th shifted mesh and its start vectors P[j].  A common shift of k and
 * k' leaves q = k' - k, and so W_q, unchanged: every plan takes the same W_q.
 * plans[n_off] (same problem sizes), P[n_off] device c128 [N][nb] each,
 * weights host [n_off]; S host [nb][n_w] (overwritten); steps_done host
 * [n_off][nb] or NULL.  Each chain runs as in bse_haydock_spectrum;
 * BSE_INFO_BREAKDOWN if any chain ended early (the result is still valid).
 * ------------------------------------------------------------------------- */
bse_status bse_offset_spectrum(bse_plan* const* plans, const void* const* P, const double* weights,
                               int32_t n_off, int32_t nb, int32_t n_steps, const double* omega,
                               int32_t n_w, double eta, double* S, int32_t* steps_done,
                               void* hip_stream);

/* The paper's offset set: the four classes of a 3x3x3 grid of offsets, (0,0,0)
 * with weight 1/27, (1/3,0,0) 8/27, (1/3,1/3,0) 6/27, (2/3,1/3,0) 12/27.
 * *n = 4; offsets host [4][3] and weights host [4] may each be NULL. */
bse_status bse_offset_set(int32_t* n, double* offsets, double* weights);

/* ---------------------------------------------------------------------------
 * Vector-Jacobian product of the Haydock spectrum: for L = sum_{b,w} gamma[b][w] S_b(w)
 * the gradients with respect to W(R) / W(q) and the energies, through
 *   dS(w) = -(1/(pi N_k)) Im( yt^H dA y ),  y = (z - A)^-1 p,  yt = (conj z - A)^-1 p,
 * with y ~ b_0 Q (z - T)^-1 e_1 from the chain's Lanczos basis Q and tridiagonal T
 * (the derivative of the converged spectrum; resolvents solved on the host in FP64,
 * Krylov recombination and the adjoint contractions on the device).
 * basis device c128 [nb][n_steps][N] as returned by bse_haydock_spectrum; a, b, steps,
 * omega, gamma host arrays as there ([nb][n_steps], [nb][n_steps+1], [nb], [n_w],
 * [nb][n_w]).  Outputs as in bse_apply_adjoint (each may be NULL); overwritten.
 * ------------------------------------------------------------------------- */
bse_status bse_haydock_vjp(bse_plan* plan, const void* basis, const double* a, const double* b,
                           const int32_t* steps, int32_t nb, int32_t n_steps, const double* omega,
                           int32_t n_w, double eta, const double* gamma, void* g_WR, void* g_Wq,
                           double* g_eps, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Lowest exciton by block LOBPCG (Knyazev 2001) on the FP64 apply, with
 * Rayleigh-Ritz in FP64 on the host:  Omega_1 and its eigenvector (Sec. IV.B.3:
 * E_B = min_k (E_c1k - E_vtop k) - Omega_1).
 * n_block >= 1 (block size), max_iter, tol (relative residual |r| <= tol |Omega|).
 * X0 device c128 [N][n_block] start block (NULL: deterministic pseudo-random);
 * omega host f64 [n_block] ascending Ritz values; x_out device c128 [N][n_block]
 * (NULL allowed); iters host int32 (NULL allowed).  Converged means every Ritz pair
 * has |A x - omega x| <= tol |omega|; otherwise the last iterate is returned with
 * BSE_INFO_NOT_CONVERGED.  Synchronises the stream every iteration.
 * ------------------------------------------------------------------------- */
bse_status bse_lowest_excitons(bse_plan* plan, int32_t n_block, int32_t max_iter, double tol,
                               const void* X0, double* omega, void* x_out, int32_t* iters,
                               void* hip_stream);

/* ---------------------------------------------------------------------------
 * Full BSE (Eq. (Hamiltonian) with its coupling block; the paired solutions of
 * Eqs. (right)/(left); the spectrum of Eq. (full_BSE_epsilon2)), for plans of
 * either kind of LRI coefficients (on two-centre plans the cross pair densities
 * are formed from both one-sided products, as the resonant ones) and zero
 * exciton momentum.
 *
 * bse_apply_coupling: Y = B X with
 *   B_{cvk,c'v'k'} = (alpha/N_k) sum_munu M^mu_cv(k,k) Vbar_munu M^nu_c'v'(k',k')
 *                  - (1/N_k) sum_munu M^mu_c'v(k',k) W_munu(k'-k) M^nu_cv'(k,k')
 * (every pair formed; Vbar real symmetric and W(-R) = W(R)^T make B symmetric).
 * X, Y device c128 [N][nb], 1 <= nb <= max_nb, not overlapping; Y overwritten.
 *
 * bse_apply_full: out = [[A, B], [-B*, -A*]] [X; Y].  XY and out device c128
 * [2N][nb] (rows 0..N-1 the X block, N..2N-1 the Y block); needs 2 nb <= max_nb
 * (A is applied to [X | conj Y] and B to [Y | conj X] as one block each).
 *
 * bse_full_spectrum: for each of the nb columns p of P (device c128 [N][nb],
 * velocity start vectors as from bse_velocity_start)
 *   S[b][w] = (1/N_k) sum_{Omega_S > 0} |p^H X^S - p^T Y^S|^2 L_eta(omega_w - Omega_S)
 * with X^H X - Y^H Y = 1, by n_steps of Lanczos in the inner product
 * <x, y> = x^H J H y (J = diag(I, -I); positive definite for a stable ground
 * state) from [p; p*], full re-orthogonalisation, and Gauss quadrature on the
 * leading even-sized tridiagonal (its Ritz values come in +- pairs).  Needs
 * 2 nb <= max_nb and 2 <= n_steps <= 2N.  S host f64 [nb][n_w]; a host f64
 * [nb][n_steps] (diagonal, zero up to rounding), b host f64 [nb][n_steps+1]
 * (b[0] = |[p; p*]|, then the off-diagonal); steps_done host int32 [nb].
 * A chain stops when b_j <= 1e-12 max(|a_0|, .., |a_{j-1}|, b_1, .., b_{j-1})
 * (scale of H seen by the chain, independent of |p|).  Exact once the Krylov
 * space is invariant; BSE_INFO_BREAKDOWN when a chain stopped early (its
 * spectrum uses the steps done).
 * ------------------------------------------------------------------------- */
/* bse_full_lowest: the n_block smallest positive Omega_S of the full BSE with
 * right eigenvectors [X; Y] normalised X^H X - Y^H Y = 1 (Eqs. (right)/(left);
 * the negative partners are -Omega_S with [Y*; X*]).  Block LOBPCG on the
 * Hermitian-definite pencil J z = (1/Omega) (J H) z, whose largest eigenvalues
 * are the smallest positive Omega; one bse_apply_full per iteration, Rayleigh-
 * Ritz in FP64 on the host.  Needs 2 n_block <= max_nb.  X0 device c128
 * [2N][n_block] start block (NULL: pseudo-random X part, zero Y part); omega
 * host f64 [n_block] ascending; xy_out device c128 [2N][n_block] (NULL
 * allowed); iters host int32 (NULL allowed).  Converged means
 * |H z - Omega z| <= tol Omega |z| for every pair; otherwise the last iterate
 * with BSE_INFO_NOT_CONVERGED.  Synchronises the stream every iteration. */
bse_status bse_full_lowest(bse_plan* plan, int32_t n_block, int32_t max_iter, double tol, const void* X0,
                           double* omega, void* xy_out, int32_t* iters, void* hip_stream);
bse_status bse_apply_coupling(bse_plan* plan, const void* X, void* Y, int32_t nb, void* hip_stream);
bse_status bse_apply_full(bse_plan* plan, const void* XY, void* out, int32_t nb, void* hip_stream);
bse_status bse_full_spectrum(bse_plan* plan, const void* P, int32_t nb, int32_t n_steps, const double* omega,
                             int32_t n_w, double eta, double* S, double* a, double* b, int32_t* steps_done,
                             void* hip_stream);

/* ---------------------------------------------------------------------------
 * Stage timing (tracing): when enabled, HIP events are recorded on the call's
 * stream around every stage launched by bse_apply / bse_apply_adjoint /
 * bse_haydock_spectrum, and bse_plan_stage_times() synchronises on them and
 * returns accumulated milliseconds and launch counts per stage.
 * ------------------------------------------------------------------------- */
typedef enum {
    BSE_STAGE_PAIRDENS_V = 0, /* valence pair densities M_vv' from the halves (1 kernel)    */
    BSE_STAGE_WSTEP = 1,      /* P = conj(M_v) W(q) (1 kernel)                             */
    BSE_STAGE_DBLOCK = 2,     /* direct block T = M_c P (1 kernel)                         */
    BSE_STAGE_TX = 3,         /* Y(k) -= T X(k') (1 kernel)                                */
    BSE_STAGE_EXCHANGE = 4,   /* rho Vbar rho^H X                                          */
    BSE_STAGE_DIAG = 5,       /* transition energies                                       */
    BSE_STAGE_LANCZOS = 6,    /* recurrence, CGS2 and continued fraction                   */
    BSE_STAGE_ADJOINT = 7,    /* adjoint-only contractions                                 */
    BSE_STAGE_PAIRDENS_C = 8, /* conduction pair densities M_cc' from the halves (1 kernel) */
    BSE_STAGE_TABLES = 9,     /* gather tables of a q batch                                */
    BSE_STAGE_COUPLING = 10,  /* direct term of the coupling block B (full BSE)            */
    BSE_NSTAGES = 11
} bse_stage;
bse_status bse_plan_set_timing(bse_plan* plan, int enable);
/* ms, launches: host arrays of BSE_NSTAGES entries; reset != 0 clears the totals */
bse_status bse_plan_stage_times(bse_plan* plan, double* ms, int64_t* launches, int reset);

const char* bse_status_string(bse_status s);
const char* bse_last_error(void);
/* Library version string. */
const char* bse_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BSE_H */
