/*
 * hrom.h -- C ABI of the MI355X (gfx950) hyper-reduced RVE evaluation.
 *
 * The library evaluates the hyper-reduced RVE of the monolithic hyper ROM FE2
 * method (Lange, Huetter, Kiefer, arXiv 2306.02687) at every macroscopic
 * Gauss point ("macro point"), on one GPU.  At each ECM point q of the RVE
 * cluster it forms the reduced kinematics F_q = Fr + sum_m a_m G_qm
 * (Sec. 3.2.1, eq. ROM_assumption), evaluates the compressible Neo-Hooke
 * stress P_q and tangent A_q, and accumulates with the ECM weights
 * (Sec. 3.3):
 *   r   = sum_q w_q G_q^T P_q           (eq. ROMintforce)
 *   Kaa = sum_q G_q^T (w_q A_q) G_q     (eq. ROMstiffness)
 *   KaF = sum_q w_q G_q^T A_q,  KFF = sum_q w_q A_q,  Pr = sum_q w_q P_q.
 * It then condenses the ROM amplitudes statically (Sec. 3.2.3):
 *   Palg = Pr - KaF^T Kaa^{-1} r,   Cr = KFF - KaF^T Kaa^{-1} KaF
 * (eq. Biot_Tangent), applies the monolithic update
 *   a <- a - Kaa^{-1} (r + KaF dFr)
 * and differentiates the converged map by an adjoint solve.
 *
 * Frames.  With HROM_OBJECTIVE the RVE sees only the right stretch Ubar of
 * the polar split Fbar = Rbar Ubar (Sec. 3.2.2, eq. ploar_decomp), so Fr =
 * Ubar; the returned macro stress is Pbar = Fbar S with Ubar S + S Ubar =
 * 2 sym(Palg) (the second-Piola form of eqs. workconjugacy / biotstress) and
 * Cbar = dPbar/dFbar.  Without the flag Fr = Fbar and Pbar = Palg, Cbar = Cr.
 * For codes in the Updated-Lagrangian form, hrom_cauchy returns the Cauchy
 * stress of the same state and the tangent dsigma/dD of the paper's App. A.
 *
 * Conventions.
 *  - 3x3 tensors are flattened row-major, I = 3 i + j; tangents are
 *    C[I][J] = dP_I / dF_J.
 *  - Per-point arrays are component-major ("SoA"): X[k * N + b] is component
 *    k of macro point b, so consecutive points are contiguous.
 *  - Mode-indexed per-point arrays (a, r, and the optional Kaa, KaF outputs)
 *    hold one block per cluster, in cluster order; cluster c's block starts
 *    at offset hrom_plan_offset(plan, c, kind) and is [k][count_c].
 *  - All array arguments are DEVICE pointers owned by the caller, except the
 *    cluster descriptor array of hrom_plan_create (host memory).
 *  - Every compute call only enqueues work on `stream` (no host sync, no
 *    allocation after plan creation).  Per-point results and status are
 *    valid after the stream is synchronised.
 *
 * Return codes: HROM_OK, or a negative HROM_E_* (nothing was enqueued).
 * Per-point failures do not fail the call; they set bits in status[N].
 */
#ifndef HROM_H
#define HROM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HROM_OK 0
#define HROM_E_INVALID (-1)   /* invalid argument (null pointer, bad size) */
#define HROM_E_HIP (-2)       /* a HIP runtime call failed */
#define HROM_E_ORDER (-3)     /* call sequence violated, e.g. condense before eval */
#define HROM_E_NOMEM (-4)     /* device allocation failed at plan creation */
#define HROM_E_UNSUPPORTED (-5) /* size outside the supported range (m > 96, ...), or an
                                 output the plan's mode does not provide */
#define HROM_E_SCRATCH (-6)   /* hrom_newton_noalloc: the request does not fit its static scratch */
#define HROM_E_NOCONV (-7)    /* an iteration did not reach its tolerance (ECM: SVD sweeps, NNLS) */
#define HROM_E_RANK (-8)      /* ECM: truncation beyond the rank of the training matrix, or a
                                 selected column dependent on the others */

/* per-point status bits */
#define HROM_PT_JNONPOS 1    /* det F <= 0 at an ECM point (or det Fbar <= 0) */
#define HROM_PT_NOT_SPD 2    /* Cholesky of Kaa hit a non-positive pivot; LU used */
#define HROM_PT_NOCONV 4     /* Newton did not reach the tolerance */
#define HROM_PT_NONFINITE 8  /* non-finite input or output, or singular Kaa */
#define HROM_PT_NOREFINE 16  /* hrom_backward with HROM_REFINE: after the last of the 3
                                refinement steps the adjoint correction was still above 1e-5
                                of lambda (lambda not known to the mixed path's accuracy) */

/* arithmetic of the evaluation (Sec. 3.2 blocks).  The mixed modes require
 * HROM_SPLIT (plan creation returns HROM_E_UNSUPPORTED without it): they are
 * within 1e-5 (relative, per point) of the FP64 result on Pbar, Cbar and the
 * adjoint gradients; the FP64 mode within 1e-12. */
#define HROM_FP64 0          /* everything in double precision (FP64 MFMA) */
#define HROM_MIXED_BF16 1    /* Kaa, KaF, KFF contraction on BF16 MFMA, FP32 accumulation;
                                residual, factorisation, Schur complement in FP64 */
#define HROM_MIXED_FP16 2    /* same with FP16 MFMA */

/* plan flags */
#define HROM_OBJECTIVE 1u    /* RVE sees Ubar of Fbar = Rbar Ubar (Sec. 3.2.2) */
#define HROM_SPLIT 2u        /* mixed modes: hi/lo split operands (3 MFMA terms); required */
#define HROM_J2 8u           /* material: small-strain J2 plasticity with linear isotropic
                                hardening and history at the ECM points (Sec. 5 Example 1,
                                Sec. 4); FP64 or mixed (split) plans, the law and the
                                history in FP64; theta = device [8] */
#define HROM_BIOT6 16u       /* objective plans: condense only the six coordinates of the
                                symmetric stretch (KaU = KaF E6, six right-hand sides; the
                                paper's Biot form, Sec. 3.2.2-3.2.3): the same Pbar, Cbar,
                                update and adjoint, one trailing block less to eliminate */
#define HROM_REFINE 4u       /* mixed modes: the adjoint with the FP64 operator (FP64 tangent
                                in the re-evaluation), lambda by iterative refinement whose
                                residual uses that operator and whose correction uses the
                                low-precision factor (per point at most 3 steps, stopping once
                                a correction is below 1e-6 of lambda) */

/* offset kinds for hrom_plan_offset */
#define HROM_OFF_A 0         /* a, r, y: [m_c][count_c] */
#define HROM_OFF_KAA 1       /* Kaa output: [m_c * m_c][count_c] */
#define HROM_OFF_KAF 2       /* KaF output: [m_c * 9][count_c] */

/* One RVE cluster (Sec. 3.3, hyper integration points and weights; the
 * element ROM modes of Sec. 4 enter as mode gradients at the ECM points). */
typedef struct {
    int32_t m;              /* ROM modes, 1 <= m <= 96 */
    int32_t Q;              /* ECM points, Q >= 1 */
    const double* G;        /* device [Q][9][m]: gradient of mode m at point q */
    const double* w;        /* device [Q]: ECM weights; every ECM sum is divided by their sum,
                               the RVE measure V0 (volume averages, Sec. 3.3) */
    const int32_t* phase;   /* device [Q]: 0 = matrix, 1 = inclusion */
    int64_t first;          /* macro points [first, first + count) use this cluster */
    int64_t count;
} hrom_cluster;

typedef struct hrom_plan_s* hrom_plan;

/* Create a plan for N macro points partitioned into ncl clusters (contiguous,
 * in order, covering [0, N)): the RVE clusters of Sec. 3.4 with their hyper
 * integration points and weights of Sec. 3.3.  Reads G, w, phase once
 * (synchronously) to build the device layouts the kernels use, in the mode
 * basis orthonormal in the weighted gradient inner product (the caller's
 * arrays stay in the caller's basis); allocates the per-point workspace.
 * HROM_E_INVALID for linearly dependent mode gradients.
 * Ownership: the plan owns its workspace; the caller keeps G, w, phase. */
int hrom_plan_create(hrom_plan* out, const hrom_cluster* clusters, int32_t ncl, int64_t N,
                     int32_t precision, uint32_t flags);
int hrom_plan_destroy(hrom_plan plan);

/* offset (in elements) of cluster c's block in mode-indexed arrays, and the
 * total length of such an array (c = ncl) */
int64_t hrom_plan_offset(hrom_plan plan, int32_t c, int32_t kind);

/* Evaluate at (Fbar, a) (Sec. 3.2.1 eqs. ROM_assumption, ROMintforce,
 * ROMstiffness with the ECM sums of Sec. 3.3; the polar split of Sec. 3.2.2
 * eq. ploar_decomp in objective plans): theta = device [4] (mu_0, lam_0,
 * mu_1, lam_1), or [8] for J2 plans.  Fbar [9][N], a (mode-indexed).  Writes
 * status[N] (overwrites).  Optional test outputs (NULL = not written), all in
 * the RVE frame: r (mode-indexed), Pr [9][N], Kaa [m*m][count] blocks, KaF
 * [m*9][count] blocks, KFF [81][N]. */
int hrom_eval(hrom_plan plan, const double* theta, const double* Fbar, const double* a,
              double* r, double* Pr, double* Kaa, double* KaF, double* KFF,
              int32_t* status, hipStream_t stream);

/* Condense the state left by the last hrom_eval (Sec. 3.2.3, eq.
 * Biot_Tangent: Palg = Pr - KaF^T Kaa^{-1} r, Cr = KFF - KaF^T Kaa^{-1} KaF,
 * factorised, never inverted, Sec. 4), then push out to the macro frame
 * (Sec. 3.2.2 eqs. workconjugacy, biotstress): Pbar [9][N] (algorithmic
 * stress, macro frame), Cbar [81][N], rnorm [N] = ||r||_2.  ORs status bits. */
int hrom_condense(hrom_plan plan, double* Pbar, double* Cbar, double* rnorm,
                  int32_t* status, hipStream_t stream);

/* Updated-Lagrangian output of the state left by the last hrom_condense
 * (objective plans only, else HROM_E_UNSUPPORTED; HROM_E_ORDER before a
 * condense): the Cauchy stress sigma [9][N] (3x3 row-major, symmetric) from
 * the Biot stress sym(Palg_r) by Sec. 3.2.2 eq. (biotstress), and, unless
 * dsdD is NULL, the consistent tangent dsdD [81][N], entry 9 (3i+j) + 3k+l =
 * dsigma_ij / dD_kl, by the product rule of App. A with C^B = the condensed
 * RVE-frame tangent on symmetric stretch rates and dUdot/dD ~ R_ki F_lj
 * (constant rotation over the step).  Device pointers owned by the caller;
 * ORs HROM_PT_NONFINITE into status for non-finite outputs.  Allocates
 * nothing; does not change the plan's state. */
int hrom_cauchy(hrom_plan plan, double* sigma, double* dsdD, int32_t* status, hipStream_t stream);

/* Biot form of the state left by the last hrom_condense (objective plans,
 * else HROM_E_UNSUPPORTED; HROM_E_ORDER before a condense): the Biot stress
 * T [6][N] = sym(Palg_r) in Voigt order (11, 22, 33, 12, 23, 13), work
 * conjugate to the stretch Ubar (Sec. 3.2.2 eq. workconjugacy), and unless
 * CB is NULL the condensed Biot tangent CB [36][N], entry 6 k + l =
 * dT_k / dgamma_l with gamma = (U11, U22, U33, 2 U12, 2 U23, 2 U13) (Sec.
 * 3.2.3 eq. Biot_Tangent on symmetric stretch increments), the interface of
 * codes that impose the stretch.  ORs HROM_PT_NONFINITE into status. */
int hrom_biot(hrom_plan plan, double* T, double* CB, int32_t* status, hipStream_t stream);

/* Monolithic update a <- a - (y + X dFr) with the y, X of the last condense
 * (Sec. 3.2.3, the amplitude increment of the monolithic scheme).  dFbar [9][N] macro-frame increment (linearised to the stretch
 * increment in objective mode), or NULL for a pure micro Newton step; with
 * dFbar == NULL, points whose last rnorm < tol are left unchanged (frozen).
 * Points whose status (of the last eval/condense) has JNONPOS or NONFINITE
 * are never changed.  After an update, the next call must be hrom_eval. */
int hrom_update(hrom_plan plan, const double* dFbar, double tol, double* a,
                const int32_t* status, hipStream_t stream);

/* Micro Newton at fixed Fbar (the staggered micro solve that the monolithic
 * scheme of Sec. 3.2.3 replaces by one update per macro iteration; used to
 * converge the RVE state), max_it evaluations with no host sync (so it can
 * be captured in a HIP graph): max_it - 1 times {eval, condense, update with
 * converged points frozen}, then a final eval + condense.  Points still at
 * rnorm >= tol get HROM_PT_NOCONV.  Pbar, Cbar, rnorm as in hrom_condense. */
int hrom_newton(hrom_plan plan, const double* theta, const double* Fbar, double* a, double tol,
                int32_t max_it, double* Pbar, double* Cbar, double* rnorm, int32_t* status,
                hipStream_t stream);

/* Adjoint backward of the converged map (Fbar, theta) -> Pbar (the
 * derivative of the condensed problem of Sec. 3.2.3: the adjoint system is the
 * transpose of eq. Biot_Tangent's Kaa solve) at the state of the last eval +
 * condense (which must have been at this a and theta, i.e.
 * no update in between).  gPbar [9][N] = dL/dPbar.  Pull-back to the RVE
 * frame g_r, adjoint solve lambda = Kaa^{-T} KaF g_r with the stored solve
 * (mixed modes: plus one refinement step with the accurate operator),
 * re-evaluation of F_q and A_q at every ECM point (nothing of size Q is
 * stored), then dL/dFbar [9][N] and dL/dtheta [4] (sum over all points in a
 * fixed order: bitwise reproducible). */
int hrom_backward(hrom_plan plan, const double* theta, const double* a, const double* gPbar,
                  double* gFbar, double* gtheta, int32_t* status, hipStream_t stream);

/* J2 plans (HROM_J2): every evaluation starts from the committed history
 * of the ECM points (plastic strain xx yy zz xy yz xz and equivalent plastic
 * strain alpha, zero at plan creation) and leaves the history of its state;
 * theta = device [8], per phase (mu, lambda, sigma_y0, H): strain
 * eps = sym(F) - I, radial return with linear isotropic hardening
 * sigma_y = sigma_y0 + H alpha, P = sigma and A = the consistent tangent
 * (Sec. 5 Example 1 material; a phase with sigma_y0 beyond reach stays
 * elastic).  hrom_commit makes the history of the last evaluation the
 * committed one (call it after the macro increment is accepted, e.g. after a
 * converged hrom_newton); hrom_history copies the committed (which = 0) or
 * last-evaluated (which = 1) history into out, one [count_c][Q_c][7] block
 * per cluster in cluster order.  HROM_E_UNSUPPORTED for plans without
 * HROM_J2; hrom_backward returns HROM_E_UNSUPPORTED for J2 plans. */
int hrom_commit(hrom_plan plan, hipStream_t stream);
int hrom_history(hrom_plan plan, int32_t which, double* out, hipStream_t stream);

/* Launch variants of the tangent contraction, chosen by the autotuner.
 * Single-cluster plans, variants 0..3: bit 0 asks for four wavefronts per
 * SIMD instead of three (mixed kernels), bit 1 turns off the prefetch of the
 * next ECM point's mode-gradient operands; variants 4 and 5 (mixed kernels,
 * m <= 64; otherwise as variant 2 and 0) put two macro points on each
 * wavefront, sharing every mode-gradient operand, without / with that
 * prefetch (the FP64 kernel reads both as variant 0).  Plans with
 * several clusters: FP64 plans give their persistent tangent launch
 * (variant + 1) x #CUs workgroups; mixed plans launch the tangent once per
 * cluster with that cluster's variant, as above.  c = -1 applies to every
 * cluster.  Results do not depend on the
 * variant (same arithmetic, same order). */
int32_t hrom_num_variants(void);
int hrom_plan_set_variant(hrom_plan plan, int32_t c, int32_t variant);

/* Launch variants of the other kernels (autotuner hooks; results never change,
 * only speed), per cluster c (-1: every cluster):
 *  HROM_VK_TANGENT  the tangent contraction (same as hrom_plan_set_variant);
 *  HROM_VK_KIN      the kinematics: 0 four wavefronts per 32-point workgroup
 *                   (two workgroups per CU), 1 eight wavefronts;
 *  HROM_VK_CONDENSE the register condensation: 0 the register budget of three
 *                   wavefronts per SIMD, 1 of two (no spills) -- m <= 64 only,
 *                   larger mode counts always run at two.
 * hrom_num_kernel_variants returns the count of a kind (0 for an unknown one). */
#define HROM_VK_TANGENT 0
#define HROM_VK_KIN 1
#define HROM_VK_CONDENSE 2
int32_t hrom_num_kernel_variants(int32_t kind);
int hrom_plan_set_kernel_variant(hrom_plan plan, int32_t kind, int32_t c, int32_t variant);

/* Measurement hook (not part of the method): with enable != 0 every later
 * hrom_eval records two HIP events on its stream around the tangent
 * contraction (all tangent launches of a plan with several clusters, the
 * single tangent launch of a one-cluster plan).  hrom_plan_tangent_ms waits for the second
 * event and returns the elapsed milliseconds of the last recorded launch;
 * HROM_E_ORDER if profiling is off.  The events are created on the first
 * enable and destroyed with the plan. */
int hrom_plan_profile(hrom_plan plan, int32_t enable);
int hrom_plan_tangent_ms(hrom_plan plan, float* ms);

/* Allocation-free micro Newton, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same work and the same results as hrom_plan_create
 * + hrom_newton (launch variant 0, one launch per cluster for every step),
 * with every buffer of the plan -- device layouts of G, w, phase and the
 * per-point workspace -- carved from a static device array of
 * hrom_noalloc_scratch_bytes() bytes (64 MiB) that each GPU the library runs
 * on holds until the process ends.  The layouts are rebuilt from the
 * caller's G, w, phase on `stream` at every call.  Arguments are those of
 * hrom_plan_create (clusters: host array, at most 16 entries) and
 * hrom_newton (device pointers owned by the caller; a updated in place).
 * Calls no hipMalloc / hipFree and performs no host sync.
 * Returns HROM_E_SCRATCH (nothing enqueued) when the plan would need more
 * than the scratch, HROM_E_UNSUPPORTED for more than 16 clusters.  Every call
 * on one GPU shares that GPU's array, which keeps the last call's contents
 * (no buffer needs to start at zero): calls on one GPU must be ordered (the
 * same stream, or synchronised); calls that overlap on one GPU race. */
int hrom_newton_noalloc(const hrom_cluster* clusters, int32_t ncl, int64_t N, int32_t precision,
                        uint32_t flags, const double* theta, const double* Fbar, double* a,
                        double tol, int32_t max_it, double* Pbar, double* Cbar, double* rnorm,
                        int32_t* status, hipStream_t stream);
size_t hrom_noalloc_scratch_bytes(void);

/* ---------------------------------------------------------------------------
 * Empirical cubature: the offline selection of the ECM points and weights
 * (Sec. 3.3).  The three calls run in order on the full set of M candidate
 * integration points; each allocates its own device workspace, runs on
 * `stream` and returns after synchronising it.  All array arguments are
 * device pointers owned by the caller unless marked host.
 * ------------------------------------------------------------------------- */

/* Training matrix x_f (Sec. 3.3, eq. ECM1 and the matrix after it).  The
 * candidates: mode gradients G [M][9][m] (the layout of hrom_cluster.G),
 * weights w [M] (V0 = sum w), phase [M]; theta [4] Neo-Hooke moduli.  The p
 * snapshots: RVE-frame macro input Fr [p][9] and converged mode
 * coefficients a [p][m].  For snapshot k and candidate g the integrand is the
 * point's force vector f^{kg} = [G_g^T P(F_g); P(F_g)] (m mode forces and the
 * nine first Piola components), F_g = Fr^k + G_g a^k.  Outputs:
 * xf [p (m + 9)][M], row k (m + 9) + i holding f^{kg}_i - f^k_i / V0, and
 * fint [p (m + 9)] the integrals f^k_i = sum_g w_g f^{kg}_i.  *nbad (host,
 * may be null) receives the number of (snapshot, candidate) pairs with
 * det F_g <= 0, whose entries are zero.  Errors: HROM_E_INVALID (sizes,
 * null pointers), HROM_E_NOMEM, HROM_E_HIP. */
int hrom_ecm_training(int32_t m, int32_t M, const double* G, const double* w, const int32_t* phase,
                      const double* theta, int32_t p, const double* Fr, const double* a, double* xf,
                      double* fint, int32_t* nbad, hipStream_t stream);

/* Truncated basis of eq. SVDlambda: x_f^T = lambda sigma v^T.  xf [P][M] is
 * read only.  lam [M][r] receives the r leading left singular vectors of
 * x_f^T (candidate-major: lam[g r + j]); sigma [P] all singular values in
 * decreasing order.  tol: orthogonality of the Jacobi columns relative to
 * their norms (<= 0: 1e-13); max_sweeps (<= 0: 40).  method: 1 runs the
 * one-sided Jacobi sweeps on x_f^T itself; 2 first factors x_f^T = Q R by
 * Householder reflectors (needs M >= Ppad, P rounded up to an even number of
 * 32-column blocks), then R^T Pi = Q2 R2 with column pivoting, sweeps the
 * P x P matrix R2^T and returns Q Pi times its left vectors (the same
 * singular values; every sweep over P rows in place of M, and a third of the
 * sweeps on the pivoted triangle); 0 takes 2 when M >= 2 Ppad, else 1.  *sweeps (host, may be null) the
 * sweeps used; off_hist (host, may be null, max_sweeps entries) the largest
 * relative off-diagonal Gram entry met in each sweep.  Singular vectors are
 * determined up to sign (and rotation within equal singular values), which
 * the selection does not see.  Errors: HROM_E_INVALID (r > P, method outside
 * 0..2, method 2 with M < Ppad, ...), HROM_E_NOCONV (sweeps exhausted;
 * outputs written), HROM_E_RANK (sigma_r <= max(M, P) eps sigma_1: x_f has
 * fewer than r numerically independent directions; outputs written),
 * HROM_E_NOMEM, HROM_E_HIP. */
int hrom_ecm_svd(int32_t P, int32_t M, const double* xf, int32_t r, double* lam, double* sigma, double tol,
                 int32_t max_sweeps, int32_t method, int32_t* sweeps, double* off_hist, hipStream_t stream);

/* Greedy selection of Box 1 on J = [lambda 1]^T, b = [0 ... 0 V0]: picks the
 * available candidate of largest j_k . res / |j_k| (lowest index on ties),
 * solves the least-squares problem on the selection, falls back to the
 * non-negative one when a weight is negative and drops the points it gives
 * zero weight for good, with res = b - J_z w; ends at mt points or when no
 * candidate is left.  lam [M][r] as returned by hrom_ecm_svd, r + 1 <= 1024,
 * 1 <= mt <= r + 1.  Outputs: z [mt] candidate indices in pick order and
 * w [mt] their weights (the first *n_sel entries are valid; host n_sel),
 * *iters (host) the iterations, trace [trace_cap][4] (may be null) per
 * iteration: picked candidate, 1 if the NNLS ran, points dropped, selection
 * size after it.  Errors: HROM_E_INVALID, HROM_E_RANK (a picked column
 * dependent on the selection), HROM_E_NOCONV (NNLS iteration limit),
 * HROM_E_NOMEM, HROM_E_HIP. */
int hrom_ecm_select(int32_t M, int32_t r, const double* lam, double V0, int32_t mt, int32_t* z, double* w,
                    int32_t* n_sel, int32_t* trace, int32_t trace_cap, int32_t* iters, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Clustered training (Sec. 3.4, Box 2) and the POD basis (Sec. 3.2.1).
 * Each call allocates its own device workspace and returns after
 * synchronising `stream`; array arguments are device pointers owned by the
 * caller unless marked host.
 * ------------------------------------------------------------------------- */

/* Box 2, steps 2 and 3: E [d][N] (component-major) macro strain states of N
 * points, d <= 8 components; every component is scaled by its root mean square
 * over the points, then Lloyd's k-means (k <= 1024 centres, started from the
 * points init_idx [k]) runs until no label changes: every point to its nearest
 * centre (squared Euclidean distance, ties to the lowest centre index), every
 * centre to the mean of its points (a centre without points stays).  Outputs:
 * centres [k][d] in the units of E, labels [N]; *iters (host, may be null) the
 * iterations.  Errors: HROM_E_INVALID, HROM_E_NOCONV (max_iter reached;
 * outputs of the last iteration written), HROM_E_NOMEM, HROM_E_HIP. */
int hrom_training_clusters(int64_t N, int32_t d, const double* E, int32_t k, const int32_t* init_idx,
                           int32_t max_iter, double* centres, int32_t* labels, int32_t* iters,
                           hipStream_t stream);

/* Monotonic training trajectories from cluster centres (Box 2, step 4):
 * centres [k][6] (strain xx yy zz xy yz xz, tensor shear components); for step
 * j = 1 .. n_steps, Fr[c n_steps + j - 1] = I + (j / n_steps) H(c), H
 * symmetric, as [k n_steps][9] row-major 3x3 (RVE-frame macro inputs).  Only
 * enqueues on `stream`.  Errors: HROM_E_INVALID, HROM_E_HIP. */
int hrom_training_paths(int32_t k, const double* centres, int32_t n_steps, double* Fr, hipStream_t stream);

/* POD with the elastic-inelastic split (Sec. 3.2.1, eqs. SVD_displacement and
 * snapshots_displacement): X_el [s_el][nd] elastic and X_in [s_in][nd]
 * inelastic displacement snapshots (one snapshot of nd nodal values per row).
 * Phi [nd][n_el + n_in] receives the n_el leading left singular vectors of the
 * elastic snapshots, then the n_in leading ones of the inelastic snapshots
 * without their part in that span; sigma_el [s_el], sigma_in [s_in] all
 * singular values.  Errors: HROM_E_INVALID (n_el > s_el, ...), HROM_E_RANK
 * (fewer independent snapshots than modes asked), HROM_E_NOCONV, HROM_E_NOMEM,
 * HROM_E_HIP. */
int hrom_pod(int32_t nd, int32_t s_el, const double* X_el, int32_t s_in, const double* X_in, int32_t n_el,
             int32_t n_in, double* Phi, double* sigma_el, double* sigma_in, hipStream_t stream);

const char* hrom_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* HROM_H */
