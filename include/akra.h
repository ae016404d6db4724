/*
 * akra.h -- C ABI of libakra: the matrix-free normal-equation operator of AKRA 3.0
 * (Shi, Zhang, Cui, Qin, Yao) on an AMD Instinct MI355X (gfx950).
 *
 * The method (paper Sec. II.B, "AKRA 3.0: matrix-free inversion framework"):
 *   convergence harmonics x = (kappa_E, kappa_B)  --  joint E/B unknowns, App. A eq. joint_forward
 *   A = Y o K : harmonic diagonal K_l = sigma_D D_l (eq. Dl_kernel), then the inverse spin-2
 *               transform Y to shear gamma = gamma_1 + i gamma_2 at HEALPix RING pixel centres
 *               (shear expansion eq. shear_SH with 2a = -(a_E + i a_B), eq. EB_decomp)
 *   N^-1, M  : per-pixel inverse noise and binary mask, folded once into W_p = M_p N^-1_p
 *              (pixel-space diagonal of the storage problem; eq. noise_var, eq. mask)
 *   H v = K Y^H ( W (Y (K v)) ) + lambda_eff v                  (eq. normal_eq, eq. ML_estimator_reg)
 *   b   = K Y^H ( W gamma_obs )
 *   solved by preconditioned conjugate gradient with P = (<M^2 N^-1> + lambda_eff)^-1 I
 *   (eq. precond), x0 = 0 by default, stopping at ||r_k|| / ||b|| < tol (Sec. III.C).
 * Y^H is the exact adjoint of Y for the pixel product <g,h> = sum_p Omega Re(conj(g_p) h_p),
 * Omega = 4 pi / Npix, and the full-m harmonic product
 *   <a,b> = sum_l [ Re(a_l0* b_l0) + 2 sum_{m>0} Re(a_lm* b_lm) ].
 * lambda_eff = lambda <N^-1>_M (mean of N^-1 over unmasked pixels), lambda = 1e-3 by default.
 *
 * Data layout (all arrays are DEVICE pointers owned by the caller unless stated):
 *   alm   complex128 interleaved (re, im), m >= 0 only, index i(l,m) = m (2 lmax + 1 - m)/2 + l,
 *         n_alm = (lmax+1)(lmax+2)/2 entries per field.  A real field has a_{l,-m} = (-1)^m conj(a_lm).
 *         On input, entries with l < 2 are ignored by Y and Im(a_l0) is ignored everywhere;
 *         on output Im(a_l0) = 0 and Y^H / b have zero entries at l < 2.
 *   maps  float64 [Npix] in HEALPix RING order, Npix = 12 nside^2 (gamma_1 and gamma_2 separate).
 *   ninv  float64 [Npix] (>= 0, finite), mask uint8 [Npix] (0 = masked, nonzero = observed).
 *   Batched plans (nrhs > 1): alm, maps and ninv carry a leading [nrhs] dimension, contiguous;
 *   the mask is shared by all right-hand sides.
 *
 * Streams and ownership: every call is ordered on the plan's HIP stream.  The plan owns all
 * tables and scratch; calls allocate no device memory after akra_plan_create, except that
 * akra_cg_solve* allocate nothing either (all solver vectors live in the plan).  Outputs must
 * not alias inputs, except x in akra_cg_solve*, which is both the start vector (opts->use_x0)
 * and the result.  Calls on one plan must not overlap from several host threads.
 *
 * Errors: every call returns an akra_status; nothing throws across the ABI and nothing aborts.
 * akra_last_error() returns a thread-local message for the last failing call on this thread.
 */
#ifndef AKRA_H
#define AKRA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct akra_plan_s *akra_plan;

typedef enum {
    AKRA_OK = 0,
    AKRA_ERR_ARG = 1,        /* invalid argument (sizes, null pointers, negative weights)        */
    AKRA_ERR_ALLOC = 2,      /* device or host allocation failed                                 */
    AKRA_ERR_HIP = 3,        /* a HIP runtime call or kernel launch failed                        */
    AKRA_ERR_NUMERIC = 4,    /* NaN/Inf in the inputs, or CG breakdown (p^T H p <= 0)             */
    AKRA_NOT_CONVERGED = 5,  /* maxiter reached; x holds the last iterate                         */
    AKRA_STAGNATED = 6       /* ||r|| reached no new minimum in opts->stall_iters iterations;     */
                             /* x holds the last iterate                                          */
} akra_status;

typedef enum {
    AKRA_FP64 = 0,           /* transforms in FP64                                                */
    AKRA_FP32 = 1            /* transforms in FP32 (recurrence seeds and rescaling in FP64);      */
                             /* solves refine in FP64 to the requested tolerance                  */
} akra_precision;

/*
 * Unknowns of a solve (App. A, eq. normal_block).  JOINT_EB solves the full 2x2 block system for
 * x = (kappa_E, kappa_B).  E_ONLY solves the E block (H_EE + lambda_eff) kappa_E = b_E of the E-mode
 * reconstruction of the main text: kappa_B is held at zero and returned as zero.  B_ONLY solves
 * (H_BB + lambda_eff) kappa_B = b_B with kappa_E held at zero (the reduced system of eq.
 * Bmode_reduced when the right-hand side is given, see akra_cg_solve_cond_b).
 */
typedef enum {
    AKRA_JOINT_EB = 0,
    AKRA_E_ONLY = 1,
    AKRA_B_ONLY = 2
} akra_mode;

typedef struct {
    double lambda;           /* regulariser lambda (default 1e-3, Sec. II.B)                      */
    double tol;              /* ||r|| / ||b|| target (default 1e-3, Sec. III.C)                  */
    int maxiter;             /* iteration cap (default 1000)                                      */
    int use_x0;              /* nonzero: x holds the start vector on entry (default 0: x0 = 0)   */
    const double *kernel_l;  /* HOST array [lmax+1]: harmonic kernel K_l; NULL = sigma_D D_l     */
                             /* with sigma_D = -1 (eq. Dl_kernel)                                  */
    double reliable_delta;   /* FP32 plans: replace the residual by the FP64 true residual once  */
                             /* ||r|| drops by this factor (default 0.1)                         */
    double *resid_hist;      /* HOST, optional: relative residual after each iteration           */
    int resid_hist_len;
    int mode;                /* akra_mode of the unknowns (default AKRA_JOINT_EB)                 */
    int stall_iters;         /* > 0: stop with AKRA_STAGNATED once the relative residual has not  */
                             /* fallen below its smallest earlier value for this many iterations  */
                             /* (the residual the convergence test sees); 0 (default): off        */
    int check_every;         /* > 1: iterations between convergence tests, run back to back with */
                             /* one host synchronisation per test (single-RHS and flat solves);   */
                             /* the history is written at tested iterations only, stall_iters    */
                             /* counts tests, and a solve may run up to check_every - 1           */
                             /* iterations past the one that met tol; 0 or 1 (default): every     */
                             /* iteration                                                        */
} akra_cg_opts;

typedef struct {
    int iters;               /* CG iterations (operator applies in the iteration's precision)    */
    int fp64_applies;        /* FP64 applies used for true residuals (FP32 plans)                */
    double rel_resid;        /* last recursive ||r|| / ||b||                                      */
    double rel_resid_true;   /* ||b - H x|| / ||b|| recomputed in FP64 at exit                    */
    double lambda_eff;       /* lambda <N^-1>_M actually used                                     */
    double precond;          /* scalar P actually used                                            */
    double ms_total;         /* wall time of the call                                             */
    int status;              /* akra_status of the solve                                          */
} akra_cg_info;

/* Default options (lambda 1e-3, tol 1e-3, maxiter 1000, x0 = 0, kernel sigma_D D_l, joint E/B,
 * no stagnation test). */
void akra_cg_opts_default(akra_cg_opts *opts);

/*
 * Create a plan for HEALPix nside with band limit lmax (2 <= lmax <= 4 nside, nside <= 2048 for FP64
 * plans, 1 <= nrhs <= 64), on the HIP stream `hip_stream` (hipStream_t, NULL = default stream) of the
 * current device.  Builds the ring geometry, the Wigner-d recurrence tables and per-(m, ring) seeds
 * (scaled-exponent FP64), FFT twiddles and all workspaces.  Errors: AKRA_ERR_ARG, AKRA_ERR_ALLOC,
 * AKRA_ERR_HIP.  The plan is released with akra_plan_destroy.
 */
akra_status akra_plan_create(int nside, int lmax, int nrhs, int precision, void *hip_stream, akra_plan *out);
void akra_plan_destroy(akra_plan plan);
const char *akra_last_error(void);

/* Device bytes held by the plan (tables + workspaces). */
int64_t akra_plan_device_bytes(akra_plan plan);

/*
 * Y: spin-2 synthesis (shear expansion eq. shear_SH, eq. EB_decomp), no harmonic kernel:
 *   g1 + i g2 = sum_{l>=2} sum_{m=-l..l} 2a_lm 2Y_lm(pixel centre),  2a_lm = -(almE_lm + i almB_lm).
 * In: almE, almB (alm layout).  Out: g1, g2 (maps).
 */
akra_status akra_synth2(akra_plan plan, const double *almE, const double *almB, double *g1, double *g2);

/*
 * Y^H: exact adjoint of akra_synth2 (pixel product with Omega = 4 pi/Npix, full-m harmonic product):
 *   2h_lm = sum_p Omega conj(2Y_lm(p)) h_p,  -2h_lm = sum_p Omega conj(-2Y_lm(p)) conj(h_p),
 *   almE = -(2h + -2h)/2,  almB = (i/2)(2h - -2h)   (eq. EB_decomp), h = g1 + i g2.
 * In: g1, g2 (maps).  Out: almE, almB (alm layout).
 */
akra_status akra_adjoint2(akra_plan plan, const double *g1, const double *g2, double *almE, double *almB);

/*
 * H v = K Y^H (W (Y (K v))) + lambda_eff v with W_p = mask_p * ninv_p (eq. normal_eq; the operator
 * chain diagonal -> SHT^-1 -> diagonal -> SHT of the storage problem).  kernel_l: HOST [lmax+1] or
 * NULL (sigma_D D_l).  lambda_eff is used as given.  In: ninv, mask, xE, xB.  Out: yE, yB.
 * Errors: AKRA_ERR_NUMERIC when ninv holds NaN/Inf, AKRA_ERR_ARG when a weight is negative.
 */
akra_status akra_apply_H(akra_plan plan, const double *ninv, const uint8_t *mask, const double *kernel_l,
                         double lambda_eff, const double *xE, const double *xB, double *yE, double *yB);

/* b = K Y^H (W gamma_obs) (right-hand side of eq. normal_eq).  In: g1, g2, ninv, mask.  Out: bE, bB. */
akra_status akra_rhs(akra_plan plan, const double *g1, const double *g2, const double *ninv, const uint8_t *mask,
                     const double *kernel_l, double *bE, double *bB);

/*
 * Regularised ML estimate x = (H)^-1 b for the shear maps g1, g2 (eq. ML_estimator_reg) by PCG
 * (Sec. II.B inversion problem).  FP64 plans iterate in FP64; FP32 plans iterate with the FP32
 * operator and replace the residual by the FP64 true residual b - H x whenever it has dropped by
 * opts->reliable_delta (reliable updates), so the result meets tol in FP64.  Should the FP32 operator
 * no longer resolve a search direction (p^T H p <= 0, which can happen for tolerances near its
 * accuracy on ill-conditioned systems), the solve restarts from the true residual and finishes
 * with the FP64 operator; info->fp64_applies counts those iterations too.  If that stalls as well
 * (tol below the attainable accuracy of the system), the call returns AKRA_NOT_CONVERGED with the
 * last iterate and its true residual in info.
 * Out: xE, xB (alm layout), info (HOST, may be NULL).  Returns AKRA_NOT_CONVERGED (x valid) at maxiter,
 * AKRA_STAGNATED (x valid) when opts->stall_iters is set and the residual stops falling,
 * AKRA_ERR_NUMERIC on breakdown.  ||b|| = 0 gives x = 0 after 0 iterations.  With several right-hand
 * sides the status is the most severe of theirs (NOT_CONVERGED over STAGNATED over OK); a batched
 * FP32 plan stops each right-hand side on its own.
 */
akra_status akra_cg_solve(akra_plan plan, const double *g1, const double *g2, const double *ninv,
                          const uint8_t *mask, const akra_cg_opts *opts, double *xE, double *xB, akra_cg_info *info);

/*
 * Conditional B-mode solve (App. A, eq. lower_block and eq. Bmode_reduced).  Given a converged
 * E-mode solution kE (device, alm layout, [nrhs] leading), forms the effective right-hand side
 * b~_B = b_B - H_BE kE, with b_B the B block of b = K Y^H (W gamma_obs) and H_BE kE the B block of
 * H (kE, 0), both in FP64, then solves (H_BB + lambda_eff) kB = b~_B by PCG as akra_cg_solve does
 * (opts->mode is ignored; opts->use_x0 must be 0).  The stopping rule is relative to ||b~_B||.
 * In: g1, g2, ninv, mask, kE.  Out: kB (device, alm layout; must not alias kE), info (HOST, may be
 * NULL).  Errors and statuses as akra_cg_solve; AKRA_ERR_ARG for use_x0.
 */
akra_status akra_cg_solve_cond_b(akra_plan plan, const double *g1, const double *g2, const double *ninv,
                                 const uint8_t *mask, const akra_cg_opts *opts, const double *kE, double *kB,
                                 akra_cg_info *info);

/* As akra_cg_solve for a given right-hand side (bE, bB) in alm layout (used by the adjoint solve of the
 * differentiable form). */
akra_status akra_cg_solve_b(akra_plan plan, const double *ninv, const uint8_t *mask, const double *bE,
                            const double *bB, const akra_cg_opts *opts, double *xE, double *xB, akra_cg_info *info);

/*
 * Gradient of the solve (the differentiable form): for x = (xE, xB) returned by akra_cg_solve with
 * the same g1, g2, ninv, mask and opts, and the gradient vE, vB of a real loss L with respect to the
 * stored (Re, Im) of x (the convention of torch autograd), writes dL/dg1, dL/dg2 and dL/dninv
 * (maps, layout of g1 / ninv).  x enters H^-1 b through eq. normal_eq; the backward pass is one more
 * CG solve with the same self-adjoint H,
 *   u = H^-1 (v / w)   (w = 1 for m = 0, 2 for m > 0: the full-m harmonic product; Im(v_l0) ignored),
 *   dL/dg = Omega W (Y K u),   dL/dninv = M [Omega (Y K u).(g - Y K x) - (lambda / sum M) <u, x>]
 * where the last term follows lambda_eff = lambda <ninv>_M.  opts->use_x0 must be 0.  info reports
 * the backward solve.  Returns AKRA_NOT_CONVERGED (outputs valid) when that solve hits maxiter.
 */
akra_status akra_cg_solve_vjp(akra_plan plan, const double *g1, const double *g2, const double *ninv,
                              const uint8_t *mask, const akra_cg_opts *opts, const double *xE, const double *xB,
                              const double *vE, const double *vB, double *dg1, double *dg2, double *dninv,
                              akra_cg_info *info);

/*
 * Step-wise PCG on the plan's device-resident solver state (first right-hand side of the plan):
 *   akra_cg_start  forms b = K Y^H (W gamma_obs), lambda_eff and P as akra_cg_solve does, sets x0 = 0,
 *                  r0 = b, p0 = P r0 (one host synchronisation).  opts->use_x0 must be 0.
 *   akra_cg_step   runs nsteps PCG iterations (Sec. II.B inversion problem) in the plan precision,
 *                  stream-ordered with no host synchronisation and no convergence test:
 *                  w = H p, alpha = rz/<p,w>, x += alpha p, r -= alpha w, beta = P<r,r>/rz, p = P r + beta p.
 *   akra_cg_state  synchronises and returns ||r||/||b|| of the recursive residual, the iteration count,
 *                  and (if xE, xB are non-NULL device pointers) copies the iterate.  AKRA_ERR_NUMERIC on
 *                  breakdown.
 */
akra_status akra_cg_start(akra_plan plan, const double *g1, const double *g2, const double *ninv, const uint8_t *mask,
                          const akra_cg_opts *opts);
akra_status akra_cg_step(akra_plan plan, int nsteps);
akra_status akra_cg_state(akra_plan plan, double *rel_resid, int *iters, double *xE, double *xB);

/*
 * Graph replay of the PCG iteration (Sec. II.B inversion problem; the loop of akra_cg_step and of the
 * solves of akra_cg_solve, single-right-hand-side and batched lockstep): when on (the default), the
 * plan records the kernel launches of one iteration once as a HIP graph, on a private capture stream
 * of default priority, and replays it on the plan stream; it records again when lambda_eff, the
 * preconditioner, the K_l table, the precision, the right-hand side, the E/B unknowns, the Legendre
 * launch shapes or (batched) the set of right-hand sides still iterating change.  Results
 * are bit-identical to direct launches.  Stage timing (akra_plan_set_timing) always launches directly.
 * akra_plan_set_graph synchronises the plan stream; off releases the recorded graph.
 */
akra_status akra_plan_set_graph(akra_plan plan, int on);

/*
 * Stage timing: when on, every operator apply records HIP events on the plan stream around its
 * stages; akra_plan_stage_times synchronises, returns the summed milliseconds and launch counts per
 * stage in HOST arrays of AKRA_NSTAGES entries, and resets the counters.
 * Stages: 0 prologue (K_l), 1 Legendre synthesis, 2 ring stage (DFTs and weights), 3 Legendre
 * adjoint, 4 epilogue (E/B combination, K_l, lambda_eff), 5 CG vector updates.
 */
#define AKRA_NSTAGES 6

/*
 * Launch shapes of the Legendre kernels (chosen by the autotuner; results do not depend on them
 * beyond the rounding order of the adjoint's ring sums):
 *   syn_variant  0 two steps per trip, 1 four steps per trip with look-ahead loads
 *   syn_rings    ring pairs per lane of the synthesis (1, 2, 4)
 *   adj_rings, adj_waves, adj_chunk   ring pairs per lane, waves per workgroup and l-chunk of the
 *                adjoint: (R,1,8) and (R,1,4) for R = 1..8, and (1,2,8) (1,4,8) (2,2,8) (2,4,8)
 *                (4,2,8) (4,4,8) (8,2,8) (2,4,4) (4,2,4) (4,4,4).  Single-wave shapes spread a list of
 *                n 64-pair groups evenly over ceil(n / R) workgroups (at most R groups each, none
 *                with an empty slot); the others take R W consecutive groups per workgroup.  A shape
 *                covering fewer ring pairs per workgroup than the plan's partial-sum buffer allows
 *                (at least 256 pairs per workgroup when Nside > 512) is rejected with AKRA_ERR_ARG.
 * akra_plan_get_tuning writes the five current values to out5 (HOST).
 * These shapes apply to every group of an unweighted transform and to the ring groups weighted on
 * both sides in weighted applies (see akra_plan_set_skip_unweighted); akra_plan_set_tuning_one_sided
 * sets the same five values for the groups weighted on one side only (their contraction has half
 * the FMAs per loaded record or adjoint chunk, so another shape can pay), with the same rules, and
 * akra_plan_get_tuning_one_sided reads them.  A new plan starts with both equal.
 */
akra_status akra_plan_set_tuning(akra_plan plan, int syn_variant, int syn_rings, int adj_rings, int adj_waves,
                                 int adj_chunk);
akra_status akra_plan_get_tuning(akra_plan plan, int *out5);
akra_status akra_plan_set_tuning_one_sided(akra_plan plan, int syn_variant, int syn_rings, int adj_rings,
                                           int adj_waves, int adj_chunk);
akra_status akra_plan_get_tuning_one_sided(akra_plan plan, int *out5);
/*
 * Launch shapes of the batched matrix-core Legendre kernels (FP32 plans with nrhs > 1): syn_waves
 * 64-pair ring groups (one per wave) per workgroup of the batched synthesis, in {1, 2, 4, 8};
 * adj_waves groups per workgroup of the batched adjoint, in {2, 4, 8}, whose waves are summed in LDS
 * into one partial-sum slab per workgroup (fewer waves: more slabs for the epilogue to add).  The
 * default is (4, 4); results do not depend on the shapes beyond the rounding order of the adjoint's
 * sums.  Synchronises the plan stream and drops a recorded iteration.  akra_plan_get_tuning_batched
 * writes the two current values to out2 (HOST).  Errors: AKRA_ERR_ARG (other values, or a plan that
 * is not FP32 with several right-hand sides), AKRA_ERR_HIP.
 */
akra_status akra_plan_set_tuning_batched(akra_plan plan, int syn_waves, int adj_waves);
akra_status akra_plan_get_tuning_batched(akra_plan plan, int *out2);
/*
 * Work of one Legendre launch, in (l, m, ring pair) triples, written to out3 (HOST): [0] all triples
 * with max(2, m) <= l <= lmax; [1] those the synthesis evaluates and [2] those the adjoint evaluates
 * with the current launch shapes.  Below the degree where the recurrence values of a whole 64-pair
 * ring group first reach 2^-100 (FP64 plans; their sum is far under FP64 rounding) or 2^-44 (FP32
 * plans; the FP32 kernels mask them) the terms are skipped, and the kernels start from recurrence
 * states stored at plan creation.
 */
akra_status akra_plan_work(akra_plan plan, int64_t *out3);
/*
 * Work of the batched matrix-core Legendre kernels (FP32 plans with nrhs > 1), written to out1 (HOST):
 * the (l, m, ring pair) triples evaluated per right-hand side when every 64-pair ring group starts
 * at its own entry degree, as those kernels do.  One batched synthesis or adjoint of K right-hand
 * sides performs (10 + 16 K) flop per such triple: two recurrence steps shared by the right-hand
 * sides and eight multiply-adds per right-hand side (the transform of eq. shear_SH and its adjoint).
 */
akra_status akra_plan_work_batched(akra_plan plan, int64_t *out1);
/*
 * Rings without weight.  H v and the right-hand side depend on a ring only through its weights
 * W = M N^-1 (Sec. II.B: the pixel diagonal between the inverse and the forward SHT), so a ring whose
 * weights are all zero -- outside the survey footprint, eq. mask -- contributes nothing.  Every weight
 * set-up (akra_apply_H, akra_rhs and the solves) records which rings carry weight; the weighted
 * operator's ring stage then transforms only those rings, and its Legendre stages skip the 64-pair
 * ring groups none of whose rings (north ring p or south ring nrings - 1 - p) carries weight and
 * contract only the weighted side of groups with weight on one side.  The results are those of the
 * full transforms up to the rounding order of the adjoint's sums.  akra_synth2, akra_adjoint2 and
 * the gradient's synthesis always transform every ring.
 *
 * akra_plan_set_skip_unweighted: on != 0 (the default) as above; on = 0 runs every ring and group in
 * weighted applies too (for comparisons).  Synchronises the plan stream and drops a recorded
 * iteration.  Errors: AKRA_ERR_ARG (null plan), AKRA_ERR_HIP.
 *
 * akra_plan_work_weighted writes to out6 (HOST): [0] the rings that carry weight in the last weight
 * set-up (all rings before one), then the (l, m, ring pair) triples the weighted Legendre launches
 * evaluate with the current shapes: [1] synthesis in groups weighted on both sides, [2] synthesis in
 * groups weighted on one side, [3] adjoint on both sides, [4] adjoint on one side, [5] the batched
 * kernels per right-hand side (FP32 plans with nrhs > 1; they contract both sides of every weighted
 * group).  A two-sided triple costs 26 flop per direction (two recurrence steps and eight
 * multiply-adds), a one-sided one 18 (the same recurrence and four multiply-adds).  Errors:
 * AKRA_ERR_ARG.
 */
akra_status akra_plan_set_skip_unweighted(akra_plan plan, int on);
akra_status akra_plan_work_weighted(akra_plan plan, int64_t *out6);
akra_status akra_plan_set_timing(akra_plan plan, int on);
/*
 * Sustained fused multiply-add rate of the current device in TFLOP/s, written to *tflops (HOST):
 * 16 independent FMA chains per thread, 8 waves per SIMD on every compute unit, plain (not packed)
 * FP32 or FP64 by precision (AKRA_FP32 / AKRA_FP64), the fastest of 12 back-to-back launches of a
 * few ms each, timed with HIP events on a private stream.  It is the ceiling an ALU-bound kernel meets at the clock the device holds
 * under that load, beside the published peak.  Allocates and frees a scratch buffer of 8 B per
 * thread of the grid; synchronises its own stream only.  Errors: AKRA_ERR_ARG (null output,
 * unknown precision), AKRA_ERR_HIP.
 */
akra_status akra_fma_rate(int precision, double *tflops);
/*
 * Sustained rate of the matrix-core product v_mfma_f32_32x32x2_f32 (4096 flop each) on the current
 * device in TFLOP/s, written to *tflops (HOST): chains (1, 2 or 4) independent 32 x 32 FP32
 * accumulators per wave, valu (0, 4 or 8) pairs of plain FP32 FMAs on two other chains of each lane
 * after every product, waves (1 or 2) single-wave workgroups per SIMD on every compute unit; the
 * fastest of 6 launches, timed with HIP events on a private stream.  The rate counts the products'
 * flops only.  It measures how far VALU work between products slows the matrix cores, the bound of
 * the batched Legendre kernels, whose recurrence is such work.  Allocates and frees a scratch buffer
 * of 4 B per thread of the grid; synchronises its own stream only.  Errors: AKRA_ERR_ARG (null
 * output, a value outside the lists), AKRA_ERR_HIP.
 */
akra_status akra_mfma_rate(int chains, int valu, int waves, double *tflops);
/*
 * Ring-stage kernel choice of plans created afterwards (process-wide, not thread-safe against
 * concurrent akra_plan_create).  A ring whose length N is not a power of two is transformed whole by
 * Bluestein when its convolution length (the power of two M >= 2N - 1) is at most maxm, else as two
 * sub-transforms of length N / 2.  maxm: a power of two in [2, 8192]; default 8192, the largest
 * convolution LDS holds in FP64.  Results do not depend on the choice beyond rounding; smaller values
 * exist to exercise the split kernel at small sizes.  Errors: AKRA_ERR_ARG.
 */
akra_status akra_set_ring_whole_maxm(int maxm);
/*
 * Register engine of the ring stage for plans created afterwards (process-wide, not thread-safe
 * against concurrent akra_plan_create).  on != 0 (the default): rings whose transform length is 4096
 * or 8192 (whole power-of-two rings and whole-ring Bluestein convolutions) run the kernels that hold
 * a transform in registers and exchange through LDS; on = 0: every ring runs the LDS kernels.  The
 * results agree to rounding; the switch exists for tests and timing comparisons.  Returns AKRA_OK.
 */
akra_status akra_set_ring_register_engine(int on);
akra_status akra_plan_stage_times(akra_plan plan, double *ms, int *calls);

/*
 * Shape-noise realisations and power spectra (Sec. IV, power spectrum results).  The paper estimates
 * the shape-noise bias N_l of an auto spectrum, and the error bars of auto and cross spectra, from
 * realisations made by permuting the observed shear at random among the unmasked pixels and passing
 * each permuted map through the full reconstruction; the cross spectrum correlates the
 * reconstructions of two disjoint random halves of the sample.  The random permutations are
 * inputs.  The paper gives no formula for the spectrum; these calls take, for coefficient sets X, Y
 * of real fields (m >= 0 storage),
 *   C_l^{XY} = (2l+1)^-1 [ Re(X_l0 conj Y_l0) + 2 sum_{m>0} Re(X_lm conj Y_lm) ]   (l >= 2),
 *   C_0 = C_1 = 0,
 * with no mask, f_sky or shear-calibration correction.  The shuffle moves the shear only: the
 * weights W = M N^-1 stay with their pixels.
 */

/*
 * Ascending RING indices of the unmasked pixels (mask != 0).
 *   mask   device uint8 [Npix];
 *   idx    device int32 [Npix] capacity; the first n_obs entries are written;
 *   n_obs  HOST int64, out.
 * Synchronises the plan stream.  Errors: AKRA_ERR_ARG (null pointers), AKRA_ERR_HIP.
 */
akra_status akra_unmasked_index(akra_plan plan, const uint8_t *mask, int32_t *idx, int64_t *n_obs);

/*
 * Shear permuted among the unmasked pixels, for realisations k < n_real and j < n_obs:
 *   g1_out[k][idx[j]] = g1[idx[perm[k][j]]],  g2_out[k][idx[j]] = g2[idx[perm[k][j]]],
 * and 0 at every other pixel of g1_out[k], g2_out[k].
 *   g1, g2          device float64 [Npix];
 *   idx             device int32 [n_obs], the list akra_unmasked_index returns (0 <= n_obs <= Npix);
 *   perm            device int32 [n_real][n_obs]; each row should be a permutation of 0 .. n_obs-1
 *                   (not checked), every entry must lie in [0, n_obs) (checked);
 *   g1_out, g2_out  device float64 [n_real][Npix]; must not overlap the inputs or each other.
 * Synchronises the plan stream.  Errors: AKRA_ERR_ARG for null pointers, counts out of range,
 * overlapping outputs, or an entry of perm or idx out of range (entries out of range are skipped and
 * the outputs are then incomplete), AKRA_ERR_HIP.
 */
akra_status akra_shuffle_shear(akra_plan plan, const double *g1, const double *g2, const int32_t *idx, int64_t n_obs,
                               const int32_t *perm, int n_real, double *g1_out, double *g2_out);

/*
 * Spectra C_l^{XY} of coefficient pairs: for q < npairs, cl[q] = C^{x[i] y[j]} with
 * (i, j) = (pairs[2q], pairs[2q+1]).
 *   x      device complex128 [nx][n_alm];  y  device complex128 [ny][n_alm] (y == x allowed), both
 *          16-byte aligned;
 *   pairs  HOST int32 [npairs][2], 0 <= i < nx, 0 <= j < ny;
 *   cl     device float64 [npairs][lmax+1].
 * Stream-ordered, no host synchronisation; the sum over m has a fixed order, so results repeat
 * bit for bit.  Errors: AKRA_ERR_ARG (null pointers, negative counts, a pair out of range),
 * AKRA_ERR_HIP.
 */
akra_status akra_alm_spectra(akra_plan plan, const double *x, int nx, const double *y, int ny, const int32_t *pairs,
                             int npairs, double *cl);

/*
 * Allocation-free form of akra_alm_spectra, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  It needs no
 * plan: the band limit is an argument, and the partial sums live in a static device array of the
 * library (SPEC pairs x chunks x degrees of float64, 16.3 MiB at AKRA_NOALLOC_LMAX_MAX), one copy
 * per GPU held until the process ends.  The call allocates nothing; its device address is looked
 * up once per device, at the first call with that device current.
 *   lmax      0 <= lmax <= AKRA_NOALLOC_LMAX_MAX (AKRA_ERR_ARG beyond it, before any HIP call);
 *   x, y, nx, ny, pairs, npairs, cl   as for akra_alm_spectra, with n_alm = (lmax+1)(lmax+2)/2;
 *   hip_stream  a stream of the current device (NULL: the null stream).
 * Stream-ordered, no host synchronisation; results equal akra_alm_spectra's bit for bit.  Calls that
 * overlap on one GPU (other threads or other streams) share the scratch array and race: serialise
 * them.  Errors: AKRA_ERR_ARG as for akra_alm_spectra, lmax out of range, or a stream of another
 * device; AKRA_ERR_HIP.
 */
#define AKRA_NOALLOC_LMAX_MAX 4096
akra_status akra_alm_spectra_noalloc(int lmax, const double *x, int nx, const double *y, int ny,
                                     const int32_t *pairs, int npairs, double *cl, void *hip_stream);

/*
 * Device bytes of the workspace akra_noise_spectra needs for nset (1 or 2) shear sets, written to
 * *bytes (HOST): the unmasked list, the shuffled maps and the solutions of max(nrhs, nset) right-hand
 * sides.  Errors: AKRA_ERR_ARG.
 */
akra_status akra_noise_work_size(akra_plan plan, int nset, int64_t *bytes);

/*
 * Shape-noise realisations through the full solve, and their spectra.
 *   nset = 1  g1, g2, ninv: device float64 [Npix].  Realisation k solves the shear shuffled by
 *             perm[k] (the akra_shuffle_shear rule) with the unshuffled ninv and mask, and keeps the
 *             auto spectra of its solution x = (E, B).
 *   nset = 2  split halves A, B: g1, g2, ninv are [2][Npix].  Realisation k shuffles half q with
 *             perm[q][k], solves both halves and keeps the cross spectra of the two solutions.
 *   mask      device uint8 [Npix], shared by every solve;
 *   perm      device int32 [nset][n_real][n_obs], n_obs = the number of unmasked pixels (checked);
 *   opts      as for akra_cg_solve.  opts->mode picks the unknowns and the spectra kept:
 *             AKRA_JOINT_EB  nspec = 3: (EE, BB, EB); for nset = 2 (A_E B_E, A_B B_B, A_E B_B),
 *             AKRA_E_ONLY    nspec = 1: EE,   AKRA_B_ONLY  nspec = 1: BB;
 *   work      device workspace of work_bytes >= akra_noise_work_size(plan, nset) bytes, 256-byte
 *             aligned;
 *   cl        device float64 [n_real][nspec][lmax+1];
 *   cl_mean, cl_std  device float64 [nspec][lmax+1] or NULL: the mean over the realisations (for
 *             nset = 1 the noise-bias estimate N_l) and the sample standard deviation (n_real - 1 in
 *             the denominator; 0 when n_real < 2);
 *   info      HOST, nullable: iters and fp64_applies summed over the solves, the worst rel_resid and
 *             rel_resid_true, lambda_eff and precond of the first solve, the worst status.
 * The right-hand sides are solved in groups of the plan's nrhs (the batched solver on FP32 plans
 * with nrhs > 1); with nset = 2 and nrhs > 1, nrhs must be even.  A last, partial group is filled
 * with zero shear, which the solver finishes without iterating.  Synchronises the plan stream.
 * Errors: AKRA_ERR_ARG (null pointers, sizes, n_obs differing from the mask, a perm entry out of
 * range, a small workspace), the errors of akra_cg_solve, AKRA_NOT_CONVERGED when some solve stopped
 * at maxiter (its spectra are those of the last iterate).
 */
akra_status akra_noise_spectra(akra_plan plan, int nset, const double *g1, const double *g2, const double *ninv,
                               const uint8_t *mask, const int32_t *perm, int64_t n_obs, int n_real,
                               const akra_cg_opts *opts, void *work, int64_t work_bytes, double *cl,
                               double *cl_mean, double *cl_std, akra_cg_info *info);

/*
 * Catalogue pixelisation (Sec. III.B pixelization).  Galaxies j with direction (z_j = cos theta_j,
 * phi_j), ellipticities (e1_j, e2_j) and weights w_j >= 0 are binned onto the plan's HEALPix RING
 * grid, and per pixel i:
 *   g_i^nu  = sum_j w_j e^nu_j / (R sum_j w_j)      (eq. gamma_obs; 0 where sum_j w_j = 0)
 *   N_eff,i = (sum_j w_j)^2 / sum_j w_j^2           (eq. Neff_pixel; 0 where sum_j w_j^2 = 0)
 *   N^-1_i  = N_eff,i / sigma_e^2                   (eq. noise_var)
 *   M_i     = N_eff,i >= n_th                       (eq. mask)
 * The sums of a pixel run over its galaxies in catalogue order, each product rounded before it is
 * added, and R sum_j w_j is formed before the division: the results are a fixed function of the
 * catalogue (no atomics), reproducible bit for bit.  The outputs feed akra_cg_solve directly
 * (g1, g2, ninv, mask).
 */

/*
 * RING pixel of each direction: z = cos theta in [-1, 1], phi in [0, 2 pi) (the inverse of the
 * pixel boundaries of Gorski et al. 2005, computed in FP64 with every operation rounded on its own).
 *   z, phi  device float64 [n];  pix  device int32 [n].
 * Synchronises the plan stream.  Errors: AKRA_ERR_ARG (null pointers, n < 0, a direction out of
 * range), AKRA_ERR_HIP.
 */
akra_status akra_ang2pix(akra_plan plan, const double *z, const double *phi, int64_t n, int32_t *pix);

/* Device bytes of the workspace akra_pixelize needs for n_gal galaxies (0 <= n_gal < 2^31), written
 * to *bytes (HOST): a 32-byte record {w, w e1, w e2, w^2} per galaxy, pixel keys, their sorted copy
 * and galaxy order, per-pixel runs and the radix-sort storage.  Errors: AKRA_ERR_ARG. */
akra_status akra_pixelize_work_size(akra_plan plan, int64_t n_gal, int64_t *bytes);

/*
 * Pixelise a catalogue of n_gal galaxies (definitions above).
 *   z, phi, e1, e2, w   device float64 [n_gal] (may be NULL when n_gal = 0);
 *   R                   mean shear response (finite, nonzero); sigma_e > 0; n_th finite;
 *   work                device workspace of work_bytes >= akra_pixelize_work_size(plan, n_gal), 256-byte
 *                       aligned;
 *   g1, g2, ninv, neff  device float64 [Npix];  mask  device uint8 [Npix].
 * Synchronises the plan stream.  Errors: AKRA_ERR_ARG (null pointers, sizes, a direction out of
 * range, a negative or non-finite weight, a non-finite ellipticity, a small workspace; the outputs
 * are then not written), AKRA_ERR_HIP.
 */
akra_status akra_pixelize(akra_plan plan, const double *z, const double *phi, const double *e1, const double *e2,
                          const double *w, int64_t n_gal, double R, double sigma_e, double n_th, void *work,
                          int64_t work_bytes, double *g1, double *g2, double *ninv, double *neff, uint8_t *mask);

/*
 * Flat-sky variant (Sec. II.B, storage problem: on a flat field each spherical harmonic transform
 * becomes a 2-D FFT, the four-step operator and the CG solver otherwise unchanged).
 *   field    nx x ny square pixels, periodic; maps float64 [ny][nx] (x index fastest);
 *   unknown  z = kappa_E + i kappa_B on the grid (joint E/B);
 *   A z      = F^-1 (D . F z), F the unitary 2-D DFT, D(k) = (k1 + i k2)^2 / |k|^2 the flat-sky
 *            Kaiser-Squires kernel with D(0) = 0 (it depends only on the direction of k, so the
 *            pixel size does not enter); gamma = gamma_1 + i gamma_2 = A z;
 *   H z      = A^H (W . A z) + lambda_eff z,  b = A^H (W . gamma_obs), W = M N^-1,
 *            lambda_eff = lambda <N^-1>_M, P = (<W> + lambda_eff)^-1 (as on the sphere);
 * with A^H z = F^-1 (conj(D) . F z), the adjoint for <u, v> = sum_p Re(conj(u_p) v_p).  FP64.
 * The solver holds x = F z, so one H apply costs two 2-D FFTs.
 */
typedef struct akra_flat_plan_s *akra_flat_plan;

/* Plan for an nx x ny field (powers of two in [4, 8192]) on HIP stream hip_stream (NULL = default
 * stream).  Allocates all device memory of the flat calls.  Errors: AKRA_ERR_ARG, AKRA_ERR_ALLOC,
 * AKRA_ERR_HIP. */
akra_status akra_flat_plan_create(int nx, int ny, void *hip_stream, akra_flat_plan *out);
void akra_flat_plan_destroy(akra_flat_plan plan);
int64_t akra_flat_plan_device_bytes(akra_flat_plan plan);

/* gamma = A z: kE, kB, g1, g2 device float64 [ny][nx].  Stream-ordered.  Errors: AKRA_ERR_ARG. */
akra_status akra_flat_synth(akra_flat_plan plan, const double *kE, const double *kB, double *g1, double *g2);
/* (yE + i yB) = A^H (g1 + i g2).  Stream-ordered.  Errors: AKRA_ERR_ARG. */
akra_status akra_flat_adjoint(akra_flat_plan plan, const double *g1, const double *g2, double *yE, double *yB);
/* (yE + i yB) = H (kE + i kB) for W from ninv (device float64 [ny][nx], finite, >= 0) and mask (device
 * uint8 [ny][nx]) and the given lambda_eff.  Synchronises once (weight validation).  Errors:
 * AKRA_ERR_ARG (null pointers, negative weights), AKRA_ERR_NUMERIC (non-finite weights). */
akra_status akra_flat_apply_H(akra_flat_plan plan, const double *ninv, const uint8_t *mask, double lambda_eff,
                              const double *kE, const double *kB, double *yE, double *yB);
/* (bE + i bB) = A^H (W (g1 + i g2)).  Errors as akra_flat_apply_H. */
akra_status akra_flat_rhs(akra_flat_plan plan, const double *g1, const double *g2, const double *ninv,
                          const uint8_t *mask, double *bE, double *bB);
/* Regularised estimate (kappa_E, kappa_B) of the flat field by PCG (opts as for akra_cg_solve:
 * lambda, tol, maxiter, use_x0 with kE/kB as the start maps, resid_hist; mode must be AKRA_JOINT_EB,
 * kernel_l NULL, reliable_delta unused).  Outputs kE, kB device float64 [ny][nx]; info as for
 * akra_cg_solve (fp64_applies 0).  ||b|| = 0 gives zero maps.  Errors: AKRA_ERR_ARG, AKRA_ERR_NUMERIC
 * (non-finite data, CG breakdown), AKRA_NOT_CONVERGED (maxiter; kE, kB hold the last iterate),
 * AKRA_STAGNATED (opts->stall_iters; kE, kB hold the last iterate). */
akra_status akra_flat_cg_solve(akra_flat_plan plan, const double *g1, const double *g2, const double *ninv,
                               const uint8_t *mask, const akra_cg_opts *opts, double *kE, double *kB,
                               akra_cg_info *info);
/* Step-wise PCG on the plan's state: akra_flat_cg_start forms W, lambda_eff = lambda <N^-1>_M, P and b,
 * and sets x0 = 0 (one synchronisation); akra_flat_cg_step runs nsteps iterations stream-ordered with no
 * host synchronisation and no convergence test (for timing).  Errors: AKRA_ERR_ARG. */
akra_status akra_flat_cg_start(akra_flat_plan plan, const double *g1, const double *g2, const double *ninv,
                               const uint8_t *mask, double lambda);
akra_status akra_flat_cg_step(akra_flat_plan plan, int nsteps);

#ifdef __cplusplus
}
#endif
#endif /* AKRA_H */
