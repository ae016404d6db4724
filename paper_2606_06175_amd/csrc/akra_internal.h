// Internal declarations of libakra (HIP, gfx950).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/akra.h"

namespace akra {

// ------------------------------------------------------------------------------------------------
// Scaled-exponent representation of the Wigner-d recurrence values.
// A value is mant * 2^(UNIT * k) with an integer k <= 0.  While k < 0 the value is below
// 2^-(UNIT/2) and contributes nothing; the mantissa is rescaled by 2^-UNIT whenever it exceeds
// 2^(UNIT/2), and k then grows by one.  Once k == 0 the mantissa is the value itself.
// ------------------------------------------------------------------------------------------------
// padding (in entries) after the coefficient table and the kernel-scaled alm buffers
constexpr int ALM_PAD = 64;
// unmasked-pixel compaction: threads per block, contiguous pixels per thread, pixels per tile
constexpr int CMP_T = 256, CMP_PER = 16, CMP_TILE = CMP_T * CMP_PER;
// spectra: degrees per block, orders per partial sum, pairs per launch
constexpr int SPEC_LT = 256, SPEC_MC = 64, SPEC_NP = 8;
struct SpecArgs {
    const double2 *x[SPEC_NP];  // coefficient sets X of the pairs (m >= 0 storage)
    const double2 *y[SPEC_NP];  // coefficient sets Y
    double *cl[SPEC_NP];        // [lmax+1] outputs
};

template <typename T> struct Scale;
template <> struct Scale<double> {
    static constexpr int UNIT = 512;
};
template <> struct Scale<float> {
    static constexpr int UNIT = 64;
};

// Per-(l, m) recurrence coefficients of the normalised spin-weighted functions
//   2lambda_{l+1} = (a x + b) 2lambda_l - g 2lambda_{l-1},   -2lambda_{l+1} = (a x - b) -2lambda_l - g -2lambda_{l-1}
// stored at the alm index i(l, m) (entries at l = lmax are zero).
struct alignas(32) Coef64 {
    double a, b, g, pad;
};
struct alignas(16) Coef32 {
    float a, b, g, pad;
};
// Scaled form of the same recurrence, run by the Legendre kernels away from the poles.  With
// lambda_l = c_l mu_l, where c_{l0} = c_{l0+1} = 1 and c_{l+1} = g_l c_{l-1},
//   mu_{l+1} = (a' x +- b') mu_l - mu_{l-1},   a' = a c_l / c_{l+1},  b' = b c_l / c_{l+1},
// two FMAs per spin and step instead of three operations and a shared product.  Every g_l < 1 and
// their products stay of order one (c_l > 2^-3.1 at lmax 16384 over a dense sample of m), so mu
// has lambda's range.
// Synthesis records carry the alm multiplied by c_l; the adjoint multiplies its sums by c_l.
struct alignas(32) Coef64S {
    double a, b, c, ic;  // a', b', c_l, 1 / c_l
};
struct alignas(16) Coef32S {
    float a, b, c, ic;
};
// Near the poles FP32 kernels run the recurrence in difference form, with d_l = lambda_l - lambda_{l-1}
// and y = 1 - x:
//   d_{l+1} = (e - a y) lambda_l + g d_l,   lambda_{l+1} = lambda_l + d_{l+1},   e = a +- b - g - 1.
// There a x + b - g - 1 is small while a x + b is close to 2 and the plain form loses its
// information to rounding; e is formed in extended precision at plan creation.
struct alignas(16) Coef32D {
    float a, ep, em, g;  // a, e for spin +2, e for spin -2, g
};

// State of the recurrence of one (m, ring pair) at the entry degree of the pair's 64-pair group:
// lambda_l and lambda_{l-1} for spin +2 and -2, sharing one scale exponent (kept beside it).
// Below the entry degree every value of the group is under the scale threshold and contributes
// nothing, so the Legendre kernels start there instead of at l = max(m, 2).
struct alignas(32) Ent64 {
    double c2, p2, cm, pm;
};
// entry degree of a group whose values never reach the threshold up to lmax
constexpr int ENT_SKIP = 0x3fffffff;

// One iso-latitude ring of the pixelisation.
struct RingInfo {
    double z;      // cos(theta): the ring is defined by this double value
    int64_t ofs;   // first pixel (RING order)
    int nphi;      // pixels on the ring, N = 4 * sub
    int sub;       // N / 4: length of the four interleaved sub-transforms
    int shift;     // phi0 = pi * shift / N
    int M;         // Bluestein FFT length (0: sub is a power of two): of the whole ring when the
                   // ring is transformed whole, else of the sub-transform
    int64_t bofs;  // Bluestein rings: offset of the chirp spectrum of the transformed length
    int64_t rofs;  // Bluestein rings of the register engine: offset of that spectrum in register order
};

// Rings that carry weight.  A ring whose weights W = M N^-1 are all zero contributes nothing to
// H v or to the right-hand side (its G is zero), so with a weight set in place the ring stage skips
// such rings and the Legendre stages skip the 64-pair groups none of whose rings carry weight.  A
// group of ring pairs (north ring p, south ring nrings - 1 - p) falls in one of three classes:
// weight on north and south rings (GCLS_BOTH), on north rings only (GCLS_NORTH; the equatorial ring
// counts as a north ring) or on south rings only (GCLS_SOUTH).  A one-ring class contracts with half
// of the FMAs of the two-ring class.
enum { GCLS_BOTH = 0, GCLS_NORTH = 1, GCLS_SOUTH = 2, GCLS_N = 3 };
// 64-pair groups of one apply: per class an ascending list whose first npol entries are near-polar
// groups of FP32 plans (difference form), then nmain others; list_any holds every listed group
// (the union of the classes, for the batched kernels, which have no one-ring form).
struct GroupSet {
    const int *list[GCLS_N] = {nullptr, nullptr, nullptr};
    int npol[GCLS_N] = {0, 0, 0}, nmain[GCLS_N] = {0, 0, 0};
    const int *list_any = nullptr;
    int npol_any = 0, nmain_any = 0;
};
// rings of one ring-stage launch set, by kernel kind: whole power-of-two rings in LDS (RK_P2), whole-ring
// Bluestein (RK_BF), two half-length Bluestein transforms (RK_BL), and the register engine's six
// lists (RK_REG + q, q as in Plan::d_order_r)
enum { RK_P2 = 0, RK_BF = 1, RK_BL = 2, RK_REG = 3, RING_KINDS = 9 };
// ring blocks a class-split adjoint may write beyond the unsplit layout (each of up to two polar
// and two further main parts rounds up by at most one block)
constexpr int LIVE_NRB_EXTRA = 4;
// values keying a recorded PCG iteration (see iter_key)
constexpr int ITER_KEY_N = 18;
struct RingSet {
    const int *order[RING_KINDS] = {};
    int n[RING_KINDS] = {};
};

struct Plan {
    int nside = 0, lmax = 0, nrhs = 1, prec = AKRA_FP64;
    int dev = 0;
    hipStream_t stream = nullptr;
    int nrings = 0, npairs = 0;
    int64_t npix = 0, nalm = 0;
    double omega = 0;

    // tables
    RingInfo *d_rings = nullptr;
    double *d_pair_z = nullptr;
    Coef64 *d_coef64 = nullptr;  // plain form: entry states (plan build)
    Coef32 *d_coef32 = nullptr;  // plain form: batched matrix-core synthesis
    Coef64S *d_coef64s = nullptr;  // scaled form (Legendre kernels, FP64), and c_l for every form
    Coef32S *d_coef32s = nullptr;  // scaled form (Legendre kernels, FP32)
    Coef32D *d_coef32d = nullptr;
    double *d_seed2 = nullptr, *d_seedm2 = nullptr;  // [m][pair] seeds at l = max(m,2) (plan build only)
    int *d_seedk = nullptr;
    Ent64 *d_ent = nullptr;     // [m][pair] entry states
    int *d_entk = nullptr;      // [m][pair] their scale exponents
    int *d_entl = nullptr;      // [m][group] entry degree of each 64-pair group (ENT_SKIP: none)
    int ng64 = 0;               // 64-pair groups
    std::vector<int> h_entl;
    int *d_wgstart = nullptr;   // [m][adjoint ring block] first degree the block wrote
    int64_t work[3] = {0, 0, 0};  // (l, m, pair) triples: all, evaluated by synthesis, by adjoint
    int64_t work_b = 0;           // triples per right-hand side of the batched kernels (each group from its entry)
    void *d_tw64 = nullptr, *d_tw32 = nullptr;  // e^{-2 pi i k / twn}, k < twn/2
    void *d_bhat64 = nullptr, *d_bhat32 = nullptr;  // Bluestein chirp spectra per distinct sub length
    int twn = 1;
    int *d_lof = nullptr;  // l of every alm index
    int *d_order_p2 = nullptr, *d_order_bl = nullptr, *d_order_bf = nullptr;
    int n_p2 = 0, n_bl = 0, n_bf = 0, maxM_p2 = 1, maxM_bl = 1, maxM_bf = 1;
    // rings of the register engine (transform length 4096 or 8192): [0] direct M = 4096, [1] direct
    // 8192, [2] whole-ring Bluestein M = 4096, [3] 8192, [4] two-half Bluestein M = 4096, [5] 8192
    int *d_order_r[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int n_r[6] = {0, 0, 0, 0, 0, 0};
    void *d_bhatr64 = nullptr, *d_bhatr32 = nullptr;  // their chirp spectra in register order
    std::vector<RingInfo> h_rings;

    // every ring and group (transforms without weights), and those of the current weights: the
    // lists of the weighted set are rebuilt at every weight set-up (setup_weights)
    RingSet rs_all, rs_live;
    // the weighted rings of rs_live by the class of their 64-pair group: [0] groups weighted on both
    // sides, [1] on one side (each kind's list holds the first class's rings, then the second's)
    RingSet rs_cls[2];
    GroupSet gs_all, gs_live;
    std::vector<int> h_order[RING_KINDS];  // host copies of the rings of every kind
    int *d_gl_all = nullptr;      // [ng64] 0, 1, .., ng64 - 1
    int *d_live_lists = nullptr;  // [RING_KINDS][nrings] ring lists, then [GCLS_N + 1][ng64] group lists
    uint8_t *d_ring_live = nullptr;  // [nrings] 1: the ring carries weight in some right-hand side's W
    uint8_t *h_live = nullptr;       // pinned: the flags read back, then the lists staged for upload
    std::vector<uint8_t> h_live_prev;  // the flags the current lists were built from
    int live_gen = 0;                // counts weight set-ups (recorded graphs hold the lists' sizes)
    bool skip_rings = true;          // weighted applies use the weighted sets (akra_plan_set_skip_unweighted)
    int n_live_rings = 0;            // rings that carry weight in the current weights
    int nrb_cur = 1;                 // ring blocks the last single-right-hand-side adjoint wrote
    int nrb_b_cur = 1;               // ring blocks the last batched adjoint wrote
    int64_t work_live[5] = {0, 0, 0, 0, 0};  // evaluated triples with the current weights: synthesis of
                                             // two-ring, one-ring groups, adjoint of two-ring, one-ring,
                                             // batched kernels per right-hand side

    // Legendre launch shapes
    int syn_R = 1, syn_V = 1, syn_groups = 1;
    int adj_R = 1, adj_W = 1, adj_L = 8, adj_nrb = 1;
    // the shapes of groups weighted on one side only (GCLS_NORTH, GCLS_SOUTH), tuned apart: they
    // contract with half the FMAs per loaded record or chunk
    int syn_R1 = 1, syn_V1 = 1, adj_R1 = 1, adj_W1 = 1, adj_L1 = 8;
    size_t part_rb_cap = 1;  // ring blocks the partial-sum buffer holds
    // FP32 plans: the 64-pair groups nearest the poles run the Legendre stages in the difference
    // form; the adjoint covers them with adj_nrb_polar single-wave ring blocks of at most adj_Rpol
    // groups (spread evenly): 4, or 1 where blocks of four would leave the launch with too few waves
    // for its long recurrences
    int polar_groups = 0, adj_nrb_polar = 0, adj_Rpol = 4;
    // batched matrix-core kernels: waves (64-pair groups) per workgroup of the synthesis and the
    // adjoint; nrb_b adjoint ring blocks of bat_AW groups (the buffers hold those of bat_AW = 2)
    int bat_SW = 4, bat_AW = 4, nrb_b_cap = 0;

    // workspaces (sized for FP64; FP32 views reuse them)
    void *d_FG = nullptr;       // [nrhs][nrings][lmax+1][2] complex
    void *d_part = nullptr;     // [nrb][nalm][4] adjoint partial sums
    void *d_rec = nullptr;      // [nrhs][nalm + ALM_PAD] synthesis records (64 B in FP64), scaled form
    float4 *d_recu = nullptr;   // FP32 plans with polar groups: [nrhs][nalm + ALM_PAD] unscaled alm for
                                // the difference form
    float *d_brec = nullptr;    // FP32 plans with nrhs > 1: [nalm + ALM_PAD][8 rhs][4] batched records
    int nrb_b = 0;              // FP32 plans with nrhs > 1: ring blocks of the batched adjoint
    int *d_wgstart_b = nullptr; // [m][nrb_b] first degree each batched adjoint block wrote
    int64_t rec_stride = 0;     // records per right-hand side
    double *d_W = nullptr;      // [nrhs][npix] weights
    double *d_kern = nullptr;   // [lmax+1]
    double *d_kuser = nullptr;  // [lmax+1] caller-supplied kernel
    double *d_red = nullptr;    // reduction partials
    double *d_red_cg = nullptr; // [nrhs][2][CG_RED_BLOCKS] partials of the PCG iteration's inner products
    double *d_scal = nullptr;   // device scalars
    int *d_flag = nullptr;
    // solver vectors [nrhs][2][nalm] complex FP64
    double *d_x = nullptr, *d_r = nullptr, *d_p = nullptr, *d_w = nullptr, *d_b = nullptr, *d_xs = nullptr;
    double *h_pin = nullptr;    // pinned host scalars
    // unmasked-pixel list (compaction scratch) and spectrum partial sums
    int64_t cmp_ntile = 0;        // tiles of CMP_TILE pixels
    void *d_cmp = nullptr;        // one allocation holding the four members below
    int *d_cmp_cnt = nullptr;     // [cmp_ntile] unmasked pixels per tile
    int64_t *d_cmp_offs = nullptr;  // [cmp_ntile] first list position of each tile
    int64_t *d_cmp_nobs = nullptr;  // number of unmasked pixels
    int *d_cmp_flag = nullptr;    // nonzero: a shuffle met an index out of range
    int spec_nmc = 0;             // m-chunks of the spectrum partial sums
    double *d_spec = nullptr;     // [SPEC_NP][spec_nmc][lmax+1]
    int64_t device_bytes = 0;

    // solver state of the right-hand side in progress
    bool cg_ready = false;
    int cg_rhs = 0, cg_iters = 0, cg_fp64_applies = 0;
    // unknowns of the running solve (App. A block systems): 0 joint E/B, 1 E only (the epilogue
    // zeroes the B block of every output), 2 B only (E block zeroed); cg_proj is kept for akra_cg_step
    int proj = 0, cg_proj = 0;
    double cg_bn = 0, cg_rr = 0, cg_lam = 0, cg_pc = 1;
    const double *cg_kern = nullptr;

    // one single-right-hand-side PCG iteration recorded as a HIP graph (on a private capture stream)
    // and replayed on the plan stream; cg_graph_key holds every by-value kernel argument it baked in
    bool use_graph = true;
    bool capturing = false;  // recording the graph: host-side trace ranges are not emitted
    hipStream_t cap_stream = nullptr;
    // a second stream at the default priority: independent launches of one stage (the Legendre
    // classes, the ring-kernel kinds) run on it beside the plan stream, forked from and joined back
    // to the plan stream with events, so that one launch fills the other's tail
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool in_fork = false;  // inside a fork_join: a nested one runs its halves in order
    hipGraphExec_t cg_graph = nullptr;
    double cg_graph_key[ITER_KEY_N] = {};
    // the lockstep iteration of the batched solve, keyed by its by-value arguments and active set
    hipGraphExec_t cg_graph_b = nullptr;
    std::vector<double> cg_graph_b_key;

    // stage timing with HIP events on the plan stream
    bool timing = false;
    std::vector<std::array<hipEvent_t, 2>> ev_pool;
    std::vector<int> ev_stage;
    int ev_used = 0;
};

// Host-side trace range for the duration of a scope (shown by rocprofv3 --marker-trace, which
// attributes the kernels dispatched inside it; without a tracer the calls return at once).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// Solves that stopped with a valid iterate (maxiter or stagnation), and the status of several such
// solves together: NOT_CONVERGED over STAGNATED over OK.
inline bool stopped_early(akra_status s) { return s == AKRA_NOT_CONVERGED || s == AKRA_STAGNATED; }
inline akra_status merge_stops(akra_status a, akra_status b)
{
    if (a == AKRA_NOT_CONVERGED || b == AKRA_NOT_CONVERGED) return AKRA_NOT_CONVERGED;
    if (a == AKRA_STAGNATED || b == AKRA_STAGNATED) return AKRA_STAGNATED;
    return AKRA_OK;
}
// Stagnation test: true once `window` consecutive observed residuals have failed to go below the
// smallest one seen before them (window <= 0: never).
struct StallWatch {
    int window = 0;
    double best = 0.0;
    int since = 0;
    StallWatch(int w = 0, double start = 0.0) : window(w), best(start) {}
    bool step(double rel)
    {
        if (window <= 0) return false;
        if (rel < best) {
            best = rel;
            since = 0;
            return false;
        }
        return ++since >= window;
    }
};

// Runs side() with the plan's launches going to the side stream and main() on the plan stream,
// the side stream forked from the plan stream before and joined to it after (stream-ordered, and
// captured the same way into a recorded graph).  Without a side stream, or nested inside another
// fork_join, both run in order on the current stream.  A failing event call leaves its error for
// the launch check that follows every stage.
template <class A, class B> void fork_join(Plan &P, A &&side, B &&main)
{
    if (!P.side_stream || P.in_fork) {
        side();
        main();
        return;
    }
    P.in_fork = true;
    (void)hipEventRecord(P.ev_fork, P.stream);
    (void)hipStreamWaitEvent(P.side_stream, P.ev_fork, 0);
    const hipStream_t s = P.stream;
    P.stream = P.side_stream;
    side();
    P.stream = s;
    main();
    (void)hipEventRecord(P.ev_join, P.side_stream);
    (void)hipStreamWaitEvent(P.stream, P.ev_join, 0);
    P.in_fork = false;
}

// error handling
void set_error(const std::string &msg);
akra_status hip_fail(hipError_t e, const char *what);

// ---- kernel launchers (akra_kernels.hip) -------------------------------------------------------
// the weighted apply's Legendre and ring stages (single right-hand side, W of the plan's weights) as
// one chain per class of ring groups on two streams (requires the side stream and both classes)
void launch_weighted_chains(Plan &P, bool fp32, const double *W);
// prologue: records {a, b, g, 0, K_l x_E, K_l x_B} per (l, m) in the transform precision (Im(a_l0) dropped)
void launch_prologue(Plan &P, bool fp32, const double *xE, const double *xB, const double *kern, int nrhs);
// entry states of the recurrence from the seeds (plan build)
void launch_entry(Plan &P);
// FP32 plans with nrhs > 1: kernel-scaled records and matrix-core synthesis of all right-hand sides
// (alm of right-hand side r at xE/xB + 2 r rstride doubles)
// (live: only the 64-pair groups with a ring that carries weight in the current weights)
void launch_synth_batched(Plan &P, const double *xE, const double *xB, int64_t rstride, const double *kern,
                          bool live);
// Legendre synthesis of the prologue's records (d_rec) into d_FG: every group (live false) or the
// groups of the current weights by class (live true: F only of rings that carry weight)
void launch_leg_synth(Plan &P, bool fp32, int nrhs, bool live);
// ring stage: mode 0 = F -> maps, 1 = maps -> G, 2 = F -> W -> G (in place); every ring (live false)
// or only the rings that carry weight (live true: the others' G is left as it was, and adjoints with
// live true read it as zero)
void launch_ring(Plan &P, bool fp32, int mode, const double *g1, const double *g2, double *o1, double *o2,
                 const double *W, int nrhs, bool live);
// Legendre adjoint of d_FG into the partial sums d_part (live as for the synthesis; with live true,
// rings without weight are read as G = 0); sets nrb_cur for the epilogue
void launch_leg_adj(Plan &P, bool fp32, int rhs, bool live);
// ring blocks an adjoint launch set writes
int adj_blocks_total(const Plan &P, bool live);
// per-ring flags (any weight nonzero on the ring, over the nrhs maps of W) into d_ring_live
void launch_ring_live(Plan &P, int nrhs);
// gradient of the solve (ring MODE 3, FP64): F = Y K x in d_FG, q = Y K u in (q1, q2) on entry;
// dninv = M (Omega q . (g - Y K x) - c), (q1, q2) <- Omega W q
void launch_ring_grad(Plan &P, const double *g1, const double *g2, double *q1, double *q2, const double *W,
                      double *dninv, const uint8_t *mask, const double *cdev);
// b = upstream alm gradient / full-m weight (Im(a_l0) dropped), for the backward solve
void launch_vjp_rhs(Plan &P, const double *vE, const double *vB, double *bE, double *bB);
void launch_scale_scalar(Plan &P, double *out, const double *in, double f);
// epilogue: sum partials, E/B combination, out = K_l * c + lam * x; with dot_red (and x), also the
// workgroup partials of the full-m <x, out> (cg_red_blocks(P) of them)
void launch_epilogue(Plan &P, bool fp32, const double *kern, double lam, const double *xE, const double *xB,
                     double *outE, double *outB, double *dot_red = nullptr);
// batched FP32 adjoint (matrix cores) of right-hand-side group q, and the epilogue of one right-hand
// side from its slabs
void launch_adj_batched(Plan &P, int q, bool live);
void launch_epilogue_batched(Plan &P, int rhs, const double *kern, double lam, const double *xE, const double *xB,
                             double *outE, double *outB, double *dot_red = nullptr);
// chirp spectra of the Bluestein sub lengths Ls (FFT lengths Ms, table offsets ofs; device arrays)
void launch_bhat(Plan &P, const int *Ls, const int *Ms, const int64_t *ofs, int n, int maxM);
void launch_bhat_reorder(Plan &P, int logm, const int64_t *src_ofs, const int64_t *dst_ofs, int n);
// weights W = mask * ninv, plus the sums needed for lambda_eff / P and input validation; right-hand
// side r reads the N^-1 map r mod ncount of ninv ([ncount][npix])
void launch_weights(Plan &P, const double *ninv, const uint8_t *mask, int nrhs, int ncount);

// full-m dot products and CG vector updates on [2][nalm] complex FP64 vectors
void launch_dot(Plan &P, const double *a, const double *b, double *out_dev, int64_t n_complex);
void launch_cg_p(Plan &P, double *p, const double *r, const double *beta_dev, double precond, int64_t n_complex);
// The PCG iteration's fused scalar path: at most CG_RED_BLOCKS workgroup partials per inner
// product (the epilogue's <p, w>, the update's <r, r>), summed in a fixed order by the kernels that
// form alpha and beta (scal[0] rz, [1] <p, w>, [2] alpha, [3] <r, r>, [4] beta)
constexpr int CG_RED_BLOCKS = 1024;
int cg_red_blocks(const Plan &P);
void launch_cg_alpha_sum(Plan &P, const double *red, double *scal, int *flag);
void launch_cg_xr_rr(Plan &P, double *x, double *r, const double *p, const double *w, const double *alpha_dev,
                     int64_t n_complex, double *rr_red);
void launch_cg_beta_sum(Plan &P, const double *red, double *scal, double precond);
// the same iteration in two vector kernels for one right-hand side (scal[7] holds rz between them)
void launch_cg_xr_alpha(Plan &P, double *x, double *r, const double *p, const double *w, const double *red_pw,
                        double *scal, int *flag, int64_t n_complex, double *rr_red);
void launch_cg_p_beta(Plan &P, double *p, const double *r, const double *red_rr, double *scal, double precond,
                      int64_t n_complex);
void launch_axpby(Plan &P, double *y, double a, const double *x, double b, int64_t n_complex);
void launch_scalar_div(Plan &P, double *out, const double *num, const double *den);
// shape-noise realisations and spectra (akra_spectra.hip)
// ascending indices of the unmasked pixels into idx (capacity npix), their count into d_cmp_nobs
void launch_unmasked_index(Plan &P, const uint8_t *mask, int32_t *idx);
// o = shear permuted by perm among the n_obs unmasked pixels idx, zero elsewhere (o all zero when
// perm is null); indices out of range set d_cmp_flag and are skipped
void launch_shuffle(Plan &P, const double *g1, const double *g2, const int32_t *idx, int64_t n_obs,
                    const int32_t *perm, double *o1, double *o2);
// C_l of the first n (<= SPEC_NP) pairs of a
void launch_spectra(Plan &P, const SpecArgs &a, int n);
// mean and sample standard deviation over n realisations of len values (either output nullable)
void launch_cl_moments(Plan &P, const double *cl, int n, int64_t len, double *mean, double *sd);
// catalogue pixelisation (akra_pixel.hip)
// device bytes of the pixelisation workspace for n_gal galaxies (sort keys, runs, sort storage)
hipError_t pixelize_work_bytes(Plan &P, int64_t n_gal, int64_t *bytes);
// where the pixel keys and the galaxy records live inside that workspace
uint32_t *pixelize_keys(Plan &P, int64_t n, void *work, double4 **rec);
// RING pixel of every galaxy into pix; out-of-range inputs set d_cmp_flag[0] (position) or
// d_cmp_flag[1] (weight / ellipticity, checked when e1 is non-null, which also writes the galaxy
// records {w, w e1, w e2, w^2} into rec)
void launch_ang2pix(Plan &P, const double *z, const double *phi, const double *e1, const double *e2, const double *w,
                    int64_t n, uint32_t *pix, double4 *rec);
// sort by pixel, per-pixel sums in catalogue order and the pixel products (keys and records written)
hipError_t launch_pixelize(Plan &P, int64_t n, double R, double se2, double n_th, void *work, double *g1, double *g2,
                           double *ninv, double *neff, uint8_t *mask);
bool pow2(int n);
bool adj_shape_supported(int r, int w, int l);

// Workgroups of the adjoint over a list of n 64-pair groups with R groups per wave and W waves per
// workgroup.  Workgroups of several waves take W R consecutive list entries each (the last one
// possibly fewer, its empty slots computing zeros).  Single-wave workgroups spread the list evenly
// instead, so that no slot is empty: q = ceil(n / R) workgroups, the first nA of RA = ceil(n / q)
// groups, the others of RA - 1 (RA <= R, and the count of workgroups is the same).
struct AdjSplit {
    int q, RA, nA;
};
inline AdjSplit adj_split(int n, int R, int W)
{
    AdjSplit s{0, R, 0};
    if (n <= 0) return s;
    if (W > 1) {
        s.q = (n + R * W - 1) / (R * W);
        s.nA = s.q;
        return s;
    }
    s.q = (n + R - 1) / R;
    s.RA = (n + s.q - 1) / s.q;
    s.nA = n - s.q * (s.RA - 1);
    return s;
}
// first list entry and number of groups of workgroup b of a split (W as in adj_split)
inline void adj_block(const AdjSplit &s, int n, int W, int b, int &first, int &count)
{
    if (W > 1) {
        first = b * s.RA * W;
        count = std::min(n - first, s.RA * W);
    } else if (b < s.nA) {
        first = b * s.RA;
        count = s.RA;
    } else {
        first = s.nA * s.RA + (b - s.nA) * (s.RA - 1);
        count = s.RA - 1;
    }
}

}  // namespace akra
