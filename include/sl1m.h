/*
 * sl1m.h -- C ABI of the SL1M hot path on MI355X (gfx950).
 *
 * SL1M deconvolves interferometer data by minimising
 *     F(I) = 1/2 |V - M I|^2 + lambda * sum_j I_j   over I >= 0
 * (Hardy 2013, eq. (cme) together with the iteration of Section
 * "Implementation of SL1M"), where M maps pixel fluxes to ungridded
 * visibilities and every entry of M is recomputed from its closed form each
 * time it is used (Section "On-the-fly computation versus in-memory
 * computation"); no matrix is ever stored.
 *
 * Notation: j = pixel, k = visibility.  Phases are in turns.
 *
 * Conventions for every call below
 *  - Array arguments are DEVICE pointers owned by the caller unless the
 *    comment says "host".  The library never frees them.
 *  - The library allocates no device memory: a plan's workspace is sized by
 *    sl1m_plan_workspace_bytes() and provided by the caller; it must stay
 *    alive and untouched until sl1m_plan_destroy().
 *  - Calls are asynchronous on the given stream (a hipStream_t passed as
 *    void*; NULL means the default stream) unless the comment says they
 *    synchronise.
 *  - Every call returns sl1m_status (0 = OK, negative = error).  Arguments
 *    are validated on the host before any launch; on error nothing is
 *    launched and sl1m_last_error() returns a thread-local message.
 *  - No C++ exception crosses this interface.
 *  - Calls that share a plan must not run concurrently (the plan's workspace
 *    holds per-call scratch such as split-K partial sums).
 *  - Real/complex element types follow the plan's precision: float32 and
 *    complex64 (interleaved re, im) for SL1M_PREC_FP32, SL1M_PREC_FP32_HILO
 *    and the MFMA precisions, float64 and complex128 for SL1M_PREC_FP64.
 */
#ifndef SL1M_H_
#define SL1M_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SL1M_OK = 0,
  SL1M_EINVAL = -1,     /* bad argument (null pointer, size, enum value)          */
  SL1M_EDOMAIN = -2,    /* a pixel with l^2 + m^2 >= 1, sigma < 0, non-finite input */
  SL1M_ENOMEM = -3,     /* workspace too small                                    */
  SL1M_EHIP = -4,       /* a HIP runtime call failed                              */
  SL1M_EDIVERGED = -5,  /* solver produced a non-finite objective (L too small)   */
  SL1M_ECANCELLED = -6  /* reserved for the serving layer                         */
} sl1m_status;

/* Pixel basis functions (Section "Defining the direct solution"). */
typedef enum {
  SL1M_PIX_DELTA = 0,          /* eq. (deltam): Dirac delta pixels                    */
  SL1M_PIX_GAUSS_PARAXIAL = 1, /* eq. (samlm4): Gaussian pixel, paraxial w phase      */
  SL1M_PIX_GAUSS_WIDE = 2      /* eq. (samlm5): Gaussian pixel, centre w phase kept   */
} sl1m_pixel_kind;

typedef enum {
  SL1M_PREC_FP64 = 0,      /* everything in float64                              */
  SL1M_PREC_FP32 = 1,      /* float64 phase with exact reduction to [-1/2, 1/2]
                              turn; sincos, gains and accumulation in float32   */
  SL1M_PREC_MFMA_F16 = 2,  /* the FP32 plan's phase and sincos; the matrix
                              entries and the images / residuals they multiply
                              rounded to float16 and contracted on the matrix
                              cores, float32 accumulation (see below)           */
  SL1M_PREC_MFMA_BF16 = 3, /* as SL1M_PREC_MFMA_F16 with bfloat16 operands      */
  SL1M_PREC_FP32_HILO = 4  /* the FP32 plan with the phase formed in float32
                              hi/lo arithmetic instead of float64 (see below)   */
} sl1m_precision;

/*
 * Matrix-core precisions.  The paper treats the polarisations of one
 * observation as independent problems through the same matrix (Section
 * "Defining the direct solution"); with R right-hand sides the operators are
 * products of the N_v x N_p matrix with an N_p x R (forward) or N_v x R
 * (adjoint) matrix, and these plans contract them with the gfx950 MFMA
 * v_mfma_f32_4x4x4_16b (16 blocks of 4 x 4 x 4; four right-hand sides per
 * instruction, 4 pixels or visibilities per step, each lane forming the
 * entries of its own visibility (forward) or pixel (adjoint) from the FP64
 * phase).  Per call the images (times the pixel amplitude) or the residual
 * records are scaled by a power of two that brings their largest magnitude
 * into [2^13, 2^14) and rounded to the operand type; the result is scaled
 * back exactly.  Error per entry of the result: at most
 * (2u + N 2^-24 + 2^-17) sum_j |M_kj x_j| (forward; the adjoint likewise over
 * k), u = 2^-11 (float16) or 2^-8 (bfloat16) the operands' rounding, N the
 * length of the sum (float32 accumulation), 2^-17 the float32 entry itself;
 * float16 operands below 2^-14 of the scale add at most 2^-38 of the largest
 * operand per term (subnormal spacing).  Only delta pixels (every pixel
 * SL1M_PIX_DELTA) and gains without per-pair beam widths are accepted
 * (SL1M_EINVAL otherwise); there is no tuning or serving with these
 * precisions.  When all pixels form one square delta grid (see "Evaluation
 * order" below) the plan also evaluates on the grid: sl1m_plan_info.grid_mfma
 * is 1, and calls with fewer sides than the matrix cores pay off for (float16:
 * 1 and 2 sides, bfloat16: 1, 2 and 4 sides, and bfloat16's adjoint at 8)
 * run the FP32 grid evaluation.  The others contract the grid's products
 * of the per-|l|, per-|m| and per-radius phasors (sixteen basis values per
 * mirrored pair of cells) on the matrix cores; float16 forms them with
 * packed float16 products, so each basis value carries up to five float16
 * roundings and the per-entry bound above becomes
 * (2 ((1 + u)^6 - 1) + N 2^-24 + 2^-17) sum_j |M_kj x_j| for the forward and
 * 2 sqrt(2) times that relative term for the adjoint, plus N 2^-19 (forward)
 * or N 2^-21 (adjoint) of the largest operand times the largest |M_kj| for
 * float16's subnormal range.  Real and complex arrays at the ABI are float32
 * and complex64 as for SL1M_PREC_FP32.
 *
 * FP32 hi/lo phase (SL1M_PREC_FP32_HILO).  theta = u l + v m + w (n - 1) is
 * formed without float64: every coordinate is split once into a float32 pair
 * a = a_hi + a_lo, each product's leading part a_hi b_hi is split exactly into
 * its rounding p and error e (an FMA), p is reduced exactly to p - rint(p) in
 * [-1/2, 1/2], and the three reduced parts, the errors and the cross terms
 * a_hi b_lo + a_lo b_hi are added in float32: about three roundings of 2^-24
 * turn, as the float64 phase.  It costs about twenty float32 operations per
 * entry against three float64 FMAs, so it is slower on the MI355X; it exists
 * for precision studies.  Delta pixels only, no per-pair beam widths, no grid
 * evaluation, no tuning or serving (SL1M_EINVAL otherwise); float32 and
 * complex64 arrays at the ABI.
 */

/*
 * Evaluation order of the operators.  The element of eq. (deltam) factorises
 * exactly:
 *     exp(-2 pi i (u l + v m + w (n - 1)))
 *       = exp(-2 pi i u l) * exp(-2 pi i v m) * exp(-2 pi i w (n - 1)),
 * and n - 1 depends on l^2 + m^2 only.  When the pixels of a segment (the
 * delta pixels, or one Gaussian (kind, sigma) group) lie on a product set
 * symmetric under l -> -l and m -> -m (a centred image grid, or a subset of
 * one), the four positions (+-|l|, +-|m|) share the last factor, the first
 * two come from per-|l| and per-|m| phasors, and one sincos serves four
 * matrix entries.  Gaussian pixels, eqs. (samlm4)/(samlm5), factorise the
 * same way: the taper exp(-pi sigma^2 D |(u,v) - w(l,m)|^2) is a product of
 * an l part and an m part, the phase is linear in l and m plus terms in
 * l^2 + m^2.  The "grid" evaluation uses that; the "direct" evaluation forms
 * every entry on its own.  Both compute the same operator; they differ by
 * float32 rounding only.  Applies to float32 plans without per-pair beams:
 * to single right-hand-side calls, and to multi-RHS calls of 2, 4 or 8 sides when
 * every grid segment of the plan is a square delta grid (the forward shares
 * each phasor among the sides; sl1m_plan_info.grid_multi); float64 plans,
 * other multi-RHS calls and segments that do not qualify use the direct
 * evaluation.
 */
typedef enum {
  SL1M_GRID_AUTO = 0,    /* grid evaluation when the delta pixels qualify        */
  SL1M_GRID_OFF = 1,     /* direct evaluation always                             */
  SL1M_GRID_REQUIRE = 2  /* grid evaluation; SL1M_EINVAL if the pixels do not
                            qualify (for tests and benchmarks)                   */
} sl1m_grid_mode;

/*
 * One deconvolution problem.  All arrays are device pointers.
 *  l, m      [n_pix] float64  direction cosines of the pixel centres; the
 *                             paper allows arbitrary (off-grid) positions
 *                             (Section "Delta function pixels"); l^2+m^2 < 1.
 *  sigma     [n_pix] float64  Gaussian scale of eq. (gaus),
 *                             f = exp(-pi r^2 / sigma^2) / sigma^2; NULL = all 0.
 *  kind      [n_pix] uint8    sl1m_pixel_kind; NULL = DELTA where sigma == 0,
 *                             GAUSS_WIDE elsewhere.
 *  u, v, w   [n_vis] float64  baseline coordinates in wavelengths.
 *  ant_p, ant_q [n_vis] int32 antennas of each visibility; NULL = unit gains.
 *  ant_gain  [2*n_ant] float64 complex gain constant c_a (re, im) per antenna;
 *                             NULL = 1.
 *  ant_fwhm  [n_ant] float64  power-beam full width at half maximum F_a
 *                             (radians of l, m) per antenna; NULL = flat beam.
 *    The direction-dependent gain of eq. (samdelta) is taken as
 *    A_jk = E_p(l_j,m_j) conj(E_q(l_j,m_j)), E_a = c_a exp(-2 ln2 r^2 / F_a^2),
 *    evaluated at the pixel centre for Gaussian pixels (as eq. (samlm3)
 *    assumes).
 *  precision sl1m_precision.
 *  max_rhs   largest n_rhs that sl1m_forward_multi/sl1m_adjoint_multi will be
 *            called with (sizes the workspace); 0 means 1.
 *  tile_blocks  number of thread blocks the split of one operator application
 *            aims at (more blocks: more parallelism, larger partial-sum
 *            buffers); 0 means 4096, enough to fill the 256 compute units.
 *  grid_mode sl1m_grid_mode.  A segment qualifies for the grid evaluation
 *            when (a) the plan is float32 without per-pair beams, (b) no two
 *            of its pixels share a position, (c) it has at least 1024 pixels
 *            with at least 16 distinct |l| values, and (d) the product set of
 *            its distinct |l| and |m| values (padded to a multiple of 8 |m|
 *            values), times four signs, holds at most 2.5 times as many
 *            positions as it has pixels.  SL1M_GRID_REQUIRE needs at least
 *            one qualifying segment.
 */
typedef struct {
  int64_t n_pix;
  const double* l;
  const double* m;
  const double* sigma;
  const uint8_t* kind;
  int64_t n_vis;
  const double* u;
  const double* v;
  const double* w;
  const int32_t* ant_p;
  const int32_t* ant_q;
  int32_t n_ant;
  const double* ant_gain;
  const double* ant_fwhm;
  int32_t precision;
  int32_t max_rhs;      /* right-hand sides per operator call: 0 or 1, 2, 4, 8 */
  int32_t tile_blocks;  /* blocks one operator launch aims at; 0 = 4096       */
  int32_t grid_mode;    /* sl1m_grid_mode                                     */
  int32_t fwd_vpl;      /* direct forward: visibilities per lane 1, 2, 4; 0 = plan's choice
                           (matrix-core precisions: visibilities per lane of the MFMA
                           forward, each one A operand)                                 */
  int32_t adj_ppl;      /* direct adjoint: pixels per lane 1, 2, 4; 0 = plan's choice
                           (matrix-core precisions: pixels per lane of the MFMA adjoint) */
} sl1m_problem;

typedef struct sl1m_plan sl1m_plan;

/* Bytes of device workspace that sl1m_plan_create() needs for `problem`.
 * Reads sigma, kind, ant_p, ant_q and ant_fwhm with blocking device-to-host
 * copies when they are given (the grouping of pixels and the gain mode set the
 * layout), and l and m unless grid_mode is SL1M_GRID_OFF, the plan is float64
 * or no segment has 1024 pixels (the grid evaluation's tables depend on them);
 * the other arrays are not read.  At most 16 distinct (kind, sigma)
 * Gaussian groups per problem; more gives SL1M_EINVAL. */
sl1m_status sl1m_plan_workspace_bytes(const sl1m_problem* problem, size_t* bytes);

/* Build a plan: derives per-pixel quantities (n, n - 1, 1/n, the wide-field
 * remainder n - 1 + r^2/2, beam factors) and per-visibility gains into the
 * workspace, groups pixels by (kind, sigma) and checks the domain.  The
 * problem's device arrays are read during this call only.  Synchronises
 * `stream` once.  On success *out owns host memory released by
 * sl1m_plan_destroy(). */
sl1m_status sl1m_plan_create(const sl1m_problem* problem, void* workspace, size_t workspace_bytes,
                             void* stream, sl1m_plan** out);

sl1m_status sl1m_plan_destroy(sl1m_plan* plan);

/* ---------------------------------------------------------------------------
 * Autotuning of a problem's launch shapes.  sl1m_tune builds candidate plans of
 * `problem` one after another in `workspace` (size from
 * sl1m_tune_workspace_bytes) and times `reps` forward and adjoint applications
 * of each with HIP events on `stream`: the grid evaluation on and off (when
 * some segment qualifies), split targets tile_blocks of 1024 .. 16384 blocks,
 * and for direct plans 1, 2 or 4 visibilities (forward) and pixels (adjoint)
 * per lane.  The fastest forward + adjoint pair is returned in *out (host),
 * where a candidate replaces the earlier choice (first: every field left at 0)
 * only when at least 1 % faster; copy its fields into the problem before
 * sl1m_plan_create.  The problem's
 * own tile_blocks, grid_mode, fwd_vpl and adj_ppl are ignored (all are
 * searched).  Synchronises `stream` after every candidate; the workspace holds
 * nothing useful afterwards.
 * --------------------------------------------------------------------------- */
typedef struct {
  int32_t tile_blocks, grid_mode, fwd_vpl, adj_ppl;  /* the choice                */
  double forward_ms, adjoint_ms;          /* median per application, the choice  */
  double default_forward_ms;              /* ... with every field left at 0      */
  double default_adjoint_ms;
  int32_t candidates;                     /* configurations timed                */
  int32_t reserved[3];
} sl1m_tuning;

sl1m_status sl1m_tune_workspace_bytes(const sl1m_problem* problem, size_t* bytes);
sl1m_status sl1m_tune(const sl1m_problem* problem, void* workspace, size_t workspace_bytes,
                      int32_t reps, void* stream, sl1m_tuning* out);

/* What a plan decided: evaluation order and split of the operators.  Host
 * call, no device work.  `info` is a host pointer filled on success. */
typedef struct {
  int64_t n_pix, n_vis;
  int32_t precision;        /* sl1m_precision                                   */
  int32_t max_rhs;
  int32_t grid;             /* segments single-RHS calls evaluate on their grid */
  int32_t grid_abs_l;       /* distinct |l| of the delta segment, if on its grid */
  int32_t grid_abs_m;       /* distinct |m| of the delta segment, if on its grid */
  int32_t n_layers;         /* Gaussian (kind, sigma) groups                    */
  int64_t grid_positions;   /* 4 x grid cells evaluated (>= delta pixels)       */
  int32_t fwd_vpl;          /* visibilities per lane, direct forward            */
  int32_t adj_ppl;          /* pixels per lane, direct adjoint                  */
  int32_t n_fchunks;        /* split-K partial rows of the forward (direct)     */
  int32_t n_fchunks_grid;   /* ... of the forward with the grid evaluation      */
  int32_t n_achunks;        /* visibility chunks of the adjoint                 */
  int32_t grid_pairs;       /* grid segments evaluated as mirrored cell pairs   */
  int32_t grid_multi;       /* multi-RHS calls of 2, 4 (and 8) sides up to
                               this count evaluate on the grid (every grid
                               segment a square delta grid); 0: direct        */
  int32_t grid_mfma;        /* matrix-core plan whose forward runs on the grid
                               evaluation (all pixels one square delta grid) */
  int32_t reserved[2];
} sl1m_plan_info;

sl1m_status sl1m_plan_query(const sl1m_plan* plan, sl1m_plan_info* info);

/* Forward operator, eq. (sme): vis[k] = sum_j M_kj x[j] with M from eq. (deltam),
 * (samlm4) or (samlm5) per pixel.  x: real [n_pix]; vis: complex [n_vis].
 * x may be any sign. */
sl1m_status sl1m_forward(sl1m_plan* plan, const void* x, void* vis, void* stream);

/* Adjoint (back-projection of the gradient step, Section "Implementation of
 * SL1M"): g[j] = Re sum_k conj(M_kj) r[k].  r: complex [n_vis]; g: real [n_pix]. */
sl1m_status sl1m_adjoint(sl1m_plan* plan, const void* r, void* g, void* stream);

/* Several real right-hand sides through the same operator in one pass: the
 * paper treats each polarisation independently through the same M (Section
 * "Defining the direct solution"), so Stokes I, Q, U, V share every phasor.
 *   forward: vis[r][k] = sum_j M_kj x[r][j],  x: real [n_rhs][n_pix],
 *            vis: complex [n_rhs][n_vis];
 *   adjoint: g[r][j] = Re sum_k conj(M_kj) rr[r][k],  rr: complex [n_rhs][n_vis],
 *            g: real [n_rhs][n_pix].
 * n_rhs is 1, 2, 4 or 8 and at most the plan's max_rhs (else SL1M_EINVAL).
 * Every pixel kind and gain mode is supported; accumulation is FP32 (FP64 in
 * SL1M_PREC_FP64 plans), each right-hand side summed in the same order as a
 * single-right-hand-side call. */
sl1m_status sl1m_forward_multi(sl1m_plan* plan, int32_t n_rhs, const void* x, void* vis,
                               void* stream);
sl1m_status sl1m_adjoint_multi(sl1m_plan* plan, int32_t n_rhs, const void* rr, void* g,
                               void* stream);

/* Largest eigenvalue of Re(M^H M) (the step-size constant L of the FISTA
 * iteration; the paper leaves the method open) by `iters` steps of power
 * iteration.  Start vector: x0 (device, real [n_pix]) if not NULL, else
 * U[0,1) values from the SplitMix64 generator (Steele, Lea & Flood 2014) at
 * counter j+1 from state `seed` for pixel j.  *rayleigh_out (host) receives
 * the last Rayleigh quotient <x, A x> with |x| = 1.  Synchronises. */
sl1m_status sl1m_estimate_L(sl1m_plan* plan, int32_t iters, uint64_t seed, const void* x0,
                            double* rayleigh_out, void* stream);

typedef struct {
  double lambda;        /* regularisation weight of eq. (cme)                        */
  double eps;           /* stop when |F_k - F_prev| <= eps F_prev between two checks;
                           0 disables (the paper stops on a small relative change)   */
  int32_t max_iter;     /* iteration cap                                             */
  int32_t check_every;  /* iterations between objective checks when eps > 0 (>= 1)   */
  double L;             /* step constant; <= 0 runs sl1m_estimate_L first            */
  double L_safety;      /* factor applied to an estimated L (e.g. 1.01); <= 0 -> 1.01 */
  int32_t power_iters;  /* power-iteration steps when L <= 0 (e.g. 30)               */
  int32_t method;       /* sl1m_method (0: the printed FISTA)                        */
  uint64_t seed;        /* SplitMix64 state for the power-iteration start            */
  double nnz_eps;       /* stop when |nnz_k - nnz_prev| < nnz_eps max(nnz_prev, 1)
                           between two checks (the paper's other stopping rule:
                           the count of non-zero pixels has nearly settled); 0
                           disables.  Checks run every check_every iterations when
                           eps > 0 or nnz_eps > 0.                                   */
} sl1m_solve_params;

/* The iteration sl1m_solve runs.  SL1M_MFISTA is the monotone variant the
 * paper names after its algorithm (Section "Implementation of SL1M"; Beck &
 * Teboulle): from x_0 = y_1 = I_0, t_1 = 1,
 *   z_k = T^{lambda/L}(y_k - Re M^H (M y_k - V) / L);
 *   x_k = z_k if F(z_k) <= F(x_{k-1}) else x_{k-1};
 *   y_{k+1} = x_k + (t_k/t_{k+1})(z_k - x_k) + ((t_k - 1)/t_{k+1})(x_k - x_{k-1}),
 * so F never increases, at the cost of one more forward operator per
 * iteration (F(z_k) is formed and compared on the device).  The server runs
 * SL1M_FISTA only. */
typedef enum { SL1M_FISTA = 0, SL1M_MFISTA = 1 } sl1m_method;

typedef struct {
  int32_t iters;        /* iterations run                                            */
  int32_t converged;    /* 1 if stopped by eps, 2 if stopped by nnz_eps              */
  double L;             /* step constant used                                        */
  double F;             /* objective at the returned image                           */
  double l2_term;       /* 1/2 |V - M I|^2                                           */
  double l1_term;       /* sum_j I_j                                                 */
  int64_t nnz;          /* non-zero pixels                                           */
  int32_t status;       /* sl1m_status of the solve                                  */
  int32_t reserved;
} sl1m_solve_info;

/* The L1 solve of Section "Implementation of SL1M" (FISTA, Beck & Teboulle
 * 2009, with the positive threshold of eq. (threshp)), started from a zero
 * image.  One iteration is one captured graph: the forward operator at the
 * extrapolated point y, the residual against V, the adjoint, then one fused
 * update kernel that takes the gradient step of size 1/L, applies the
 * positive threshold lambda/L, forms the next extrapolated point with the
 * momentum weight of the step sequence t_k, and advances t_k; t_k, 1/L and
 * lambda/L live on the device, so every replay is the same graph.
 * vis: complex [n_vis] data V; img_out: real [n_pix] final I; info: host.
 * Synchronises at the end (and at each objective check when eps > 0).
 * Returns SL1M_EDIVERGED if the final objective is not finite. */
sl1m_status sl1m_solve(sl1m_plan* plan, const void* vis, const sl1m_solve_params* params,
                       void* img_out, sl1m_solve_info* info, void* stream);

/* Warm start (Section "Acceleration strategies": starting from the dirty
 * image, or from an upscaled coarser solution, cuts the iterations, not the
 * cost of one).  The iteration of sl1m_solve from y_1 = I_0 = x0 instead of
 * 0 (t_1 = 1, so the first momentum coefficient is 0).  x0: device, real
 * [n_pix], caller order; not NULL when n_pix > 0 (SL1M_EINVAL); it may alias
 * img_out.  Otherwise as sl1m_solve. */
sl1m_status sl1m_solve_from(sl1m_plan* plan, const void* vis, const void* x0,
                            const sl1m_solve_params* params, void* img_out,
                            sl1m_solve_info* info, void* stream);

/* Iteration state of the FISTA solve after iteration k (the paper's
 * iteration is fully determined by it, with L and lambda): the image I_k and
 * the extrapolated point y_{k+1} (device, real [n_pix], caller order, owned
 * by the caller) and the step-sequence value t_{k+1}; k counts the
 * iterations run so far.  t = 0 marks a fresh start from I_0 = img. */
typedef struct {
  void* img;
  void* y;
  double t;
  int64_t k;
} sl1m_fista_state;

/* Checkpoint and exact resume: runs params->max_iter iterations starting
 * from *state (a fresh start from state->img when state->t == 0) and leaves
 * in *state the state after the last one (img, y, t updated, k advanced by
 * info->iters).  A solve of K1 + K2 iterations equals a resume of K1
 * followed by a resume of K2, bit for bit.  FISTA only (SL1M_EINVAL for
 * MFISTA); state arrays may not alias img_out.  Otherwise as sl1m_solve. */
sl1m_status sl1m_solve_resume(sl1m_plan* plan, const void* vis, sl1m_fista_state* state,
                              const sl1m_solve_params* params, void* img_out,
                              sl1m_solve_info* info, void* stream);

/* Dirty image, the warm start the paper names: img_out[j] =
 * max(0, Re(M^H V)_j / n_vis) (device, real [n_pix], caller order); for unit
 * gains a point source of flux S at pixel j gives S / n_j^2 there.  The
 * division by n_vis and the clip at 0 (the solution is positive) are this
 * library's choice; the paper does not state a normalisation.  Asynchronous
 * on `stream`. */
sl1m_status sl1m_dirty_image(sl1m_plan* plan, const void* vis, void* img_out, void* stream);

/* Kernel timing (tracing).  Between sl1m_timing_begin() and sl1m_timing_end()
 * the plan records a pair of HIP events around every launch of its operator
 * kernels on the launch stream (at most max_launches launches per kind; later
 * launches are not timed).  sl1m_timing_end() synchronises on the recorded
 * events and reports, per kind, the number of timed launches and the sum of
 * their durations in milliseconds.  Kinds: 0 = forward operator kernels,
 * 1 = adjoint operator kernels, 2 = FISTA vector update; and single launches
 * of the grid evaluation inside kinds 0 and 1: 3 = delta forward
 * (k_grid_fwd_delta_pairs or k_grid_fwd_delta), 4 = delta adjoint
 * (k_grid_adj_delta_square or k_grid_adj_delta), 5 = Gaussian forward (one
 * launch per layer), 6 = Gaussian adjoint (every layer in one launch);
 * 7 is unused.
 *
 * Host trace ranges: sl1m_plan_create, sl1m_tune, the power iteration, every
 * solve ("sl1m solve"), sl1m_server_step and each plan build of the server's
 * admission thread are roctx ranges, shown on the host timeline of
 * `rocprofv3 --marker-trace` beside the kernels of `--kernel-trace`. */
typedef struct {
  int64_t launches[8];
  double total_ms[8];
} sl1m_timing;

sl1m_status sl1m_timing_begin(sl1m_plan* plan, int32_t max_launches);
sl1m_status sl1m_timing_end(sl1m_plan* plan, sl1m_timing* out /* host */);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of many solves on one GPU.
 *
 * The paper solves every channel as an independent deconvolution (Sections
 * "NGC5921" and "NGC2403": 63 and 61 per-channel solves).  A server runs many
 * such solves of different sizes together.  It sub-allocates each admitted
 * request's plan and FISTA state from one caller-provided device arena
 * (admission by footprint; a request waits while its footprint does not fit
 * or no slot is free).  Work advances in rounds: one launch of each batched
 * kernel covers the work items of every active request.  A round holds about
 * `round_budget_evals` pixel-visibility evaluations: under the FAIR policy
 * each of the n active requests advances by at most max(budget / n,
 * budget / 32) evaluations (at least one work item, never past the end of its
 * current phase), so small requests finish a whole FISTA iteration per round
 * while large ones advance part of one; under OLDEST_FIRST a round holds
 * max(budget, one FISTA iteration of the earliest admitted request), at most
 * 4 budgets, of which that request may take the whole, requests of at most
 * 128 budgets of work in total a quarter, and the others 1/1024 (close to
 * first-come-first-served for the large requests, small requests not queued
 * behind them).
 * A request whose pixels form one grid segment (see sl1m_grid_mode) runs the
 * grid evaluation; other requests the direct one.  A request's arithmetic and
 * summation order depend only on its own problem: its image is bitwise the
 * same alone and in any mix.  FP32 plans, one right-hand side; the solve runs
 * the power iteration when params->L <= 0, then params->max_iter FISTA
 * iterations (params->eps is not used), then the objective terms.
 * --------------------------------------------------------------------------- */
typedef struct sl1m_server sl1m_server;

typedef struct {
  int64_t rounds;            /* rounds launched                              */
  int64_t completed_rounds;  /* rounds known to have finished on the GPU     */
  double evals_scheduled;    /* operator evaluations launched so far          */
  uint64_t arena_bytes;      /* usable arena bytes                            */
  uint64_t arena_used;       /* bytes held by admitted and reserved requests  */
  int32_t active;            /* requests on the GPU                           */
  int32_t pending;           /* requests waiting for admission or being admitted */
} sl1m_server_stats_t;

/* arena: device memory owned by the caller (256-byte aligned), kept alive
 * until sl1m_server_destroy(); max_slots: at most this many requests on the
 * GPU at once (1..64); round_budget_evals: work per round (<= 0 selects 3e10,
 * about 4 ms of operator work); under OLDEST_FIRST a round grows to one FISTA
 * iteration of the oldest request, at most 4 budgets, so that large requests
 * run in rounds that fill the GPU while small ones keep short rounds.  The
 * server creates its own non-blocking streams (rounds, second lane,
 * admission, result read-back) and one host thread that builds admitted
 * requests' plans on the current device; sl1m_server_destroy() ends it after
 * the build in progress.  Calls on one server from several host threads are
 * serialised by the server's lock (sl1m_server_destroy excepted: no other
 * call may be in progress or follow it). */
sl1m_status sl1m_server_create(void* arena, size_t arena_bytes, int32_t max_slots,
                               double round_budget_evals, sl1m_server** out);

typedef enum {
  SL1M_SERVE_FAIR = 0,         /* equal shares of each round                    */
  SL1M_SERVE_OLDEST_FIRST = 1  /* the earliest admitted request first (it
                                  keeps at least 4/5 of each round), small
                                  requests expedited in the rest, a floor for
                                  the others (default)                          */
} sl1m_serve_policy;

/* Selects how rounds are shared from the next round on.  SL1M_EINVAL for an
 * unknown policy.  Results do not depend on the policy. */
sl1m_status sl1m_server_set_policy(sl1m_server* server, int32_t policy);

/* Queue one solve.  problem: as for sl1m_plan_create (FP32, max_rhs <= 1); its
 * arrays must stay valid until the request is admitted (sl1m_server_poll's
 * times[1] > 0) or done; its tile_blocks sets
 * the request's work-item split (0: 2048, the best of a sweep on a saturated
 * stream of mixed requests).  vis: complex64
 * [n_vis] data and img_out: float32 [n_pix] result, both device pointers valid
 * until the request is done.  Non-blocking apart from reading the problem's
 * grouping arrays (see sl1m_plan_workspace_bytes).  *ticket identifies the
 * request.  SL1M_ENOMEM if its footprint exceeds the whole arena. */
sl1m_status sl1m_server_submit(sl1m_server* server, const sl1m_problem* problem,
                               const void* vis, const sl1m_solve_params* params,
                               void* img_out, uint64_t* ticket);

/* One scheduling step: release finished requests; move requests whose plans
 * the server's admission thread has built into the rounds (in submission
 * order); reserve arena memory and a slot for waiting requests that fit and
 * hand them to that thread; launch the next round (asynchronous; at most 4
 * rounds are in flight, after which the step waits for the oldest).  Plans
 * are built on the thread's own stream while rounds run, so a request becomes
 * active a step or more after its reservation.  Reports the numbers of active
 * requests and of waiting ones, those being admitted included (either pointer
 * may be NULL). */
sl1m_status sl1m_server_step(sl1m_server* server, int32_t* n_active, int32_t* n_pending);

/* *done = 1 once the request's image is in img_out and info (host) is final;
 * for a cancelled request, once no launched round can still read its vis or
 * write its img_out (its memory has been released), so both may then be
 * freed; poll itself releases requests whose rounds have completed;
 * times (host, may be NULL): [submit, admit, finish] in seconds since the
 * server was created (finish = when a step observed the completion). */
sl1m_status sl1m_server_poll(sl1m_server* server, uint64_t ticket, sl1m_solve_info* info,
                             int32_t* done, double* times);

/* Cancel a waiting or running request; its memory is released once no
 * launched round uses it; other requests are unaffected. */
sl1m_status sl1m_server_cancel(sl1m_server* server, uint64_t ticket);

sl1m_status sl1m_server_stats(sl1m_server* server, sl1m_server_stats_t* out);

/* Waits for launched work, releases host resources (not the arena). */
sl1m_status sl1m_server_destroy(sl1m_server* server);

/* Issue rates of the instruction classes the operator kernels consist of.
 * Every matrix entry is evaluated from its closed form (Section "On-the-fly
 * computation versus in-memory computation"), so the operators are bound by
 * instruction issue, and an issue-slot roofline needs the rates of the
 * running GPU.  sl1m_issue_rates runs, on `stream`, one warm-up and one
 * timed kernel per class (eight independent dependency chains per lane,
 * 32 wavefronts per compute unit, 65,536 instructions of the class per
 * lane), synchronises, and writes rates[0..3] = wave64 instructions per
 * second per compute unit of v_fma_f32, v_fma_f64, v_sin_f32 (v_cos_f32
 * issues alike) and v_exp_f32 on the current device.  `scratch` is memory
 * of that device, at least sl1m_issue_scratch_bytes() (one float per
 * thread; contents overwritten; the caller owns it);
 * `rates` is host memory of 4 doubles.  SL1M_ENOMEM when the scratch is
 * too small, SL1M_EHIP on a launch or event failure. */
sl1m_status sl1m_issue_scratch_bytes(size_t* bytes);
sl1m_status sl1m_issue_rates(void* scratch, size_t scratch_bytes, double* rates, void* stream);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, e.g. tight serving loops or harnesses that forbid it): the
 * forward operator of sl1m_forward for one problem, with the plan built in
 * a library-owned device scratch of SL1M_NOALLOC_SCRATCH_BYTES per device
 * (a static array each GPU holds until the process ends) instead of a
 * caller workspace.  problem, x, vis as for sl1m_plan_create and
 * sl1m_forward (the result is the same as theirs, bit for bit).  Allocates
 * no device memory; plans, runs and synchronises `stream` before returning.
 * SL1M_ENOMEM when sl1m_plan_workspace_bytes(problem) exceeds the scratch
 * (e.g. 65,536 pixels x 97,536 visibilities); other errors as
 * sl1m_plan_create / sl1m_forward.  Every call on a GPU reuses that GPU's
 * scratch and overwrites the last call's contents, so two calls that
 * overlapped on one GPU would race: the library serialises the calls of a
 * process (a lock held until the call's kernels have finished), and each
 * process holds its own copy of the scratch. */
#define SL1M_NOALLOC_SCRATCH_BYTES (64u << 20)
sl1m_status sl1m_forward_noalloc(const sl1m_problem* problem, const void* x, void* vis,
                                 void* stream);

/* Message of the last error on this thread ("" if none). */
const char* sl1m_last_error(void);

/* Library version string. */
const char* sl1m_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SL1M_H_ */
