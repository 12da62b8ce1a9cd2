/*
 * kpme.h -- C ABI of the MI355X reciprocal-space Kroneckerised PME library.
 *
 * The library evaluates the long-range (reciprocal) part of the periodic
 * Coulomb sum (Sec. 1.1, Eq. qmutheta_coulomb; Sec. 1.2, Eqs. tau, hexpr,
 * sumhexpr) in the particle-mesh form of Thm. 1 / Eq. formfinale:
 *
 *     phi = S* ( sum_r  A_r (x) B_r (x) C_r ) S q  -  c 1 1^T q
 *
 * with S the order-p cardinal B-spline spread onto a periodic K1 x K2 x K3
 * grid (the B-spline option of Sec. 2.2; or, by plan option, the paper's
 * per-cell Lagrange interpolation), the Kronecker terms from the nested
 * SVD of the smooth-PME kernel (Sec. 2.1.1; or its sinc quadrature,
 * Sec. 2.1.2) expanded into real circulant
 * per-axis factors (Sec. 2.3-2.4), applied as three mode products per term
 * (Sec. 3.2-3.3, Alg. 1 and Alg. 2), and c the constant correction
 * (Sec. 4.1, Eq. termbonsum; Alg. 4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units      Coulomb constant 1; orthorhombic box L1 x L2 x L3, volume V.
 * Grids      K1*K2*K3 values, row-major [k1][k2][k3] (k3 fastest).
 * Particles  positions n x 3 row-major (x, y, z), charges n.  Positions
 *            outside [0, L) are wrapped, never rejected.
 * Types      the plan's precision fixes the element type of every particle
 *            and grid buffer: double for KPME_FP64, float for every other
 *            precision.  Energies are always double.
 * Memory     every pointer argument except those of kpme_factors_compute and
 *            kpme_plan_create's box/grid arrays is a DEVICE pointer owned by
 *            the caller; the plan owns its factors and workspace, allocated
 *            once in kpme_plan_create.  No call other than kpme_plan_create,
 *            kpme_batch_create and the destroy calls allocates or frees
 *            device memory.
 * Streams    `stream` is a hipStream_t (NULL = default stream).  All calls are
 *            asynchronous and stream-ordered; results are valid once the
 *            stream has reached them.  A plan has one workspace: do not use
 *            one plan on two streams concurrently.
 * Errors     every call returns a kpme_status, never aborts or exits, and
 *            validates its arguments before launching anything.  HIP errors
 *            map to KPME_ERROR_DEVICE; kpme_last_error() returns a message
 *            for the calling thread's last failure.
 */
#ifndef KPME_H
#define KPME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kpme_plan_s* kpme_plan_t;
typedef struct kpme_batch_s* kpme_batch_t;

typedef enum {
  KPME_SUCCESS = 0,
  KPME_ERROR_INVALID_VALUE = 1,  /* bad argument; nothing was launched      */
  KPME_ERROR_NOT_SUPPORTED = 2,  /* valid but unsupported (odd p, too large) */
  KPME_ERROR_OUT_OF_MEMORY = 3,  /* device allocation failed                 */
  KPME_ERROR_DEVICE = 4,         /* no usable gfx950 device, or a HIP error  */
  KPME_ERROR_NUMERICAL = 5       /* factor construction failed to converge   */
} kpme_status;

/* Arithmetic of the SKP mode products.  Spread, gather and the intermediate
 * grids use float for every precision but KPME_FP64; the factor
 * construction, the correction and the energy reduction are always FP64.
 *   KPME_FP64   double everywhere, FP64 matrix cores.
 *   KPME_FP32   float grids, FP32 matrix cores.
 *   KPME_BF16X3 every operand split x = hi + lo into two bfloat16 (round to
 *               nearest even); products hi*hi + hi*lo + lo*hi accumulated in
 *               FP32 on the bf16 matrix cores.
 *   KPME_FP16X3 as BF16X3 with IEEE half hi and lo (22 significand bits).
 *               Every half operand is brought into range by a power of two:
 *               one plan-time scale per factor kind (A, B, C; uniform over
 *               terms), bound-derived scales for the intermediates, and a
 *               run-time scale for the input grid from its largest value. */
typedef enum {
  KPME_FP64 = 0,
  KPME_FP32 = 1,
  KPME_BF16X3 = 2,
  KPME_FP16X3 = 3
} kpme_precision;

/* How the kernel tensor is compressed into Kronecker terms. */
typedef enum {
  /* Nested SVD (Sec. 2.1.1, Eq. last_decomp_kron): axis 2 separated first,
   * terms kept by weight; kernel-independent. */
  KPME_SKP_NESTED_SVD = 0,
  /* Sinc quadrature of 1/|m|^2 (Sec. 2.1.2, Eqs. one_over_r_int and
   * quaddecompalpham): nodes lambda_l = log(1 + e^{lh}), weights
   * omega_l = h / (1 + e^{-lh}), l = -N..N, one Kronecker term per node
   * (R = 2N + 1, every term its own axis-2 factor, so r0 = R), applied to
   * x = s |m_hat|^2 with s = max_j L_j^2 so that x >= 1 for m != 0.
   * skp_rank > 0 must be odd and fixes N = (skp_rank - 1) / 2; skp_rank <= 0
   * takes the smallest N whose best h gives a symbol error
   * max_{m != 0} |theta_Lambda(m) - theta_hat(m)| / max theta_hat <= svd_tol
   * (a max-norm tolerance, unlike the nested SVD's Frobenius one). */
  KPME_SKP_SINC_QUADRATURE = 1
} kpme_skp_method;

/* Interpolation between particles and the grid. */
typedef enum {
  /* order-p cardinal B-splines on the periodic grid (smooth PME); the kernel
   * is theta_hat with the B-spline moduli over every DFT mode */
  KPME_INTERP_BSPLINE = 0,
  /* the paper's own scheme (Sec. 2.2, Eqs. interp1d and interpnd; Sec. 4.1):
   * K_j / (L - 1) cells per axis, on each an equispaced product grid of
   * L = spline_order nodes per axis with the end points shared by
   * neighbouring cells (so the nodes form the periodic K_j-point grid), each
   * particle interpolated by the Lagrange basis of its cell; the kernel is
   * the mode-truncated alpha_M, exp(-pi^2 |m_hat|^2 / beta^2) /
   * (pi V |m_hat|^2) for 0 < |m'_j| <= mode_cutoff on every axis, zero
   * elsewhere (no B-spline moduli).  Needs K_j a multiple of L - 1 and
   * 1 <= mode_cutoff with 2 mode_cutoff + 1 <= K_j (no aliasing);
   * L even, 4..12. */
  KPME_INTERP_LAGRANGE = 1
} kpme_interpolation;

/* Form in which the Kronecker terms are applied. */
typedef enum {
  /* real symmetric circulant K_j x K_j factors, three mode products per term
   * on the matrix cores, terms grouped by their axis-2 factor (every
   * precision) */
  KPME_FORM_CIRCULANT = 0,
  /* the rectangular real cos/sin factors of Sec. 2.3-2.4 (Eqs. kronw, VtV):
   * each factor is F^T diag(d_r) F with F the min(2M + 1, K) x K real
   * Fourier rows (M the mode cutoff, or K / 2), so every term shares F and
   * the operator is three thin products into the real mode basis, one
   * scaling by D = sum_r omega_r d_r1 (x) d_r2 (x) d_r3, and three thin
   * products back (plain GEMMs, rocBLAS).  KPME_FP64 and KPME_FP32 only
   * (KPME_ERROR_NOT_SUPPORTED otherwise). */
  KPME_FORM_RECT = 1
} kpme_skp_form;

/* Options of kpme_plan_create_ex (NULL = all defaults, which is what
 * kpme_plan_create uses). */
typedef struct {
  int skp_method;     /* kpme_skp_method, default KPME_SKP_NESTED_SVD        */
  double quad_h;      /* sinc rule: lifting factor h > 0, or <= 0 to choose
                         it by brute force (the h of a geometric scan around
                         pi / sqrt(2N + 1) with the smallest symbol error)  */
  int interpolation;  /* kpme_interpolation, default KPME_INTERP_BSPLINE     */
  int mode_cutoff;    /* Lagrange: M, the largest |m_j| kept; B-spline: 0    */
  int skp_form;       /* kpme_skp_form, default KPME_FORM_CIRCULANT          */
} kpme_plan_options;

typedef struct {
  int grid[3];          /* K1, K2, K3                                        */
  int spline_order;     /* p                                                 */
  int precision;        /* kpme_precision                                    */
  int rank;             /* R, number of Kronecker terms kept                 */
  int r0;               /* distinct axis-2 factors among them (outer SVD)    */
  int total_terms;      /* terms available before truncation                 */
  int64_t max_particles;
  double beta;
  double theta_norm;    /* ||theta_hat||_F                                   */
  double trunc_err;     /* ||theta_hat - theta_hat_R||_F (exact tail)        */
  double zero_mode;     /* c = theta_hat_R(0), the correction constant       */
  size_t workspace_bytes;
  int skp_method;       /* kpme_skp_method of the plan                       */
  int quad_N;           /* sinc rule: N (R = 2N + 1); -1 for the nested SVD  */
  double quad_h;        /* sinc rule: lifting factor h                       */
  double sym_err;       /* sinc rule: max-norm symbol error (relative)       */
  int interpolation;    /* kpme_interpolation of the plan                    */
  int mode_cutoff;      /* Lagrange: M; B-spline: 0                          */
  int skp_form;         /* kpme_skp_form of the plan                         */
} kpme_plan_info_t;

/* Build a plan: the smooth-PME kernel theta_hat on the K1 x K2 x K3 mode grid,
 * its nested SVD (Sec. 2.1.1, Eq. last_decomp_kron; axis 2 separated first),
 * the R largest terms by weight (or, if skp_rank <= 0, the smallest R whose
 * exact Frobenius tail is <= svd_tol * ||theta_hat||_F; Eqs. eym and
 * estimate_svd bound it), the real circulant per-axis factors (Sec. 2.3-2.4,
 * Eq. VtV) in the requested precision, and all device workspace for up to
 * max_particles particles.
 *   box[3]        host, L1..L3 > 0 and finite.
 *   grid[3]       host, 4 <= K_j <= 256 and K_j >= spline_order
 *                 (KPME_ERROR_INVALID_VALUE otherwise).  The operator
 *                 kernels further need K1 <= 128, and, for KPME_BF16X3 and
 *                 KPME_FP16X3, K2 <= 128; and the K1 x K2 slab must fit in
 *                 the 160 KiB of LDS at the plan's precision (K1 = K2 = 128
 *                 fits every precision).  Grids outside these limits return
 *                 KPME_ERROR_NOT_SUPPORTED before any device work.
 *   spline_order  even, 4..12 (odd orders: KPME_ERROR_NOT_SUPPORTED).
 *   ewald_beta    > 0, the Ewald splitting parameter (xi in Eq. hexpr).
 *   skp_rank      R >= 1, or <= 0 to select R by svd_tol; R larger than the
 *                 number of available terms is clamped to it.
 *   max_particles capacity for n in later calls, 0 < max_particles < 2^31.
 *   device        HIP device ordinal the plan lives on.
 * The kernel construction and SVD run on the host in FP64 at plan time.
 * On failure *plan is set to NULL and nothing is left allocated. */
kpme_status kpme_plan_create(kpme_plan_t* plan, const double box[3],
                             const int grid[3], int spline_order,
                             double ewald_beta, int skp_rank, double svd_tol,
                             int precision, int64_t max_particles, int device);

/* kpme_plan_create with options (NULL: defaults): the kernel compression
 * method (nested SVD or sinc quadrature) and its parameters.  Arguments,
 * errors and ownership as for kpme_plan_create; invalid options give
 * KPME_ERROR_INVALID_VALUE, options the library does not implement
 * KPME_ERROR_NOT_SUPPORTED. */
kpme_status kpme_plan_create_ex(kpme_plan_t* plan, const double box[3],
                                const int grid[3], int spline_order,
                                double ewald_beta, int skp_rank,
                                double svd_tol, int precision,
                                int64_t max_particles, int device,
                                const kpme_plan_options* options);

kpme_status kpme_plan_destroy(kpme_plan_t plan);

/* Plan description (host struct filled by the call). */
kpme_status kpme_plan_info(kpme_plan_t plan, kpme_plan_info_t* info);

/* Spread: Q(k) = sum_i q_i prod_j M_p(u_ij - k_j) on the periodic grid,
 * u_ij = K_j (x_ij / L_j mod 1) (the interpolation matrix S_Y of Eq.
 * sxsyfromB, realised with B-splines).  Writes every grid value of `grid`
 * (K1*K2*K3, row-major).  0 <= n <= max_particles. */
kpme_status kpme_spread(kpme_plan_t plan, int64_t n, const void* pos,
                        const void* q, void* grid, void* stream);

/* Reciprocal operator on the grid: phi_grid = sum_r omega_r (A_r (x) B_r (x) C_r)
 * grid_in - c * sum(grid_in) (Eq. formfinale between S and S*, Alg. 2 for
 * each term, Eq. termbonsum for the correction).  grid_in and phi_grid are
 * K1*K2*K3 row-major and must not overlap. */
kpme_status kpme_skp_apply(kpme_plan_t plan, const void* grid_in,
                           void* phi_grid, void* stream);

/* Gather (the transpose interpolation S_X* of Eq. formfinale):
 * pot_i = sum_k W_i(k) phi_grid(k) and force_i = -q_i sum_k grad W_i(k)
 * phi_grid(k), grad W through dM_p/du = M_{p-1}(u) - M_{p-1}(u-1) and
 * d/dx_j = (K_j / L_j) d/du_j.  pot (n) and force (n x 3 row-major) may each
 * be NULL to skip them; q may be NULL when force is NULL. */
kpme_status kpme_gather(kpme_plan_t plan, int64_t n, const void* pos,
                        const void* q, const void* phi_grid, void* pot,
                        void* force, void* stream);

/* Energies from potentials, reduced in FP64 in a fixed order (deterministic):
 * energy4[0] = E_rec = 1/2 sum_i q_i pot_i, energy4[1] = E_self =
 * -(beta / sqrt(pi)) sum q_i^2, energy4[2] = E_neutral = -pi (sum q)^2 /
 * (2 V beta^2), energy4[3] = their sum.  The real-space part of Ewald is not
 * included.  energy4 is a device array of 4 doubles. */
kpme_status kpme_energy(kpme_plan_t plan, int64_t n, const void* q,
                        const void* pot, double* energy4, void* stream);

/* kpme_energy for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid allocation):
 * the same reduction and results, with its scratch -- the per-block FP64
 * partial sums, 3 x 256 doubles (6 KiB) -- in a fixed device array of the
 * library instead of the plan's workspace.  Each GPU holds one such array
 * until the process ends, shared by every call on that GPU: calls that
 * overlap in time on one GPU (on different streams, or from different
 * plans) race on it and must be serialised by the caller.  No call makes
 * any allocation; n is limited only by the plan's max_particles.  Errors as
 * for kpme_energy. */
kpme_status kpme_energy_noalloc(kpme_plan_t plan, int64_t n, const void* q,
                                const void* pot, double* energy4, void* stream);

/* The whole reciprocal path in one call (Alg. 4 on one device): bin the
 * particles by grid brick once, spread, apply the Kronecker operator with its
 * correction, gather potentials and forces, reduce the energies.  pot, force
 * and energy4 as above (pot and force may be NULL; energy4 may be NULL);
 * here E_rec is taken as 1/2 sum_k Q(k) Phi(k) over the grid, which equals
 * 1/2 sum_i q_i pot_i because each particle's B-spline weights sum to one
 * (the same value up to rounding).  Uses the plan's internal grids. */
kpme_status kpme_evaluate(kpme_plan_t plan, int64_t n, const void* pos,
                          const void* q, void* pot, void* force,
                          double* energy4, void* stream);

/* Adjoint of kpme_evaluate for reverse-mode differentiation of
 *   L = g_E * energy4[3] + sum_i g_pot_i * pot_i,
 * the chain rule through the spread, the symmetric corrected operator Theta
 * (Eq. formfinale with Eq. termbonsum) and the gather:
 *   grad_pos_i = grad W_i . [ (g_E q_i + g_pot_i) Phi + q_i Psi ],
 *   grad_q_i   = g_E (pot_i - 2 beta q_i / sqrt(pi) - pi sum(q) / (V beta^2))
 *                + W_i . Psi,
 * with Phi = Theta S q and Psi = Theta S g_pot.
 *   g_energy  DEVICE pointer to one double (NULL: 0).
 *   g_pot     device, n values (NULL: 0).
 *   grad_pos  device, n x 3 (NULL: not computed); grad_q device, n (NULL: not
 *             computed).
 * Costs two spreads, two operator applications and one gather over both
 * grids; allocates nothing. */
kpme_status kpme_evaluate_backward(kpme_plan_t plan, int64_t n,
                                   const void* pos, const void* q,
                                   const double* g_energy, const void* g_pot,
                                   void* grad_pos, void* grad_q,
                                   void* stream);

/* Host-only factor construction, exactly as kpme_plan_create performs it,
 * for inspection and for tests without a device.  All pointers are HOST.
 * Fills, for the n_terms <= max_terms kept terms in order of decreasing
 * weight: omega[r], the Fourier-domain mode vectors vec0[r*K1 + m],
 * vec1[r*K2 + m], vec2[r*K3 + m] (even in m, unit norm) and group[r] (the
 * outer singular-vector index i), plus info3 = {||theta||_F, trunc_err,
 * zero_mode}.  Any output pointer may be NULL.  max_terms must be >= the
 * number kept, else KPME_ERROR_INVALID_VALUE. */
kpme_status kpme_factors_compute(const double box[3], const int grid[3],
                                 int spline_order, double ewald_beta,
                                 int skp_rank, double svd_tol, int max_terms,
                                 int* n_terms, double* omega, double* vec0,
                                 double* vec1, double* vec2, int* group,
                                 double* info3);

/* kpme_factors_compute with options (NULL: defaults).  info6 (host, may be
 * NULL) receives {||theta||_F, ||theta - theta_R||_F, zero_mode, N, h,
 * symbol error}; the last three are -1, 0, 0 for the nested SVD.  With the
 * sinc quadrature the terms come in node order l = -N..N and group[r] = r. */
kpme_status kpme_factors_compute_ex(const double box[3], const int grid[3],
                                    int spline_order, double ewald_beta,
                                    int skp_rank, double svd_tol,
                                    const kpme_plan_options* options,
                                    int max_terms, int* n_terms, double* omega,
                                    double* vec0, double* vec1, double* vec2,
                                    int* group, double* info6);

/* Batched evaluation of independent systems (each with its own box, grid,
 * spline order and rank R = skp_rank[s] >= 1; the batched form of the
 * Kronecker-product method's term independence, Conclusion).
 * kpme_batch_create builds one plan per system (one precision for all; host
 * arrays box3[3*count], grid3[3*count], spline_order, beta, skp_rank,
 * max_particles), autotunes every distinct (grid, order, R, precision) class
 * once, caps every system's stage-2 split at the smallest value that still
 * gives the batch two stage-2 workgroups per CU (the systems fill the device
 * together; override KPME_BATCH_PARTS), and orders the systems by
 * longest-processing-time on an estimated cost.  kpme_batch_evaluate records, for a new argument signature (n[] and
 * the five pointers), one HIP graph and replays it as a single launch on
 * `stream`; an unchanged signature only replays.  The recording is, where
 * every system's kernels have a batched form (the mixed-precision paths),
 * one kernel launch per stage and kernel instance whose grid holds every
 * system's workgroups (a per-launch table of argument tuples and system
 * slices in device memory, largest systems first); otherwise every system's
 * kpme_evaluate launch sequence on parallel graph branches.  The environment
 * variable KPME_BATCH_FUSED=0 forces the second form; KPME_BATCH_PERSISTENT=1
 * records the batched launches in their persistent form (a grid of the
 * resident workgroups that takes the concatenated grid's workgroups from a
 * device counter in cost order, zeroed by a fill kernel at the head of the
 * recording).  A signature change after
 * the first recording synchronises `stream` and then the whole device
 * before the previous recording is released and the new one captured, so
 * no recording ever overlaps a running replay; callers that evaluate in a
 * loop should therefore keep their output buffers.  pos/q/pot/force are device
 * arrays concatenated in system order (offsets = prefix sums of n[s]);
 * energy4 (device) receives 4 doubles per system; pot/force/energy4 may be
 * NULL.  n[s] <= max_particles[s] (host array).  Errors as for the single
 * calls; creation failures name the system. */
kpme_status kpme_batch_create(kpme_batch_t* batch, int count,
                              const double* box3, const int* grid3,
                              const int* spline_order, const double* beta,
                              const int* skp_rank, int precision,
                              const int64_t* max_particles, int device);
kpme_status kpme_batch_destroy(kpme_batch_t batch);
/* The form of the batch's current recording (host outputs, may be NULL):
 * *form = 2 persistent batched launches, 1 batched launches, 0 per-system
 * graph, -1 nothing recorded yet;
 * *launches = kernel launches (graph nodes) replayed per evaluation. */
kpme_status kpme_batch_info(kpme_batch_t batch, int* form, int* launches);
kpme_status kpme_batch_evaluate(kpme_batch_t batch, const int64_t* n,
                                const void* pos, const void* q, void* pot,
                                void* force, double* energy4, void* stream);

/* Native per-stage profiler.  While enabled, every call brackets each of its
 * stages with a pair of hipEvents recorded on the call's stream (at most 2048
 * pairs per stage between two reads; later stages go unrecorded).
 * kpme_plan_profile_read waits for the recorded events and returns, per
 * stage, the summed elapsed milliseconds and the number of recorded launches
 * (host arrays of KPME_NUM_STAGES), then starts a new accumulation.  A stage
 * that launches nothing in a call (the grid sum when the split stage 1
 * reduces the spread's partials itself) records nothing.
 * Enabling creates the events (host-side, no device memory); disabling
 * synchronizes the device and destroys them. */
#define KPME_NUM_STAGES 7
enum {
  KPME_STAGE_SPREAD = 0,     /* grid clear + spread (binning included)      */
  KPME_STAGE_GRID_SUM = 1,   /* FP64 sum of the input grid (correction)     */
  KPME_STAGE_SKP1 = 2,       /* axis-2 mode products of the r0 groups      */
  KPME_STAGE_SKP2 = 3,       /* fused axis-0/axis-1 products of all terms  */
  KPME_STAGE_FINALIZE = 4,   /* partial-slab sum, transpose, correction    */
  KPME_STAGE_GATHER = 5,     /* potentials and forces                      */
  KPME_STAGE_ENERGY = 6      /* FP64 energy reduction                      */
};
kpme_status kpme_plan_profile(kpme_plan_t plan, int enable);
kpme_status kpme_plan_profile_read(kpme_plan_t plan, double* total_ms, int64_t* counts);

/* Project autotuner for the work shapes of the Kronecker operator: for
 * BF16X3/FP16X3 the stage-2 term streams per workgroup (1 or 2: each stream
 * has its own waves over the shared Y slab, so this sets the waves per
 * workgroup), for each of them the stage-2 split (the number of term ranges
 * per k3 slab, 1..8); the stream count of the fastest pair is kept, with the
 * smallest split within 3% of that count's fastest (other precisions: the
 * split alone); and, for BF16X3/FP16X3 with K3 <= 160, the stage-1 split
 * (workgroups per tile of 64 grid positions, 1..6; the fastest is kept).  Times every candidate on `stream` with hipEvents and
 * records the choices in a process-wide cache and, when the environment
 * variable KPME_TUNE_CACHE names a file, on disk ("key value" lines keyed by
 * what is tuned, grid, order, R, r0 and precision), which later plans of the
 * same class read at creation.  Synchronizes the stream.  The contents of
 * the plan's internal grids are overwritten. */
kpme_status kpme_plan_autotune(kpme_plan_t plan, void* stream);
/* The stage-2 work split in use (-1 for an invalid handle). */
int kpme_plan_stage2_parts(kpme_plan_t plan);
/* The stage-1 split in use (workgroups per 64-position tile; used by BF16X3
 * and FP16X3 with K3 <= 160), -1 for an invalid handle. */
int kpme_plan_stage1_split(kpme_plan_t plan);
/* The stage-2 term streams per workgroup in use (BF16X3/FP16X3: 1 or 2;
 * other precisions 1), -1 for an invalid handle. */
int kpme_plan_stage2_streams(kpme_plan_t plan);

const char* kpme_status_string(kpme_status s);
const char* kpme_last_error(void);
/* Number of gfx950 devices visible (0 without one); never fails. */
int kpme_device_count(void);

#ifdef __cplusplus
}
#endif
#endif /* KPME_H */
