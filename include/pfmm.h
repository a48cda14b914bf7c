/*
 * pfmm.h — C ABI of libpfmm, a natively periodic Fast Multipole Method for
 * MI355X (gfx950).
 *
 * Method: N. Y. Gnedin, "Natively Periodic Fast Multipole Method:
 * Approximating the Optimal Green's Function" (ApJ).  The library computes
 * the potential of a density sampled on a uniform N^3 periodic mesh with the
 * paper's FMM (Sec. 2): an oct-tree whose nodes carry p^3 "gridlet" effective
 * masses (the Cartesian-multipole representation of Sec. 2, p being the
 * paper's N_g), the upward projection of Eq. 5, the interaction-zone
 * convolution of Eq. 6 with a periodic Green's function at level 2 and the
 * non-periodic algorithm with periodic neighbour selection below it (Sec. 2),
 * the downward projection of Eq. 7, and the direct 27-node near zone of a leaf.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Unit periodic box, N^3 cells of side h = 1/N, C order with x slowest:
 *    cell (i, j, k) is element (i*N + j)*N + k.
 *  - Green's-function normalisation G_0 = -1/(4 pi r) (Sec. 1), so that the
 *    potential solves lap(Phi) = rho and
 *        Phi_i  ~=  h^3 * sum_j G((x_i - x_j) wrapped) rho_j       (Eq. 4).
 *    The FMM approximates this periodic convolution; the self term G(0) of
 *    the real-space kinds is the potential at the centre of a uniform cube
 *    cell, -c0/(4 pi h) with c0 = 3 ln((sqrt3+1)/(sqrt3-1)) - pi/2.
 *  - Device pointers are HIP device addresses (e.g. a torch tensor's
 *    data_ptr()); the caller owns them.  The plan owns its tables and
 *    workspaces.  No entry point takes ownership of caller memory.
 *  - Plan and batch handles are opaque tokens, not addresses.  Each carries
 *    a generation count: once its object is destroyed the handle is refused
 *    with PFMM_ERR_BAD_HANDLE, also after the library has reused its slot.
 *    Calls on one handle must not overlap with its destroy.
 *  - Every entry point returns a pfmm_status.  Host-side argument checks run
 *    before anything is enqueued.  Asynchronous device faults surface as
 *    PFMM_ERR_HIP from a later call that synchronises.  pfmm_last_error()
 *    returns a message for the calling thread's last failure.
 */
#ifndef PFMM_H
#define PFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pfmm_plan_s* pfmm_plan_t;

typedef enum {
  PFMM_OK = 0,
  PFMM_ERR_INVALID_ARG = 1,   /* bad size, kind, option or pointer          */
  PFMM_ERR_UNSUPPORTED = 2,   /* valid but outside what the library handles  */
  PFMM_ERR_OUT_OF_MEMORY = 3, /* a plan-time allocation failed              */
  PFMM_ERR_HIP = 4,           /* a HIP runtime call or a kernel failed      */
  PFMM_ERR_CAPTURE = 5,       /* a call that allocates or synchronises was
                                 made while the plan's stream is being
                                 captured into a graph                      */
  PFMM_ERR_BAD_HANDLE = 6     /* not a live plan or batch handle            */
} pfmm_status;

/* Periodic Green's functions. */
typedef enum {
  /* "Exact-in-real-space" G_X(x) = -1/(4 pi |x wrapped|)  (Eq. 2). */
  PFMM_GREEN_X = 0,
  /* "Exact-in-Fourier-space" G_K, the inverse transform of -1/k^2 with the
   * k = 0 mode removed, k = 2 pi n, n_i in [-N/2+1, N/2]  (Eq. 1).  Between
   * mesh points it is the real even trigonometric interpolant that splits
   * the Nyquist term equally between n_i = +N/2 and -N/2. */
  PFMM_GREEN_K = 1,
  /* Approximately optimal G_S1 (Eq. 9): G_X of the mapped separation
   * x_hat = (9/(8 pi)) sin(pi x) - (1/(24 pi)) sin(3 pi x), per component. */
  PFMM_GREEN_S1 = 2,
  /* The ansatz G_S of Sec. 3 with free a_1 and a_2 (n <= 2):
   * xi(t) = sin(pi t)/pi + a_1 (sin(3 pi t)/(3 pi) - sin(pi t)/pi)
   *                      + a_2 (sin(5 pi t)/(5 pi) - sin(pi t)/pi),
   * set by PFMM_OPT_GS_A1 (default -1/8) and PFMM_OPT_GS_A2 (default 0).
   * The defaults give G_S1; a_1 = -25/128, a_2 = 3/128 give the variant whose
   * map is t + O(t^7). */
  PFMM_GREEN_S = 3,
  /* The Ewald Green's function of Sec. 1:
   *   G_E(x) = G_X(x) erfc(r/r_S) + 1/(2 pi^(3/2) r_S)
   *            + inverse transform of -exp(-k^2 r_S^2/4)/k^2 (k != 0),
   * the real-space part on the nearest image, the Fourier part over the mesh
   * frequencies as for G_K.  r_S is set by PFMM_OPT_EWALD_RS (default 0.1 of
   * the box).  At zero separation the Newtonian part of G_X erfc takes the
   * cube self value and the rest its limit 1/(2 pi^(3/2) r_S). */
  PFMM_GREEN_E = 4,
  /* A learned approximation of the optimal G_* (Sec. 3 defines G_* as the G
   * with which FMM and PM agree; Sec. 4 proposes parameterising it): G_S1's
   * tables with the interaction-zone entries corrected by the network of
   * pfmm_learned_set (weights also through PFMM_OPT_LEARNED_WEIGHTS).
   * Without weights a solve uses the uncorrected G_S1 tables (the fallback),
   * returns PFMM_OK and records the fallback in pfmm_last_error(). */
  PFMM_GREEN_LEARNED = 5
} pfmm_green;

/* Arithmetic of the two contraction-heavy steps (interaction-zone
 * convolution and near zone).  Tabulation of G always runs in FP64. */
typedef enum {
  /* FP32 products and FP32 accumulation.  The spectral interaction zones
   * (PFMM_OPT_M2L) are FP64 in every precision.  With GEMM zones the leaf
   * level's FP32 sums, which cancel 10^2-10^3 fold, are amplified toward the
   * leaf corners by L2P's extrapolation beyond the outer gridlet nodes: at
   * 256^3, p = 8 that leaves 8e-5 of max|phi| against the FP64 reference
   * FMM (2e-5 relative L2 against PM), against 3e-6 for the spectral zones;
   * PFMM_OPT_FP64_LEVELS = L - 1 removes it. */
  PFMM_PREC_FP32 = 0,
  /* Split precision: each FP32 operand x is held as hi = bf16(x) and
   * lo = bf16(x - hi); products hi*hi + hi*lo + lo*hi on the BF16 matrix
   * cores with FP32 accumulation. */
  PFMM_PREC_BF16X3 = 1,
  /* FP64 throughout: every level's gridlets and interaction zones, the mesh
   * transfers and the near zone (direct summation in FP64, whatever
   * PFMM_OPT_NEAR says).  pfmm_solve then rounds only its FP32 result;
   * pfmm_solve_f64 takes and returns FP64 arrays.  Needs the leaf's FP64
   * transfers to fit in 64 KiB of LDS (p (s + 1) + s^2 (s + 1) + s^2 p + s p^2
   * <= 8192 doubles, and the same for L2P; every s <= 16 with p <= 9): else
   * PFMM_ERR_UNSUPPORTED.  Not accepted by batches. */
  PFMM_PREC_FP64 = 2
} pfmm_precision;

/* Options for pfmm_plan_set. */
typedef enum {
  /* value: int32 pfmm_precision.  Default PFMM_PREC_FP32. */
  PFMM_OPT_PRECISION = 1,
  /* value: hipStream_t (pointer-sized).  The stream solve enqueues on.
   * Default: the null stream. */
  PFMM_OPT_STREAM = 2,
  /* value: double a_1 of the G_S ansatz (Sec. 3); only for PFMM_GREEN_S.
   * Re-tabulates G synchronously. */
  PFMM_OPT_GS_A1 = 3,
  /* value: int32 0, 1 or 2.  Non-zero: solve records a start and an end
   * HIP event around every stage's launches, and around each kernel of the
   * spectral interaction zones and of the FFT near zone, on the stream each
   * runs on (the events are created when profiling is first switched on;
   * recording them allocates nothing); pfmm_plan_stage_times,
   * pfmm_plan_level_times and pfmm_plan_kernel_times read them.  1: the
   * near zone runs on the plan's stream before the tree, so every interval
   * is a stage alone on the device.  2: the near zone stays beside the tree
   * as in an unprofiled solve (live durations of overlapped kernels).
   * Default 0. */
  PFMM_OPT_PROFILE = 4,
  /* value: int32 in [0, 30]: keep the gridlet masses and potentials of the
   * coarsest levels 2 .. 1+value (those the tree has) in FP64, with their M2M, interaction-zone
   * sums (on the FP64 matrix cores at p = 8) and L2L in FP64.  The downward
   * interpolation (Eq. 7, and its leaf analogue when s > p) extrapolates past
   * a parent's outermost gridlet nodes, so rounding noise in a coarse field
   * is amplified on its way to the mesh, most at leaf corners.  Default
   * max(2, L - 2): levels 2 .. L - 1, every level above the leaf, for
   * L >= 4 (at 512^3, L = 5, an FP32 level 4 would leave 1e-4 of max|phi|,
   * FP64 storage 7e-7), and levels 2 and 3 for L <= 3; L - 1 or more also
   * keeps the leaf level in FP64. */
  PFMM_OPT_FP64_LEVELS = 5,
  /* value: int32 0 or 1.  1 makes the plan the non-periodic twin used to
   * separate the multipole-expansion error from the Green's-function error
   * (Sec. 3, Eq. 3): the free-space G_0(x) = -1/(4 pi |x|) with no periodic
   * images in every table, and every zone (level-2 zone: all non-neighbour
   * nodes of the 4^3 level, offsets in [-3, 3]^3 \ [-1, 1]^3) keeps only
   * source nodes inside the box.  Needs PFMM_GREEN_X and a plan without
   * learned tables; re-tabulates (plan time).  Isolated plans are not
   * accepted by batches, the learned-table calls, pfmm_plan_direct or the
   * FFT interaction zones.  With PFMM_ACCEL_FD4 the accelerations use the
   * periodic stencil (the two outermost cell layers of each face are not
   * meaningful); PFMM_ACCEL_EXPANSION gives them everywhere.  Default 0. */
  PFMM_OPT_ISOLATED = 6,
  /* value: double a_2 of the G_S ansatz (Sec. 3); only for PFMM_GREEN_S.
   * Re-tabulates G synchronously. */
  PFMM_OPT_GS_A2 = 7,
  /* value: int32 pfmm_accel, how pfmm_solve forms `accel`.  Switching to
   * PFMM_ACCEL_EXPANSION allocates and tabulates its near-zone kernels
   * (plan time; re-tabulated with G).  Default PFMM_ACCEL_FD4. */
  PFMM_OPT_ACCEL = 8,
  /* value: double r_S in (0, 1/4] (box units), the Ewald splitting radius of
   * PFMM_GREEN_E; only for that kind.  Re-tabulates G synchronously. */
  PFMM_OPT_EWALD_RS = 9,
  /* value: int32 pfmm_m2l, how the interaction zones are summed.  Switching
   * to PFMM_M2L_FFT creates FFT plans and up to 1 GiB of grids and transforms
   * the level tables (plan time; transformed again when G changes).  Not for
   * isolated plans, batches or learned tables.  Default PFMM_M2L_GEMM. */
  PFMM_OPT_M2L = 10,
  /* value: int32 pfmm_near, how the leaf near zone is summed.  Switching to
   * PFMM_NEAR_FFT creates FFT plans and about 100 bytes of buffers per cell
   * and transforms the near-zone kernels (plan time; transformed again when G
   * or PFMM_OPT_ACCEL changes).  Batches take such plans for leaf edges
   * s = 4, 8, 16 (the library's own transforms).  Default PFMM_NEAR_DIRECT. */
  PFMM_OPT_NEAR = 11,
  /* value: PFMM_MLP_PARAMS floats, the weights of the table-correction
   * network (same as pfmm_learned_set with BF16 inference), meant for
   * PFMM_GREEN_LEARNED plans.  Synchronises. */
  PFMM_OPT_LEARNED_WEIGHTS = 12,
  /* value: int32 0 or 1.  1 folds P2M into the FFT near zone's forward leaf
   * transforms and L2P into the potential's inverse ones (Sec. 2: the leaf
   * steps read and write the same cells), when the library's own transforms
   * run (leaf edge 8 or 16, p = 4 or 8) and the leaf level is FP32: the
   * density is read once and the potential written once, two launches fewer.
   * The tree then starts only after the forward transforms and the inverse
   * waits for the whole tree, so the near zone no longer runs beside the
   * coarse levels' small kernels: at 256^3, L = 4, p = 8 (FP32 leaf-level
   * zones) a solve takes about 1.00 ms folded against 0.96 ms unfolded.
   * Default 0. */
  PFMM_OPT_FOLD = 13,
  /* value: int32 0 or 1.  1 sums the spectral interaction zones (PFMM_M2L_SPECTRAL,
   * Eq. 6 per frequency) of a 16^3 leaf level (L = 4) in FP32: the level's
   * spectra stored in FP32 (the node transforms compute in FP64), each of a
   * target's 36 zone columns (six or three offsets along a line, both
   * parities) summed in FP32 and the column sums added in FP64.  Every
   * other level and tree keeps FP64 stencils.  At 256^3, p = 8 the level's
   * transforms and stencil take 0.25 instead of 0.37 ms and the potential
   * moves by up to 1.5e-5 of max|phi| (at leaf corners, where L2P
   * extrapolates), relative L2 against PM with the same G 1.3e-6 instead of
   * 1.0e-6.  Default 0. */
  PFMM_OPT_ZONES_FP32 = 14
} pfmm_option;

/* Leaf near-zone algorithm (the 27 neighbour leaves, Sec. 2). */
typedef enum {
  /* Direct summation as a block-Toeplitz GEMM over the 27 leaf offsets
   * (matrix cores or the portable kernel, as PFMM_OPT_PRECISION selects). */
  PFMM_NEAR_DIRECT = 0,
  /* FFT convolution on the doubled grid, the route the paper takes (Sec. 2
   * and 3): each leaf's cells zero-padded to (2s)^3 and transformed once
   * (rocFFT, FP32), the 27 neighbours' transforms multiplied by the
   * transformed kernels G(h (m - s e)) (FP64 DFT at plan time, stored FP32)
   * and added per frequency, one inverse transform per leaf.  The cyclic
   * convolution on 2s points equals the linear one at the target cells.
   * Same sums as the direct route up to rounding; the precision option
   * does not apply to it.  With PFMM_ACCEL_EXPANSION the three acceleration
   * kernels reuse the forward transforms.  For leaf edges s = 4, 8, 16 the
   * transforms are the library's own (one workgroup per leaf, in LDS, reading
   * and writing the mesh directly); other s use rocFFT on zero-padded blocks.
   * pfmm_solve then needs density, potential and accel 16-byte aligned
   * (PFMM_ERR_INVALID_ARG otherwise). */
  PFMM_NEAR_FFT = 1
} pfmm_near;

/* Interaction-zone (M2L, Eq. 6) algorithm. */
typedef enum {
  /* Block-Toeplitz GEMM over the zone's offsets (matrix cores or the
   * portable kernel, as PFMM_OPT_PRECISION selects). */
  PFMM_M2L_GEMM = 0,
  /* The Hierarchical Particle-Mesh form the paper runs (Sec. 2): per target
   * node the effective masses of its whole zone on one uniform grid, one FFT
   * convolution with G (rocFFT; FP64 transforms for the levels kept in FP64,
   * PFMM_OPT_FP64_LEVELS, FP32 for the rest).  Levels >= 3: the 6^3 children of the
   * parent's neighbours with the target's neighbours zeroed, padded to
   * (8p)^3; level 2: the periodic (4p)^3 level.  A comparator: same sums as
   * the GEMM up to rounding. */
  PFMM_M2L_FFT = 1,
  /* Spectral stencils, for p = 4, 6 and 8: every node's gridlet transformed
   * once on its (2p)^3 cyclic grid (exact for the block convolutions of
   * Eq. 6, whose separations |a - a'| <= p - 1 have distinct residues), the
   * zone's offsets (189 per parity class, the level-2 zone) summed per
   * frequency with the transformed kernels G(eta_l (m - p d)), one inverse
   * per node.  All in FP64 on the vector ALUs, whatever
   * PFMM_OPT_PRECISION and PFMM_OPT_FP64_LEVELS say; masses are read and
   * potentials added in each level's precision.  Allocates about
   * 2 (2p)^2 (p + 1) x 16 bytes per leaf-level node (0.3 GB at 16^3 nodes,
   * p = 8) and transforms the kernels of the 343 offsets in [-3, 3]^3 per
   * level (plan time; again when G changes).  Periodic and isolated plans
   * and batches (the zones then run as the plan's own launches in the
   * batch graph); not with learned tables. */
  PFMM_M2L_SPECTRAL = 2
} pfmm_m2l;

/* How accelerations are formed (Sec. 3: PM differences its potential, the
 * FMM takes them from its expansion). */
typedef enum {
  /* -grad(potential) by periodic 4th-order central differences of the mesh
   * potential. */
  PFMM_ACCEL_FD4 = 0,
  /* From the expansion: the far part is minus the analytic gradient of each
   * leaf's local expansion (the degree p-1 interpolant that L2P evaluates) at
   * the cell centre; the near part is the direct sum over the 27 leaves of
   * each source cell's acceleration as PM's 4th-order difference of the
   * potential gives it, D_i(x) = -(8 (G(x + h e_i) - G(x - h e_i))
   * - (G(x + 2h e_i) - G(x - 2h e_i))) / (12 h).  Three more near-zone
   * contractions (on the near zone's stream) and one gradient interpolation
   * per component. */
  PFMM_ACCEL_EXPANSION = 1
} pfmm_accel;

/* Stages reported by pfmm_plan_stage_times (durations summed over levels). */
typedef enum {
  PFMM_STAGE_P2M = 0,
  PFMM_STAGE_M2M = 1,
  PFMM_STAGE_M2L = 2,   /* interaction zones of all levels (Eq. 6)      */
  PFMM_STAGE_L2L = 3,
  PFMM_STAGE_L2P = 4,
  PFMM_STAGE_NEAR = 5,  /* direct near zone of the leaves               */
  PFMM_STAGE_FD4 = 6,
  PFMM_STAGE_COUNT = 7
} pfmm_stage;

/* Intermediate buffers readable with pfmm_plan_read (for testing a stage). */
typedef enum {
  /* Gridlet effective masses of level l: [8^l nodes][p^3], nodes and gridlet
   * points both in C order, as float (FP64 levels are rounded).  Output of
   * P2M (l = L) and M2M (Eq. 5). */
  PFMM_BUF_MULTIPOLE = 0,
  /* Gridlet potentials of level l, same layout: the interaction-zone sum of
   * Eq. 6 plus the parent's field carried down by Eq. 7. */
  PFMM_BUF_LOCAL = 1,
  /* FP64 samples G(j / (2^l p)) used by the interaction-zone convolution of
   * level l (Eq. 6 arguments), j in [-(4p-1), 4p-1]^3, C order: (8p-1)^3
   * doubles.  `dst` is then a double*. */
  PFMM_BUF_TABLE_LEVEL = 2,
  /* FP64 mesh samples G(j h) of the near zone, j in [-(2s-1), 2s-1]^3 with
   * the cube self term at j = 0: (4s-1)^3 doubles (`level` ignored). */
  PFMM_BUF_TABLE_NEAR = 3
} pfmm_buffer;

/*
 * Create a plan for an N^3 box, a uniform tree of depth L (levels 2..L,
 * 2^l nodes per axis at level l, leaves of s = N/2^L cells per axis), p^3
 * gridlet masses per node and the Green's function `green_kind`.
 *
 *   N     power of two, 8 <= N <= 1024 (else PFMM_ERR_INVALID_ARG)
 *   L     2 <= L and 2^L <= N (else PFMM_ERR_INVALID_ARG); a leaf width
 *         s = N/2^L above 16 is refused with PFMM_ERR_UNSUPPORTED (the mesh
 *         transfers stage one leaf in 64 KiB of LDS)
 *   p     1 <= p <= 10
 *
 * Tabulates G on the device in FP64 (plan time) and allocates every
 * workspace, so that pfmm_solve never allocates.  Synchronises the device.
 * On success *out receives the handle; on failure *out is set to NULL.
 */
pfmm_status pfmm_plan_create(int N, int L, int p, int green_kind, pfmm_plan_t* out);

/*
 * Set a plan option (pfmm_option).  `value` points to `bytes` bytes holding
 * the option's type (see the enum).  May synchronise; never called by solve.
 */
pfmm_status pfmm_plan_set(pfmm_plan_t plan, int option, const void* value, size_t bytes);

/*
 * Solve: potential = FMM approximation of h^3 sum_j G(x_i - x_j) rho_j.
 *
 *   density    device, const float[N*N*N], C order (read only)
 *   potential  device, float[N*N*N], overwritten
 *   accel      device, float[3][N*N*N] (components x, y, z), overwritten with
 *              the accelerations -grad(potential) formed as PFMM_OPT_ACCEL
 *              selects (default: periodic 4th-order central differences of
 *              the potential, Sec. 3), or NULL to skip
 *
 * Enqueues on the plan's stream; does not allocate and does not synchronise.
 * The near zone (which reads only the density) runs on a second stream owned
 * by the plan, forked from the plan's stream and joined back to it by events
 * before the interpolation to the mesh is added, so the two parts of the
 * potential (Sec. 2) overlap; the whole solve is still ordered on the plan's
 * stream and may be captured into a HIP graph from it.  The order of the
 * arithmetic, and so the result, is the same as with profiling on.
 * No mean is removed: the density normally has zero mean (G_K ignores the
 * mean by construction).  `potential` and `accel` must not alias `density`.
 */
pfmm_status pfmm_solve(pfmm_plan_t plan, const float* density, float* potential, float* accel);

/*
 * The same solve with FP64 arrays, for PFMM_PREC_FP64 plans (the plain FP64
 * periodic FMM; PFMM_ERR_INVALID_ARG for other plans):
 *
 *   density    device, const double[N*N*N], C order (read only)
 *   potential  device, double[N*N*N], overwritten
 *   accel      device, double[3][N*N*N], or NULL
 *
 * Same ordering, stream and no-allocation rules as pfmm_solve.  With L = 2
 * and s = p the FMM is the exact periodic convolution of Eq. 4 (Sec. 3:
 * identical by construction), here up to FP64 rounding.
 */
pfmm_status pfmm_solve_f64(pfmm_plan_t plan, const double* density, double* potential,
                           double* accel);

/*
 * Copy a plan buffer (pfmm_buffer) at tree level `level` (2..L) into the
 * device array `dst`: 8^level * p^3 floats for the gridlet buffers of the
 * last solve, or the FP64 tables described with the enum.  Enqueued on the
 * plan's stream like solve.
 */
pfmm_status pfmm_plan_read(pfmm_plan_t plan, int buffer, int level, void* dst);

/*
 * Per-solve durations in milliseconds of each stage, pfmm_stage, as the sum of its
 * timed intervals, averaged over the most recent (at most 16) solves made
 * since PFMM_OPT_PROFILE was switched on, and the timed intervals of each
 * stage in one solve, into ms[PFMM_STAGE_COUNT] and
 * launches[PFMM_STAGE_COUNT] (host arrays; launches may be NULL).  Waits for
 * those solves' events.  PFMM_ERR_INVALID_ARG if no profiled solve has run.
 */
pfmm_status pfmm_plan_stage_times(pfmm_plan_t plan, double* ms, int* launches);

/*
 * Per-level split of a stage with one launch per tree level (PFMM_STAGE_M2M,
 * PFMM_STAGE_M2L or PFMM_STAGE_L2L; Eqs. 5-7): ms[l] for l = 0..L (host
 * array of L + 1 doubles; entries of levels without a launch are 0), averaged
 * over the same profiled solves as pfmm_plan_stage_times.  The M2L entry of
 * a level covers its whole interaction-zone convolution, operand splitting and
 * group reduction included.  PFMM_ERR_INVALID_ARG for another stage or if no
 * profiled solve has run.
 */
pfmm_status pfmm_plan_level_times(pfmm_plan_t plan, int stage, double* ms);

/*
 * Durations of the kernels of one stage at one tree level (level 0 for the
 * stages without levels), averaged over the same profiled solves: ms[part]
 * for part = 0 .. *count - 1 (host array of 8 doubles).  The spectral
 * interaction zones of a level have three parts (0 node transforms, 1
 * stencil, 2 inverse transforms); the FFT near zone has the forward
 * transforms (0), then the stencil (1 + 2t) and the inverse (2 + 2t) of
 * each kernel t (the potential's, then one per acceleration component);
 * every other stage and level is one part.  *count = 0 when none ran.
 */
pfmm_status pfmm_plan_kernel_times(pfmm_plan_t plan, int stage, int level, double* ms, int* count);

/* Query plan geometry: leaf width s and the number of table entries
 * per tree level ((8p-1)^3) into *s and *table_entries (either may be NULL). */
pfmm_status pfmm_plan_info(pfmm_plan_t plan, int* s, int64_t* table_entries);

/* Release a plan and everything it owns.  Synchronises its stream.  NULL is
 * accepted and ignored.  Batches that pfmm_solve_batch made with the plan
 * are released with it; a plan bound to a live batch of pfmm_batch_create
 * is refused (PFMM_ERR_INVALID_ARG): destroy the batch first. */
pfmm_status pfmm_plan_destroy(pfmm_plan_t plan);

/*
 * Batches of independent fields (fields of different N and p in one solve).
 *
 * pfmm_batch_create binds n plans to their density and potential device
 * arrays (density[i], potential[i] as for pfmm_solve on plans[i]) and builds
 * work lists of independent contraction items for the whole batch (every
 * interaction-zone level and near zone of every field, split into workgroup
 * tiles of targets of one class):
 *   - the near zone of a plan in PFMM_PREC_BF16X3 with 8^3-cell sub-blocks
 *     (leaf width 8 or 16) runs on the BF16 matrix cores, 2-term split, as in
 *     pfmm_solve;
 *   - FP64 levels at p = 8 run on the FP64 matrix cores;
 *   - everything else runs in the portable kernel: FP64 levels in FP64, the
 *     rest in FP32 with FP64 per-offset running totals.
 * Each list is drained by one persistent kernel through an atomic counter.
 * A plan with PFMM_NEAR_FFT (leaf edges 4, 8, 16 only) has no near-zone
 * items, and one with PFMM_M2L_SPECTRAL no interaction-zone items: their
 * transforms and stencils run as their own kernels in the same graph,
 * beside the matrix-core persistent kernels.
 * The portable items fall into groups by block edge (p for interaction zones,
 * min(s, 8) for near zones), FP32 or FP64 and near or interaction zone; the
 * tile width (targets per thread: 1, 2 or 4) of each FP32 group is picked by
 * timing the group's own items at each width (or read from the JSON file
 * named by the environment variable PFMM_TUNE_CACHE, key "batch-q<q>-f32-
 * <near|zone>", which it then updates).  The whole batch solve -- upward
 * passes, the persistent launches, downward passes -- is captured into a HIP
 * graph on the batch's own stream, ordered with the stream of plans[0].  It
 * allocates, runs solves and synchronises; it is plan time.
 *
 * Requirements: 1 <= n <= 4096; live plans on one device, p <= 8, not
 * PFMM_PREC_FP64; the plans are not solved concurrently with the batch (it
 * uses their workspaces); density and potential 16-byte aligned for plans
 * with PFMM_NEAR_FFT.  Precision and FP64 levels are those of each plan at
 * batch creation.  While the batch lives its plans refuse pfmm_plan_destroy
 * and the options that change what its graph uses (precision, isolated
 * twin, FP64 levels, M2L and near-zone routes).  PFMM_ERR_CAPTURE while the
 * stream of plans[0] is being captured.
 */
typedef struct pfmm_batch_s* pfmm_batch_t;
pfmm_status pfmm_batch_create(int n, const pfmm_plan_t* plans, const float* const* density,
                              float* const* potential, pfmm_batch_t* out);

/* Solve the whole batch: one graph launch on the stream of plans[0].  Does
 * not allocate or synchronise.  Potentials are overwritten. */
pfmm_status pfmm_batch_solve(pfmm_batch_t batch);

/* Work items in all lists and the number of portable item groups (either
 * pointer may be NULL). */
pfmm_status pfmm_batch_info(pfmm_batch_t batch, int* items, int* groups);

/* Portable item group `group` (0 <= group < groups): desc[4] = {block edge q,
 * FP64 (0/1), near zone (0/1), chosen tile width} and ms[3] = the timed
 * launch of the group's items at widths 1, 2, 4 in ms (negative when not
 * timed: FP64 groups, or widths read from the cache).  Either pointer may be
 * NULL; PFMM_ERR_INVALID_ARG for a group out of range. */
pfmm_status pfmm_batch_group(pfmm_batch_t batch, int group, int* desc, double* ms);

/* Release a batch (not its plans). NULL is accepted and ignored. */
pfmm_status pfmm_batch_destroy(pfmm_batch_t batch);

/*
 * Solve n independent fields as one batch: potential[i] from density[i]
 * with plans[i] (arguments as for pfmm_batch_create).  The first call with
 * a given set of (plan, density, potential) triples builds and captures its
 * batch (plan time: allocates and synchronises; PFMM_ERR_CAPTURE under
 * capture) and keeps it; later calls with the same set only launch its
 * graph on the stream of plans[0] and do not allocate.  The kept batch is
 * released with the first of its plans to be destroyed.
 */
pfmm_status pfmm_solve_batch(int n, const pfmm_plan_t* plans, const float* const* density,
                             float* const* potential);

/*
 * Direct periodic convolution  potential_i = h^3 sum_j G((x_i - x_j) wrapped) rho_j
 * over the whole box with the plan's G (Eq. 4, "PM with G": the exact result
 * the FMM approximates), by the block-Toeplitz kernel in FP32 with FP64
 * per-offset totals.  O(N^6) work: a reference for moderate N.  Allocates
 * its table on the first call; enqueued on the plan's stream.
 */
pfmm_status pfmm_plan_direct(pfmm_plan_t plan, const float* density, float* potential);

/*
 * pfmm_plan_direct for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and result as pfmm_plan_direct, bit for bit,
 * without its first-call allocation: the lattice table of G is tabulated on
 * every call into a static device array of the library (8 MiB, one per
 * device, held until the process ends), which limits it to N <= 64
 * (PFMM_ERR_UNSUPPORTED above; isolated plans too).  Allocates and
 * synchronises nothing; enqueued on the plan's stream.  Every call on a
 * device shares that device's array: calls that overlap on one device (two
 * streams, or two threads) race.
 */
pfmm_status pfmm_plan_direct_noalloc(pfmm_plan_t plan, const float* density, float* potential);

/*
 * Learned correction of the interaction-zone tables (Sec. 3 defines the
 * optimal G_* as the G with which FMM and PM agree; Sec. 4 proposes
 * parameterising it with many values).  A network of the table offset
 * j = a - a' - p d (Eq. 6), the level and p,
 *     f(|j| sorted / (4p), (|j| sorted mod p) / p, level / 8, p / 10),
 * with layers 8 -> 64 -> 64 -> 1 and SiLU activations, sets
 * T_l[j] = G(eta_l j) (1 + 1e-4 f) for every interaction-zone table entry;
 * the near zone keeps G.  Its inputs are invariant under the cube's 48
 * symmetries, so the corrected tables keep the FMM symmetric.  Weights:
 * PFMM_MLP_PARAMS floats, W1[64][8] b1[64] W2[64][64] b2[64] W3[64] b3.
 */
#define PFMM_MLP_PARAMS 4801

/* Set the network (host weights) and rebuild the tables by running it on the
 * device, in BF16 with FP32 accumulation when bf16 != 0, else in FP32.
 * weights == NULL restores the uncorrected G (the fallback).  Synchronises. */
pfmm_status pfmm_learned_set(pfmm_plan_t plan, const float* weights, int bf16);

/* Start training from the host weights with Adam step size lr (> 0).
 * Tables follow the network in FP32 from here on.  Allocates; synchronises. */
pfmm_status pfmm_learned_train_begin(pfmm_plan_t plan, const float* weights, double lr);

/* One training field: solve `density` (device) with the current tables,
 * compare with `target` (device, the potential to reproduce, e.g. from
 * pfmm_plan_direct), and add the gradient of
 *     loss = sum r^2 / sum (target - mean)^2,  r = phi - target - mean(phi - target)
 * with respect to the weights to the plan's accumulator (adjoint sweep,
 * table gradient, network backward pass, all on the device).  *loss
 * receives the field's loss (may be NULL).  Synchronises. */
pfmm_status pfmm_learned_accumulate(pfmm_plan_t plan, const float* density, const float* target,
                                    double* loss);

/* The loss above for one field with the plan's current tables, without a
 * gradient (a forward solve and the residual).  Synchronises. */
pfmm_status pfmm_learned_loss(pfmm_plan_t plan, const float* density, const float* target,
                              double* loss);

/* Adam step with the accumulated gradient averaged over the accumulated
 * fields; clears the accumulator and rebuilds the tables.  Synchronises. */
pfmm_status pfmm_learned_step(pfmm_plan_t plan);

/* Current weights into the host array `weights` (PFMM_MLP_PARAMS floats). */
pfmm_status pfmm_learned_get(pfmm_plan_t plan, float* weights);

/* Gradients of the last pfmm_learned_accumulate: d loss / d T_level[j] into
 * the host array table_grad ((8p-1)^3 doubles, same layout as
 * PFMM_BUF_TABLE_LEVEL) and the accumulated weight gradient into weight_grad
 * (PFMM_MLP_PARAMS floats); either may be NULL. */
pfmm_status pfmm_learned_read_grad(pfmm_plan_t plan, int level, double* table_grad,
                                   float* weight_grad);

/*
 * Grid-valued interaction-zone tables (Sec. 3 defines G_* by FMM = PM; Sec. 4
 * proposes treating G_* as a grid of free values).  Every table value of
 * Eq. 6 is free up to the 48 symmetries of the cube:
 *     T_l[j] = G(eta_l j) (1 + delta_l[u(j)]),
 * u(j) the orbit of the sorted |j_i|, one delta per orbit and level (levels
 * 2 .. L).  delta[(l - 2) nu + u]: nu = orbits per level, u the position of
 * (a >= b >= c) = sorted |j_i| in the order a = 0 .. 4p-1, b = 0 .. a,
 * c = 0 .. b, i.e. u = a(a+1)(a+2)/6 + b(b+1)/2 + c.  The near zone keeps G.  Training uses pfmm_learned_accumulate,
 * pfmm_learned_loss and pfmm_learned_step (Adam on delta) with the same loss
 * and target as the network; pfmm_learned_set(plan, NULL, 0) restores G.
 */

/* Number of free values, (L - 1) x orbits per level, into *count.  Prepares
 * the orbit tables (allocates on first use; synchronises). */
pfmm_status pfmm_table_params(pfmm_plan_t plan, int* count);

/* Set delta from the host (count floats, see pfmm_table_params) and rebuild
 * the tables; NULL restores the uncorrected G.  Synchronises. */
pfmm_status pfmm_table_set(pfmm_plan_t plan, const float* delta);

/* Copy the current delta to the host (count floats).  Fails unless the plan
 * holds grid-valued tables. */
pfmm_status pfmm_table_get(pfmm_plan_t plan, float* delta);

/* Start training the grid-valued tables from delta = 0 (exactly G) with Adam
 * step size lr > 0 (a change of the relative correction per step).
 * Allocates; synchronises. */
pfmm_status pfmm_table_train_begin(pfmm_plan_t plan, double lr);

/* Copy the gradient summed over the fields accumulated since the last step
 * (d loss / d delta, count floats) to the host and clear it, for a driver
 * that takes its own steps (pfmm_table_set) instead of pfmm_learned_step.
 * The loss is exactly quadratic in delta (the FMM is linear in its tables),
 * so a line search along any direction needs one more loss evaluation.
 * Synchronises. */
pfmm_status pfmm_table_grad(pfmm_plan_t plan, float* grad);

/*
 * G_* as one grid-valued function everywhere (Sec. 3: G_* is the G with which
 * the FMM and PM, both using it, agree, which gives Eq. 8; Sec. 4: G_* as a
 * grid of free values).  On the periodic mesh,
 *     G_*(x) = G(x) (1 + delta[u(x)]),
 * one free value per orbit u of mesh separations x under the cube's 48
 * symmetries: each component folded to min(|x_i| mod N, N - |x_i| mod N),
 * sorted a >= b >= c, u = a(a+1)(a+2)/6 + b(b+1)/2 + c, (N/2 + 1)(N/2 + 2)
 * (N/2 + 3)/6 values.  G_* replaces G in the near-zone table G(h m), in every
 * level's interaction-zone table G(eta_l j), and in the exact periodic
 * convolution (pfmm_plan_direct), which is the PM solution with G_* that
 * the FMM is compared with.  The level tables sample the mesh only when p
 * divides the leaf width N / 2^L, which is required (UNSUPPORTED otherwise),
 * as are a periodic plan, interaction zones other than the FFT comparator,
 * and the potential alone (no PFMM_OPT_ACCEL expansion accelerations).
 * While G_* is set, the interaction-zone table corrections (pfmm_learned_*,
 * pfmm_table_*) are refused, and they must be cleared before G_* is set.
 * The loss of a density is that of pfmm_learned_accumulate with the target
 * PM(G_*), which moves with delta.  The first call allocates (tables,
 * orbit maps, an FP64 FFT plan of N^3); every call synchronises.
 */

/* Number of free values into *count. */
pfmm_status pfmm_gstar_params(pfmm_plan_t plan, int* count);

/* Set delta from the host (count floats) and rebuild every table; NULL
 * restores G everywhere. */
pfmm_status pfmm_gstar_set(pfmm_plan_t plan, const float* delta);

/* Copy the current delta to the host (count floats). */
pfmm_status pfmm_gstar_get(pfmm_plan_t plan, float* delta);

/* Loss of one density (device, N^3 FP32) against PM with the plan's G_*:
 * a forward solve, the exact periodic convolution and the residual. */
pfmm_status pfmm_gstar_loss(pfmm_plan_t plan, const float* density, double* loss);

/* The same, and add d loss / d delta to the plan's accumulator: the FMM's
 * adjoint (level tables through the adjoint sweep, the near-zone table by a
 * sum over neighbouring-leaf pairs) minus the PM side (a periodic
 * cross-correlation by FP64 FFT), including the change of the PM norm.
 * *loss may be NULL. */
pfmm_status pfmm_gstar_accumulate(pfmm_plan_t plan, const float* density, double* loss);

/* Copy the accumulated gradient (count floats) to the host and clear it. */
pfmm_status pfmm_gstar_grad(pfmm_plan_t plan, float* grad);

/* Message describing the calling thread's last failure ("" if none). */
const char* pfmm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PFMM_H */
