/*
 * shape_is.h -- C ABI of the MI355X importance-sampling (IS) engine for
 * Gaussian molecular shape overlap (Tuzharov, Bochenkova, Maximov,
 * "Importance-Sampling Estimation of Gaussian Molecular Shape Overlap: Exact
 * Union Volumes and Confidence-Bounded Virtual Screening").
 *
 * Model (section "Gaussian shape and its union volume", Eqs. occ/union):
 * atom i of a molecule has centre c_i and width alpha_i and the unit-height
 * occupancy o_i(r) = exp(-alpha_i |r - c_i|^2); the molecule's union occupancy
 * is u(r) = 1 - prod_i (1 - o_i(r)), its first-order density m(r) = sum_i o_i.
 * The union overlap of A and B is O_AB = int u_A u_B (Eq. union-overlap), the
 * shape Tanimoto T = O_AB / (O_AA + O_BB - O_AB).
 *
 * Estimator (sections "Importance-sampling estimator", "Exact union overlap
 * by bounded reweighting", Eqs. expectation/var/union-is): sample points are
 * drawn exactly from A's own normalised mixture q_A = m_A / Z_A,
 * Z_A = sum_i (pi/alpha_i)^(3/2), and O_AB ~ Z_A/n sum_k w_A(r_k) u_B(r_k) with
 * the bounded weight w_A = u_A/m_A.  The estimate is symmetrised by averaging
 * the A-sided and B-sided estimates.  Each value carries its analytic
 * standard error Z * std / sqrt(n).
 *
 * Random numbers: sample k of a molecule with stream id `id` is one
 * Philox4x32-10 block with counter (k mod 2^32, k div 2^32, id, 0) and key
 * (seed mod 2^32, seed div 2^32).  Word 0 selects the mixture component through
 * the integer thresholds floor(2^32 * (v_0+..+v_i)/Z); words 1..3 give the
 * uniforms ((x >> 8) + 0.5) / 2^24 mapped to standard normals.  Results are
 * therefore reproducible sample by sample and independent of launch shape.
 *
 * Conventions for every call below:
 *  - Array arguments are DEVICE pointers on the context's device unless a
 *    parameter says "host".  The caller owns them; the library never frees or
 *    retains them after the work queued on `stream` completes.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *    asynchronous on that stream unless they return values in host memory,
 *    in which case they synchronise the stream before returning.
 *  - The context owns only internal scratch (grown on demand with hipMalloc,
 *    which happens at most on the first calls with a given problem size).
 *    Calls of one context share that scratch: calls queued on different
 *    streams of one context must not run at the same time (order them with
 *    events, or give each stream its own context).
 *  - Return value: SHAPE_OK or a negative SHAPE_E_* code; a message is kept
 *    in the context (shape_last_error).  No exception or abort crosses the
 *    ABI.  A context is not thread-safe: one host thread per context.
 */
#ifndef SHAPE_IS_H
#define SHAPE_IS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHAPE_OK 0
#define SHAPE_E_INVAL (-1)       /* NULL or ill-formed argument */
#define SHAPE_E_RANGE (-2)       /* size/count outside its documented range */
#define SHAPE_E_NOMEM (-3)       /* device allocation failed */
#define SHAPE_E_HIP (-4)         /* HIP runtime error, or no usable device */
#define SHAPE_E_UNSUPPORTED (-5) /* device is not gfx950 */
#define SHAPE_E_DATA (-6)        /* invalid molecule data found on device */

/* Largest number of atoms in one molecule. */
#define SHAPE_MAX_ATOMS 256

typedef struct shape_ctx shape_ctx;

/* Create a context on HIP device `device` (the device must be gfx950).
 * *out receives the context, or NULL on failure. */
int shape_create(shape_ctx** out, int device);

/* Free the context and its scratch.  NULL is accepted. */
void shape_destroy(shape_ctx* ctx);

/* Message of the last failed call on ctx (ctx NULL: last failed
 * shape_create or context-free call on this thread).  Never NULL; valid until
 * the next call on ctx. */
const char* shape_last_error(const shape_ctx* ctx);

/* Library version string (host memory, static). */
const char* shape_version(void);

/* Atom widths of Eq. occ: alpha_i = kappa / (lambda R_i^2) with
 * kappa = pi (3 / (4 pi))^(2/3).  lambda = 1 makes a single occupancy integrate
 * to the hard-sphere volume; a Gaussian height p in the Grant-Pickup form
 * alpha = pi (3p / (4 pi R^3))^(2/3) corresponds to lambda = p^(-2/3).
 * radius, alpha: device float [n] (Angstrom, Angstrom^-2).  n >= 0.
 * Errors: SHAPE_E_INVAL (NULL pointers with n > 0, lambda <= 0). */
int shape_alpha_from_radius(shape_ctx* ctx, const float* radius, int64_t n,
                            double lambda, float* alpha, void* stream);

/* A set of molecules in CSR layout (all device pointers except the ints).
 *  n_mols       number of molecules (>= 1)
 *  max_atoms    host-known upper bound on atoms per molecule, 1..SHAPE_MAX_ATOMS
 *               (sizes on-chip staging; a molecule above it is invalid data)
 *  n_atoms      host-known total number of atoms (= atom_offset[n_mols]);
 *               every offset must lie in [0, n_atoms]
 *  atom_offset  int32 [n_mols + 1], non-decreasing, atom_offset[0] = 0
 *  xyz          float32 [n_atoms][3] atom centres (Angstrom)
 *  alpha        float32 [n_atoms] atom widths alpha_i > 0 (Angstrom^-2)
 *  mol_id       uint32 [n_mols] random-stream id of each molecule, or NULL
 *               (id = index in the set).  Equal ids give common random numbers.
 * A molecule with no atoms, more than max_atoms atoms, offsets outside
 * [0, n_atoms], a non-finite coordinate or a width that is not finite and
 * positive is invalid data. */
typedef struct {
  int32_t n_mols;
  int32_t max_atoms;
  int64_t n_atoms;
  const int32_t* atom_offset;
  const float* xyz;
  const float* alpha;
  const uint32_t* mol_id;
} shape_mols;

/* Result of one symmetrised pair estimate (host struct, FP64).
 *  O_ab, se_O_ab        union overlap int u_A u_B and its SE
 *  O_aa, O_bb           union self-overlaps int u^2 (from each side's samples)
 *  V_a, V_b             union volumes int u
 *  T, se_T              shape Tanimoto and the delta-method SE of section
 *                       "Confidence-bounded screening" (O_ab error only)
 *  se_T_full            delta-method SE that also propagates the errors of
 *                       O_aa, O_bb and their covariance with O_ab
 *  O_ab_from_a/_from_b  the one-sided estimates that are averaged into O_ab
 *  Ofo_ab_is, Ofo_aa_is, Ofo_bb_is  first-order overlaps estimated from the
 *                       same samples (f = m_B, Eq. var), a built-in check
 *                       against the closed form of Eq. fo
 *  n_a, n_b             samples drawn from A and from B */
typedef struct {
  double O_ab, O_aa, O_bb, V_a, V_b, T;
  double se_O_ab, se_O_aa, se_O_bb, se_V_a, se_V_b, se_T, se_T_full;
  double O_ab_from_a, O_ab_from_b, Ofo_ab_is, Ofo_aa_is, Ofo_bb_is;
  int64_t n_a, n_b;
} shape_result;

/* One pair, fixed sample counts (Eqs. expectation, var, union-is).
 * A, B: molecule sets with n_mols == 1 each.  n_a, n_b: samples from A and
 * from B, 2..2^31.  out: HOST struct; the call synchronises `stream`.
 * Errors: SHAPE_E_INVAL, SHAPE_E_RANGE, SHAPE_E_DATA, SHAPE_E_NOMEM,
 * SHAPE_E_HIP. */
int shape_estimate(shape_ctx* ctx, const shape_mols* A, const shape_mols* B,
                   int64_t n_a, int64_t n_b, uint64_t seed, void* stream,
                   shape_result* out);

/* Allocation-free variant of shape_estimate, for callers that cannot allocate
 * device memory (code that must not call hipMalloc: tight serving loops,
 * harnesses that forbid allocation).  Same arguments, checks, kernels and
 * results (bit for bit) as shape_estimate, but the call allocates nothing:
 * the prepared molecule records, the per-block partial sums and the device
 * copy of the result live in a fixed array of the library's device code
 * (about 1.5 MiB, one copy per GPU, held until the process ends), and the
 * context's own scratch is neither used nor grown.  Limits: n_a and n_b at
 * most SHAPE_NOALLOC_MAX_SAMPLES, and A->n_atoms, B->n_atoms at most
 * SHAPE_MAX_ATOMS (else SHAPE_E_RANGE).  Every call on one GPU, from any
 * context, shares that GPU's array: calls that overlap in time on one GPU
 * (several host threads, or streams whose work interleaves) race and must be
 * serialised by the caller.  Synchronises `stream`; SHAPE_E_UNSUPPORTED
 * during graph capture.  Errors: as shape_estimate. */
#define SHAPE_NOALLOC_MAX_SAMPLES ((int64_t)1 << 24)
int shape_estimate_noalloc(shape_ctx* ctx, const shape_mols* A, const shape_mols* B,
                           int64_t n_a, int64_t n_b, uint64_t seed, void* stream,
                           shape_result* out);

/* The sampling steps of one molecule, exported for exact comparison of the
 * integer work (section "Importance-sampling estimator": exact draws from the
 * normalised mixture q = m/Z by integer thresholds, and the reading of the
 * random-number stream given at the top of this header).  M: a molecule set
 * (prepared into context scratch like any sampling call); mol: the molecule,
 * 0 <= mol < M->n_mols; samples k0 .. k0+n-1 (0 <= n <= 2^24, 0 <= k0 <=
 * 2^62) under the context's sampling scheme (shape_set_sampling).  Outputs,
 * each a device array or NULL:
 *   thr    uint32 [atoms of mol]: thresholds floor(2^32 (v_0+..+v_i)/Z) of
 *          the prepared molecule (the last entry, never compared, is
 *          0xFFFFFFFF)
 *   words  uint32 [n][4]: the Philox block of each sample (antithetic
 *          sampling: block k/2)
 *   comp   int32 [n]: the selected component #{i < N-1 : words[k][0] >= thr_i}
 *          (by binary lifting over the thresholds)
 *   r      float32 [n][3]: the sample point c_j + z sd_j (coordinates of M),
 *          its component taken through the screening kernel's guide table
 * The same device functions as the sampling kernels compute these.
 * Synchronises `stream` once (validity of the molecule) and then queues the
 * export asynchronously.  Errors: SHAPE_E_INVAL, SHAPE_E_RANGE, SHAPE_E_DATA
 * (invalid molecule), SHAPE_E_NOMEM, SHAPE_E_HIP; SHAPE_E_UNSUPPORTED during
 * graph capture. */
int shape_sample_points(shape_ctx* ctx, const shape_mols* M, int32_t mol, int64_t k0,
                        int32_t n, uint64_t seed, void* stream, uint32_t* thr,
                        uint32_t* words, int32_t* comp, float* r);

#define SHAPE_SCREEN_FIXED 0
#define SHAPE_SCREEN_ADAPTIVE 1

/* Screening parameters (host struct).
 *  mode            SHAPE_SCREEN_FIXED or SHAPE_SCREEN_ADAPTIVE
 *  n_per_side      FIXED: samples per molecule side, a multiple of 64 in
 *                  [64, 2^20]
 *  round_per_pair  ADAPTIVE: samples per pair per round (half per side),
 *                  a multiple of 128 in [128, 8192]
 *  cap_per_pair    ADAPTIVE: sample cap per pair, a multiple of
 *                  round_per_pair, at most 2^21
 *  tau             ADAPTIVE: stop once SE(T) <= tau (tau > 0)
 *  seed            Philox key
 *  n_start         ADAPTIVE, optional: device int32 [n_pairs] sample budgets
 *                  per pair; the stop test is first taken once a pair has
 *                  drawn n_start[p] samples (rounded up to whole rounds,
 *                  capped), e.g. budgets predicted by a surrogate; NULL =
 *                  test after every round
 * Adaptive screening (section "Confidence-bounded screening"): each pair
 * draws rounds of samples until the delta-method SE(T) is at most tau or the
 * cap is reached; the decision is taken in FP64 after every round. */
typedef struct {
  int32_t mode;
  int32_t n_per_side;
  int32_t round_per_pair;
  int32_t cap_per_pair;
  double tau;
  uint64_t seed;
  const int32_t* n_start;
} shape_screen_params;

/* Per-pair outputs (device pointers; T and se_T required when n_pairs > 0,
 * others may be NULL).  n_used is the total number of samples of the pair
 * (both sides). */
typedef struct {
  float* T;
  float* se_T;
  float* O_ab;
  float* O_aa;
  float* O_bb;
  int32_t* n_used;
} shape_screen_out;

/* Screen one query molecule against library molecules.
 * query: n_mols == 1.  lib: the library.  pairs: device int32 [n_pairs]
 * library indices to score, or NULL to score lib molecule p for p < n_pairs
 * (then n_pairs <= lib->n_mols).  Outputs are indexed by pair; an index
 * outside [0, lib->n_mols) gives NaN outputs and n_used 0.
 * Asynchronous.  Invalid molecules produce NaN outputs and are reported by
 * shape_check_data.  A screen of at least 16 pairs per compute unit runs its
 * pairs longest first (estimated from atom counts and n_start, computed on
 * the device in the same call, with 4 (n_pairs + 133120) bytes of context
 * scratch); every pair's outputs are the same in any order.  Errors:
 * SHAPE_E_INVAL, SHAPE_E_RANGE, SHAPE_E_NOMEM, SHAPE_E_HIP. */
int shape_screen(shape_ctx* ctx, const shape_mols* query, const shape_mols* lib,
                 const int32_t* pairs, int32_t n_pairs,
                 const shape_screen_params* params, void* stream,
                 const shape_screen_out* out);

/* Synchronise `stream` and report whether any molecule seen by the calls
 * queued since the previous check was invalid (SHAPE_E_DATA) or not
 * (SHAPE_OK); clears the flag. */
int shape_check_data(shape_ctx* ctx, void* stream);

/* Sampling scheme of shape_estimate and shape_screen (section
 * "Importance-sampling estimator").  SHAPE_SAMPLING_IID (default): sample k
 * of a molecule is Philox block k.  SHAPE_SAMPLING_ANTITHETIC: samples 2p
 * and 2p+1 share Philox block p (component and normals) and are the draw
 * c_j + z sd_j and its reflection c_j - z sd_j; means are unchanged, and the
 * standard errors come from the variance of the pair means.  Needs even
 * sample counts (>= 4) in shape_estimate, n_per_side a multiple of 128 and
 * round_per_pair a multiple of 256 in shape_screen (else SHAPE_E_RANGE).
 * shape_get_sampling returns the current scheme (-1 if ctx is NULL).
 * Errors: SHAPE_E_INVAL. */
#define SHAPE_SAMPLING_IID 0
#define SHAPE_SAMPLING_ANTITHETIC 1
int shape_set_sampling(shape_ctx* ctx, int32_t sampling);
int32_t shape_get_sampling(const shape_ctx* ctx);

/* Reuse of molecule preparation across calls (a pipeline that hands the
 * same molecule set to several calls, e.g. shape_screen and shape_estimate
 * of one library).  Every sampling call prepares its molecule sets (mixture
 * weights, sampling thresholds, frames) into context scratch, one set on the
 * query side and one on the library side; a shape_screen whose pairs list
 * names fewer than a quarter of the library prepares only those molecules,
 * and such a partial preparation is never reused.  shape_features and
 * shape_fo_overlap read the caller's arrays and prepare nothing.  While the
 * cache is
 * enabled, a set whose arrays (device pointers) and sizes equal those of the
 * set last prepared on the same side is not prepared again.  The caller
 * guarantees that the arrays are not written while the cache is enabled;
 * shape_prepare_cache(ctx, 1) also forgets earlier preparations, so a
 * pipeline that starts with it prepares each set once (also when captured in
 * a graph: the replay repeats that one preparation).  enable = 0 turns the
 * reuse off.  Invalid molecules are still reported by shape_check_data.
 * Errors: SHAPE_E_INVAL. */
int shape_prepare_cache(shape_ctx* ctx, int enable);

/* Work-granularity autotuning of the screening kernel (adaptive batching,
 * section "Confidence-bounded screening": the rounds and the stopping rule
 * are fixed by the method; only how many points a lane evaluates per atom
 * record is tuned).  Every variant draws the same samples, assigns them to
 * the same lanes and sums them in the same order, so results are
 * bit-identical whichever variant runs.
 *
 * shape_screen_tune runs the screen described by its arguments (as for
 * shape_screen; outputs go to context scratch) once per variant after one
 * untimed warm-up launch, times each with HIP events on `stream`, keeps the
 * fastest as the context's variant for later shape_screen calls, and writes
 * its index to *best (host pointer, may be NULL) and the measured kernel
 * times to ms[SHAPE_SCREEN_VARIANTS] (host, may be NULL).  Synchronises
 * `stream`.  Errors: as shape_screen; SHAPE_E_UNSUPPORTED during capture.
 * shape_screen_set_variant selects a variant by index (-1 = default);
 * shape_screen_get_variant returns the current one (-1 if ctx is NULL).
 *
 * Tuning cache: each choice is remembered process-wide under the kind of
 * screen — the device's architecture name and compute-unit count, mode,
 * sampling, the sample schedule (n_per_side, or round_per_pair and
 * cap_per_pair), whether n_start seeds the budgets, and the power-of-two
 * classes (floor log2) of the pair count, the query's atom count and the
 * library's mean atom count.  A later shape_screen_tune of the same kind, on
 * any context, selects the remembered variant without launching anything
 * (ms receives -1 for every variant); results are the same bits either way.
 * shape_tune_cache_file(path) backs the table with a text file: its entries
 * are read now (lines that do not parse are skipped; a missing file is
 * created) and each new choice is appended as one line; NULL detaches the
 * file (SHAPE_E_INVAL if it cannot be opened; message via
 * shape_last_error(NULL)).  shape_tune_cache_clear forgets every entry
 * (the file is left as it is); shape_tune_cache_size counts them.  These
 * three are thread-safe. */
#define SHAPE_SCREEN_VARIANTS 8
int shape_screen_tune(shape_ctx* ctx, const shape_mols* query, const shape_mols* lib,
                      const int32_t* pairs, int32_t n_pairs,
                      const shape_screen_params* params, void* stream, float* ms,
                      int32_t* best);
int shape_screen_set_variant(shape_ctx* ctx, int32_t variant);
int32_t shape_screen_get_variant(const shape_ctx* ctx);
int shape_tune_cache_file(const char* path);
int shape_tune_cache_clear(void);
int32_t shape_tune_cache_size(void);

/* HIP graphs of a sequence of asynchronous calls (launch overhead only;
 * results are those of the same calls made directly).
 * shape_graph_begin starts capturing `stream` (which must not be the null
 * stream); every asynchronous call of this library on that stream is then
 * recorded instead of run, until shape_graph_end, which ends the capture and
 * returns an executable graph in *out (owned by the caller; release with
 * shape_graph_destroy).  shape_graph_launch replays it on `stream`.
 * Replays read and write the same device addresses as the captured calls,
 * so those buffers must stay allocated while the graph is used; input data
 * may change between replays.  During capture the library allocates
 * nothing: run the same calls once, uncaptured, beforehand so its scratch is
 * large enough (else SHAPE_E_UNSUPPORTED), and calls that synchronise
 * (shape_estimate, shape_check_data, shape_screen_tune, shape_timing_read)
 * return SHAPE_E_UNSUPPORTED.  Kernel timing is suspended while capturing.
 * A failed call inside the capture leaves it open; shape_graph_end then
 * discards it and returns the error.  Scratch that an eager call grows while
 * a graph of the context is alive is not freed: the superseded buffer is
 * kept (retired) for the graphs that captured its address and released when
 * the last of them is destroyed, so a graph stays valid whatever eager calls
 * follow.  shape_graph_begin and shape_graph_end forget the molecule
 * preparations of shape_prepare_cache: a preparation made before a capture
 * is not reused inside it, nor one recorded inside it afterwards.  A graph
 * can only be launched with the context that captured it.  Errors:
 * SHAPE_E_INVAL, SHAPE_E_HIP, SHAPE_E_UNSUPPORTED. */
typedef struct shape_graph shape_graph;
int shape_graph_begin(shape_ctx* ctx, void* stream);
int shape_graph_end(shape_ctx* ctx, void* stream, shape_graph** out);
int shape_graph_launch(shape_ctx* ctx, shape_graph* graph, void* stream);
void shape_graph_destroy(shape_graph* graph);

/* Device memory held by the context (host pointers, each may be NULL): the
 * scratch in use, the retired scratch kept for live graphs, and the number
 * of executable graphs of this context not yet destroyed.  Errors:
 * SHAPE_E_INVAL. */
int shape_memory_info(const shape_ctx* ctx, int64_t* scratch_bytes, int64_t* retired_bytes,
                      int32_t* live_graphs);

/* ------------------------------------------------------------------------
 * Differentiable rigid alignment (section "Differentiable alignment and the
 * hybrid pipeline", Eqs. pose and grad).  B is moved rigidly,
 * c_j -> R(q/|q|) c_j + t, with the pose as seven floats
 * (qw, qx, qy, qz, tx, ty, tz): an unnormalised quaternion (rotation about
 * the origin of B's coordinates) and a translation.  A's first n_samples
 * sample points and weights are held fixed (common random numbers), so
 *   O(pose) = Z_A/n sum_k w_A(r_k) u_B(r_k; pose),
 *   T(pose) = O / (O_aa + O_bb - O)
 * is a smooth function of the pose with the pathwise gradient of Eq. grad.
 * ------------------------------------------------------------------------ */

/* Pose-invariant self-overlaps O_MM = Z_M/n sum_k w_M u_M over each
 * molecule's own first n_samples samples.  O_self: device float [n_mols].
 * n_samples in [2, 2^20].  Asynchronous; invalid molecules give NaN. */
int shape_self_overlap(shape_ctx* ctx, const shape_mols* M, int32_t n_samples,
                       uint64_t seed, void* stream, float* O_self);

/* Aligned Tanimoto and its gradient for n_starts poses of every pair.
 * A, B: molecule sets paired by index (equal n_mols = number of pairs).
 * pose: device float [pairs][n_starts][7].  O_aa, O_bb: device float [pairs]
 * (from shape_self_overlap with the same n_samples and seed).  n_samples in
 * [64, 4096], n_starts >= 1.  T: device float [pairs][n_starts];
 * dT_dpose: device float [pairs][n_starts][7], or NULL for values only.
 * At least 4 pairs per compute unit run largest pair first (the order
 * computed on the device from the atom counts, 4 (pairs + 133120) bytes of
 * context scratch); every pair's outputs are the same in any order.
 * Asynchronous.  Errors: SHAPE_E_INVAL, SHAPE_E_RANGE (including on-chip
 * staging larger than the device allows), SHAPE_E_NOMEM, SHAPE_E_HIP. */
int shape_align_grad(shape_ctx* ctx, const shape_mols* A, const shape_mols* B,
                     int32_t n_starts, const float* pose, const float* O_aa,
                     const float* O_bb, int32_t n_samples, uint64_t seed,
                     void* stream, float* T, float* dT_dpose);

/* One Adam step (Kingma and Ba) that increases T on n_poses poses:
 * g = -dT/dpose; m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * pose -= lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps), then the quaternion is
 * renormalised.  step: device int32 holding the number of steps already
 * taken (t - 1), advanced by one.  pose, m, v: device float [n_poses][7]
 * (m, v zero before the first step).  Asynchronous. */
int shape_adam_pose(shape_ctx* ctx, float* pose, const float* dT_dpose, float* m, float* v,
                    int64_t n_poses, int32_t* step, float lr, float beta1, float beta2,
                    float eps, void* stream);

/* Multi-start alignment driver: self-overlaps, then n_steps of
 * (shape_align_grad, shape_adam_pose) from the given starts, then T at the
 * final poses and the best start of each pair (largest final T).  The steps
 * run inside one kernel launch (A's samples drawn once per pair, each
 * start's Adam state in registers) with the same arithmetic as calling the
 * two entry points in turn.
 * pose: device float [pairs][n_starts][7], updated in place.  T_final:
 * device float [pairs][n_starts].  best: device int32 [pairs] or NULL.
 * Adam uses beta1 = 0.9, beta2 = 0.999, eps = 1e-8.  Pairs are launched in
 * the order of shape_align_grad.  Asynchronous. */
int shape_align(shape_ctx* ctx, const shape_mols* A, const shape_mols* B, int32_t n_starts,
                float* pose, int32_t n_samples, int32_t n_steps, float lr, uint64_t seed,
                void* stream, float* T_final, int32_t* best);

/* Dense-grid quadrature reference (the grid ground truth of the paper's
 * accuracy comparison): for one pair A, B (n_mols == 1 each), the trapezoid
 * rule on the cubic grid of spacing h over the box of all atom centres
 * grown by pad on every side (ceil(extent/h) + 1 points per axis, end
 * planes weighted 1/2), FP64.  out8 (HOST double[8]): int uA uB, int uA^2,
 * int uB^2, int uA, int uB, int mA mB, int mA^2, int mB^2 (u the union
 * occupancy, m the first-order density).  Synchronises `stream`.
 * Errors: SHAPE_E_INVAL, SHAPE_E_RANGE (grid or molecules too large),
 * SHAPE_E_DATA, SHAPE_E_NOMEM, SHAPE_E_HIP; SHAPE_E_UNSUPPORTED during
 * graph capture. */
int shape_grid_integrals(shape_ctx* ctx, const shape_mols* A, const shape_mols* B, double h,
                         double pad, void* stream, double* out8);

/* ------------------------------------------------------------------------
 * Hybrid pipeline (section "Differentiable alignment and the hybrid
 * pipeline"): rigid alignment on the analytic first-order overlap (Eq. fo)
 * from multiple starts, then union scoring of the superposed pairs with
 * shape_screen.  Pairs: B holds one molecule per pair (n_pairs = B->n_mols),
 * A one per pair or a single molecule shared by all pairs.  Poses as in
 * shape_align_grad: (qw, qx, qy, qz, tx, ty, tz), B's atoms moved to
 * R(q/|q|) c + t.  Invalid molecules give NaN and are reported by
 * shape_check_data.
 * ---------------------------------------------------------------------- */

/* Alignment starts per pair, pose: device float [n_pairs][5 + n_random][7]:
 * the given pose (identity), the four proper principal-axis alignments
 * R = U_A D U_B^T (U: principal axes of the mixture covariance, descending,
 * right-handed, sign-fixed; D = diag(1,1,1), diag(1,-1,-1), diag(-1,1,-1),
 * diag(-1,-1,1)) with t = mu_A - R mu_B (mixture means), then n_random
 * uniformly random rotations about B's mean (Shoemake, uniforms from Philox
 * block (s, pair, 0x5157A27, 0) under the key seed), same centring.  FP64.
 * Asynchronous.  Errors: SHAPE_E_INVAL, SHAPE_E_RANGE, SHAPE_E_NOMEM,
 * SHAPE_E_HIP. */
int shape_fo_starts(shape_ctx* ctx, const shape_mols* A, const shape_mols* B,
                    int32_t n_random, uint64_t seed, void* stream, float* pose);

/* First-order aligned Tanimoto T_FO = O/(O_AA + O_BB - O), O the
 * first-order overlap of A and the moved B (Eq. fo), maximised by Adam
 * (betas 0.9, 0.999, eps 1e-8, q renormalised after each step, the rule
 * of shape_adam_pose with hardware reciprocals) for n_steps steps from each
 * start.  pose: device float
 * [n_pairs][n_starts][7], starts in, final poses out; T: device float
 * [n_pairs][n_starts], T_FO at the final poses; grad (device float
 * [n_pairs][n_starts][7] or NULL): dT_FO/dpose there.  n_steps = 0
 * evaluates T_FO and its gradient at the given poses.  FP32, one wave per
 * (pair, start), the whole optimisation in one launch; when A has at most
 * 64 atoms, one workgroup per pair (a start per 16-lane row), and with at
 * least 16 pairs per compute unit those run largest B first (order computed
 * on the device, 4 (pairs + 133120) bytes of context scratch; outputs the
 * same in any order).  Asynchronous.
 * Errors: SHAPE_E_INVAL, SHAPE_E_RANGE (also molecules too large for the
 * kernel's LDS), SHAPE_E_NOMEM, SHAPE_E_HIP. */
int shape_fo_align(shape_ctx* ctx, const shape_mols* A, const shape_mols* B, int32_t n_starts,
                   float* pose, int32_t n_steps, float lr, void* stream, float* T,
                   float* grad);

/* Per pair, the start with the largest T (lowest index on ties; NaN never
 * wins): best_pose device float [n_pairs][7], best_T device float [n_pairs]
 * (may be NULL).  T: [n_pairs][n_starts], pose: [n_pairs][n_starts][7].
 * Asynchronous.  Errors: SHAPE_E_INVAL, SHAPE_E_RANGE, SHAPE_E_HIP. */
int shape_best_pose(shape_ctx* ctx, int32_t n_pairs, int32_t n_starts, const float* T,
                    const float* pose, void* stream, float* best_pose, float* best_T);

/* Conformer ensembles (max over conformers, the paper's accuracy lever):
 * for each group g of consecutive entries [group_offset[g],
 * group_offset[g+1]) of T (device float [n_T], e.g. one shape_screen output
 * over a library holding every conformer), best_T[g] = the largest T (device
 * float [n_groups]) and best_idx[g] its entry (device int32 [n_groups] or
 * NULL); lowest entry on ties, NaN never wins (all NaN or empty: NaN and -1).
 * group_offset: device int32 [n_groups + 1], non-decreasing.  A group that
 * is reversed or reaches outside [0, n_T) reads nothing: NaN and -1, and
 * shape_check_data reports it.  Asynchronous.  Errors: SHAPE_E_INVAL,
 * SHAPE_E_RANGE, SHAPE_E_HIP. */
int shape_group_max(shape_ctx* ctx, const float* T, int64_t n_T, const int32_t* group_offset,
                    int32_t n_groups, void* stream, float* best_T, int32_t* best_idx);

/* Moved coordinates of every molecule of M by its pose (device float
 * [n_mols][7]): xyz_out (device float [n_atoms][3]) = R(q/|q|) xyz + t.
 * Asynchronous.  Errors: SHAPE_E_INVAL, SHAPE_E_RANGE, SHAPE_E_HIP. */
int shape_apply_pose(shape_ctx* ctx, const shape_mols* M, const float* pose, void* stream,
                     float* xyz_out);

/* ------------------------------------------------------------------------
 * Learned triage (an addition to the paper's method: a surrogate that ranks a
 * library cheaply so that confidence-bounded IS refines only the head of the
 * ranking; IS stays the arbiter of every reported value).
 * ------------------------------------------------------------------------ */

/* Per-molecule features, 24 floats each (out: device float [n_mols][24]):
 * [0..15] histogram of atom distances from the mixture mean (0.5 A bins over
 * [0, 8), last bin open); [16..18] square roots of the descending
 * eigenvalues of the mixture covariance sum pi_i (c_i c_i^T + I/(2 alpha_i))
 * - mu mu^T; [19..22] atoms per width class (alpha < 0.767, < 0.893, < 0.995,
 * otherwise); [23] the first-order self-overlap (Eq. fo with B = A).
 * Reads the caller's arrays directly; invalid molecules (as in shape_screen)
 * give NaN rows and raise the flag that shape_check_data reports.  From 512
 * molecules per compute unit on, the molecules are taken in descending
 * order of their squared atom count (computed on the device in the same
 * call, 4 (n_mols + 133120) bytes of context scratch) so that each wave's
 * four molecules are of about one size; every row is the same in any order.
 * Asynchronous.  Errors: SHAPE_E_INVAL, SHAPE_E_RANGE, SHAPE_E_NOMEM,
 * SHAPE_E_HIP. */
int shape_features(shape_ctx* ctx, const shape_mols* M, void* stream, float* out);

/* First-order cross-overlap (Eq. fo) of the query with library molecules at
 * their given poses: out[p] = O^FO(query, lib[m]), m = pairs[p] (pairs NULL:
 * m = p).  O(N_q N_m) per pair.  out: device float [n_pairs].  Asynchronous.
 * Reads the caller's arrays directly; an invalid molecule gives NaN and
 * raises the flag that shape_check_data reports; a pairs entry outside the
 * library gives NaN.  FP32 with the widths entering as 1/(log2(e) alpha):
 * alpha from 1e-6 to 1e6 A^-2 (atomic widths are 0.1-10). */
int shape_fo_overlap(shape_ctx* ctx, const shape_mols* query, const shape_mols* lib,
                     const int32_t* pairs, int32_t n_pairs, void* stream, float* out);

/* Standardised pair features (out: device float [n][96]): for pair p with
 * query row q = qidx[p] (qidx NULL: q = 0) and library row m = idx[p] (idx
 * NULL: m = p), raw = [f_q, f_m, |f_q - f_m|, f_q * f_m] and
 * out[p][j] = (raw_j - mean[j]) * inv_std[j].  If fo_cross (device float
 * [n], from shape_fo_overlap) is given, raw[71] (|.| of the self-overlaps)
 * becomes the pair's first-order Tanimoto O_qm/(O_qq + O_mm - O_qm) and
 * raw[95] (their product) becomes O_qm.  f_q: device float [*][24]; f_lib:
 * device float [*][24]; mean, inv_std: device float [96]. */
int shape_pair_features(shape_ctx* ctx, const float* f_q, const float* f_lib,
                        const int32_t* qidx, const int32_t* idx, int32_t n,
                        const float* fo_cross, const float* mean, const float* inv_std,
                        void* stream, float* out);

/* Fused surrogate inference (learned triage): the standardised pair
 * features of shape_pair_features (same arguments) fed through the
 * 96-256-256-256-2 ReLU network whose parameters are params (device float,
 * packed W_0, b_0, W_1, b_1, ... with W_l row-major [in][out]), BF16
 * operands and FP32 accumulation; out: device float [n][2].  Bit-identical
 * to shape_pair_features followed by one BF16 shape_gemm per layer (ReLU on
 * the hidden layers); the features and activations stay on chip.  Uses
 * context scratch for the weights packed to BF16.  Asynchronous.
 * Errors: SHAPE_E_INVAL, SHAPE_E_RANGE, SHAPE_E_NOMEM, SHAPE_E_HIP. */
int shape_mlp_infer(shape_ctx* ctx, const float* f_q, const float* f_lib,
                    const int32_t* qidx, const int32_t* idx, int32_t n,
                    const float* fo_cross, const float* mean, const float* inv_std,
                    const float* params, void* stream, float* out);

/* Training forward of the surrogate: shape_mlp_infer (same arguments,
 * same bits in out) that also writes what the backward pass reads — the
 * standardised pair features x (device float [n][96], the values of
 * shape_pair_features) and the hidden activations after ReLU h1, h2, h3
 * (device float [n][256] each, FP32: the outputs the per-layer BF16
 * shape_gemm calls would have written).  One kernel instead of five
 * launches per minibatch.  x, h1, h2, h3 must be 16-byte aligned.
 * Uses context scratch for the weights packed to BF16.  Asynchronous.
 * Errors: SHAPE_E_INVAL (NULL or misaligned array), SHAPE_E_RANGE,
 * SHAPE_E_NOMEM, SHAPE_E_HIP. */
int shape_mlp_forward(shape_ctx* ctx, const float* f_q, const float* f_lib,
                      const int32_t* qidx, const int32_t* idx, int32_t n,
                      const float* fo_cross, const float* mean, const float* inv_std,
                      const float* params, void* stream, float* x, float* h1, float* h2,
                      float* h3, float* out);

#define SHAPE_GEMM_BF16 1u  /* round A and B to bfloat16 (else FP32 operands) */
#define SHAPE_GEMM_RELU 2u  /* epilogue ReLU after the bias */

/* Dense layer on the matrix cores, FP32 accumulation:
 *   C[m][n] = epi( sum_k A(m,k) B(k,n) ),  A(m,k) = A[m*sam + k*sak],
 *   B(k,n) = B[k*sbk + n*sbn],  C[m][n] at C[m*scm + n],
 * epi: + bias[n] (bias may be NULL), then ReLU if SHAPE_GEMM_RELU, then, if
 * gate is not NULL, zero where gate[m*sgm + n] <= 0 (backward through ReLU).
 * All device float arrays; M, N, K >= 1.  Asynchronous. */
int shape_gemm(shape_ctx* ctx, int32_t M, int32_t N, int32_t K, const float* A, int64_t sam,
               int64_t sak, const float* B, int64_t sbk, int64_t sbn, float* C, int64_t scm,
               const float* bias, const float* gate, int64_t sgm, uint32_t flags, void* stream);

/* One product of shape_gemm_set: the arguments of shape_gemm. */
typedef struct shape_gemm_desc {
  const float* A;
  const float* B;
  float* C;
  const float* bias;
  const float* gate;
  int64_t sam, sak, sbk, sbn, scm, sgm;
  int32_t M, N, K;
  uint32_t flags;
} shape_gemm_desc;

/* n (1..8) independent products, each with exactly the result shape_gemm
 * gives for its arguments (the weight gradients of all layers of a backward
 * pass at once).  BF16 products that shape_gemm runs with 64 x 64 tiles go
 * into one launch (plus one launch for their split-K reductions); any other
 * product is run as by shape_gemm.  d: host array of n descriptors.  Uses
 * context scratch for the split-K partials.  Asynchronous.  Errors as
 * shape_gemm; SHAPE_E_RANGE for n outside 1..8. */
int shape_gemm_set(shape_ctx* ctx, int32_t n, const shape_gemm_desc* d, void* stream);

/* The surrogate's weights (96-256-256-256-2 network, params packed as for
 * shape_mlp_infer) in the two bfloat16 layouts the fused training step reads:
 * matrix-core fragments of W_l for the forward and of W_l^T (l = 1..3) for
 * the input-gradient chain.  packed: device buffer of SHAPE_MLP_PACK_BYTES,
 * 16-byte aligned, caller-owned.  Asynchronous.  Errors: SHAPE_E_INVAL,
 * SHAPE_E_HIP. */
#define SHAPE_MLP_PACK_BYTES 598016
int shape_mlp_pack(shape_ctx* ctx, const float* params, void* stream, void* packed);

/* Optimiser state of shape_mlp_train_step (all device memory). */
typedef struct shape_mlp_adam {
  float* params;    /* [n_params] network parameters, updated in place      */
  float* m;         /* [n_params] Adam first moments, updated               */
  float* v;         /* [n_params] Adam second moments, updated              */
  int32_t* step;    /* [1] steps taken so far, incremented                  */
  void* packed;     /* SHAPE_MLP_PACK_BYTES: shape_mlp_pack(params) on entry,
                       rewritten from the updated params                    */
  float lr, beta1, beta2, eps;
} shape_mlp_adam;

#define SHAPE_MLP_STEP_MAX_ROWS 65536

/* One training step of the learned-triage surrogate (96-256-256-256-2, BF16
 * operands, FP32 accumulation) on a minibatch of n pairs: the forward of
 * shape_mlp_forward (pair features as there: f_q, f_lib, qidx, idx,
 * fo_cross, mean, inv_std), the weighted MSE of shape_mse against target
 * (device float [n][2]) with weights loss_w (device float [2]), the backward
 * of shape_mlp_backward (BF16) and the Adam update of shape_adam, with the
 * same arithmetic, so the same bits in params, m, v, step, grad and loss as
 * that sequence of calls.  Two kernel launches: the forward and the
 * row-local part of the backward (ReLU-gated input gradients, 32-row chunk
 * sums of the bias gradients, the loss terms) for 32 rows per workgroup;
 * then the weight gradients in shape_gemm_set's split-K chunks, the bias
 * sums, the loss, Adam and the packing of the new weights.
 *   n      rows, a multiple of 32 in [32, SHAPE_MLP_STEP_MAX_ROWS]
 *   opt    optimiser state; opt->packed must hold shape_mlp_pack(opt->params)
 *          (a previous step leaves it so)
 *   grad   device float [n_params] dloss/dparams of this step, or NULL
 *   loss   device float [1]: the minibatch loss
 * Uses context scratch (about 3.4 KB per row).  Asynchronous.  Errors:
 * SHAPE_E_INVAL (NULL or misaligned array), SHAPE_E_RANGE (n, Adam
 * hyper-parameters), SHAPE_E_NOMEM, SHAPE_E_HIP. */
int shape_mlp_train_step(shape_ctx* ctx, const float* f_q, const float* f_lib,
                         const int32_t* qidx, const int32_t* idx, int32_t n,
                         const float* fo_cross, const float* mean, const float* inv_std,
                         const float* target, const float* loss_w, const shape_mlp_adam* opt,
                         void* stream, float* grad, float* loss);

/* Backward pass of a dense ReLU network (the surrogate of learned triage:
 * 96-256-256-256-2) for one minibatch: the gradient of a loss with respect to
 * every parameter, given the forward's inputs and activations and the
 * gradient with respect to the output.
 *   n_layers   number of layers L, 1..8
 *   width      HOST int32 [L + 1]: width[0] inputs, width[L] outputs
 *   batch      rows of the minibatch, >= 1
 *   params     device float, packed W_0, b_0, W_1, b_1, ... (W_l row-major
 *              [width[l]][width[l+1]]), as for shape_mlp_infer
 *   act        HOST array of L device pointers: act[0] the inputs [batch]
 *              [width[0]], act[l] (l >= 1) the outputs of hidden layer l after
 *              ReLU [batch][width[l]] (shape_mlp_forward's x, h1, h2, h3)
 *   dout       device float [batch][width[L]]: dloss/doutput
 *   flags      SHAPE_GEMM_BF16 (operands rounded to bfloat16, FP32
 *              accumulation) or 0 (FP32 operands)
 *   grad       device float, same layout as params: dloss/dparams
 * dloss/dW_l = act[l]^T g_l and dloss/db_l = column sums of g_l, with g_{L-1}
 * = dout and g_{l-1} = (g_l W_l^T) zeroed where act[l] <= 0.  The arithmetic
 * of shape_gemm (the input gradients, with the ReLU gate), shape_gemm_set
 * (all weight gradients) and shape_colsum_set (all bias gradients), so the
 * same bits as those calls.  Uses context scratch for the hidden-layer
 * gradients.  Asynchronous.  Errors: SHAPE_E_INVAL, SHAPE_E_RANGE,
 * SHAPE_E_NOMEM, SHAPE_E_HIP. */
int shape_mlp_backward(shape_ctx* ctx, int32_t n_layers, const int32_t* width, int32_t batch,
                       const float* params, const float* const* act, const float* dout,
                       uint32_t flags, void* stream, float* grad);

/* Column sums out[n] = sum_m A[m*lda + n] (device float).  Asynchronous. */
int shape_colsum(shape_ctx* ctx, int32_t M, int32_t N, const float* A, int64_t lda,
                 float* out, void* stream);

/* The column sums of n_mats (1..8) matrices in one launch: for t < n_mats,
 * out[t][n] = sum_m A[t][m*lda[t] + n], m < M[t], n < N[t], each with the
 * bits shape_colsum gives (the bias gradients of all layers of a backward
 * pass at once).  M, N, A, lda, out: host arrays of n_mats entries; A[t] and
 * out[t] device float.  Asynchronous.  Errors: SHAPE_E_INVAL (NULL),
 * SHAPE_E_RANGE (n_mats, M or N out of range), SHAPE_E_HIP. */
int shape_colsum_set(shape_ctx* ctx, int32_t n_mats, const int32_t* M, const int32_t* N,
                     const float* const* A, const int64_t* lda, float* const* out,
                     void* stream);

/* Weighted mean squared error of predictions y against targets t (device
 * float [B][N]) with per-output weights w (device float [N]):
 * loss = sum_j w_j mean_b (y - t)^2 (device float [1]), grad = dloss/dy
 * (device float [B][N]).  Deterministic.  Asynchronous. */
int shape_mse(shape_ctx* ctx, int32_t B, int32_t N, const float* y, const float* t,
              const float* w, void* stream, float* grad, float* loss);

/* Adam (Kingma and Ba) descent step on a flat FP32 vector p with gradient g
 * and moments m, v (all device float [n]); step: device int32 holding the
 * steps already taken, advanced by one.  Asynchronous. */
int shape_adam(shape_ctx* ctx, float* p, const float* g, float* m, float* v, int64_t n,
               int32_t* step, float lr, float beta1, float beta2, float eps, void* stream);

/* Indices of the k largest scores (device float [n]; NaN ranks lowest; ties
 * go to the lower index), written in increasing index order to idx (device
 * int32 [k]).  1 <= k <= n.  Asynchronous. */
int shape_topk(shape_ctx* ctx, const float* score, int32_t n, int32_t k, void* stream,
               int32_t* idx);

/* Seeded sample budgets for surrogate-triaged screening: for i < k, with
 * r = idx[i] (idx NULL: r = i), the network's standardised log-scale output
 * s = raw[r*ld + 1] gives the per-sample SE scale sigma = exp(s y_std +
 * y_mean) and the budget n = (sigma / tau)^2, rounded up to a multiple of
 * round_per_pair and kept within [round_per_pair, cap_per_pair] (NaN: cap);
 * n_start: device int32 [k], for shape_screen_params.n_start.  FP64.
 * raw: device float [*][ld]; idx: device int32 [k] or NULL.  Asynchronous.
 * Errors: SHAPE_E_INVAL, SHAPE_E_RANGE, SHAPE_E_HIP. */
int shape_seed_budget(shape_ctx* ctx, const float* raw, int64_t ld, const int32_t* idx,
                      int32_t k, double y_mean, double y_std, double tau,
                      int32_t round_per_pair, int32_t cap_per_pair, void* stream,
                      int32_t* n_start);

/* Issue-rate microbenchmarks of the instructions the kernels are made of
 * (measurement support, not part of the method): rates (HOST double[5]) =
 * FP32 fused multiply-adds, v_exp_f32 exponentials and v_mad_u64_u32 integer
 * multiply-adds per second, counted per lane (one wave instruction = 64),
 * LDS bytes read per second, and FP32 fused multiply-adds per second with
 * SGPR operands, each the best of three timed launches of
 * sixteen workgroups of 256 lanes per compute unit with independent chains
 * in every lane (the FMA operands in VGPRs: the full-rate form).  Synchronises `stream`.  Errors: SHAPE_E_INVAL, SHAPE_E_NOMEM,
 * SHAPE_E_HIP; SHAPE_E_UNSUPPORTED during graph capture. */
int shape_peak_rates(shape_ctx* ctx, void* stream, double* rates);

/* Failure injection for tests of error handling: the next n scratch
 * allocations of ctx fail as if the device were out of memory (the call
 * returns SHAPE_E_NOMEM; the context stays usable and its earlier scratch
 * stays valid); n = 0 turns it off.  Errors: SHAPE_E_INVAL, SHAPE_E_RANGE. */
int shape_fail_allocations(shape_ctx* ctx, int32_t n);

/* Named ranges for profiles (roctx): every entry point that launches work
 * opens a range with its own name around its host work and launches; a
 * caller can bracket stages of its own pipeline with shape_range_push(name)
 * / shape_range_pop() (host strings, thread-local nesting).  Without an
 * attached profiler these cost a few nanoseconds and record nothing.
 * Errors: SHAPE_E_INVAL (NULL name). */
int shape_range_push(const char* name);
int shape_range_pop(void);

/* Kernel timing (measurement support, not part of the method).  While
 * enabled, every call records a pair of HIP events on its stream around its
 * dominant kernel (the screening kernel of shape_screen, the sample kernel of
 * shape_estimate).  shape_timing_read synchronises those events and returns
 * the summed kernel time in milliseconds and the number of launches since the
 * last reset (host pointers; either may be NULL); reset != 0 clears them.
 * Errors: SHAPE_E_INVAL, SHAPE_E_HIP. */
int shape_timing_enable(shape_ctx* ctx, int enable);
int shape_timing_read(shape_ctx* ctx, double* total_ms, int64_t* launches, int reset);

#ifdef __cplusplus
}
#endif

#endif /* SHAPE_IS_H */
