/*
 * mf.h -- C ABI of the MI355X messenger-field Gibbs sampler.
 *
 * The library samples the joint posterior of a signal s on a periodic N^3 grid
 * and its isotropic power spectrum P(k), given data d = R s + noise with a
 * diagonal noise covariance N (Jasche & Lavaux 2014, "Matrix-free large scale
 * Bayesian inference in cosmology", Sec. 2 model, Sec. 3 sampler).  One Gibbs
 * sweep (Algs. 1 and 2 of that paper, P(k) averaged over |k| shells):
 *   1. messenger t ~ Pi(t | T, d, s), voxel by voxel (eqs. for mu^t, sigma^t),
 *   2. forward 3D FFT of t,
 *   3. signal s^ ~ Pi(s^ | S, T, t^), mode by mode (eqs. for mu^s, sigma^s),
 *   4. shell sums of |s^|^2 and P_b ~ InvGamma(n_b/2, sigma_b/(2M)) under
 *      Jeffreys' prior (eq. of the inverse-gamma conditional, Alg. 2),
 *   5. inverse 3D FFT of s^.
 * T = tau * 1 with tau = the smallest observed noise variance (Sec. 2, the
 * positivity bound on the augmented noise N - R^T T R).
 *
 * Conventions
 *  - Grids are C order (ix, iy, iz), iz fastest, M = N^3 voxels.
 *  - Unobserved voxels are marked by noise_var = +INF (R_i = 0); their data
 *    value is ignored.
 *  - Power is given and returned per bin in physical units (volume, h^-3
 *    Mpc^3 when the box side is in h^-1 Mpc); bin b holds the modes with
 *    b*dk <= |k| < (b+1)*dk, dk = sqrt(3) * pi * N / (box * n_bins), edges
 *    compared in exact integer arithmetic, the corner mode in the last bin,
 *    k = 0 in no bin.
 *  - Random numbers: Philox4x32-10 keyed by the 64-bit seed, counter
 *    (element, sweep, phase, chain id).  A chain is a pure function of
 *    (inputs, seed, chain id, sweep index): there is no generator state.
 *  - Memory: the caller owns every host array (copied during the call) and the
 *    device workspace (size from mf_workspace_bytes, at least 256-byte
 *    aligned), which must outlive the problem handle; the library allocates
 *    no device memory.  The handle owns small host metadata only.
 *  - Streams: `stream` is a hipStream_t (NULL = default stream).  Sweeps are
 *    enqueued asynchronously; functions that return host data synchronise the
 *    stream.
 *  - Errors: every call returns an mf_status; mf_last_error() gives a
 *    thread-local message for the last non-OK status.  No call throws.
 */
#ifndef MF_H
#define MF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MF_OK = 0,
  MF_E_INVALID_ARG = -1,      /* null pointer, bad count, bad descriptor field */
  MF_E_UNSUPPORTED_SIZE = -2, /* N is not a supported FFT size */
  MF_E_TAU = -3,              /* tau above the smallest observed noise variance */
  MF_E_NONFINITE = -4,        /* NaN input, or a non-finite P / shell sum on device */
  MF_E_DEVICE = -5,           /* a HIP call or kernel launch failed */
  MF_E_WORKSPACE = -6,        /* workspace missing, misaligned or too small */
  MF_E_STATE = -7             /* chain index out of range, or handle misuse */
} mf_status;

typedef enum {
  MF_PREC_FP64 = 0, /* every step in FP64 */
  MF_PREC_FP32 = 1  /* fields, FFTs and pointwise draws in FP32; shell sums,
                       inverse-gamma draws and per-bin tables in FP64 */
} mf_precision;

typedef struct {
  int32_t n;          /* grid side N: 8, 16, 32, 48, 64, 80, 96, 128, 256 or 512 */
  int32_t n_bins;     /* number of |k| bins, 1 <= n_bins <= 1024 */
  double box;         /* box side L (> 0) */
  double tau;         /* messenger variance; <= 0 selects min observed N_i */
  uint64_t seed;      /* Philox key */
  uint32_t chain_id;  /* counter word 3 of chain 0; chain c uses chain_id + c */
  int32_t precision;  /* mf_precision */
  int32_t sample_pk;  /* 1: Gibbs update of P(k) each sweep; 0: P held fixed */
  int32_t n_chains;   /* independent chains sharing N, bins, box and seed (>= 1) */
  int32_t has_response; /* 1: mf_init_problem takes a per-voxel response R per
                           chain; 0: R = 1 on every observed voxel */
  /* Prior on every P_b: the conjugate InvGamma(a0, b0), density
   * ~ P^-(a0+1) exp(-b0 / P), with a0 = pk_prior_shape >= 0 and
   * b0 = pk_prior_scale >= 0 in physical units (volume).  (0, 0) is Jeffreys'
   * prior 1/P of Sec. 3.2, the paper's choice, under which the joint
   * posterior is improper as P_b -> 0 wherever the noise is finite; b0 > 0
   * makes it proper.  The P step then draws InvGamma(n_b/2 + a0,
   * sigma_b/(2M) + b0 / V_cell) in grid units, and the mixing sweep's
   * Metropolis-Hastings move accepts with min(1, (U/U')^(2 a0 + 1)
   * exp(M b0 / V_cell (1/U^2 - 1/U'^2))). */
  double pk_prior_shape;
  double pk_prior_scale;
} mf_chain_desc;

typedef struct mf_problem mf_problem;

/* Number of sweep kernels reported by mf_gibbs_sweep_timed, in launch order:
 * 0 z-pass (inverse z-FFT, messenger draw, forward z-FFT), 1 forward y-FFT,
 * 2 x-pass (forward x-FFT, signal draw, shell sums, inverse x-FFT),
 * 3 inverse y-FFT together with the P(k) draw. */
#define MF_NUM_KERNELS 4

/* Returns 1 if N is a supported grid side, else 0. */
int32_t mf_supported_n(int32_t n);

/* Device workspace bytes needed by a problem with this descriptor.
 * Errors: MF_E_INVALID_ARG, MF_E_UNSUPPORTED_SIZE. */
mf_status mf_workspace_bytes(const mf_chain_desc* desc, size_t* bytes);

/* Set up a problem (model of Sec. 2: data model d = R s + eps with diagonal
 * response R and noise covariance N, messenger covariance tau).
 *  data[c], noise_var[c]: host, M doubles each, chain c's data and noise
 *      variance (+INF = unobserved).  Observed voxels need finite d and N > 0.
 *  response: NULL when desc->has_response = 0 (R = 1); otherwise a host array
 *      of n_chains pointers, each M finite doubles R_i.  R_i = 0 marks an
 *      unobserved voxel (its d and N are then ignored), as N_i = +INF does.
 *  pk_init[c]: host, n_bins doubles, initial P per bin (physical units, >= 0).
 *  s_init: NULL (every chain starts at s = 0) or host array of n_chains
 *      pointers, each M doubles (a NULL entry also means s = 0).
 *  workspace: device pointer of workspace_bytes >= mf_workspace_bytes(desc).
 * Per chain, tau is the smallest observed N_i / R_i^2 (the bound of Sec. 2)
 * unless desc->tau > 0, which must not exceed it (MF_E_TAU).  The messenger
 * conditional of Sec. 3.1 is folded into per-voxel coefficients
 * alpha = 1 - tau R^2 / N and beta = tau R d / N, formed in FP64 on the host
 * and uploaded; the sweep itself does not depend on R otherwise.  Enqueues on
 * `stream` and synchronises it.
 * Errors: MF_E_INVALID_ARG (also a response given or missing against
 * desc->has_response), MF_E_UNSUPPORTED_SIZE, MF_E_TAU, MF_E_NONFINITE,
 * MF_E_WORKSPACE, MF_E_DEVICE.  On error *out is NULL. */
mf_status mf_init_problem(const mf_chain_desc* desc, const double* const* data,
                          const double* const* noise_var, const double* const* response,
                          const double* const* pk_init, const double* const* s_init,
                          void* workspace, size_t workspace_bytes, void* stream,
                          mf_problem** out);

/* Enqueue n_sweeps >= 0 Gibbs sweeps of every chain (Algs. 1 and 2 with shell
 * averaging; the P(k) step only when sample_pk = 1).  Asynchronous.
 * The sweep index is Philox counter word 1 (32 bits): sweeps that would take
 * it beyond 2^32 - 1 are refused, since they would repeat the random numbers
 * of earlier sweeps.  This holds for every call that sweeps.
 * Errors: MF_E_INVALID_ARG (also that bound), MF_E_DEVICE. */
mf_status mf_gibbs_sweep(mf_problem* p, int32_t n_sweeps, void* stream);

/* As mf_gibbs_sweep, but times the kernels with HIP events, synchronises,
 * and writes the mean duration in milliseconds of each of the first
 * min(n_kernels, MF_NUM_KERNELS) sweep kernels to kernel_ms (host).  Sweep i
 * brackets only its kernel i mod MF_NUM_KERNELS, with events that skip the
 * system-scope fence, so every kernel is timed on n_sweeps / MF_NUM_KERNELS
 * sweeps (NaN for a kernel never timed: n_sweeps < MF_NUM_KERNELS). */
mf_status mf_gibbs_sweep_timed(mf_problem* p, int32_t n_sweeps, void* stream,
                               double* kernel_ms, int32_t n_kernels);

/* As mf_gibbs_sweep_timed, with every timed kernel preceded by a stream
 * through the caller's device buffer `evict` (contents overwritten):
 * evict_mode 0 copies its first half onto its second half, 1 reads all of
 * it, 2 does both, copy then read.  A buffer several times the device's
 * last-level (fabric) cache, 256 MB on MI355X, leaves that cache holding none
 * of the kernel's data, so the times are those of passes that find their
 * inputs in DRAM only; the difference to mf_gibbs_sweep_timed is what the
 * cache gives each pass.  A copy leaves the cache full of dirty lines, whose
 * write-back may then fall inside the timed kernel; a read leaves clean
 * lines, if the cache allocates on reads.  The streams are not inside the
 * timed intervals.  The chain advances as with mf_gibbs_sweep.
 * Errors: as mf_gibbs_sweep_timed, and MF_E_INVALID_ARG for an eviction
 * buffer that is NULL, not 16-byte aligned, not a multiple of 32 bytes or
 * smaller than 64 MiB, or a mode outside 0..2. */
mf_status mf_gibbs_sweep_timed_cold(mf_problem* p, int32_t n_sweeps, void* stream,
                                    double* kernel_ms, int32_t n_kernels, void* evict,
                                    size_t evict_bytes, int32_t evict_mode);

/* Copy chain `chain`'s state to the host: s_out (M doubles, may be NULL),
 * pk_out (n_bins doubles, physical units, may be NULL), sweep_out (number of
 * sweeps done, may be NULL).  Synchronises `stream`.
 * Errors: MF_E_STATE (bad chain), MF_E_NONFINITE (the device flagged a
 * non-finite shell sum or P draw), MF_E_DEVICE. */
mf_status mf_get_chain_state(mf_problem* p, int32_t chain, double* s_out, double* pk_out,
                             uint64_t* sweep_out, void* stream);

/* Overwrite chain `chain`'s s (M doubles, NULL keeps s) and P (n_bins
 * doubles, NULL keeps P) and set the sweep counter of the whole problem to
 * `sweep` (the counter is shared by all chains; at most 2^32 - 1).
 * Continuing from a state read by mf_get_chain_state reproduces the original
 * chain.
 * Errors: MF_E_STATE, MF_E_INVALID_ARG (also sweep >= 2^32, with nothing
 * changed), MF_E_NONFINITE, MF_E_DEVICE. */
mf_status mf_set_chain_state(mf_problem* p, int32_t chain, const double* s, const double* pk,
                             uint64_t sweep, void* stream);

/* Checkpoints: the exact device state of one chain (its half-complex field in
 * the working precision, P per bin in FP64, and the sweep index), so that a
 * chain resumed from a checkpoint continues bitwise identically -- the random
 * numbers carry no state beyond the sweep index.  mf_checkpoint_bytes gives
 * the size of one chain's checkpoint; mf_save_checkpoint writes it to the
 * host buffer `buf` (synchronises `stream`); mf_load_checkpoint restores it
 * into chain `chain` of a problem with the same N, n_bins and precision, and
 * sets the problem's sweep counter to the checkpoint's.
 * Errors: MF_E_INVALID_ARG (size or header mismatch, a sweep index >= 2^32),
 * MF_E_STATE, MF_E_DEVICE. */
mf_status mf_checkpoint_bytes(mf_problem* p, size_t* bytes);
mf_status mf_save_checkpoint(mf_problem* p, int32_t chain, void* buf, size_t bytes, void* stream);
mf_status mf_load_checkpoint(mf_problem* p, int32_t chain, const void* buf, size_t bytes,
                             void* stream);

/* Mixing sweeps (Sec. 3.3, Alg. 3, in the shell form), grid sides 32 to 256.
 * One mixing sweep draws the messenger t | s, then updates (s^, P) jointly
 * given t^ in the coordinates s^ = sqrt(S^) x^, S^_b = M P_b.  It draws x^
 * (the signal conditional at the current P, divided by sqrt(S^)).  Then per
 * bin it makes a Metropolis-Hastings move of U = sqrt(S^_b) with the
 * truncated-normal independence proposal N(R_b/X_b, T^/X_b) | U > 0, where
 * X_b = sum |x^|^2 and R_b = sum Re(conj(x^) t^) over the bin's modes.  The
 * move is accepted with probability min(1, U/U'), the ratio that Jeffreys'
 * prior gives.  Finally s^ = sqrt(S^') x^ and the inverse transform.  Draws
 * use Philox phase 3 (counter (b 2^16 + attempt, sweep, 3, chain)) besides
 * the messenger and signal phases.  Mixing and Gibbs sweeps may be
 * interleaved freely; both advance the sweep index.  Enqueued on `stream`.
 * The move changes P, so a problem that holds P fixed (sample_pk = 0) is
 * refused.
 * Errors: MF_E_UNSUPPORTED_SIZE, MF_E_INVALID_ARG (also sample_pk = 0),
 * MF_E_DEVICE. */
mf_status mf_mixing_sweep(mf_problem* p, int32_t n_sweeps, void* stream);

/* How Gibbs sweeps run the transforms, and their autotuner.
 * Path 0 (split, 32 <= N <= 256): the y-passes also run the radix-N/16 half
 * of the x-DFT, and the x-pass runs 16-point DFTs in registers.
 * Path 1 (whole): the x-pass runs whole x pencils through LDS.  It is the
 * only path for N = 8, 16, 512.
 * On the split path three choices are open:
 *  - x_tile: the x-pass workgroup (variant 0 is the library's tile rule,
 *    e.g. 128 iy columns x 2 k1 values at 256, with 8 LDS shell histograms
 *    per wave, for at most 255 bins; 1 is the same tile with 2 histograms
 *    per wave, for any bin count; 2 splits every column over two
 *    neighbouring lanes, 8 of its 16 rows each, e.g. 128 columns x 1 k1
 *    value at 256, with 8 histograms per wave, for at most 255 bins);
 *  - y_group: (kz, q) units per y-pass workgroup, the rule's G, G/2, G/4
 *    (at least 1);
 *  - y_radix: the order of the y transform's radix stages, 0 the library's
 *    schedule (e.g. 6 x 4 x 4 at 96), 1 its reverse (4 x 4 x 6).
 * Every choice gives the same chain up to rounding (the shell sums are
 * grouped by workgroup, the transforms factor differently) and leaves the
 * same state between sweeps, so choices may change at any time.  The
 * default is the split path where it exists, x tile 0 (1 above 255 bins),
 * y group 0 and y_radix 0.  Mixing sweeps and the Wiener filter always use
 * the split path with x tile 1.
 * mf_set_x_path: MF_E_UNSUPPORTED_SIZE for the split path outside 32..256.
 * mf_set_tuning / mf_get_tuning: the path and the three choices at once;
 *   mf_get_tuning also fills the geometry they stand for.  MF_E_INVALID_ARG
 *   for a variant outside 0..2, a y_radix other than 0 or 1, or an x tile
 *   whose histograms cannot hold the problem's bins, MF_E_UNSUPPORTED_SIZE
 *   as mf_set_x_path.
 * mf_autotune: coordinate search over the split path's x tiles (y group 0),
 * then its y groups (with the best x tile), then the y radix order where
 * the schedule differs from its reverse, then that tuned split path against
 * the whole-pencil path.  Each stage times its candidates in turn,
 * three rounds of `trials` Gibbs sweeps each (after one warm-up sweep, and a
 * warm-up of the device first), and keeps every candidate's fastest round;
 * an alternative replaces the first candidate of its stage (the incumbent)
 * only if faster by more than 1%.  ms (host, MF_TUNE_SLOTS doubles) receives
 * the mean sweep time in ms of every candidate: [0] the tuned split path,
 * [1] whole, [2 + v] x tile v, [5 + v] y group v, [8 + r] y radix order r,
 * NaN for a candidate not available or equal to another.  picked (may be
 * NULL)
 * receives the choice as mf_get_tuning gives it.  Every chain's state
 * (spectrum, P, sweep index) is saved to host memory first and restored
 * bitwise afterwards.  Diagnostic recording is suspended meanwhile.
 * Synchronises `stream`. */
typedef struct {
  int32_t x_path;   /* 0 split, 1 whole */
  int32_t x_tile;   /* split x-pass tile variant, 0..2 */
  int32_t y_group;  /* split y-pass workgroup variant, 0..2 */
  int32_t x_cols;   /* out (mf_get_tuning): iy columns per x-pass workgroup */
  int32_t x_k1;     /* out: k1 values per split x-pass workgroup */
  int32_t y_units;  /* out: (kz, q) units per split y-pass workgroup */
  int32_t x_hist;   /* out: LDS shell histograms per wave of the split x-pass */
  int32_t y_radix;  /* split y-pass radix stages: 0 schedule order, 1 reversed */
} mf_tuning;
#define MF_TUNE_SLOTS 10
mf_status mf_set_x_path(mf_problem* p, int32_t path);
mf_status mf_get_x_path(const mf_problem* p, int32_t* path);
mf_status mf_set_tuning(mf_problem* p, const mf_tuning* t);
mf_status mf_get_tuning(const mf_problem* p, mf_tuning* t);
mf_status mf_autotune(mf_problem* p, int32_t trials, void* stream, double* ms, mf_tuning* picked);

/* Algorithmic HBM bytes of one sweep, per kernel (bytes[MF_NUM_KERNELS], in
 * sweep order), summed over the problem's chains.  Each pass reads and
 * writes the half-complex field once, 2 (N/2 + 1) N^2 reals each way.  On
 * top of that:
 *  - the z-pass reads the two messenger coefficients of every voxel in the
 *    chunks of its tiles that hold an observed voxel (a chunk is one element
 *    of every lane of a tile; chunks with none skip the read);
 *  - the x-pass writes one FP64 shell partial per bin and workgroup;
 *  - the inverse y-pass reads those partials and updates P and its table.
 * These are the per-unit figures behind the roofline of each kernel. */
mf_status mf_sweep_bytes(const mf_problem* p, size_t* bytes);

/* The messenger variance tau of a chain (host value). */
mf_status mf_get_tau(mf_problem* p, int32_t chain, double* tau_out);

/* Diagnostics (used by the tests to check single passes).
 * mf_debug_run_kernel: enqueue one sweep kernel (numbering as in
 * MF_NUM_KERNELS) for every chain with sweep index `sweep` (it rewrites the
 * device sweep counter; reset it with mf_set_chain_state before sweeping).
 * mf_debug_spectrum: copy chain `chain`'s half-complex working buffer to
 * (to_device = 0) or from (to_device = 1) the host array `buf` of
 * 2 * (N/2 + 1) * N * N doubles, laid out [kz][ix][iy][re, im] with
 * kz in [0, N/2] -- the buffer holds the field transformed along whichever
 * axes the passes run so far have transformed (for 32 <= N <= 256 the
 * y-passes also run half of the x transform, so after kernel 1 the rows of a
 * kz plane hold that intermediate).  Synchronises `stream`. */
mf_status mf_debug_run_kernel(mf_problem* p, int32_t kernel, uint64_t sweep, void* stream);
mf_status mf_debug_spectrum(mf_problem* p, int32_t chain, double* buf, int32_t to_device,
                            void* stream);

/* Graphs of sweeps, for batches of problems (different grid sizes or
 * precisions) run as independent chains (Sec. 3.4: independent chains need no
 * communication).  mf_graph_create captures one Gibbs sweep of each of the n
 * problems into one HIP graph; problems are independent branches of the graph
 * and may run concurrently.  mf_graph_launch replays it n_sweeps times on
 * `stream` (asynchronously) and advances every problem's sweep counter; the
 * replays draw the same random numbers as mf_gibbs_sweep would.  The problems
 * must outlive the graph and must not be swept on another stream while a
 * replay is in flight.  A graph replays the diagnostic recording set when it
 * was created (mf_set_diagnostics), buffers included, so that call is refused
 * for a problem while a graph over it exists.  It also keeps the x path and
 * tile variants chosen when it was created: a later mf_set_tuning or
 * mf_autotune changes eager sweeps only (every choice gives the same chain
 * up to rounding).  The graph owns its side streams and events.
 * Errors: MF_E_INVALID_ARG, MF_E_DEVICE. */
typedef struct mf_graph mf_graph;
mf_status mf_graph_create(mf_problem* const* problems, int32_t n, void* stream, mf_graph** out);
mf_status mf_graph_launch(mf_graph* g, int32_t n_sweeps, void* stream);
void mf_graph_destroy(mf_graph* g);

/* Deterministic messenger Wiener filter and its adjoint (grid sides 32 to
 * 256).
 *
 * With every unit normal of the sweep set to zero and P held fixed, one
 * sweep becomes the iteration s_{k+1} = C (alpha s_k + beta): the means of
 * the messenger and signal conditionals (Sec. 3.1).  Here C = F^-1 diag(f) F
 * with f_b = P_b / (P_b + tau) and f = 0 at k = 0, alpha = 1 - tau R_i^2 / N_i
 * and beta = tau R_i d_i / N_i on observed voxels, and (1, 0) elsewhere.  The
 * iteration converges to the Wiener filter S R (R S R + N)^-1 d.  Starting
 * from s_0 = 0, K iterations give s_K, and the loss is
 *   chi2_K = sum_i d_i (d_i - R_i s_K,i) / N_i   over observed voxels,
 * which tends to d^T (R S R + N)^-1 d as K grows.  The noise model (N_i, R_i,
 * the mask and tau) is the chain's; d and P are inputs of each call.  With a
 * response the library runs the same iteration on d / R with noise N / R^2
 * (an exact rescaling: s_K and chi2_K are unchanged) and scales the gradient
 * with respect to d by 1 / R.
 *
 * chain >= 0 selects one chain.  chain = -1 runs every chain of the problem
 * in the same launches (arrays then hold the chains one after another).
 *
 * mf_wiener_workspace_bytes: size of the caller-owned device workspace for
 *   that chain selection, K iterations and a checkpoint every `ckpt_every`.
 *   Per chain it holds ceil(K / E) checkpoints plus E stored spectra, about
 *   (ceil(K/E) + E + 6) * 8 M bytes in FP32 mode, and 8 M bytes more with a
 *   response.
 * mf_wiener_forward: d (FP64, M per chain, [ix][iy][iz]; ignored where
 *   unobserved) and pk (FP64, n_bins per chain, physical units) are device
 *   arrays.  d is data in the problem's model d = R s + eps, and
 *   chi2_K = sum over observed i of d_i (d_i - R_i s_K,i) / N_i.  Writes
 *   chi2_K to the device doubles `chi2` (one per chain) and,
 *   when `s_out` (device FP64, M per chain) is not NULL, s_K.  Checkpoints of
 *   s_k every `ckpt_every` iterations stay in the workspace for
 *   mf_wiener_backward.  The chains' Gibbs state is not touched.
 * mf_wiener_backward: the gradient of the last forward run's chi2_K with
 *   respect to d (device FP64, M per chain; zero where unobserved) and to
 *   P_b (device FP64, n_bins per chain, physical units).  It takes the same
 *   chain selection, the same d and the same workspace as that run, and
 *   recomputes each segment from its checkpoint: 2 K iterations.
 *
 * Both calls enqueue on `stream` without synchronising.  They use the
 * problem's state staging buffer and its shell partials as scratch, so they
 * must not overlap sweeps or state calls on the same problem.
 * Errors:
 *  - MF_E_UNSUPPORTED_SIZE for grid sides outside 32..256;
 *  - MF_E_STATE for a bad chain, or a backward call without a matching
 *    forward run;
 *  - MF_E_WORKSPACE for a workspace that is too small or not aligned;
 *  - MF_E_INVALID_ARG, MF_E_DEVICE. */
mf_status mf_wiener_workspace_bytes(const mf_problem* p, int32_t chain, int32_t n_iter,
                                    int32_t ckpt_every, size_t* bytes);
mf_status mf_wiener_forward(mf_problem* p, int32_t chain, const double* d, const double* pk,
                            int32_t n_iter, int32_t ckpt_every, void* workspace, size_t ws_bytes,
                            double* chi2, double* s_out, void* stream);
mf_status mf_wiener_backward(mf_problem* p, int32_t chain, const double* d, void* workspace,
                             size_t ws_bytes, double* grad_d, double* grad_pk, void* stream);

/* The log-determinant term of the likelihood's power-spectrum gradient (grid
 * sides 32 to 256).  The data d = R s + eps of Sec. 2 are Gaussian with
 * covariance A = (R S R + N) over the observed voxels, so
 *   d ln L / d P_b = -1/2 d chi2_inf / d P_b - 1/2 T_b,
 *   T_b = tr(A^-1 R (dS/dP_b) R),
 * where chi2_inf is the converged chi2_K of mf_wiener_forward (whose P-gradient
 * mf_wiener_backward gives).  mf_wiener_logdet_trace estimates T_b by
 * Hutchinson's method with probes of covariance N: z = sgn(R) sqrt(N) xi on
 * observed voxels, xi = +-1 from Philox counter (v div 4, probe, 4, chain_id +
 * chain), word v mod 4 (top bit set -> -1) for voxel v in [ix][iy][iz] order.
 * Each probe is filtered by K messenger iterations (as in mf_wiener_forward),
 * u = N^-1 (z - R s_K) -> A^-1 z, and contributes
 *   (1/M) sum over the modes of bin b of Re(conj(FT(R u)) FT(R z / N)),
 * whose expectation is T_b once the filter has converged.
 *   pk: device FP64, n_bins per chain, physical units.
 *   trace_out: device FP64, n_bins per chain: the mean over probes probe0 ..
 *     probe0 + n_probes - 1, per unit of physical P_b.
 * chain = -1 runs every chain in the same launches.  The workspace (size from
 * mf_wiener_logdet_workspace_bytes, 256-byte aligned) holds the probe
 * coefficients and four spectra per chain.  One probe costs K + 3 iterations.
 * Enqueues on `stream`; uses the problem's shell partials as scratch, so it
 * must not overlap sweeps on the same problem.  The chains' Gibbs state is
 * not touched.
 * Errors: MF_E_UNSUPPORTED_SIZE, MF_E_STATE (bad chain), MF_E_INVALID_ARG
 * (n_iter or n_probes < 1, NULL pointers), MF_E_WORKSPACE, MF_E_DEVICE. */
mf_status mf_wiener_logdet_workspace_bytes(const mf_problem* p, int32_t chain, size_t* bytes);
mf_status mf_wiener_logdet_trace(mf_problem* p, int32_t chain, const double* pk, int32_t n_iter,
                                 int32_t n_probes, uint32_t probe0, void* workspace,
                                 size_t ws_bytes, double* trace_out, void* stream);

/* For callers that cannot allocate device memory (code being captured into
 * a HIP graph, serving loops, harnesses that forbid allocation):
 * mf_wiener_logdet_trace without the workspace argument.  The estimator's
 * scratch (the size mf_wiener_logdet_workspace_bytes reports) lives in a
 * static device array of MF_LOGDET_SCRATCH_BYTES (64 MiB) inside the
 * library, one per device, held from the first call on that device until the
 * process ends; the call allocates nothing.  That covers one 128^3 FP32
 * chain, or several chains at 64^3.  Arguments, results and the other errors
 * are those of mf_wiener_logdet_trace, with the problem on the calling
 * thread's current device.  Every call on a device uses the same array and
 * rewrites all of it that it reads, so calls do not see each other's
 * results; calls that overlap in time on one device (other streams or host
 * threads) race on it and must be serialised by the caller.
 * Errors: MF_E_WORKSPACE when the estimate needs more scratch than
 * MF_LOGDET_SCRATCH_BYTES, MF_E_DEVICE if the array's address cannot be
 * found, and those of mf_wiener_logdet_trace. */
#define MF_LOGDET_SCRATCH_BYTES (64ull << 20)
mf_status mf_wiener_logdet_trace_noalloc(mf_problem* p, int32_t chain, const double* pk,
                                         int32_t n_iter, int32_t n_probes, uint32_t probe0,
                                         double* trace_out, void* stream);

/* Streaming reference for the roofline (not part of the sampler): what
 * plain HBM streaming reaches on the device.  mode 0 copies `bytes` from src
 * to dst; mode 1 does the same with non-temporal loads and stores; mode 2
 * reads src and writes one 32-bit sum per workgroup to dst (dst holds at
 * least 4 * blocks bytes); mode 3 reads with non-temporal loads.  `blocks`
 * workgroups of 256 threads stride over the buffer, each thread moving four
 * 16-byte vectors per step.  Enqueues on `stream`.
 * Errors: MF_E_INVALID_ARG (NULL or unaligned pointers, bytes not a positive
 * multiple of 16, mode or blocks out of range), MF_E_DEVICE. */
mf_status mf_stream_reference(const void* src, void* dst, size_t bytes, int32_t mode,
                              int32_t blocks, void* stream);

/* Chain diagnostics (Sec. 5.1, "Statistical efficiency").
 *
 * Recording.  mf_set_diagnostics makes sweeps record sample n, the chain
 * state after n sweeps, as sweep n begins, for n = start + j * thin
 * (j = 0, 1, ...).  Two kinds of record can be kept, each optional (NULL
 * switches it off):
 *  - trace: caller-owned device FP64 array [n_chains][trace_cap][n_bins].
 *    Entry j holds P_b of recorded sample j in physical units; recording
 *    stops after trace_cap samples.
 *  - moments: caller-owned device FP64 array of n_chains * 2 * N^3 doubles,
 *    in the library's own order.  It holds running (Welford) sums for the
 *    posterior mean and variance of s.  It is zeroed here, and the z-pass
 *    updates it on every recorded sweep.
 * Sizes are given by mf_diagnostics_bytes.  The settings apply to sweeps
 * enqueued afterwards and to graphs created afterwards.  Calling again
 * resets the recording, and both NULL stops it.  Errors: MF_E_INVALID_ARG
 * (thin < 1, start >= 2^32, unaligned buffers), MF_E_STATE (a graph created
 * by mf_graph_create still holds this problem: it would keep recording into
 * the previous buffers).
 * mf_recorded_samples: samples recorded so far, from the problem's sweep
 * count (the trace holds min(count, trace_cap) of them).
 * mf_get_moments: writes the posterior mean and variance (population form,
 * 1/K over the K recorded samples) of chain `chain` to the device FP64
 * arrays mean and var (N^3 each, [ix][iy][iz]).  Enqueued on `stream`.
 * MF_E_STATE without a moment buffer or before the first recorded sample.
 *
 * Autocorrelation.  mf_acf takes a device FP64 trace [t][n_bins] (one
 * chain's records).  It writes the autocorrelation
 *   acf[n][b] = sum_{i < t-n} (x_i - mu)(x_{i+n} - mu) / ((t - n) var)
 * for n = 0 .. max_lag (Eq. CORR_COEFF: mean and variance taken over the t
 * samples, the average over the t - n available pairs), and the correlation
 * length nc[b], the first lag with acf < 0.1 or -1 if there is none
 * (device int32, n_bins).  A constant series gives NaN.  Enqueued on
 * `stream`.  MF_E_INVALID_ARG unless t >= 2 and 0 <= max_lag < t. */
mf_status mf_diagnostics_bytes(const mf_problem* p, int32_t trace_cap, size_t* trace_bytes,
                               size_t* moments_bytes);
mf_status mf_set_diagnostics(mf_problem* p, uint64_t start, int32_t thin, double* trace,
                             int32_t trace_cap, double* moments, void* stream);
mf_status mf_recorded_samples(const mf_problem* p, uint64_t* count);
mf_status mf_get_moments(mf_problem* p, int32_t chain, double* mean, double* var, void* stream);
mf_status mf_acf(const double* trace, int32_t t, int32_t n_bins, int32_t max_lag, double* acf,
                 int32_t* nc, void* stream);

/* Release the handle (not the workspace).  NULL is ignored. */
void mf_destroy_problem(mf_problem* p);

/* Thread-local message describing the last non-OK status (never NULL). */
const char* mf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MF_H */
