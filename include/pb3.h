/*
 * pb3.h -- C ABI of the MI355X binned power-spectrum / bispectrum library.
 *
 * The library computes the idealized (periodic-box, uniform density,
 * global line of sight, ell = 0) estimators of PolyBin3D (Philcox & Floss,
 * arXiv:2404.07249) on one gfx950 GPU:
 *
 *   P_b     = (V / N_pix^2) (1/N_b) sum_{n in b} |D(n)|^2
 *             -- eq. (pk-limit) over the ideal Fisher (bin volume,
 *                eq. fish-ideal-continuous), Sec. III.D.1;
 *   B_abc   = (V^2 / N_pix^3) (1/T_abc) sum_{n1+n2+n3=0} D(n1) D(n2) D(n3)
 *           = (V^2 / N_pix) sum_x G_a G_b G_c / T_abc on the N grid
 *             -- eq. (ideal-bk) and the closing full estimator of
 *                Sec. IV.D.1, evaluated through the separable form
 *                eq. (beta-def) with G_b = IDFT[Theta_b D] (eq. g-ell-def);
 *   T_abc   = number of closed mode triangles in the three shells
 *             -- N_0 of eq. (N-ell-def) with P_fid = 1 (Sec. IV.C.1).
 *
 * D(n) is the unnormalised DFT of the real field on the Nx x Ny x Nz grid
 * ("N^3" below: x slowest, z fastest; N_pix = Nx Ny Nz, V = Lx Ly Lz), n the
 * integer wave-vector, k_i = k_f,i n_i with k_f,i = 2 pi / L_i.  Bins are
 * half-open shells [e_b, e_{b+1}): for a box with equal sides in units of
 * k_f, decided on the integer |n|^2; otherwise in h/Mpc on the FP64 |k|^2.
 * Triplets are (a <= b <= c) with e_c < e_{a+1} + e_{b+1}, ordered with c
 * fastest; triplets with T_abc = 0 are dropped from the plan.
 *
 * Conventions for every entry point:
 *  - every function returns pb3_status and never aborts; on failure
 *    pb3_last_error() gives a thread-local message;
 *  - device pointers are caller-owned; work is enqueued asynchronously on
 *    the given HIP stream (a hipStream_t passed as void*, NULL = default
 *    stream); host outputs are written before the call returns;
 *  - a plan may have one call in flight at a time (its workspace is
 *    shared); different plans may run concurrently on different streams.
 */
#ifndef PB3_H
#define PB3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pb3_plan pb3_plan;

typedef enum {
  PB3_OK = 0,
  PB3_EINVAL = 1,        /* bad argument: null pointer, bad grid, unsorted edges, empty bin */
  PB3_ENOMEM = 2,        /* device or host allocation failed, or bound workspace too small */
  PB3_EDEVICE = 3,       /* a HIP call failed; message carries hipGetErrorString */
  PB3_EUNSUPPORTED = 4,  /* grid length or bin count outside what the kernels implement */
  PB3_EBUSY = 5          /* reserved */
} pb3_status;

/* Failure handling: every entry point returns a status and never aborts; a
 * call that fails for want of memory frees what it allocated and leaves the
 * plan or batch as it was (a plan creation that fails returns no plan).
 * Test hook: with the environment variable PB3_FAIL_ALLOC_AT=n, the n-th
 * device allocation of the library, counted from when that value was first
 * seen, fails as out of memory, which the call reports as PB3_ENOMEM.  A
 * changed value restarts the count; text after the number is ignored, so
 * "3:a" and "3:b" both arm the third allocation. */

typedef enum {
  PB3_FP32 = 0,          /* FP32 FFTs and FP32 MFMA contraction */
  PB3_MIXED_BF16X3 = 1   /* FP32 FFTs, contraction as split-BF16 (hi*hi + hi*lo + lo*hi) MFMA, FP32 accumulation */
} pb3_precision;

/* plan flags */
#define PB3_FLAG_EDGES_HMPC   0x1u  /* edges are in h/Mpc (else in units of k_f) */
#define PB3_FLAG_HOST_ONLY    0x2u  /* build host tables only (no device, no counts) */
#define PB3_FLAG_FULL_GRID    0x4u  /* contract on the N grid even when a smaller alias-free grid exists */
#define PB3_FLAG_STRICT       0x8u  /* fail with PB3_EINVAL if a triangle-valid triplet has T = 0 */
#define PB3_FLAG_EXT_WORKSPACE 0x10u /* never allocate the large workspace; caller binds one */
#define PB3_FLAG_STAGE_TIMING 0x20u /* record a HIP event pair around every kernel launch */
#define PB3_FLAG_NO_FUSION    0x40u /* run the inverse z pass as its own kernel and keep G in HBM
                                       (otherwise it is fused into the contraction when the
                                       contraction grid is 32..192 and there are <= 32 bins) */
#define PB3_FLAG_AUTOTUNE     0x80u /* choose the launch shape (fused or separate z pass, number of
                                       contraction work-groups) by timing the candidates on this
                                       device at plan creation; with the environment variable
                                       PB3_AUTOTUNE_CACHE naming a text file, choices are read
                                       from it and new ones appended (key: architecture, N, M,
                                       bin thresholds).  Overrides PB3_FLAG_NO_FUSION. */
#define PB3_FLAG_LMAX2        0x200u /* multipoles up to l = 2 (pb3_multipoles) */
#define PB3_FLAG_LMAX4        0x400u /* multipoles up to l = 4 (pb3_multipoles) */
#define PB3_FLAG_BK_FISHER    0x800u /* with PB3_FLAG_LMAX2/4: bispectrum multipoles normalised by
                                        the discrete ideal Fisher matrix (see pb3_multipoles) */
#define PB3_FLAG_POWER_ONLY   0x100u /* power spectra only (pb3_power, pb3_masked_power): no
                                        triplets, no triangle counts, no contraction buffers;
                                        pb3_bispectrum and batches refuse such a plan */

/* Build a plan for an Nx x Ny x Nz grid on an Lx x Ly x Lz box (the
 * estimators hold for any box; the paper's survey grids are non-cubic,
 * Sec. VI.A).
 *   grid[3]   grid points along x, y, z; each even with prime factors in
 *             {2, 3} (the FFT radices implemented), 16..384;
 *   box[3]    box sides in Mpc/h;
 *   edges     n_edges >= 2 strictly increasing bin edges.  Box with equal
 *             sides: k_f units, or h/Mpc with PB3_FLAG_EDGES_HMPC, then
 *             snapped to the nearest multiple of k_f/2 when within 1e-9
 *             relative; modes are binned on the integer |n|^2.  Box with
 *             unequal sides: h/Mpc (PB3_FLAG_EDGES_HMPC required); modes
 *             are binned on the FP64 value
 *             k^2 = (kfx^2 nx^2 + kfy^2 ny^2) + kfz^2 nz^2, kf_i = 2 pi / L_i,
 *             evaluated in that order;
 *   flags     PB3_FLAG_*.
 * On the device (unless PB3_FLAG_HOST_ONLY) it uploads the bin and triplet
 * tables and computes the triangle counts T_abc once in FP64 (N_0 is
 * data-independent, Sec. IV.D.1), on the default stream, synchronously.
 * The contraction grid is chosen per axis (the smallest implemented length
 * above 3 K_i, K_i the largest |n_i| of a binned mode, else N_i).
 * With the environment variable PB3_PLAN_CACHE naming a directory, the
 * counts (and, with PB3_FLAG_BK_FISHER, the multipole mixing blocks) are
 * read from a file there keyed by device architecture, grids and bins, and
 * written there after they are computed; a file whose key, length or
 * checksum does not match is ignored and rewritten.
 * Errors: PB3_EINVAL (bad grid/box/edges, a bin with no modes, strict-mode
 * empty triplet, unequal box sides without h/Mpc edges), PB3_EUNSUPPORTED
 * (grid length, more than 2^31 - 1 cells or > 48 bins), PB3_ENOMEM,
 * PB3_EDEVICE.  *out is NULL on failure. */
pb3_status pb3_plan_create(const int grid[3], const double box[3], const double* edges, int n_edges,
                           unsigned flags, pb3_plan** out);
pb3_status pb3_plan_destroy(pb3_plan* plan);

/* Bytes of device workspace one call needs (FP32 filtered fields on the
 * contraction grid, FFT intermediates, partial sums). */
size_t pb3_plan_workspace_bytes(const pb3_plan* plan);
/* Bind caller-owned device memory (>= pb3_plan_workspace_bytes) as the
 * workspace; replaces (and frees) any workspace the plan allocated. */
pb3_status pb3_plan_bind_workspace(pb3_plan* plan, void* dev, size_t bytes);

int pb3_n_bins(const pb3_plan* plan);
int pb3_n_triplets(const pb3_plan* plan);  /* after dropping T = 0 (host-only plans: before) */
int pb3_grid(const pb3_plan* plan);        /* Nx */
int pb3_contract_grid(const pb3_plan* plan); /* Mx: Nx, or the smaller alias-free length */
/* Grid (Nx, Ny, Nz) and contraction grid (Mx, My, Mz); either pointer may be NULL (not both). */
pb3_status pb3_grid3(const pb3_plan* plan, int* grid_out, int* contract_out);
/* Launch shape in use: fused (1) or separate (0) inverse z pass, contraction
 * work-groups, and how it was chosen (0 default, 1 autotune cache, 2 timed).
 * Any output pointer may be NULL. */
pb3_status pb3_plan_launch_shape(const pb3_plan* plan, int* fused_out, int* contract_wgs_out, int* tuned_out);

/* Bin edges (n_bins+1; k_f units for a box with equal sides, h/Mpc
 * otherwise), bin centres |k| in h/Mpc (mean |k| of the modes in the bin)
 * and mode counts N_b; any pointer may be NULL. */
pb3_status pb3_get_bins(const pb3_plan* plan, double* edges_kf_out, double* kmean_out, int64_t* n_modes_out);
/* Triplets (n_trip x 3 int32, a <= b <= c, c fastest). */
pb3_status pb3_get_triplets(const pb3_plan* plan, int32_t* abc_out);
/* Host copies of N_b (n_bins) and T_abc (n_trip, exact integers stored as
 * double); either pointer may be NULL.  Needs a device plan. */
pb3_status pb3_norm(const pb3_plan* plan, int64_t* n_modes_out, double* counts_out);

/* P_b for every bin.  delta_dev: N^3 float32, C order (x slowest, z
 * fastest), device memory, 8-byte aligned (the forward pass reads pairs of
 * values; PB3_EINVAL otherwise; the same holds for every field argument
 * below: data, windows, random fields, simulations and batch fields).
 * pk_dev: n_bins float64, device memory, (Mpc/h)^3. */
pb3_status pb3_power(pb3_plan* plan, const float* delta_dev, double* pk_dev, void* stream);

/* B_abc for every plan triplet: bk_dev n_trip float64 device memory,
 * (Mpc/h)^6. */
pb3_status pb3_bispectrum(pb3_plan* plan, const float* delta_dev, double* bk_dev, pb3_precision prec,
                          void* stream);

/* Both statistics from one forward FFT (pk_dev or bk_dev may be NULL). */
pb3_status pb3_polyspectra(pb3_plan* plan, const float* delta_dev, double* pk_dev, double* bk_dev,
                           pb3_precision prec, void* stream);

/* Conventional windowed normalisation for masked data d = w * delta
 * (the FKP-limit estimators of Sec. III.D.2 and Sec. IV.D.2 with the
 * linear and noise terms dropped): divides the plan's P by <w^2> and B by
 * <w^3> in place, the means taken over the N^3 voxels in FP64 with a fixed
 * summation order.  w_dev: N^3 float32 window (device); pk_dev / bk_dev:
 * outputs of pb3_polyspectra for d (either may be NULL, not both);
 * scratch_dev: PB3_WINDOW_SCRATCH doubles of device memory, whose first two
 * entries receive <w^2> and <w^3>.  Enqueued on `stream`. */
#define PB3_WINDOW_SCRATCH 514
pb3_status pb3_window_normalize(const pb3_plan* plan, const float* w_dev, double* pk_dev, double* bk_dev,
                                double* scratch_dev, void* stream);

/* Masked power spectrum with a Monte Carlo Fisher matrix (Sec. III.C.2:
 * eq. fish-from-Q with the Girard-Hutchinson trace of eq. girard-hutchinson;
 * global line of sight (eq. Q-alpha-global), l = 0, unit weighting, the
 * window as pointing matrix):
 *   p_b   = N_b P_box_b(d) / 2                       (numerator)
 *   F_ab  = (1 / 2 n_grf N_pix) sum_i sum_{n in b} conj(DFT[w g_a^i](n)) DFT[a_i](n),
 *           g_a = IDFT[Theta_a DFT[w a_i]]  (sum over the full spectrum of bin b)
 *   P_b   = (F^-1 p)_b                               (unwindowed estimate)
 * for white unit-variance random fields a_i (so the A^-1 of the paper is the
 * identity; with w = 1 the expectation of F is diag(N_b) / 2 and P is the
 * box estimator).  The plan must contract on its own grid
 * (PB3_FLAG_FULL_GRID), since w is not band-limited.
 *   data_dev   N^3 float32, the masked data d = w * delta
 *   window_dev N^3 float32, w
 *   grfs_dev   host array of n_grf device pointers to N^3 float32 fields
 *              (the caller draws them: white, zero mean, unit variance)
 *   pk_dev     n_bins float64 output, (Mpc/h)^3
 *   fisher_dev n_bins x n_bins float64 output (row a, column b) or NULL
 *   workspace  >= pb3_masked_power_workspace_bytes, 256-byte aligned
 *              (per bin the windowed filtered field after its z transform,
 *              n_bins N^2 Kz complex values, or n_bins N^3 floats of
 *              filtered fields for N < 64; the y and x transforms of 8 bins;
 *              the plan's FFT buffers and partial sums)
 * Enqueued on `stream`; the first call on a plan also uploads a small
 * table synchronously.  Errors: PB3_EINVAL (null argument, host-only plan,
 * plan without the full grid, n_grf < 1), PB3_EUNSUPPORTED (> 48 bins,
 * unequal grid sides or box sides), PB3_ENOMEM (workspace too small),
 * PB3_EDEVICE. */
size_t pb3_masked_power_workspace_bytes(const pb3_plan* plan);
pb3_status pb3_masked_power(pb3_plan* plan, const float* data_dev, const float* window_dev,
                            const float* const* grfs_dev, int n_grf, double* pk_dev, double* fisher_dev,
                            void* workspace_dev, size_t workspace_bytes, void* stream);

/* Bispectrum with the linear term of the numerator (eq. b-numerator-practical,
 * Sec. IV.C), averaged over n_sim fields Delta_i with about the data's
 * covariance (simulations or Gaussian fields passed through the same window):
 *   B = (V^2/N_pix) [S(d) - (1/n_sim) sum_i S_lin(d; Delta_i)] / T,
 *   S_lin = sum_x (G_a[d] G_b[D] G_c[D] + G_a[D] G_b[d] G_c[D] + G_a[D] G_b[D] G_c[d]),
 * unit weighting, in the units of pb3_bispectrum (divide by <w^3> with
 * pb3_window_normalize for the windowed form).  The term vanishes in
 * expectation; it lowers the variance where a window breaks translation
 * invariance (zero in the ideal limit).  Evaluated as the part of the cubic
 * S(D + d) with one factor of d, [S(D + d) - S(D - d)] / 2 - S(d), through the
 * plan's own launch sequence (two jobs per Delta_i, up to 8 jobs per launch)
 * and combined in FP64.
 *   data_dev  N^3 float32
 *   sims_dev  host array of n_sim >= 1 device pointers to N^3 float32 fields
 *   bk_dev    n_trip float64 output
 *   workspace >= pb3_bispectrum_linear_workspace_bytes(plan, n_sim), 256-byte
 *             aligned (up to 8 copies of the plan's workspace, the D +- d
 *             fields and per-job outputs)
 * Errors: PB3_EINVAL (null argument, host-only or power-only plan, plan with
 * pb3_plan_set_weights, n_sim < 1, bad precision), PB3_ENOMEM (workspace too
 * small), PB3_EDEVICE. */
size_t pb3_bispectrum_linear_workspace_bytes(const pb3_plan* plan, int n_sim);
pb3_status pb3_bispectrum_linear(pb3_plan* plan, const float* data_dev, const float* const* sims_dev, int n_sim,
                                 double* bk_dev, pb3_precision prec, void* workspace_dev, size_t workspace_bytes,
                                 void* stream);

/* Weighted ideal estimators (Sec. III.D.1 eq. pk-limit and Sec. IV.D.1 with
 * P_fid, the pixel window m(k) and the Poisson shot-noise terms):
 *   P_b = (V/N_pix^2) sum_{n in b} |D/m|^2 / P_fid^2 / sum_{n in b} 1 / P_fid^2  -  1/nbar
 *   B_abc = (V^2/N_pix^3) sum_closed D1 D2 D3 / (m1 m2 m3 P1 P2 P3) / N_0  -  B_shot,
 *   N_0 = sum_closed 1 / (P1 P2 P3),
 *   B_shot = 1/nbar^2 + <P1 + P2 + P3>/nbar, averaged with the weights of N_0,
 *            with the power model P = P_fid - 1/nbar (P_fid includes shot noise).
 * window_order: pixel window deconvolved, m(n) = prod_i sinc(pi n_i / N_i)^order
 * (0 none, 1 nearest grid point, 2 cloud in cell, 3 triangular shaped cloud);
 * pfid: P_fid in (Mpc/h)^3 at integer |n|^2 = 0 .. n_pfid-1 (n_pfid >=
 * pb3_weights_table_len, positive at every binned |n|^2), or NULL for P_fid = 1;
 * nbar: number density in (Mpc/h)^-3, or 0 for no shot-noise terms (nbar > 0
 * needs pfid unless the plan is power-only).  Call once per plan, before its
 * first use; recomputes the (now non-integer) triangle sums in FP64
 * synchronously.  pb3_norm then returns N_0.  Applies to pb3_power,
 * pb3_bispectrum, pb3_polyspectra, batches and pb3_multipoles (shot noise on
 * the monopole); pb3_masked_power refuses a weighted plan.
 * Errors: PB3_EINVAL (host-only plan, weights already set, bad order or
 * nbar, table too short or not positive), PB3_EUNSUPPORTED (a box with
 * unequal sides: P_fid is tabulated over integer |n|^2), PB3_ENOMEM,
 * PB3_EDEVICE. */
int pb3_weights_table_len(const pb3_plan* plan);
pb3_status pb3_plan_set_weights(pb3_plan* plan, int window_order, const double* pfid, int n_pfid, double nbar);

/* Multipoles l = 0, 2 (, 4) with a global line of sight along the grid's z
 * axis, for plans made with PB3_FLAG_LMAX2 or PB3_FLAG_LMAX4:
 *   P_{b,l}   = sum_l' (F_b^-1)_{l l'} p_{b,l'},  p_{b,l} = (V/N_pix^2) sum_{n in b} L_l(mu_n) |D(n)|^2,
 *               F_b[l][l'] = sum_{n in b} L_l(mu_n) L_l'(mu_n)  -- eq. (pk-limit) with its
 *               discrete Fisher matrix, which keeps the l-l' couplings of the finite
 *               Fourier grid (Sec. III.D.1); mu_n = n_z / |n|;
 *   B_{abc,l} = (2l + 1) (V^2/N_pix) sum_x G_a G_b g_{c,l} / T_abc,
 *               g_{c,l} = IDFT[Theta_c L_l(mu) D]  -- eq. (ideal-bk), the Legendre weight on
 *               k_3 (the mode in the largest bin), evaluated through the separable
 *               form of Sec. IV.D.1 (l = 0 is pb3_bispectrum's B).
 *   With PB3_FLAG_BK_FISHER the bispectrum multipoles are instead
 *   b = F^-1 b^num with the discrete ideal Fisher matrix of eq. (bk-fish-ideal)
 *   and the degeneracy factors Delta of eq. (Delta-alpha-def) (N_l of eq.
 *   (N-ell-def) summed on the grid): per kept triplet an n_ell x n_ell block,
 *   applied as b = R B above, R = Delta Ft^+ diag(T / (2l+1)), Ft the block
 *   without its 1/(Delta Delta') and Ft^+ its pseudo-inverse (eigenvalues
 *   below 1e-12 of the largest dropped).  The blocks are summed in FP64 at
 *   plan creation (weighted unit fields on the contraction grid).  Such plans
 *   need equal box sides and refuse pb3_plan_set_weights.
 * pb3_n_ell gives the number of multipoles (lmax/2 + 1).  pk_dev: n_ell x n_bins
 * float64 (row l/2), bk_dev: n_ell x n_trip float64; either may be NULL (not
 * both).  prec: PB3_MIXED_BF16X3 runs the contraction on the matrix cores
 * (pairs of G_a G_b against columns of g_{c,l}, split-bf16 x3), PB3_FP32 on
 * FP32 FMA tiles flushed to FP64.  workspace: >= pb3_multipoles_workspace_bytes, 256-byte aligned
 * (n_ell x n_bins filtered fields on the contraction grid plus partial sums).
 * Errors: PB3_EINVAL (plan without multipoles, null arguments, power-only
 * plan asked for B; at creation: a bin whose modes cannot separate the
 * multipoles), PB3_ENOMEM (workspace too small), PB3_EDEVICE. */
int pb3_n_ell(const pb3_plan* plan);
/* The per-triplet mixing blocks R of a PB3_FLAG_BK_FISHER plan, host copy:
 * mix_out holds n_trip x n_ell x n_ell doubles (row l/2, column l'/2).
 * Errors: PB3_EINVAL (null arguments, plan without the flag). */
pb3_status pb3_multipole_mixing(const pb3_plan* plan, double* mix_out);
size_t pb3_multipoles_workspace_bytes(const pb3_plan* plan);
pb3_status pb3_multipoles(pb3_plan* plan, const float* delta_dev, double* pk_dev, double* bk_dev,
                          pb3_precision prec, void* workspace_dev, size_t workspace_bytes, void* stream);

/* Stage timing (plans made with PB3_FLAG_STAGE_TIMING): every call records
 * a HIP event pair around each kernel launch on the call's stream.
 * pb3_stage_times writes, per stage, the mean milliseconds over the calls
 * made since the last pb3_stage_timing_reset (at most the latest 256),
 * in the order fwd_z, fwd_y, fwd_x, power, inv_x, inv_y, inv_z, contract,
 * reduce (0 for stages that did not run); counts_out (may be NULL)
 * receives how many calls each mean covers.  It synchronises on the
 * recorded events.  n_out receives the number of stages written. */
pb3_status pb3_stage_times(pb3_plan* plan, float* ms_out, int* counts_out, int capacity, int* n_out);
pb3_status pb3_stage_timing_reset(pb3_plan* plan);
const char* pb3_stage_name(int stage);

/* ---------------------------------------------------------------- batches
 * Many fields through one or more plans in few launches.  The paper runs
 * its estimators independently over many simulations (Sec. VI); here those
 * evaluations share kernel launches:
 *  - jobs that use the same plan object run in the same launches, up to 8
 *    per launch (grid dimension z enumerates the jobs, each with its own
 *    workspace slice);
 *  - groups of different plans run concurrently on internal streams
 *    (default priority), forked from and joined back into the caller's
 *    stream, so the run is ordered on that stream like one call;
 *  - with PB3_BATCH_GRAPH the fork, all launch sequences and the join are
 *    captured once into a HIP graph that later runs replay; a run with other
 *    pointers, outputs or precision captures again and updates the graph.
 * Every job's results equal, bit for bit, those of pb3_polyspectra on the
 * same plan and field: the kernels and reduction orders are the same.
 * A batch has one run in flight at a time; its plans must outlive it and
 * must not be destroyed or re-bound while it exists. */
typedef struct pb3_batch pb3_batch;

#define PB3_BATCH_GRAPH         0x1u  /* capture the run into a HIP graph, replay afterwards */
#define PB3_BATCH_EXT_WORKSPACE 0x2u  /* do not allocate; caller binds pb3_batch_workspace_bytes */

/* plans: host array of n_jobs device plans (current device; repeats share
 * launches).  Allocates the workspace unless PB3_BATCH_EXT_WORKSPACE.
 * Errors: PB3_EINVAL (null or host-only plan, n_jobs < 1, unknown flag),
 * PB3_ENOMEM, PB3_EDEVICE. */
pb3_status pb3_batch_create(pb3_plan* const* plans, int n_jobs, unsigned flags, pb3_batch** out);
pb3_status pb3_batch_destroy(pb3_batch* batch);
/* Sum over jobs of their plans' workspace sizes. */
size_t pb3_batch_workspace_bytes(const pb3_batch* batch);
/* Caller-owned device memory, 256-byte aligned, >= pb3_batch_workspace_bytes. */
pb3_status pb3_batch_bind_workspace(pb3_batch* batch, void* dev, size_t bytes);
/* Run every job.  deltas: host array of n_jobs device pointers (N^3 float32
 * of the job's plan); pk / bk: host arrays of n_jobs device outputs
 * (n_bins / n_trip float64 of the job's plan), or NULL to skip that
 * statistic for all jobs (not both).  Enqueued on `stream`. */
pb3_status pb3_batch_run(pb3_batch* batch, const float* const* deltas, double* const* pk, double* const* bk,
                         pb3_precision prec, void* stream);
/* Kernel launches one run issues (with or without each statistic) and the
 * number of launch groups (plan, up to 8 jobs). */
int pb3_batch_launches(const pb3_batch* batch, int with_pk, int with_bk);
int pb3_batch_groups(const pb3_batch* batch);

/* One-shot form: builds a batch for plans[0..n_jobs), runs the bispectra of
 * all fields, waits for `stream` and frees the batch (allocates and
 * synchronises on every call; repeated use should keep a pb3_batch). */
pb3_status pb3_bispectrum_batched(pb3_plan* const* plans, const float* const* deltas, double* const* bk_outs,
                                  int n_jobs, pb3_precision prec, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the power
 * spectrum of pb3_power, with its workspace (forward-pass outputs, compact
 * spectrum, per-chunk sums: 8 Nx (Ny + Lcy) Kz + 8 Lcx Lcy Kz bytes and a
 * few KB, with Lcx, Lcy, Kz the compact extents of the binned modes) in a
 * static device array of 64 MiB that the library holds on every GPU it runs
 * on until the process ends, instead of the plan's workspace (which it
 * neither needs nor touches, so a plan made with PB3_FLAG_EXT_WORKSPACE may
 * skip binding one).  Same arguments and output as pb3_power; calls no
 * hipMalloc, hipFree or other allocating routine.  PB3_EUNSUPPORTED, with
 * the bytes needed in pb3_last_error(), when the plan needs more than the
 * array holds (54 MB at 256^3 with 30 bins of width 2 k_f fits; a 384^3
 * grid with 40 such bins does not).  All calls on one GPU share the array:
 * calls that overlap on one GPU (other streams, other threads) race and
 * must be serialised by the caller. */
pb3_status pb3_power_noalloc(pb3_plan* plan, const float* delta_dev, double* pk_dev, void* stream);

const char* pb3_status_string(pb3_status s);
const char* pb3_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PB3_H */
