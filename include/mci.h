/*
 * mci.h -- C ABI of libmci, an MI355X (gfx950) implementation of FFT multichannel
 * interpolation (MCI): Cheng & Kou, "FFT Multichannel Interpolation and Application
 * to Image Super-resolution", arXiv:1802.10291.
 *
 * Problem (Section 3, Theorem 3.3): a signal f on [0, 2 pi) with Fourier coefficients
 * a(n) on the band [n1, n1 + M N) is observed through M linear systems with Fourier
 * multipliers b_m(n) (eq. sysfunction); each output g_m = f * h_m is sampled at the N
 * points t_p = 2 pi p / N.  MCI recovers the band coefficients from the M N samples
 * (exactly when f is in the band, Theorem 3.3; as the approximation operator of
 * eq. "appxi operator" otherwise) and evaluates f, or a Fourier-multiplier image Qf of
 * it (end of Section 3), on a uniform output grid t_j = 2 pi j / n_out.
 *
 * The path a library call runs, entirely on the GPU:
 *   1. DFT of every channel (Lemma 3.1): d_m(n) = (1/N) sum_p g_m(t_p) e^{-i n t_p}
 *   2. per residue n in I_1 = [n1, n1 + N), A_n = D_n H_n^{-1} (eq. matrixeqn1) with
 *      H_n[j][k] = b_k(n + j N) (eq. defH), and the output operator o(n) applied
 *   3. the recovered coefficients placed in a spectrum of length n_out at n mod n_out
 *      (coefficients that land on the same bin add, so n_out < M N is exact)
 *   4. an inverse DFT of length n_out (eq. DFTexpression evaluated on the grid)
 * In real mode the result is the real part of the reconstruction.
 *
 * Conventions for every call:
 *  - Every function returns an mci_status; nothing throws across the ABI.
 *  - Array pointers passed to mci_reconstruct_1d / mci_upsample_2d are DEVICE pointers
 *    owned by the caller; the library never frees them.  Descriptor pointers (channel
 *    tables) are HOST pointers, read during the call and copied.
 *  - Device data pointers and workspaces given to mci_reconstruct_1d, mci_upsample_2d,
 *    mci_reconstruct_batch, mci_evaluate_1d and mci_averaged_error must be 16-byte aligned
 *    (the kernels use 8- and 16-byte vector accesses); otherwise the call returns
 *    MCI_E_INVALID_ARG.  hipMalloc'd memory always is; a view at an odd element offset may
 *    not be.
 *  - Argument errors are reported synchronously, before any work is queued.
 *  - A singular or ill-conditioned channel system is reported by mci_plan, never by a
 *    reconstruction call.
 *  - Reconstruction calls are asynchronous on the given stream; a kernel launch failure
 *    is reported as MCI_E_DEVICE by that call.
 *  - A plan may be used from several streams at once, provided each call has its own
 *    workspace.  Only mci_plan_set_variant and mci_plan_autotune change a plan; they must
 *    not run while work queued with the plan is pending.
 */
#ifndef MCI_H
#define MCI_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MCI_OK = 0,
  MCI_E_INVALID_ARG = 1,     /* bad pointer, size, enum value or layout */
  MCI_E_SINGULAR = 2,        /* some H_n is singular and MCI_ALLOW_SINGULAR_ZERO is not set */
  MCI_E_ILL_CONDITIONED = 3, /* max over n of cond_1 of the equilibrated H_n^T exceeds cond_max */
  MCI_E_UNSUPPORTED = 4,     /* valid request this build does not implement */
  MCI_E_OUT_OF_MEMORY = 5,   /* plan tables could not be allocated */
  MCI_E_DEVICE = 6           /* a HIP runtime call or kernel launch failed */
} mci_status;

/* Fourier multiplier of one channel (eq. sysfunction). */
typedef enum {
  MCI_MULT_DERIV = 0,   /* b(n) = (i n)^order: the order-th derivative (Example 3.6) */
  MCI_MULT_HILBERT = 1, /* b(n) = -i sgn n: the circular Hilbert transform (Section 2, Example 3.7) */
  MCI_MULT_TABLE = 2    /* b(n) given for n in [n1, n1 + M N) */
} mci_mult_kind;

/* Output operator o(n), applied to the recovered coefficients (Example 3.11 and the
 * closing paragraph of Section 3). */
typedef enum {
  MCI_OUT_IDENTITY = 0, /* f */
  MCI_OUT_HILBERT = 1,  /* circular Hilbert transform of f: o(n) = -i sgn n */
  MCI_OUT_DERIV = 2     /* order-th derivative of f: o(n) = (i n)^order */
} mci_out_op;

typedef enum { MCI_F32 = 0, MCI_F64 = 1 } mci_precision;

/* Storage type of the caller's input/output arrays. */
typedef enum {
  MCI_STORE_NATIVE = 0, /* float for MCI_F32 plans, double for MCI_F64 plans */
  MCI_STORE_F16 = 1     /* IEEE half (MCI_F32 plans only); arithmetic stays FP32 */
} mci_storage;

#define MCI_MAX_CHANNELS 4
#define MCI_MAX_OPS 4
#define MCI_N1_DEFAULT INT64_MIN       /* band start -floor((M N - 1) / 2) */
#define MCI_ALLOW_SINGULAR_ZERO 1u     /* Remark 3.4: a singular H_n contributes zero coefficients */

typedef struct {
  int32_t kind;         /* mci_mult_kind */
  int32_t order;        /* MCI_MULT_DERIV: derivative order, 0..8 */
  const double* table;  /* MCI_MULT_TABLE: host array of 2*M*N doubles, (re, im) of b(n) for
                           n = n1 .. n1 + M N - 1; copied by mci_plan.  NULL otherwise. */
} mci_channel;

typedef struct {
  int32_t M;                            /* channels, 1..MCI_MAX_CHANNELS */
  int32_t n_ops;                        /* output operators, 1..MCI_MAX_OPS */
  int64_t N;                            /* samples per channel (the paper's L), >= 1 */
  int64_t n1;                           /* band start (the paper's N_1), or MCI_N1_DEFAULT */
  int64_t n_out;                        /* output grid size, >= 1 */
  mci_channel ch[MCI_MAX_CHANNELS];     /* first M used */
  int32_t ops[MCI_MAX_OPS];             /* mci_out_op, first n_ops used */
  int32_t op_orders[MCI_MAX_OPS];       /* derivative order for MCI_OUT_DERIV, 0..8 */
  int32_t real_io;                      /* 1: real samples in, real part out; 0: complex in and out */
  int32_t precision;                    /* mci_precision of the transforms and the apply */
  int32_t storage;                      /* mci_storage of g and y */
  uint32_t flags;                       /* MCI_ALLOW_SINGULAR_ZERO */
  double cond_max;                      /* reject plans above this condition number; 0 => 1e12 */
} mci_plan_desc;

typedef struct mci_plan_s* mci_plan_t;

typedef struct {
  double max_cond;          /* max over residues of cond_1 of the row-equilibrated H_n^T */
  int64_t n_singular;       /* residues whose H_n was singular (zeroed under Remark 3.4) */
  int64_t first_singular;   /* band index n of the first one, or INT64_MIN */
  int64_t n1;               /* band start actually used */
  int64_t fft_len_fwd;      /* transform length executed for the channel DFTs (N, or the Bluestein length) */
  int64_t fft_len_inv;      /* transform length executed for the output grid */
  int32_t path;             /* 0: multi-pass path through the workspace, 1: fused single-pass kernel */
  int32_t variant;          /* active mci_variant */
} mci_plan_info_t;

/* mci_plan -- build a 1-D reconstruction plan on `device`.
 * Builds H_n = [b_k(n + jN)]_{jk} for every residue n of I_1 (eq. defH) and inverts it in
 * FP64 on the GPU; stores the tables q_mj(n) o(n + jN) / N for the apply step, the
 * transform twiddles and, for transform lengths with a prime factor above 7, the
 * Bluestein chirp tables.  One device synchronisation (to read back singular flags).
 * Errors: MCI_E_INVALID_ARG (bad descriptor), MCI_E_SINGULAR (first singular residue is
 * available through mci_plan_info of no plan: the call fails and *out is NULL),
 * MCI_E_ILL_CONDITIONED, MCI_E_OUT_OF_MEMORY, MCI_E_DEVICE.  *out is set only on success. */
mci_status mci_plan(const mci_plan_desc* desc, int device, mci_plan_t* out);

/* mci_plan_destroy -- release a plan's device tables.  NULL is a no-op. */
mci_status mci_plan_destroy(mci_plan_t plan);

/* mci_plan_info -- describe a plan. */
mci_status mci_plan_info(mci_plan_t plan, mci_plan_info_t* info);

/* mci_plan_kernel_name -- a description of the kernels the plan's active variant runs
 * (e.g. "k_mci1d_fused: forward split-Bluestein 1024-point, output 2 x 4096-point, M=3"),
 * NUL-terminated and truncated to len bytes.  For the autotuner's record and for profiles. */
mci_status mci_plan_kernel_name(mci_plan_t plan, char* name, size_t len);

/* mci_workspace_size -- device bytes of scratch a reconstruction of `batch` signals needs
 * (0 for plans that run fused).  The caller allocates it, so reconstruction calls never
 * allocate. */
mci_status mci_workspace_size(mci_plan_t plan, int64_t batch, size_t* bytes);

/* mci_reconstruct_1d -- reconstruct `batch` signals (Theorem 3.3 / eq. DFTexpression).
 *   g : device, samples [batch][M][N] (real_io) or [batch][M][N][2] (complex, re/im
 *       interleaved), element type per precision/storage, contiguous.
 *   y : device, output [batch][n_ops][n_out] (real_io) or [batch][n_ops][n_out][2].
 *   workspace / ws_bytes : device scratch of at least mci_workspace_size(plan, batch).
 *   stream : HIP stream the kernels are queued on (0 = null stream).
 * batch = 0 is a no-op.  g and y must not overlap. */
mci_status mci_reconstruct_1d(mci_plan_t plan, const void* g, void* y, int64_t batch, void* workspace,
                              size_t ws_bytes, hipStream_t stream);

/* mci_reconstruct_1d_strided -- mci_reconstruct_1d on signals spaced ld_g elements apart in g
 * and ld_y elements apart in y (signal b's samples start at g + b ld_g, its outputs at
 * y + b ld_y, each laid out as in mci_reconstruct_1d; elements of the storage type, a complex
 * value counting two).  ld_g >= M N (x2 for complex), ld_y >= n_ops n_out (x2 for complex),
 * both multiples of 4 (vector access); the output extents must not overlap.  The kernels and
 * results are those of mci_reconstruct_1d, the signals found through a table of offsets that
 * the call writes into the workspace (so it still allocates nothing and is graph-capturable):
 * workspace / ws_bytes of at least mci_workspace_size_strided(plan, batch), 16-byte aligned.
 * Errors: MCI_E_INVALID_ARG (strides, alignment, workspace), MCI_E_DEVICE. */
mci_status mci_reconstruct_1d_strided(mci_plan_t plan, const void* g, int64_t ld_g, void* y, int64_t ld_y,
                                      int64_t batch, void* workspace, size_t ws_bytes, hipStream_t stream);
/* mci_workspace_size_strided -- device bytes mci_reconstruct_1d_strided needs for `batch`
 * signals (1-D plans; 0 for batch = 0). */
mci_status mci_workspace_size_strided(mci_plan_t plan, int64_t batch, size_t* bytes);

/* ----------------------------------------------------------------------------------- */
/* 2-D separable upsampling (Section 5.2): every row, then every column of the result,  */
/* is reconstructed by MCI from two channels -- the line and its three-point centred     */
/* difference (x[p+1] - x[p-1]) / (2h), h = 2 pi / (line length), circular -- with       */
/* multipliers {1, i n}, band start -floor((2 len - 1) / 2), on a grid `scale` times      */
/* finer, keeping the real part after each pass.                                         */
/* ----------------------------------------------------------------------------------- */
typedef struct {
  int32_t h, w;         /* low-resolution image size, each >= 2 */
  int32_t scale;        /* upsampling factor s >= 1: output is (s h) x (s w) */
  int32_t precision;    /* MCI_F32 (MCI_F64 accepted for validation runs) */
  int32_t storage;      /* mci_storage of lr and hr */
  int32_t channels;     /* channels per line: 2 = {x, Dx} (0 also means 2), or 3 = {x, Dx, D2x} with the
                           three-point second difference (x[p+1] - 2x[p] + x[p-1]) / h^2 and multiplier
                           (i n)^2, the setting of the paper's Section 5.2 experiments */
} mci_plan2d_desc;

/* mci_plan_2d -- build a 2-D upsampling plan (two 1-D plans, rows and columns). */
mci_status mci_plan_2d(const mci_plan2d_desc* desc, int device, mci_plan_t* out);

/* mci_upsample_2d -- lr [batch][h][w] -> hr [batch][s h][s w], row-major, device pointers.
 * workspace of mci_workspace_size(plan, batch) bytes (holds the columns pass's result).
 * With the line passes at scale 2 (FP32 storage) the output rows s q are the input rows
 * (interpolation consistency, Theorem 4.1): the columns pass stores only the other rows and
 * the rows pass reads the sample rows from lr again, so lr must stay unchanged until the call's
 * work on the stream is done (as for every input).  MCI_LP_ZR=1 / MCI_LP_FULL_COLUMNS=1 in the
 * environment at plan creation take that form at every scale / at none. */
mci_status mci_upsample_2d(mci_plan_t plan, const void* lr, void* hr, int64_t batch, void* workspace,
                           size_t ws_bytes, hipStream_t stream);

/* ----------------------------------------------------------------------------------- */
/* Kernel variants and the autotuner (not in the paper: a choice among equivalent          */
/* schedules of the same arithmetic, steps 1-4 above; every variant meets the same        */
/* tolerance against the FP64 definition).                                                */
/* ----------------------------------------------------------------------------------- */
typedef enum {
  MCI_VARIANT_MULTIPASS_R8 = 0, /* multi-pass Stockham, radix-8 passes first */
  MCI_VARIANT_MULTIPASS_R4 = 1, /* multi-pass Stockham, radix-4 passes (more, lighter passes) */
  MCI_VARIANT_FUSED_T1 = 2,     /* 1-D single-pass kernel, output transforms one at a time */
  MCI_VARIANT_FUSED_T2 = 3,     /* 1-D single-pass kernel, both output transforms side by side */
  MCI_VARIANT_LINE_PASS = 4,    /* 2-D fused line passes (columns, then rows) */
  MCI_VARIANT_TWO_PASS = 5,     /* multi-pass path with each transform of length A B (A, B in
                                   {32, 48, 64, 96, 128, 192, 256, 384, 512}) in two LDS passes
                                   (one for a single such length); other lengths radix-8 */
  MCI_VARIANT_REAL_TWO_PASS = 6, /* FP32 plans in real mode (FP32 or FP16 storage) with even
                                   n_out and n_out/2 as above: channel DFTs straight from the
                                   sample rows (read as N/2 complex pairs for even N), apply, real
                                   part and a 2-phase polyphase gather in one kernel, one inverse
                                   transform of length n_out/2 written as the output row */
  MCI_NUM_VARIANTS = 7
} mci_variant;

/* Bit v of *mask is set when variant v can run this plan.  1-D plans: MULTIPASS_R8/R4
 * always, TWO_PASS for FP32 plans where a transform length factors as above (the Bluestein
 * lengths of FP32 plans are chosen so), FUSED_T1/T2 when the single-pass kernel covers the
 * descriptor (and fits the LDS), REAL_TWO_PASS as described above.  New 1-D plans start on
 * FUSED_T1, else REAL_TWO_PASS, else TWO_PASS, else MULTIPASS_R8.  2-D plans: MULTIPASS_R8 (rows then columns through the 1-D plans) always,
 * LINE_PASS for FP32 plans with h, w in {32, 48, 64, 96, 128, 192, 256, 384, 512} and scale
 * in {2, 4} (the default when available). */
mci_status mci_plan_variants(mci_plan_t plan, uint32_t* mask);

/* Make variant v the one the plan runs.  MCI_E_UNSUPPORTED when bit v of the mask is clear.
 * The workspace size (mci_workspace_size) follows the variant. */
mci_status mci_plan_set_variant(mci_plan_t plan, int32_t variant);

typedef struct {
  int32_t variant;          /* chosen (and now active) variant */
  int32_t from_cache;       /* 1: taken from the cache file without timing */
  int64_t batch;            /* batch the times were taken at */
  double ms[MCI_NUM_VARIANTS]; /* mean time per call of each variant tried, -1 if not tried */
} mci_tune_result;

/* mci_plan_autotune -- time every available variant on `batch` instances of this plan
 * (zero-filled inputs: the arithmetic, and so the time, does not depend on the values),
 * activate the fastest and record it in a JSON cache file keyed by the device (arch, CU
 * count) and the plan's shape.  cache_path NULL => the path in $MCI_TUNE_CACHE, if set;
 * no path => no cache.  With a cache entry for the key the entry is applied without
 * timing.  Plans created while $MCI_TUNE_CACHE names a file take their variant from it.
 * Allocates its own buffers and synchronises the device: call it at set-up, not inside
 * graph capture.  Errors: MCI_E_INVALID_ARG, MCI_E_OUT_OF_MEMORY, MCI_E_DEVICE (a cache file
 * that cannot be written is not an error: the result is still applied). */
mci_status mci_plan_autotune(mci_plan_t plan, int64_t batch, const char* cache_path, mci_tune_result* result);

/* ----------------------------------------------------------------------------------- */
/* Uneven batches (not in the paper): thousands of instances of different plans -- 1-D    */
/* lengths, channel counts, 2-D image sizes -- in one call on ragged packed buffers.      */
/* ----------------------------------------------------------------------------------- */
typedef struct {
  mci_plan_t plan;   /* 1-D or 2-D plan reconstructing this instance */
  int64_t in_off;    /* offset of the instance's input (g, or lr) in the packed input, in elements */
  int64_t out_off;   /* offset of its output (y, or hr) in the packed output, in elements */
} mci_batch_item;

typedef struct mci_batch_s* mci_batch_t;

/* mci_batch_create -- group the items by plan (one size class per distinct plan), upload
 * one device table of (in_off, out_off) per class, and spread the classes over `lanes`
 * streams (1..16; 0 => 16) by estimated bytes, largest first.  All plans must live on one
 * device, share one element type (FP32, FP16 or FP64 storage) and outlive the batch.
 * Offsets are >= 0 and multiples of 4 elements (vector access); output extents must not
 * overlap.  Each instance's layout inside its extent is the single-instance layout of
 * mci_reconstruct_1d / mci_upsample_2d.  With MCI_BATCH_MERGED=1 in the environment at
 * creation, the classes whose plans run the single-pass 1-D kernel, the real-mode
 * line-transform path or the 2-D line passes are recorded as jobs instead: per lane and
 * step of their launch sequences, one persistent launch per kernel template walks a device
 * table of the jobs' arguments (opt-in: slower than the classes' own launches on the mixed
 * workload).  The batch fixes each plan's variant at creation.  Allocates (the tables, the
 * lane streams and events): build batches at set-up.  Errors: MCI_E_INVALID_ARG,
 * MCI_E_OUT_OF_MEMORY, MCI_E_DEVICE. */
mci_status mci_batch_create(const mci_batch_item* items, int64_t n_items, int lanes, mci_batch_t* out);
mci_status mci_batch_destroy(mci_batch_t batch);

/* Element counts the packed input and output must hold (max over items of offset + size)
 * and the workspace bytes mci_reconstruct_batch needs with the plans' current variants. */
mci_status mci_batch_sizes(mci_batch_t batch, int64_t* in_elems, int64_t* out_elems, size_t* ws_bytes);

/* mci_reconstruct_batch -- reconstruct every instance: each class runs its plan's kernels
 * over its offset table; classes on different lanes run concurrently (the lanes fork from
 * and join back into `stream` through events), so one call queues all of it and a stream
 * capture of the call records it as one graph.  No allocation, no synchronisation, no
 * memset: the call is graph-capturable.  in and out are device pointers to the packed
 * buffers; workspace holds mci_batch_sizes' ws_bytes.  Calls sharing one batch must not
 * overlap in time (the lanes are the batch's). */
mci_status mci_reconstruct_batch(mci_batch_t batch, const void* in, void* out, void* workspace, size_t ws_bytes,
                                 hipStream_t stream);

/* ----------------------------------------------------------------------------------- */
/* Off-grid evaluation (Theorem 3.3 holds at every real t; eq. DFTexpression with the    */
/* output operator of the closing paragraph of Section 3, at caller-given points).        */
/* The band coefficients are recovered as by mci_reconstruct_1d, divided by the Fourier    */
/* coefficients of a spreading kernel, transformed onto an oversampled grid (L = the power  */
/* of two at or above 4 K + 2, K = max |n| over the band, oversampling s = L / (2 K + 1)),  */
/* and every point sums the w grid values around it weighted by the kernel                  */
/* ES(x) = exp(beta (sqrt(1 - x^2) - 1)), beta = 0.97 pi w (1 - 1 / (2 s)): a type-2         */
/* nonuniform FFT.  Its relative error is 5 to 20 times exp(-pi w sqrt(1 - 1 / s)), on top  */
/* of the plan's rounding.                                                                  */
/* ----------------------------------------------------------------------------------- */
typedef struct mci_offgrid_s* mci_offgrid_t;

/* mci_offgrid_plan -- desc as for mci_plan, except that n_out is ignored and storage must
 * be MCI_STORE_NATIVE (MCI_E_UNSUPPORTED otherwise).  width: kernel width w in grid points,
 * 2..16, or 0 for the smallest w whose estimated error is below 4e-7 (FP32 plans) or
 * 1e-12 (FP64 plans).  Errors as mci_plan, plus MCI_E_INVALID_ARG for a width out of range
 * or a band longer than 2^26. */
mci_status mci_offgrid_plan(const mci_plan_desc* desc, int32_t width, int device, mci_offgrid_t* out);
mci_status mci_offgrid_destroy(mci_offgrid_t plan);
/* Grid length L, width w, beta, and the plan that reconstructs onto the grid (owned by the
 * off-grid plan; its variant may be changed or autotuned).  Any output pointer may be NULL. */
mci_status mci_offgrid_info(mci_offgrid_t plan, int64_t* grid_len, int32_t* width, double* beta,
                            mci_plan_t* grid_plan);
/* Device scratch for a batch of `batch` signals and n_t points: the grid ([batch][n_ops][L]
 * in plan precision, complex when not real_io), a table of n_t tap starts and w n_t weights,
 * and the grid plan's workspace. */
mci_status mci_offgrid_workspace_size(mci_offgrid_t plan, int64_t batch, int64_t n_t, size_t* bytes);
/* mci_evaluate_1d -- y[b][op][j] = (o_op f_b)(t_j) for every signal b.
 *   g : device, samples as for mci_reconstruct_1d.
 *   t : device FP64 points (radians, any real value; taken modulo 2 pi): [n_t] shared by
 *       every signal when t_shared != 0, else [batch][n_t].
 *   y : device, [batch][n_ops][n_t] (real_io) or [batch][n_ops][n_t][2], plan precision.
 * workspace: mci_offgrid_workspace_size(plan, batch, n_t) bytes.  batch = 0 or n_t = 0 is a
 * no-op.  Asynchronous on stream; no allocation. */
mci_status mci_evaluate_1d(mci_offgrid_t plan, const void* g, const double* t, int64_t n_t, int32_t t_shared,
                           void* y, int64_t batch, void* workspace, size_t ws_bytes, hipStream_t stream);

/* ----------------------------------------------------------------------------------- */
/* Averaged approximation error (Theorem 4.4, eq. averageerror) and the plan of least     */
/* error per signal.  For a signal with Fourier coefficients a(n) the error of the         */
/* approximation operator averaged over the sampling phase is                             */
/*   eps^2 = sum_{n outside the band} |a(n)|^2 (1 + sum_{l=1..M} |sum_m q_{m,l}(n) b_m(n)|^2) */
/* with q the inverse entries at the residue of n; the bracket is a weight of the plan     */
/* alone, so a batch of signals is scored against several plans in one pass.              */
/* ----------------------------------------------------------------------------------- */
#define MCI_MAX_ERROR_PLANS 16

/* Device bytes of the workspace: the weight table, (n_plans rounded up to a power of two)
 * x n_span values of the given precision, plus 256 bytes for per-plan constants. */
mci_status mci_averaged_error_workspace_size(int32_t n_plans, int64_t n_span, int32_t precision, size_t* bytes);

/* mci_averaged_error -- eps[s][c] = epsilon(f_s, plan c) for n_sig signals and n_plans plans.
 *   plans : host array of 1..16 1-D plans on one device.  Channels must be derivative or
 *           Hilbert multipliers (MCI_E_UNSUPPORTED for table channels, which give no b(n)
 *           outside the band); a plan with singular residues gives MCI_E_SINGULAR.  Only
 *           the channels, N and n1 of a plan matter (not n_out, the output operators or
 *           the precision of its transforms).
 *   a     : device, [n_sig][n_span] complex (re, im interleaved), float for MCI_F32 and
 *           double for MCI_F64: a[s][i] = a_s(n_lo + i); coefficients outside the span are 0.
 *   eps   : device, [n_sig][n_plans] double.  best: device [n_sig] int32, the index of the
 *           plan of least error (first on ties), or NULL.
 *   workspace : mci_averaged_error_workspace_size bytes.
 * Asynchronous on stream; no allocation. */
mci_status mci_averaged_error(const mci_plan_t* plans, int32_t n_plans, const void* a, int64_t n_lo, int64_t n_span,
                              int64_t n_sig, int32_t precision, double* eps, int32_t* best, void* workspace,
                              size_t ws_bytes, hipStream_t stream);

/* mci_averaged_error_noalloc -- mci_averaged_error for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments and results, without the workspace.  The weight table lives in a
 * static 4 MiB device array, one per GPU, whose address is looked up on the first call on
 * each device.  The call allocates nothing; it fails with MCI_E_INVALID_ARG when
 * mci_averaged_error_workspace_size(n_plans, n_span, precision) exceeds 4 MiB (for FP32,
 * n_span up to 65532 with 16 plans).  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (different streams, or host threads) race and give wrong results;
 * calls in one stream's order are safe.  Nothing in the array needs to start at zero. */
mci_status mci_averaged_error_noalloc(const mci_plan_t* plans, int32_t n_plans, const void* a, int64_t n_lo,
                                      int64_t n_span, int64_t n_sig, int32_t precision, double* eps, int32_t* best,
                                      hipStream_t stream);

/* mci_error_bound -- the bound of eq. errorestimate (Theorem 4.4 and the definition of
 * Omega_m after it) on eps, for the same arguments:
 *   bound[s][c]^2 = sum_{n outside the band} |a(n)|^2 (1 + M (sum_k Omega_k) sum_m |b_m(n)|^2),
 *   Omega_k = sup over the band of |r_k|^2 = max over residues and blocks of |q_{k,l}(n)|^2.
 * Cauchy-Schwarz on eq. averageerror gives this form, with Omega_k entering once; the
 * printed bound squares Omega_k, which its definition already makes a square, and read
 * literally that is no bound when Omega_k < 1.  bound: device [n_sig][n_plans] double.
 * Same plan restrictions, layout of a, workspace and errors as mci_averaged_error.
 * Asynchronous on stream; no allocation. */
mci_status mci_error_bound(const mci_plan_t* plans, int32_t n_plans, const void* a, int64_t n_lo, int64_t n_span,
                           int64_t n_sig, int32_t precision, double* bound, void* workspace, size_t ws_bytes,
                           hipStream_t stream);

/* mci_plan_omega -- Omega_1..Omega_M of a 1-D plan (the definition after Theorem 4.4),
 * computed on the host from the plan's FP64 inverse entries (synchronous).  omega: host
 * array of len >= M doubles.  MCI_E_SINGULAR for a plan with singular residues. */
mci_status mci_plan_omega(mci_plan_t plan, double* omega, int32_t len);

/* ----------------------------------------------------------------------------------- */
/* Learned residual refiner (not part of the paper; its closing remarks on Section 5.2   */
/* suggest MCI as the interpolation stage of learning-based super-resolution).          */
/* y = u + CNN(u), u the MCI upsample of an RGB image, CNN = conv3x3 3->32, ReLU,        */
/* conv3x3 32->32, ReLU, conv3x3 32->32, ReLU, conv3x3 32->3 (zero padding), BF16 MFMA    */
/* with FP32 accumulation, FP32 master weights and Adam state.  Images are FP32           */
/* [batch][3][h][w] device arrays; h and w are any positive sizes.                         */
/* Parameter vector (20259 FP32): W1[32][9][3], b1[32], W2[32][9][32], b2[32],            */
/* W3[32][9][32], b3[32], W4[3][9][32], b4[3]; W[co][tap][ci], tap = 3 dy + dx.            */
/* ----------------------------------------------------------------------------------- */
typedef struct mci_refiner_s* mci_refiner_t;

/* Create a refiner on `device` with seeded He-normal hidden weights and a near-zero last
 * layer (starts close to y = u).  Fallback bound tau = 0 until set. */
mci_status mci_refiner_create(int device, uint64_t seed, mci_refiner_t* out);
mci_status mci_refiner_destroy(mci_refiner_t r);
int64_t mci_refiner_num_params(void);
/* Copy the FP32 parameters (and the fallback bound) to / from host memory (checkpointing). */
mci_status mci_refiner_get_params(mci_refiner_t r, float* host_params, float* tau);
mci_status mci_refiner_set_params(mci_refiner_t r, const float* host_params, float tau);
/* Gradient of the last backward / train step, FP32 host copy in the parameter layout. */
mci_status mci_refiner_get_grads(mci_refiner_t r, float* host_grads);
/* Training checkpoints: the FP32 parameters, both Adam moments, the Adam step count and the
 * fallback bound, as one host byte buffer of mci_refiner_state_size() bytes (header
 * "MCIRFN01", n_params, step, tau, then parameters, first and second moments).  Loading it
 * into any refiner makes the next train steps continue bit for bit where the saved one
 * stopped (the training data order is the caller's).  Synchronous.  Errors:
 * MCI_E_INVALID_ARG (NULL, short buffer, not a checkpoint of this network), MCI_E_DEVICE. */
size_t mci_refiner_state_size(void);
mci_status mci_refiner_save_state(mci_refiner_t r, void* host, size_t len);
mci_status mci_refiner_load_state(mci_refiner_t r, const void* host, size_t len);
/* Device scratch for a batch of `batch` images of h x w (activations, gradients, partials). */
mci_status mci_refiner_workspace_size(int64_t batch, int h, int w, size_t* bytes);
/* y = u + CNN(u).  With ratio != NULL, ratio[b] = ||y_b - u_b|| / ||u_b|| (device, [batch]);
 * with apply_fallback, images whose ratio exceeds tau (or is NaN) are replaced by u and
 * used[b] (device int) records 1 for refined, 0 for fallback.  Layers 2 and 3 run as one
 * pass here (the layer-2 activations stay on chip), with results bit-identical to the
 * layer-by-layer forward that training runs; MCI_REFINER_LAYERED=1 in the environment selects
 * that layer-by-layer form instead. */
mci_status mci_refiner_forward(mci_refiner_t r, const float* u, float* y, int64_t batch, int h, int w,
                               int apply_fallback, float* ratio, int* used, void* workspace, size_t ws_bytes,
                               hipStream_t stream);
/* Gradient of the loss mean((u + CNN(u) - hr)^2) over all batch*3*h*w values.  loss_parts
 * (device, >= 1024 floats) receives per-block partial sums of the squared error, *n_parts
 * their count. */
mci_status mci_refiner_backward(mci_refiner_t r, const float* u, const float* hr, int64_t batch, int h, int w,
                                float* loss_parts, int* n_parts, void* workspace, size_t ws_bytes, hipStream_t stream);
/* backward, then one Adam step (beta 0.9 / 0.999, eps 1e-8) with learning rate lr. */
mci_status mci_refiner_train_step(mci_refiner_t r, const float* u, const float* hr, int64_t batch, int h, int w,
                                  float lr, float* loss_parts, int* n_parts, void* workspace, size_t ws_bytes,
                                  hipStream_t stream);
const char* mci_refiner_last_error(void);

/* mci_status_string -- static text for a status code. */
const char* mci_status_string(mci_status s);

/* mci_last_error -- text of the last error recorded by this thread (empty if none). */
const char* mci_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MCI_H */
