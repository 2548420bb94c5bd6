/*
 * mpgemm: Ozaki-scheme multi-component matrix multiplication on AMD MI355X
 * (gfx950).  C-ABI of libmpgemm.so.
 *
 * The operation (Utsugiri & Kouya, arXiv 2301.09960, Section 3, Algorithm 1):
 * given A (m x k) and B (k x n) whose entries are multi-component numbers
 * (the sum of c binary64 or binary32 components), compute C := A B in the
 * same format.  A and B are split error-free into D slices each, whose
 * pairwise products are exact in the slice arithmetic; the slice products
 * C_ab = A_a B_b with a + b <= D + 1 are formed on the matrix cores and added
 * error-free into the multi-component C.
 *
 * Formats (Section 1 and Section 4.4):
 *   DD  2 x binary64 (106 bits)     TD  3 x binary64 (159 bits)
 *   QD  4 x binary64 (212 bits)     TS  3 x binary32 (72 bits)
 *
 * Layout (all matrices): component-planar, column-major.  For A with leading
 * dimension lda >= max(1, m), component r of A(i, p) is A[r*lda*k + i + p*lda]
 * (plane r starts at A + r*lda*k).  B: component r of B(p, j) is
 * B[r*ldb*n + p + j*ldb], ldb >= max(1, k).  C: component r of C(i, j) is
 * C[r*ldc*n + i + j*ldc], ldc >= max(1, m).  Inputs are expected to be
 * normalized expansions (|x_{r+1}| <= ulp(x_r)/2), finite, with magnitudes in
 * [2^-400, 2^400] (binary64 formats) or [2^-16, 2^40] (TS) or zero, so that no
 * slice product underflows; outside that range the result may lose accuracy.
 *
 * Memory and streams: A, B and C are device pointers owned by the caller; A and
 * B are only read, C is overwritten (there is no alpha/beta scaling).  Every call
 * enqueues its work on `stream` and returns without synchronizing; the result
 * is valid once the stream has reached the call.  Temporary device memory is
 * taken from a workspace attached with mpgemm_set_workspace, or else allocated
 * stream-ordered on `stream` and released at the end of the call.
 *
 * Return codes: 0 on success; -i when the i-th argument is invalid (1-based,
 * as the BLAS xerbla convention: m < 0 gives -1, lda < max(1, m) gives -5, a
 * NULL matrix pointer with a non-empty extent gives its position); a positive
 * MPGEMM_ERR_* code on a runtime failure.  m == 0 or n == 0 returns 0 without
 * work; k == 0 sets C to zero.  Calls are safe from several host threads on
 * different streams; options set with mpgemm_set_* are per host thread.
 */
#ifndef MPGEMM_H
#define MPGEMM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Formats. */
#define MPGEMM_DD 0
#define MPGEMM_TD 1
#define MPGEMM_QD 2
#define MPGEMM_TS 3

/* Slice forms.  FLOAT: binary64 slices on FP64 matrix cores (binary32 slices
 * on FP32 matrix cores for TS), Algorithm 1 as written.  INT8: signed 7-bit
 * digit slices on INT8 matrix cores with exact 32-bit integer sums (DD, TD, QD
 * only); more slices, each product far cheaper.  Digit s (s = 1..D) of an
 * element of a row of A (column of B) is the extraction step of Algorithm 1 on
 * the fixed grid u_s = 2^(E - 6 - 7 (s - 1)), E = 1 + the largest ilogb of the
 * row's (column's) leading components, applied to the exact value of the
 * element: d_s = RN(x / u_s) - 128 RN(x / u_(s-1)) (nearest, ties to even;
 * RN(x / u_0) taken as 0), so |d_s| <= 64 and the digits through s sum to x
 * rounded to the grid u_s. */
#define MPGEMM_MODE_FLOAT 0
#define MPGEMM_MODE_INT8 1

/* Runtime failures (positive return codes). */
#define MPGEMM_ERR_HIP 1         /* a HIP runtime call failed */
#define MPGEMM_ERR_WORKSPACE 2   /* attached workspace too small, or allocation failed */
#define MPGEMM_ERR_DEVICE 3      /* current device is not gfx950 */
#define MPGEMM_ERR_UNSUPPORTED 4 /* option not available for this format */
#define MPGEMM_ERR_TOO_LARGE 5   /* size beyond the library's limits (see below) */

/* Limits: m, n, k <= 2^20 (so every packed index fits 64 bits and every slice
 * product sum fits its accumulator); 1 <= D <= 16 (FLOAT) or 1 <= D <= 40 (INT8). */

/*
 * C := A B in DD / TD / QD (Section 3, Algorithm 1; the product set is the
 * triangle a + b <= D + 1 and every slice product is exact).  Arguments as in
 * the layout paragraph above.  Target: |C - A B| <= 2^-t (|A||B|) elementwise,
 * t = 100 (DD), 150 (TD), 200 (QD).  The automatic D meets it when the largest
 * entry of each row of A (column of B) is not far above the entries that
 * carry (|A||B|)_ij: tested on exponents spread uniformly over up to 60 bits.
 * It is an estimate, not a guarantee: a row whose grid is set by one entry
 * 2^40 above the rest needs more slices.  For any input in range, choose the
 * slices from the data (MPGEMM_SLICES_DATA below), which meets the target by
 * construction (up to 16 slices, enough for about 16 b - t bits of such
 * excess with b-bit slices), or check a product with mpgemm_certify.
 */
int mpgemm_dd(int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *C, int ldc,
              hipStream_t stream);
int mpgemm_td(int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *C, int ldc,
              hipStream_t stream);
int mpgemm_qd(int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *C, int ldc,
              hipStream_t stream);

/*
 * C := A B in TS, triple binary32 (Section 4.4: the paper's GPU format, with
 * binary32 slices, S = 24).  Bound t = 66 with the automatic D.  FLOAT mode only.
 */
int mpgemm_ts(int m, int n, int k, const float *A, int lda, const float *B, int ldb, float *C, int ldc,
              hipStream_t stream);

/*
 * D+S: a binary64 leading part and a binary32 trailing part per element (the
 * format of Section 4.4's GPU comparison; about 77 bits), stored as two
 * planes: hi (binary64) and lo (binary32), each column-major with the same
 * leading dimension (A: m x k with lda >= max(1, m), B: k x n with ldb >=
 * max(1, k), C: m x n with ldc >= max(1, m)); |lo| <= ulp(hi) / 2.
 *
 * mpgemm_ds: C := A B through the DD Ozaki product (Section 3, Algorithm 1):
 * each input read as the DD number (hi, lo) (exact), the DD product in the
 * thread's DD slice form and slice count, and C rounded to D+S (hi = RN of
 * the DD result, lo = its second part rounded to binary32), so that
 * |C - AB| <= 2^-76 (|A||B|) elementwise where the DD product meets its bound.
 * Takes workspace for the DD copies of A, B and C besides the DD product's.
 * Argument codes: -1 .. -12 for m, n, k, Ahi, Alo, lda, Bhi, Blo, ldb, Chi,
 * Clo, ldc; positive codes as above.
 */
int mpgemm_ds(int m, int n, int k, const double *Ahi, const float *Alo, int lda, const double *Bhi, const float *Blo,
              int ldb, double *Chi, float *Clo, int ldc, hipStream_t stream);

/*
 * The simple matrix multiplication that Section 4.4 compares with the Ozaki
 * scheme on the GPU: C := A B by the triple loop in the format's own
 * arithmetic (no splitting), every term a_ip b_pj multiplied and added in
 * order p = 0 .. k - 1.  DD: the classical double-double operations (TwoProd
 * with an FMA, the cross terms, TwoSum of both parts, two renormalizations);
 * TD, QD, TS: each term's exact and truncated partial products gathered with
 * the accumulator, sorted by magnitude and renormalized to c components.
 * D+S: DD arithmetic on the exact DD reading of the inputs, C rounded to D+S
 * once.  The error grows with k: about k 2^-(L - 3) (|A||B|) for L = 106, 159,
 * 212, 72 (DD, TD, QD, TS) bits (D+S: that of DD plus 2^-76 (|A||B|)).
 * staging 0: each thread reads its operands from global memory; 1: 64 x 16
 * operand panels pass through LDS (the paper's comparison with and without
 * shared memory); both give the same C bit for bit.  Layout and return codes
 * as mpgemm_<fmt> with the arguments shifted: -1 for fmt, -2 for staging,
 * then -(i + 2) for argument i of the DD signature (mpgemm_ds_simple: -1 for
 * staging, then -(i + 1) for argument i of mpgemm_ds).
 */
int mpgemm_simple(int fmt, int staging, int m, int n, int k, const void *A, int lda, const void *B, int ldb, void *C,
                  int ldc, hipStream_t stream);
int mpgemm_ds_simple(int staging, int m, int n, int k, const double *Ahi, const float *Alo, int lda,
                     const double *Bhi, const float *Blo, int ldb, double *Chi, float *Clo, int ldc,
                     hipStream_t stream);

/*
 * Batched products: C_i := A_i B_i for i < count, independent products of
 * uneven sizes, each computed exactly as the single call computes it (the same
 * per-tile kernel code, so the results are identical bit for bit).  All
 * arguments after `count` are host arrays of count entries holding what the
 * single call takes (device matrix pointers, sizes, leading dimensions).
 * The split of all operands and one persistent slice-product kernel that takes
 * (product, tile) work items, longest first from one list per XCD, run as one
 * launch sequence.  That
 * sequence is captured once per batch shape (format, count, every m, n, k and
 * slice count, device and stream) into a HIP graph and cached per host thread
 * (up to 6 shapes; releasing the least recently used one synchronizes the
 * device); later calls with the same shape replay it after one copy of this
 * call's pointers.  The cached workspace of a shape stays allocated until it
 * is released or mpgemm_batched_cache_clear is called.  Batched calls of one
 * shape on one stream must not be issued from two host threads at once.
 * Both slice forms (the thread's mode for the format).  In the INT8 form each
 * product takes the tile configuration a single call would (two persistent
 * launches, 128 x 128 and 256 x 256 tiles), its diagonals spread over several
 * work items.
 * Return codes: -1 for count < 0; -i (i = 2..10) for a NULL array or an
 * invalid entry of argument i (first failing product); positive codes as above.
 */
int mpgemm_dd_batched(int count, const int *m, const int *n, const int *k, const double *const *A, const int *lda,
                      const double *const *B, const int *ldb, double *const *C, const int *ldc, hipStream_t stream);
int mpgemm_td_batched(int count, const int *m, const int *n, const int *k, const double *const *A, const int *lda,
                      const double *const *B, const int *ldb, double *const *C, const int *ldc, hipStream_t stream);
int mpgemm_qd_batched(int count, const int *m, const int *n, const int *k, const double *const *A, const int *lda,
                      const double *const *B, const int *ldb, double *const *C, const int *ldc, hipStream_t stream);
int mpgemm_ts_batched(int count, const int *m, const int *n, const int *k, const float *const *A, const int *lda,
                      const float *const *B, const int *ldb, float *const *C, const int *ldc, hipStream_t stream);

/* Releases this host thread's cached batch plans (synchronizes the device). */
int mpgemm_batched_cache_clear(void);

/*
 * Options, per host thread and per format (fmt = MPGEMM_DD .. MPGEMM_TS).
 * mpgemm_set_mode selects the slice form (returns MPGEMM_ERR_UNSUPPORTED for
 * INT8 with TS).  mpgemm_set_num_slices sets D for (fmt, mode); 0 restores the
 * automatic choice (Section 3 ties the attainable accuracy to the number of
 * divisions; the automatic D is the smallest that met the bound above with
 * guard bits on the tested inputs, see mpgemm_dd).  mpgemm_num_slices returns
 * the D a call with inner dimension k would use.  mpgemm_last_num_slices
 * returns the D used by this thread's last call.
 *
 * D = MPGEMM_SLICES_DATA (binary64/binary32 slices only; INT8 returns
 * MPGEMM_ERR_UNSUPPORTED): the slice products are chosen from the data, as
 * Section 3 says the number of divisions must be found by running the
 * calculation and that more of the low-order products can be dropped.  The
 * split makes 16 slices; the certificate's quantities (see mpgemm_certify:
 * the slice exponents, the remainders, the row and column sums of |A_0| and
 * |B_0| and the product |A_0| |B_0|) are formed before the slice products;
 * then each 64 x 64 tile of C forms only the pairs (a, b) whose slices are
 * large enough to matter: those with the largest bounds k 2^(e_a + e_b),
 * taken until the bounds of all pairs left out, with the remainder and
 * rounding terms, fit 2^-t times the tile's smallest lower bound of |A||B|
 * (exponents relative to each row's and column's first slice, so the rows'
 * and columns' scales do not matter).  Every entry then meets the target,
 * and mpgemm_certify in this mode returns the certificate of the same C.
 * Zero slices, zero rows and tiles with |A||B| = 0 take no pairs.  Applies to
 * mpgemm_dd/td/qd/ts and mpgemm_certify; the batched, allocation-free, D+S
 * and LU calls use the automatic D.  Workspace: mpgemm_workspace_bytes with
 * D = MPGEMM_SLICES_DATA (or 0 while the thread is in this mode).  Stage
 * timing records the split with the pair selection as the split stage.
 */
#define MPGEMM_SLICES_DATA (-1)
/*
 * Environment defaults, read once per process when a host thread first uses
 * the library: MPGEMM_MODE=int8 starts every thread with the INT8 form for
 * DD, TD and QD (TS stays FLOAT); MPGEMM_SLICES=N starts it with D = N for
 * every format and form whose range holds N, and MPGEMM_SLICES=data with the
 * data-chosen pairs of the FLOAT form.  Other values are ignored.  The
 * per-thread setters override them.  (MPGEMM_TUNE_FILE: see below.)
 */
int mpgemm_set_mode(int fmt, int mode);
int mpgemm_get_mode(int fmt);

/*
 * Wavefront layout of the FLOAT-form slice-product kernel (64 x 64 tile of C
 * per workgroup): 1 = 4 wavefronts of 32 x 32, 2 = 8 of 32 x 16, 3 = 16 of
 * 16 x 16; 0 restores the tuned default.  Per host thread;
 * mpgemm_tile_layout returns the layout a call would use.
 *
 * Tuned tables (process-wide).  The default layouts and the automatic slice
 * counts are compiled in; a tuning file replaces them, read at first use from
 * the path in the environment variable MPGEMM_TUNE_FILE, or loaded with
 * mpgemm_load_tune_file (NULL restores the compiled-in tables).  Lines:
 *   "<fmt> <layout>"                  fmt one of dd, td, qd, ts
 *   "slices <fmt> <mode> <kmax> <D>"  mode float or int8: D slices for
 *                                     k <= kmax (the smallest kmax covering
 *                                     k applies; beyond them, the formula)
 * as written by the autotuner (python -m paper_2301_09960_amd.tune).
 * Returns 0, -1 if the file cannot be read, -2 for a line it does not accept
 * (tables unchanged).  Per-thread settings (mpgemm_set_tile_layout,
 * mpgemm_set_num_slices) take precedence.  Do not load while other threads
 * are inside a call.
 */
int mpgemm_set_tile_layout(int fmt, int layout);
int mpgemm_tile_layout(int fmt);
int mpgemm_load_tune_file(const char *path);

/*
 * Tile configuration of the INT8-form kernel, per host thread: 0 automatic
 * (256 x 256 tiles with 8 wavefronts unless padding to them more than doubles
 * the area padded to 128 x 128, else 128 x 128), 1 = 128 x 128 with 4
 * wavefronts, 2 = 256 x 256 with 4, 3 = 256 x 256 with 8, 4 = 256 x 256 with
 * 16.  Slices are padded to the chosen tile.  Returns -1 for other values.
 */
int mpgemm_set_int8_tile(int cfg);

/*
 * Kernel of the binary64/binary32 split (Algorithm 1), per host thread.
 * 0 (default): while the padded k of a product is short enough that a
 * workgroup holds two or more whole rows of A (columns of B) in registers
 * (k <= 8192 for DD, 5120 for TD, 4096 for QD, 8192 for TS), one fused launch
 * runs all D passes and reads each operand once; longer products use one
 * launch per pass.  1: one launch per pass always.  Both give the same slices
 * bit for bit.  Returns -1 for other values.
 */
int mpgemm_set_split_kernel(int kind);
int mpgemm_split_kernel(void);

/*
 * Last slice of the binary64/binary32 split (Algorithm 1, Section 3), per host
 * thread.  0 (default): all D slices are extracted on the grid of tau and the
 * remainder is dropped, so every slice product is exact in the slice format.
 * 1: the last slice is the leading component of the residual left by the first
 * D - 1 passes, as Algorithm 1 is printed; the products of that full-width
 * slice are then rounded by the matrix cores.  For comparison of the two
 * readings; the INT8 form ignores it.  Returns -1 for other values.
 */
int mpgemm_set_last_slice(int kind);
int mpgemm_last_slice(void);
int mpgemm_set_num_slices(int fmt, int mode, int D);
int mpgemm_num_slices(int fmt, int mode, int k);
int mpgemm_last_num_slices(void);

/*
 * Workspace.  mpgemm_workspace_bytes gives the device bytes a call of this
 * shape needs (D = 0: automatic).  mpgemm_set_workspace attaches caller-owned
 * device memory (at least 256-byte aligned) for this host thread's later calls;
 * NULL detaches it.  A call that finds the attached workspace too small returns
 * MPGEMM_ERR_WORKSPACE without enqueuing work.  Work on different streams must
 * not share one attached workspace concurrently.  Without one, each call takes
 * its workspace from the device's stream-ordered pool (hipMallocAsync, kept
 * allocated after release); callers that keep several streams busy at once
 * should attach one workspace per stream instead, since growing the pool under
 * such load has stalled the calling thread for up to seconds.
 */
size_t mpgemm_workspace_bytes(int fmt, int mode, int m, int n, int k, int D);
int mpgemm_set_workspace(void *dev_ptr, size_t bytes);

/*
 * C = AB with an a-posteriori certificate.  Computes C exactly as mpgemm_<fmt>
 * does, in the thread's slice form and with its slice count, then bounds its
 * error from the same split (Algorithm 1, Section 3; in the INT8 form digit
 * plane s is the slice, at most 2^(E - 7 (s - 1)), the remainder at most
 * 2^(E - 7 D)):
 * with A = A_s + RA (slices plus the remainder after D passes) and likewise B,
 * AB - C = (the pairs a + b > D + 1 that are not formed) + A_s RB + RA B + (the
 * rounding of the sum to c components).  Each part is bounded per entry from
 * the slice exponents, the remainder bound of the last pass, the row sums of
 * |A| and column sums of |B|, and one extra binary64 product |A_0||B_0| of the
 * leading components, which also gives a lower bound of (|A||B|)_ij.
 *
 * cert (device, 2 m n doubles): plane 0 (m x n, column-major, leading
 * dimension m) receives beta_ij >= |C_ij - (AB)_ij|, plane 1 lambda_ij <=
 * (|A||B|)_ij.  *worst (device, one double) receives the largest beta / lambda
 * (0 when every beta is 0; +inf where lambda is 0 and beta is not, e.g. a row
 * and a column with disjoint supports).  The result meets 2^-t (|A||B|) in every
 * entry if worst <= 2^-t (t = 100 / 150 / 200 / 66 for DD / TD / QD / TS).
 * Assumes |A||B| and the bounds stay in the normal binary64 range.
 *
 * Returns MPGEMM_ERR_UNSUPPORTED with the printed last slice
 * (mpgemm_set_last_slice(1)), for TS with D = 1, and in the INT8 form with
 * fewer than about 8 digits (their planes hold |A_0| and |B_0|).  Argument codes as for
 * mpgemm_<fmt>, shifted by one (fmt is argument 1); -11 / -12 for a NULL cert
 * (with m, n > 0) / worst.  Enqueued on `stream` like the other calls.
 */
int mpgemm_certify(int fmt, int m, int n, int k, const void *A, int lda, const void *B, int ldb, void *C, int ldc,
                   double *cert, double *worst, hipStream_t stream);

/*
 * mpgemm_certify with the slice count chosen from the data (the paper leaves the
 * number of splits to be found by running the calculation, Section 3): runs
 * the certified product at D = d_first, d_first + 1, ..., d_last in the
 * thread's slice form and stops at the first D whose worst ratio is at most
 * 2^-t (t as above).  C, cert and *worst hold that attempt's results, and
 * *d_used (host) its D; if no D up to d_last is certified they hold the
 * d_last attempt's, and the caller sees it in *worst.  A D the certificate does
 * not support is skipped (MPGEMM_ERR_UNSUPPORTED if none was).  Synchronizes
 * `stream` after each attempt to read *worst back, so it cannot be captured
 * in a graph.  The thread's slice-count option is not changed.  Argument codes
 * as for mpgemm_certify; -13 for d_first outside [1, the form's maximum D],
 * -14 for d_last outside [d_first, that maximum], -15 for a NULL d_used.
 */
int mpgemm_certify_adaptive(int fmt, int m, int n, int k, const void *A, int lda, const void *B, int ldb, void *C,
                            int ldc, double *cert, double *worst, int d_first, int d_last, int *d_used,
                            hipStream_t stream);

/*
 * LU factorization of a DD (TD) matrix with the Schur updates done by this
 * library's DD (TD) product (Section 4.6).  A (device; two (three) planes of
 * components, each n x n column-major with leading dimension lda, lda * n
 * doubles apart) is overwritten by L (unit lower, diagonal not stored) and U.
 * Block width K (the paper's MIN_DIM): the K x K diagonal block is factored in
 * DD (TD) arithmetic, the panels U12 = L11^-1 A12 and L21 = A21 U11^-1 are
 * solved in it, and A22 -= L21 U12 goes through mpgemm_dd (mpgemm_td) in the
 * thread's slice form and slice count (for k = K).  No pivoting, as in the paper: a
 * zero pivot gives infinities or NaNs.  Allocates its panel and product
 * buffers on the stream (and the GEMM's workspace, unless one is attached).
 *
 * mpgemm_dd_lu_solve (mpgemm_td_lu_solve): solves L U x = b with the factors
 * in LU; x (device, two (three) planes of n doubles) holds b on entry and x on
 * return.  Forward and backward
 * substitution in DD, each inner product summed in a fixed order.
 * Argument codes: -i for argument i (n < 0, NULL pointers, lda < max(1, n),
 * K < 1).
 */
int mpgemm_dd_lu(int n, double *A, int lda, int K, hipStream_t stream);
int mpgemm_dd_lu_solve(int n, const double *LU, int lda, double *x, hipStream_t stream);
int mpgemm_td_lu(int n, double *A, int lda, int K, hipStream_t stream);
int mpgemm_td_lu_solve(int n, const double *LU, int lda, double *x, hipStream_t stream);

/*
 * Parity hooks (used by the tests to compare intermediate results bit for bit).
 *
 * mpgemm_debug_split: split one operand as the GEMM does.  operand 0: the rows
 * of A (rows = m, cols = k, X is A with ldx = lda); operand 1: the columns of B
 * (rows = k, cols = n, X is B with ldx = ldb).  Writes D slices as planes of
 * rows x cols, column-major with leading dimension `rows`, into `slices`
 * (binary64 for DD/TD/QD, binary32 for TS, int8 for INT8 mode), and exponents
 * into `exps`: FLOAT mode: D x nvec int32, exps[a*nvec + v] = ceil(log2 mu_a)
 * of vector v in pass a (INT32_MIN when mu_a = 0), nvec = rows for operand 0,
 * cols for operand 1; INT8 mode: nvec int32, E_v = 1 + max ilogb of the
 * leading components (INT32_MIN for an all-zero vector).
 *
 * mpgemm_debug_products: FLOAT mode: the exact slice product C_ab (Section 3)
 * for 1-based a, b, as an m x n column-major binary64 matrix (ldo >= m; for TS
 * the values are binary32 products held in binary64).  INT8 mode: the exact
 * integer diagonal sum S_g = sum over s + t = g + 1 of A_s B_t for g = a
 * (b ignored), as int64 in `out` reinterpreted.  All pointers are device
 * pointers; D = 0 takes the automatic value.
 */
int mpgemm_debug_split(int fmt, int mode, int operand, int rows, int cols, const void *X, int ldx, int D,
                       void *slices, int *exps, hipStream_t stream);
/*
 * mpgemm_debug_pair_sets: the pair sets the data-chosen slice mode
 * (MPGEMM_SLICES_DATA) takes for C = AB: for tile (tm, tn) of 64 x 64 entries
 * (tiles_m = ceil(m / 64), tiles_n = ceil(n / 64)), 16 bytes at
 * sets + (tn * tiles_m + tm) * 16, byte a (0-based slice of A) holding how many
 * slices of B (0-based b < count) pair with it.  Device pointer sets.  Codes:
 * -1 fmt, then the DD signature's codes shifted by one, -10 for a NULL sets.
 */
int mpgemm_debug_pair_sets(int fmt, int m, int n, int k, const void *A, int lda, const void *B, int ldb,
                           int8_t *sets, hipStream_t stream);
int mpgemm_debug_products(int fmt, int mode, int m, int n, int k, const void *A, int lda, const void *B, int ldb,
                          int D, int a, int b, void *out, int ldo, hipStream_t stream);

/*
 * Stage timing (the split / multiply-and-accumulate shares that Section 4.1
 * profiles).  mpgemm_profile_enable(1) makes this host thread's later calls
 * record HIP events on their stream before the split, between split and GEMM,
 * and after the fused GEMM kernel.  mpgemm_profile_read waits for the recorded
 * events of up to max_calls calls, oldest first, writes each call's split and
 * GEMM milliseconds into split_ms[i] and gemm_ms[i] (host arrays of max_calls
 * entries), drops those calls from the log and returns how many it wrote, or
 * -MPGEMM_ERR_HIP on a HIP failure.
 */
int mpgemm_profile_enable(int on);
int mpgemm_profile_read(double *split_ms, double *gemm_ms, int max_calls);

/*
 * Longer binary64 expansions (the paper's arbitrary-precision section
 * multiplies 212- to 742-bit numbers in 53-bit steps): A, B and C hold
 * c = 2 .. 14 binary64 components per element, planes as for DD/TD/QD
 * (normalized expansions, each component below half an ulp of the one above).
 * The product uses the INT8-slice form with D digit slices (D = 0: automatic,
 * mpgemm_nd_num_slices), targeting |C - AB| <= 2^-(50 c) (|A||B|) elementwise
 * (c = 2, 3, 4 give the DD, TD and QD bounds); the automatic D met it on the
 * tested inputs (exponents spread up to 16 bits), with the same caveat as
 * mpgemm_dd for rows or columns dominated by one entry: mpgemm_nd_certify
 * checks a product.  At most 112
 * digits.  Return codes: -1 bad c, -2 bad D, then -(i + 2) for argument i of
 * the DD signature; positive codes as above.  Workspace as for the other
 * calls (mpgemm_nd_workspace_bytes; 0 for an invalid or empty shape).
 * mpgemm_nd_debug_split writes the D digit planes (int8, rows x cols,
 * column-major) and the per-row (operand 0) or per-column (operand 1)
 * exponents E of one operand; mpgemm_nd_debug_products writes the diagonal sum
 * S_g (1 <= g <= D) as int64 (m x n, leading dimension ldo).  Both return 0 or
 * a code as above (-1 bad c; then the positions of their own arguments).
 */
int mpgemm_nd(int c, int D, int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *C,
              int ldc, hipStream_t stream);
int mpgemm_nd_num_slices(int c, int k);
size_t mpgemm_nd_workspace_bytes(int c, int D, int m, int n, int k);
/*
 * mpgemm_nd_certify: mpgemm_nd with the a-posteriori certificate of
 * mpgemm_certify (INT8 form, c components; the target is 2^-(50 c)).  Codes as
 * for mpgemm_nd; -12 / -13 for a NULL cert (with m, n > 0) / worst.
 */
int mpgemm_nd_certify(int c, int D, int m, int n, int k, const double *A, int lda, const double *B, int ldb,
                      double *C, int ldc, double *cert, double *worst, hipStream_t stream);
int mpgemm_nd_debug_split(int c, int operand, int rows, int cols, const double *X, int ldx, int D, int8_t *digits,
                          int *exps, hipStream_t stream);
int mpgemm_nd_debug_products(int c, int m, int n, int k, const double *A, int lda, const double *B, int ldb, int D,
                             int g, int64_t *out, int ldo, hipStream_t stream);

/*
 * mpgemm_dd without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same product as mpgemm_dd (the thread's slice form
 * and slice count, the same kernels, the same C bit for bit), with its
 * workspace in a fixed device array of MPGEMM_NOALLOC_SCRATCH_BYTES that the
 * library holds on each device it runs on until the process ends.  A shape
 * whose workspace (mpgemm_workspace_bytes(MPGEMM_DD, mode, m, n, k, 0)) exceeds
 * it returns MPGEMM_ERR_TOO_LARGE without enqueuing work (for example
 * m = n = k = 1024 needs 128 MiB with binary64 slices).  Every call on a device
 * shares that device's array: calls that overlap on one device (on different
 * streams, or from different threads) race and must be serialized by the
 * caller; calls queued on one stream are ordered and safe.  The first call on
 * each device looks up the array's address (hipGetSymbolAddress) and keeps it.
 * Argument codes as mpgemm_dd.
 */
#define MPGEMM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int mpgemm_dd_noalloc(int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                      hipStream_t stream);

/* Text for a return code. */
const char *mpgemm_status_string(int status);

/* 0 if the current device is a gfx950, else MPGEMM_ERR_DEVICE (or MPGEMM_ERR_HIP). */
int mpgemm_check_device(void);

#ifdef __cplusplus
}
#endif

#endif /* MPGEMM_H */
