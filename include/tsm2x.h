/*
 * tsm2x.h -- C ABI of the MI355X (gfx950) tall-and-skinny matrix-multiply
 * library.  It implements the two problem classes of TSM2X (Rivera, Chen,
 * Xiong, Zhang, Song, Tao, "TSM2X: High-Performance Tall-and-Skinny
 * Matrix-Matrix Multiplication on GPUs"):
 *
 *   TSM2R  C = A*B, A a large regular m-by-k matrix, B a skinny k-by-n
 *          matrix, n <= 32 (Design of TSM2R, Algorithms 2-4).
 *   TSM2L  C = A*B, A a tall-and-skinny m-by-k matrix with k <= 32, B a
 *          small k-by-n matrix, n <= 32 (Design of TSM2L, Algorithm 6).
 *
 * plus the two products of the backward pass of C = A*B (for a scalar loss
 * with upstream gradient dC): dA = dC*B^T and dB = A^T*dC, and the hi+lo
 * low-precision storage form of A.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrices are column-major ("by convention", Design of TSM2R, Efficient
 *    Off-Chip Memory Access): element (i,j) of X with leading dimension ldX
 *    is X[i + j*ldX].  The _ex forms also take A and/or B given as their
 *    transposes (equivalently, row-major A or B).
 *  - All matrix pointers are DEVICE pointers owned by the caller; the library
 *    never frees or retains them.  `stream` is a hipStream_t (NULL = the
 *    null stream).  Every call is asynchronous on `stream`; a return value of
 *    0 means the work was enqueued.
 *  - The output is overwritten, never read (C := A*B), except in the _ex and
 *    gemm forms with beta != 0 (C := beta*C + A*B, the accumulating form of
 *    the paper's algorithms, which load C before adding to it).
 *  - m == 0 or n == 0 (or, for the gradients, an empty output) is a no-op.
 *    k == 0 writes zeros (beta*C in the _ex forms).
 *  - Results are deterministic: a repeated call on the same inputs gives the
 *    same bits (fixed reduction orders, no floating-point atomics).
 *  - Arguments are checked on the host before any HIP call.  An invalid
 *    argument returns -i, i being its 1-based position (LAPACK style).
 *    Positive codes are TSM_ERR_*; tsm2x_error_string() describes them.
 *
 * Workspace
 * ---------
 *  Kernels that split a reduction across workgroups write double-precision
 *  partial sums to a workspace of tsm2x_workspace_size() bytes and add them
 *  in a second, ordered pass.  tsm2r_ex and tsm_grad_b take the workspace
 *  from the caller when ws != NULL: device memory, 256-byte aligned, any
 *  contents.  Otherwise the library uses a grow-only per-device buffer it
 *  owns (allocated with hipMalloc on first need, released by
 *  tsm2x_finalize).  Two calls that share one workspace must not run
 *  concurrently (e.g. on two streams).
 */
#ifndef TSM2X_H
#define TSM2X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage types.
 *   TSM_F64        A, B, C double.
 *   TSM_F32        A, B, C float.
 *   TSM_BF16 / TSM_F16
 *                  A is one plane of bfloat16 / binary16 values (the "hi"
 *                  plane of tsm2x_split); B and C are float.
 *   TSM_BF16_SPLIT / TSM_F16_SPLIT
 *                  A is two planes, hi then lo, each lda*k elements, the lo
 *                  plane starting at element lda*k after the hi plane.  The
 *                  represented value is hi + lo.  B and C are float.        */
typedef enum {
    TSM_F64 = 0,
    TSM_F32 = 1,
    TSM_BF16 = 2,
    TSM_F16 = 3,
    TSM_BF16_SPLIT = 4,
    TSM_F16_SPLIT = 5
} tsm_dtype;

/* Operations, for tsm2x_workspace_size. */
typedef enum {
    TSM_OP_TSM2R = 0,
    TSM_OP_TSM2L = 1,
    TSM_OP_GRAD_A = 2,
    TSM_OP_GRAD_B = 3,
    TSM_OP_TSM2R_ROWMAJOR = 4,
    TSM_OP_KMEANS = 5
} tsm_op;

enum {
    TSM_SUCCESS = 0,
    TSM_ERR_UNSUPPORTED = 1, /* valid arguments outside the supported shapes/types */
    TSM_ERR_HIP = 2,         /* a HIP call failed; see tsm2x_last_hip_error()   */
    TSM_ERR_WORKSPACE = 3,   /* caller workspace too small or misaligned         */
    TSM_ERR_ALLOC = 4        /* the library's workspace could not be allocated   */
};

/* TSM2R: C = A*B, A m-by-k (lda >= max(1,m)), B k-by-n (ldb >= max(1,k)),
 * C m-by-n (ldc >= max(1,m)).  A is streamed from memory once (outer-product
 * form of Algorithm 2 with the on-chip B tile of Algorithms 3-4); the k range
 * is split across wavefronts and workgroups and the partial sums are added in
 * double precision in a fixed order.  n > 32 runs in panels of 32 columns of
 * B and C (A read once per panel, as the paper's t2 < n).
 * dtype: any tsm_dtype.  Errors: -1..-11 for arguments 1..11. */
int tsm2r(int64_t m, int64_t k, int64_t n, const void* A, int64_t lda,
          const void* B, int64_t ldb, void* C, int64_t ldc, int dtype,
          void* stream);

/* TSM2L: C = A*B, A m-by-k with k <= 32, B k-by-n (Algorithm 6: horizontal
 * tiles of A processed by a persistent grid; B is held on chip whole, so C
 * is written exactly once and never re-read).  k > 32 is computed by the
 * TSM2R kernels (correct for any shape; TSM2L's kernels need B on chip);
 * n > 32 in panels of 32 columns.
 * dtype: any tsm_dtype (16-bit forms of A as in tsm2r, B and C float).
 * Errors as tsm2r. */
int tsm2l(int64_t m, int64_t k, int64_t n, const void* A, int64_t lda,
          const void* B, int64_t ldb, void* C, int64_t ldc, int dtype,
          void* stream);

/* Extended forms: C := beta*C + op(A)*op(B), with a caller workspace.
 *   transA  0: A is m-by-k (lda >= max(1,m));
 *           1: A is given as its transpose, a k-by-m matrix (lda >=
 *              max(1,k)), i.e. A stored row-major.  The 16-bit forms of A
 *              (planes written by tsm2x_split) must have transA = 0.
 *   transB  0: B is k-by-n (ldb >= max(1,k));
 *           1: B is given as its transpose, n-by-k (ldb >= max(1,n)).  The
 *              TSM2R kernels first copy B into the workspace column-major.
 *   beta    C is read only when beta != 0.  Where the kernel finishes in
 *           double (TSM2R, transA = 1) beta*C is added in double and the
 *           sum rounded once; the TSM2L kernels add it in C's type.
 *   ws      device workspace, 256-byte aligned, at least
 *           tsm2x_workspace_size(op, m, k, n, dtype) bytes (op TSM_OP_TSM2R,
 *           TSM_OP_TSM2R_ROWMAJOR for transA = 1, TSM_OP_TSM2L), any
 *           contents; NULL: the library's own (see "Workspace").
 * tsm2r_ex uses the TSM2R kernels (transA = 1: the reduction along the
 * contiguous dimension, the tn kernel), tsm2l_ex the TSM2L kernels where
 * they apply (transA = 0, k <= 32) and the TSM2R ones otherwise.
 * Arguments: 1 transA, 2 transB, 3 m, 4 k, 5 n, 6 A, 7 lda, 8 B, 9 ldb,
 * 10 beta, 11 C, 12 ldc, 13 dtype, 14 ws, 15 ws_bytes, 16 stream.
 * Errors: -i for argument i; TSM_ERR_UNSUPPORTED for transA = 1 with a
 * 16-bit form; TSM_ERR_WORKSPACE if ws is too small or misaligned. */
int tsm2r_ex(int transA, int transB, int64_t m, int64_t k, int64_t n,
             const void* A, int64_t lda, const void* B, int64_t ldb,
             double beta, void* C, int64_t ldc, int dtype, void* ws,
             size_t ws_bytes, void* stream);
int tsm2l_ex(int transA, int transB, int64_t m, int64_t k, int64_t n,
             const void* A, int64_t lda, const void* B, int64_t ldb,
             double beta, void* C, int64_t ldc, int dtype, void* ws,
             size_t ws_bytes, void* stream);

/* The same contract, choosing by the paper's two shape classes (Design of
 * TSM2R / Design of TSM2L): TSM2L for a column-major A with k <= 32, TSM2R
 * otherwise.  Workspace: tsm2x_workspace_size(TSM_OP_TSM2R or
 * TSM_OP_TSM2R_ROWMAJOR, ...) covers every case. */
int tsm2x_gemm(int transA, int transB, int64_t m, int64_t k, int64_t n,
               const void* A, int64_t lda, const void* B, int64_t ldb,
               double beta, void* C, int64_t ldc, int dtype, void* ws,
               size_t ws_bytes, void* stream);

/* Gradient with respect to A of L = <dC, A*B>:  dA = dC * B^T.
 * dC m-by-n (lddc >= max(1,m)), B k-by-n (ldb >= max(1,k)),
 * dA m-by-k (ldda >= max(1,m)); n <= 32, any k.  Each dC row is read once;
 * dA is written once.  dtype: TSM_F64 or TSM_F32 (dC, B, dA all of it).
 * Arguments: 1 m, 2 k, 3 n, 4 dC, 5 lddc, 6 B, 7 ldb, 8 dA, 9 ldda,
 * 10 dtype, 11 stream. */
int tsm_grad_a(int64_t m, int64_t k, int64_t n, const void* dC, int64_t lddc,
               const void* B, int64_t ldb, void* dA, int64_t ldda, int dtype,
               void* stream);

/* Gradient with respect to B of L = <dC, A*B>:  dB = A^T * dC.
 * A m-by-k (lda >= max(1,m)), dC m-by-n (lddc >= max(1,m)),
 * dB k-by-n (lddb >= max(1,k)); n <= 32, any m and k.  The reduction over
 * m is split across wavefronts and workgroups and finished in double
 * precision in a fixed order.
 * dtype: TSM_F64, TSM_F32 (A, dC, dB all of it), or a 16-bit form of A as in
 * tsm2r (dC and dB float).  With bfloat16 planes and more than one group of
 * 16 columns of A, dC enters the bf16 matrix cores as three bf16 terms per
 * value (exact for finite dC in bfloat16's normal range), with the products
 * tsm2r keeps; a non-finite dC entry then gives NaN in its column of dB.
 * The workspace holds the slice partials and, for bfloat16 planes with
 * n > 16, dC's packed bf16 terms (192 bytes per row of dC);
 * tsm2x_workspace_size(TSM_OP_GRAD_B, m, k, n, dtype) gives its size, and a
 * caller's workspace must be 256-byte aligned (TSM_ERR_WORKSPACE otherwise).
 * Arguments: 1 m, 2 k, 3 n, 4 A, 5 lda, 6 dC, 7 lddc, 8 dB, 9 lddb,
 * 10 dtype, 11 ws, 12 ws_bytes, 13 stream (ws may be NULL: library buffer). */
int tsm_grad_b(int64_t m, int64_t k, int64_t n, const void* A, int64_t lda,
               const void* dC, int64_t lddc, void* dB, int64_t lddb,
               int dtype, void* ws, size_t ws_bytes, void* stream);

/* Fused backward of a TSM2L product C = A*B (k <= 32, n <= 32): one pass
 * over the rows of A (m x k, lda) and dC (m x n, lddc) writes
 * dA = dC * B^T (m x k, ldda) and dB = A^T * dC (k x n, lddb); B is k x n
 * (ldb).  A, dC and dA each cross HBM once (the separate tsm_grad_a and
 * tsm_grad_b read dC twice).  dB is reduced in double precision in a fixed
 * order.  dtype: any tsm_dtype; for the 16-bit forms A is the plane(s) of
 * tsm2x_split (lo plane lda*k elements after hi), widened to float, and B,
 * dC, dA, dB are float.  ws/ws_bytes as in tsm_grad_b (NULL: library
 * buffer).  Arguments: 1 m, 2 k, 3 n, 4 A, 5 lda, 6 B, 7 ldb, 8 dC,
 * 9 lddc, 10 dA, 11 ldda, 12 dB, 13 lddb, 14 dtype, 15 ws, 16 ws_bytes,
 * 17 stream.  TSM_ERR_UNSUPPORTED if k > 32 or n > 32. */
int tsm2l_backward(int64_t m, int64_t k, int64_t n, const void* A, int64_t lda,
                   const void* B, int64_t ldb, const void* dC, int64_t lddc,
                   void* dA, int64_t ldda, void* dB, int64_t lddb, int dtype,
                   void* ws, size_t ws_bytes, void* stream);

/* tsm2l_backward for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments without the workspace, the same kernels, the same grid and the
 * same results bit for bit, with the dB partials in a static device array of
 * the library (16 MiB per device, held until the process ends; room for one
 * 32 x 32 double partial per workgroup of the persistent grid, at most 2048
 * workgroups) instead of a workspace.  The array's address is looked up once
 * per device, on the first call made with that device current.  No
 * allocation of any kind is made on the device.  Every call on one device
 * shares that device's array: calls that overlap on one device (two streams,
 * two host threads) race and must be ordered by the caller.  Nothing needs
 * clearing between calls (every partial is written before it is read).
 * Returns as tsm2l_backward (arguments 1..14 checked the same way), plus
 * TSM_ERR_WORKSPACE when the grid's partials would exceed the array (not on
 * a device of at most 256 compute units) and TSM_ERR_HIP when the address
 * lookup fails. */
int tsm2l_backward_noalloc(int64_t m, int64_t k, int64_t n, const void* A, int64_t lda,
                           const void* B, int64_t ldb, const void* dC, int64_t lddc, void* dA,
                           int64_t ldda, void* dB, int64_t lddb, int dtype, void* stream);

/* K-means assignment step.  The paper's Introduction names K-means as a
 * tall-and-skinny GEMM application (far fewer centroids than points).  For
 * points X, m-by-k, either column-major (x_rowmajor 0: point i is row i,
 * ldx >= max(1,m)) or row-major (x_rowmajor 1: point i at X + i*ldx, its k
 * values contiguous, ldx >= k), and centroids Mu (k-by-n, column-major:
 * centroid c is column c, ldm >= k) it writes
 *   labels[i] = the smallest c with the smallest ||x_i - mu_c||^2  (int32),
 *   dist[i]   = that squared distance (dtype; dist may be NULL).
 * The distance is evaluated as ||x||^2 - 2 x.mu_c + ||mu_c||^2 (clamped at
 * 0): the cross terms are a TSM2L-shaped product on the matrix cores, and
 * the minimum is taken in registers, so X is read once (once per 32
 * centroids when n > 32) and only labels and dist are written.  Ties between
 * equal evaluated values go to the smaller c; NaN values never compare
 * smaller, and a row with no non-NaN value gets label 0 and dist NaN.
 * Any k >= 1 and n >= 1.  dtype: TSM_F64 or TSM_F32 (X, Mu, dist).
 * Workspace: tsm2x_workspace_size(TSM_OP_KMEANS, m, k, n, dtype) bytes,
 * 256-byte aligned (ws NULL: the library's buffer).
 * Row-major X is loaded as one contiguous stream per wavefront tile and
 * transposed through LDS; column-major X as k column streams.
 * Arguments: 1 m, 2 k, 3 n, 4 X, 5 ldx, 6 x_rowmajor, 7 Mu, 8 ldm,
 * 9 labels, 10 dist, 11 dtype, 12 ws, 13 ws_bytes, 14 stream.  Errors: -i
 * for argument i (k and n must be >= 1); TSM_ERR_WORKSPACE for a small or
 * misaligned ws. */
int tsm_kmeans_assign(int64_t m, int64_t k, int64_t n, const void* X, int64_t ldx,
                      int x_rowmajor, const void* Mu, int64_t ldm, int32_t* labels, void* dist,
                      int dtype, void* ws, size_t ws_bytes, void* stream);

/* Low-precision storage form of A: from a float m-by-k matrix A (lda),
 * write hi = RNE(a) and, if lo != NULL, lo = RNE(a - hi) (a - hi is exact in
 * float) as bfloat16 (fmt 0) or binary16 (fmt 1) planes of leading dimension
 * ldh (>= max(1,m)).  RNE = round to nearest, ties to even; NaN stays NaN;
 * values beyond the binary16 range become +-inf.
 * Arguments: 1 m, 2 k, 3 A, 4 lda, 5 hi, 6 lo, 7 ldh, 8 fmt, 9 stream. */
int tsm2x_split(int64_t m, int64_t k, const float* A, int64_t lda, void* hi,
                void* lo, int64_t ldh, int fmt, void* stream);

/* Bytes of workspace the call (op, m, k, n, dtype) needs; 0 if none. */
size_t tsm2x_workspace_size(int op, int64_t m, int64_t k, int64_t n,
                            int dtype);

/* Name of the main kernel a call (op, m, k, n, dtype) launches, as
 * profilers print it (for matching timings with profiler summaries), with
 * A 16-byte aligned and lda a multiple of 16 bytes.  Static storage; NULL
 * for ops other than TSM_OP_TSM2R, the 16-bit forms, or empty or
 * unsupported shapes. */
const char* tsm2x_kernel_name(int op, int64_t m, int64_t k, int64_t n, int dtype);

/* Launch plan of a TSM2R product (tsm2r, or a TSM2R-class call of
 * tsm2x_gemm) of column-major F64/F32 A, m-by-k, and n <= 32 columns, on the
 * current device.  The paper sizes its kernel from a performance model and
 * offline profiling (Section 3.6, Algorithm 5, and the t1 choice that
 * follows it); here the planner sizes the grid from the runtime's occupancy
 * query and a measured target, and a caller may replace its two choices per
 * shape (tsm2x_tsm2r_pin).  Outputs (each may be NULL):
 *   slices     k split S (gridDim.y): each workgroup streams k/S columns;
 *   tall       0: tiles of 16*RL*2 rows with 16-column chunks per
 *              wavefront; 1: twice the rows with 8-column chunks (RL = 16
 *              bytes / element size); both keep 8 KB of A in flight per
 *              wavefront;
 *   tiles      row tiles (gridDim.x); tile_rows: rows per tile;
 *   occupancy  resident workgroups per CU of the chosen kernel instance;
 *   cus        compute units of the device.
 * Returns 0; -1 m <= 0, -2 k <= 0, -3 n outside 1..32, -4 dtype not
 * F64/F32; TSM_ERR_UNSUPPORTED if no kernel instance covers the request. */
int tsm2x_tsm2r_plan(int64_t m, int64_t k, int64_t n, int dtype, int* slices, int* tall,
                     int64_t* tiles, int* tile_rows, int* occupancy, int* cus);

/* Pin the plan of later TSM2R products of exactly (m, k, n <= 32, dtype
 * F64/F32), on every device (the table is process-wide and thread-safe):
 * slices >= 1 forces the k split (rounded, like the planner's own choice,
 * so that every slice is a whole number of wavefront chunks; the plan query
 * reports the result), tall 0 / 1 forces the tile height, tall = -1 leaves
 * it to the planner; slices = 0 with tall = -1 removes the pin.  Results
 * are the same product for any plan, up to the order of the k sums (the
 * split sums are added in slice order, in double).  A larger S needs more
 * workspace: query tsm2x_workspace_size after pinning.  Products wider than
 * 32 columns run in panels of 32 columns, each looked up by its own width.
 * Host only, no HIP call.  Returns 0; -1 m <= 0, -2 k <= 0, -3 n outside
 * 1..32, -4 dtype not F64/F32, -5 slices outside 0..k, -6 tall outside
 * -1..1. */
int tsm2x_tsm2r_pin(int64_t m, int64_t k, int64_t n, int dtype, int slices, int tall);

/* Per-launch kernel timing, for measuring each kernel of a sequence of
 * calls while it runs (the paper times its kernels with GPU events, in its
 * Experimental Evaluation; this is the same measurement, per kernel launch).
 * Off until tsm2x_timing_start.  While on, every kernel launch of the library
 * is bracketed by a HIP event pair recorded on the stream the kernel is
 * launched on, and attributed to the kernel instance and to the tag last set
 * by tsm2x_timing_tag (an arbitrary caller label, e.g. which step of a
 * sequence is running; process-wide, so it also labels launches made from
 * other host threads).  The recording adds one event record before and after
 * each launch; with timing off a launch pays one atomic load.
 *   tsm2x_timing_start    drop earlier records and rows, start recording;
 *   tsm2x_timing_stop     stop recording (records kept);
 *   tsm2x_timing_tag      set the tag of later launches;
 *   tsm2x_timing_collect  wait for every recorded launch to finish, add it to
 *                         one row per (kernel, tag), and return the number of
 *                         rows.  Call it when no recorded work is being
 *                         enqueued by another thread;
 *   tsm2x_timing_row      row i: the kernel's demangled name without its
 *                         namespace and parameter list, e.g.
 *                         "rowtile_kernel<double, 4, 1, 1, true, false>"
 *                         (static storage, valid until the next start), its
 *                         tag, launch count and summed launch time in
 *                         milliseconds.  Returns -1 for i out of range.
 * All return 0 unless stated. */
int tsm2x_timing_start(void);
int tsm2x_timing_stop(void);
int tsm2x_timing_tag(int tag);
int tsm2x_timing_collect(void);
int tsm2x_timing_row(int i, const char** kernel, int* tag, int64_t* launches,
                     double* total_ms);

/* Bandwidth probes (measurement support, not part of any product): the HBM
 * ceilings the products are compared with, measured with the products' own
 * 16-byte non-temporal load and store forms.  The paper compares achieved
 * bandwidth with the device's peak (Performance Metrics Estimation, and the
 * bandwidth utilisation of its Experimental Evaluation); these give the
 * ceiling a real access pattern reaches on this device.
 *
 * tsm2x_probe_stream: kind 0 reads `bytes` of src (dst: at least 16 bytes,
 * normally left untouched), kind 1 copies `bytes` from src to dst, kind 2
 * writes `bytes` of a pattern to dst (src unused).  Each wavefront moves one
 * 4 KB piece per iteration of a grid-stride loop; `blocks` 256-thread
 * workgroups (0: 65536), never more than the pieces need.  Pointers 16-byte
 * aligned, bytes a multiple of 16.  Arguments: 1 kind, 2 src, 3 dst,
 * 4 bytes, 5 blocks, 6 stream.
 *
 * tsm2x_probe_tiles: the access pattern of the TSM2L kernel without its
 * arithmetic.  X is column-major m-by-kin, O column-major m-by-nout (F64 or
 * F32; 1 <= kin, nout <= 32); a persistent grid of `blocks` workgroups
 * (0: as many as are resident at once) walks the row tiles the TSM2L kernel
 * walks for (kin, nout), loading every element of X once and storing every
 * element of O once.  O receives X's columns in a fixed mapping (output
 * column 16t + j of a tile takes one input column of the same rows); only
 * the bytes moved matter.  With Y (m-by-kin, leading dimension ldy; NULL for
 * none) both X and Y are read, in the taller tiles of the fused TSM2L
 * backward, and O takes X + Y under the same mapping: the pattern of that
 * kernel (A and dC read, dA written).  Arguments: 1 m, 2 kin, 3 nout, 4 X,
 * 5 ldx, 6 Y, 7 ldy, 8 O, 9 ldo, 10 dtype, 11 blocks, 12 stream. */
int tsm2x_probe_stream(int kind, const void* src, void* dst, int64_t bytes, int64_t blocks,
                       void* stream);
int tsm2x_probe_tiles(int64_t m, int kin, int nout, const void* X, int64_t ldx, const void* Y,
                      int64_t ldy, void* O, int64_t ldo, int dtype, int64_t blocks, void* stream);

/* Static description of an error code (never NULL). */
const char* tsm2x_error_string(int code);

/* Message of the last HIP failure seen by this thread ("" if none). */
const char* tsm2x_last_hip_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int tsm2x_version(void);

/* Release the library-owned workspaces of every device.  No call may be in
 * flight. */
void tsm2x_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* TSM2X_H */
