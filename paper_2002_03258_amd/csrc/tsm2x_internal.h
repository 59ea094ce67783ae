// Internal launch descriptors shared by the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsm {

// Per-launch timing, off unless the caller turned it on (tsm2x_timing_start):
// a HIP event pair recorded on the launch's own stream around one kernel
// launch, attributed to the kernel and to the caller's current tag.
struct LaunchTimer {
    LaunchTimer(const void* fn, hipStream_t st);
    ~LaunchTimer();
    int slot;                // -1 when timing is off
    hipStream_t st;
};

}  // namespace tsm

// hipLaunchKernelGGL with the launch timed when timing is on
#define TSM_LAUNCH(KERNEL, GRID, BLOCK, LDS, ST, ...)                          \
    do {                                                                       \
        ::tsm::LaunchTimer tsm_launch_timer_((const void*)(KERNEL), (ST));     \
        hipLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, ST, __VA_ARGS__);         \
    } while (0)

namespace tsm {

enum { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_F16 = 3, DT_BF16_SPLIT = 4, DT_F16_SPLIT = 5 };

// Output rows per wavefront of the tn kernel for NP padded output columns:
// J*NP accumulators per lane, at most 64.
struct NNPlan {             // TSM2R launch plan (column-major A)
    const void* fn;         // kernel instance
    const char* name;       // its name as profilers print it
    int np;                 // padded n
    int tile_rows;
    int64_t tiles;          // row tiles (gridDim.x)
    int S;                  // k slices (gridDim.y)
    int64_t kslice;         // columns per k slice
    size_t ws;              // workspace bytes (0 when S == 1)
    int tall;               // 1: the taller of the two tile heights
    int occ;                // resident workgroups per CU of the instance
    int pf;                 // float TSM2R: the next chunk held in flight (0/1)
};

// A plan fixed by the caller for one shape: S >= 1 forces the k split (rounded
// as the planner rounds it), tall >= 0 forces the tile height.
struct NNPin {
    int S;
    int tall;
};

// Plan of tsm2r for (m, k, n, dtype) on a device with `cus` compute units;
// `vec`: A is 16-byte aligned with a 16-byte multiple leading dimension;
// `pin` (may be null) overrides the planner's choices.
// Returns nonzero if no kernel instance covers the request.
int plan_tsm2r(int64_t m, int64_t k, int64_t n, int dtype, int cus, bool vec, NNPlan* P,
               const NNPin* pin);

struct LaunchNN {           // tsm2r_nn: C = A*B, column-major A
    const void* fn;
    int64_t m, k, n;
    const void* A; int64_t lda;
    const void* B; int64_t ldb;
    void* C; int64_t ldc;
    int np;                 // padded n
    int tile_rows;
    int64_t tiles;          // row tiles (gridDim.x)
    int S;                  // k slices (gridDim.y)
    int64_t kslice;         // columns per k slice
    double* part;           // S > 1: partial sums (workspace)
    double beta;            // C := beta*C + A*B (C read only if beta != 0)
    int pf;                 // float TSM2R: the next chunk held in flight (0/1)
};

struct LaunchRT {           // rowtile: O = X*Y, X m x kin (kin <= 32)
    int64_t m; int kin; int64_t nout;
    const void* X; int64_t ldx;
    const void* Y; int64_t ys_in, ys_out;
    void* O; int64_t ldo;
    int kp;                 // padded kin: 8, 16 or 32
    int cols_per_block;
    int64_t blocks_x;       // upper bound on gridDim.x (0: none)
    int64_t blocks_y;
    int cus;                // compute units of the device
    double beta;            // O := beta*O + X*Y (O read only if beta != 0)
};

struct LaunchTN {           // tn: O = X^T*Y, X R x ncols, Y R x n
    int64_t R, ncols, n;
    const void* X; int64_t ldx;
    const void* Y; int64_t ldy;
    void* O; int64_t ldo;
    int64_t groups;         // 16-column tiles of the output (gridDim.x)
    int S;                  // reduction slices (gridDim.y)
    int64_t rslice;
    int rg;                 // stages per wavefront loop iteration (1, 2 or 4)
    int ct;                 // 16-column output tiles per workgroup (1 or 2)
    int pf;                 // 16-bit forms: the next step's X held in flight (0/1)
    double* part;           // S > 1: partial sums (workspace)
    double beta;            // O := beta*O + X^T*Y (O read only if beta != 0)
    const void* yt;         // bf16 planes, n > 16: Y's packed bf16 terms (workspace, or null)
};

// Low-precision storage forms of A (bf16 / f16, single or split planes).
int plan_tsm2r_lp(int64_t m, int64_t k, int64_t n, int dtype, int cus, bool vec, NNPlan* P);
// L.B: the packed terms of B written by launch_split_b (L.ldb unused)
int launch_tsm2r_lp(const LaunchNN& L, int dtype, hipStream_t st);
// B (k x n <= 32, B(j, p) = B[j*bsj + p*bsp]) split into three 16-bit terms
// packed as the matrix-core operand of tsm2r_lp, lp_bterms_bytes(k, n) bytes
size_t lp_bterms_bytes(int64_t k, int64_t n);
int launch_split_b(int64_t k, int64_t n, const float* B, int64_t bsj, int64_t bsp, int dtype,
                   void* out, hipStream_t st);
int launch_split(int64_t m, int64_t k, const float* A, int64_t lda, void* hi, void* lo,
                 int64_t ldh, int fmt, hipStream_t st);
// B(j, p) = B[j*bsj + p*bsp]
int launch_tsm2l_lp(int64_t m, int64_t k, int64_t n, const void* A, int64_t lda, const float* B,
                    int64_t bsj, int64_t bsp, float beta, float* C, int64_t ldc, int dtype,
                    int cus, hipStream_t st);

struct LaunchBwd {          // fused TSM2L backward: dA = dC*B^T, dB = A^T*dC
    int64_t m, k, n;
    const void* A; int64_t lda;
    const void* B; int64_t ldb;
    const void* dC; int64_t lddc;
    void* dA; int64_t ldda;
    void* dB; int64_t lddb;
    double* part;           // one k x n double partial per workgroup
    int cus;
};
// plan_only: set *blocks (workgroups, one dB partial each) without launching
int launch_tsm2l_bwd(const LaunchBwd& L, int dtype, int64_t* blocks, hipStream_t st,
                     bool plan_only);

int launch_tsm2r_nn(const LaunchNN& L, int dtype, hipStream_t st);
struct LaunchTN;
int launch_tn_lp(const LaunchTN& L, int dtype, hipStream_t st);
int launch_rowtile(const LaunchRT& L, int dtype, hipStream_t st);
int launch_tn(const LaunchTN& L, int dtype, hipStream_t st);
// C := beta*C for an m x n matrix (zeros when beta == 0, C then not read)
int launch_fill_scale(int64_t m, int64_t n, void* C, int64_t ldc, double beta, int dtype,
                      hipStream_t st);
// O (k x n, ld ldo) := the transpose of Bt (n x k, ld ldb), for a B given
// transposed
int launch_transpose(int64_t k, int64_t n, const void* Bt, int64_t ldb, void* O, int64_t ldo,
                     int dtype, hipStream_t st);
// Ordered sum over S slices of double partials laid out [g][s][NP][W] into
// O[g*W + r + p*ldo] := beta*O + sum (rows g*W + r < rows, p < n).
int launch_split_reduce(int dtype, int64_t groups, int S, int NP, int W, int64_t rows, int n,
                        const double* part, void* O, int64_t ldo, double beta, hipStream_t st);

struct LaunchKM {           // K-means assignment: points X (m x k), centroids Mu (k x n)
    int64_t m, k, n;
    const void* X; int64_t ldx;
    int x_rowmajor;         // 0: point i is row i of a column-major X; 1: X + i*ldx
    const void* Mu; int64_t ldm;
    void* mu2;              // n values of the dtype (workspace): ||mu_c||^2
    int32_t* labels;        // m
    void* dist;             // m, or null
    int cus;
};
int launch_kmeans_assign(const LaunchKM& L, int dtype, hipStream_t st);

}  // namespace tsm
