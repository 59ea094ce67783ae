// HIP kernels for gfx950 (MI355X): tall-and-skinny products of TSM2X.
//
// Three kernel families, all wave64, all reading every element of the big
// operand exactly once with 16-byte loads:
//
//  tsm2r_nn  C = A*B with column-major A (m x k, k large) and n <= 32.
//            Outer-product form of the Design of TSM2R (Algorithm 2): a lane
//            owns 16 bytes worth of consecutive rows of A and keeps their n
//            partial results of C in registers while it streams its columns.
//            B is staged in LDS one k-chunk at a time and read back as a
//            wave-wide broadcast (the shared-memory B tile of Algorithm 3),
//            and the next B chunk and the next A registers are fetched while
//            the current ones are used (the prefetching of Algorithm 4).
//            The k range is split across the wavefronts of a workgroup and
//            across workgroups; partial sums are added in double precision in
//            a fixed order, the last workgroup of a row tile to arrive doing
//            the final sum.
//
//  rowtile   O = X*Y with X tall (m x kin, kin <= 32): each lane loads its
//            rows of X once into registers and produces any number of output
//            columns from a Y panel held in LDS.  This is TSM2L (Algorithm 6:
//            a grid smaller than m walks the horizontal tiles of A) and also
//            the gradient dA = dC*B^T for both problem classes.
//
//  tn        O = X^T*Y with X (R x ncols) and Y (R x n) column-major, i.e. a
//            reduction along the contiguous dimension: TSM2R with a row-major
//            A, and the gradient dB = A^T*dC.  Lanes split the reduction,
//            wavefronts own output rows, workgroups split the reduction again
//            and finish it in double precision in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <cstdlib>

#include "tsm2x_internal.h"
#include "tsm2x_device.h"

namespace tsm {

// --------------------------------------------------------------------------
// tsm2r_nn: C = A*B, A column-major m x k (k large), n <= 16*NT16.
//
// Outer-product form of the Design of TSM2R (Algorithm 2) on the matrix
// cores: C^T = B^T * A^T.  S is a 16 x 4 block of B^T (lane l: B[j, 16t+rl]),
// T a 4 x 16 block of A^T.  A chunk of 4*ST columns at j0 is consumed in
// steps st = 0..ST-1 with columns j = j0 + ST*kk + st; a lane's ST B values
// of a chunk, B[j0+ST*kk .. j0+ST*kk+ST-1, 16t+rl], are contiguous in B's
// column.  The next chunk's A and B are loaded while the current one is
// multiplied (the prefetching of Algorithm 4).  Lane l ends up with
// C[row0 + 16*RL*g + RL*rl + q, 16t + mrow(kk, r)] in acc[g][q][t][r].
//
// The k range is split across the WK wavefronts of a workgroup and across
// workgroups; the partial sums are added in double precision in a fixed
// order (in LDS within the workgroup, then by split_reduce_kernel).
// --------------------------------------------------------------------------
// Explicit prefetch of the next chunk (Algorithm 4's nextA/nextB).
#ifndef TSM2X_NN_PREFETCH
#define TSM2X_NN_PREFETCH 1
#endif
// Waves per SIMD each instance is compiled for: three for n <= 16 (the
// register budget is then 168), two for n <= 32.
template <typename T, int NT16>
constexpr int nn_waves() { return NT16 == 1 ? 3 : 2; }

template <typename T, int NT16, int RG, int ST, int WK, bool VEC, bool PF = TSM2X_NN_PREFETCH>
__global__ __launch_bounds__(WAVE * WK)
__attribute__((amdgpu_waves_per_eu(nn_waves<T, NT16>(), 8))) void tsm2r_nn_kernel(
    int64_t m, int64_t k, int n, const T* __restrict__ A, int64_t lda,
    const T* __restrict__ B, int64_t ldb, T* __restrict__ C, int64_t ldc,
    int64_t kslice, double* __restrict__ part, int bvec) {
    typedef Mfma<T> M;
    typedef typename M::acc Acc;
    constexpr int RL = 16 / (int)sizeof(T);
    constexpr int TR = 16 * RL * RG;     // rows per tile
    constexpr int CW = 4 * ST;           // columns per chunk
    constexpr int NP = 16 * NT16;
    constexpr int PG = 4;
    // B run of a lane: ST values in vector loads of at most 16 bytes
    constexpr int BW = ST * (int)sizeof(T) > 16 ? RL : ST;
    static_assert(WK * PG * TR * 8 <= 32768, "LDS budget");
    __shared__ __align__(16) unsigned char smem[WK * PG * TR * 8];

    const int lane = threadIdx.x & (WAVE - 1);
    const int rl = lane & 15, kk = lane >> 4;
    const int w = threadIdx.x / WAVE;
    const int64_t tile = blockIdx.x;
    const int s = blockIdx.y, nsl = gridDim.y;
    const int64_t row0 = tile * TR;
    const bool full = (row0 + TR <= m);
    const int64_t kb0 = (int64_t)s * kslice;
    const int64_t kb1 = (kb0 + kslice < k) ? kb0 + kslice : k;
    const int64_t lw = kslice / WK;
    const int64_t wk0 = kb0 + w * lw;
    const int64_t wk1 = (wk0 + lw < kb1) ? wk0 + lw : kb1;

    Acc acc[RG][RL][NT16];
#pragma unroll
    for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int q = 0; q < RL; ++q)
#pragma unroll
            for (int t = 0; t < NT16; ++t) acc[g][q][t] = Acc{0, 0, 0, 0};

    auto loadA = [&](int64_t j0, T (&av)[ST][RG][RL]) {
#pragma unroll
        for (int st = 0; st < ST; ++st) {
            const int64_t j = j0 + ST * kk + st;
#pragma unroll
            for (int g = 0; g < RG; ++g) {
                const int64_t r = row0 + 16 * RL * g + RL * rl;
                if (j < wk1)
                    load_run<T, RL, VEC>(A + r + j * lda, m - r, full, av[st][g]);
                else
#pragma unroll
                    for (int q = 0; q < RL; ++q) av[st][g][q] = T(0);
            }
        }
    };
    // a lane's ST values of B in a chunk are contiguous in B's column; B is
    // re-read by every row tile, so these are ordinary (cached) loads
    auto loadB = [&](int64_t j0, T (&bv)[NT16][ST]) {
#pragma unroll
        for (int t = 0; t < NT16; ++t) {
            const int p = 16 * t + rl;
            const int64_t jb = j0 + ST * kk;
            const T* __restrict__ src = B + jb + (int64_t)p * ldb;
            if (p < n && bvec && jb + ST <= wk1) {
                typedef typename VecOf<T, BW>::type V;
#pragma unroll
                for (int h = 0; h < ST / BW; ++h) {
                    const V v = *reinterpret_cast<const V*>(src + h * BW);
#pragma unroll
                    for (int e = 0; e < BW; ++e) bv[t][h * BW + e] = v[e];
                }
            } else {
#pragma unroll
                for (int st = 0; st < ST; ++st)
                    bv[t][st] = (p < n && jb + st < wk1) ? src[st] : T(0);
            }
        }
    };

    if (wk1 > wk0) {
        const int ng = (int)((wk1 - wk0 + CW - 1) / CW);
        T av[ST][RG][RL], bv[NT16][ST];
        if (PF) {
            loadA(wk0, av);
            loadB(wk0, bv);
        }
        for (int gc = 0; gc < ng; ++gc) {
            T an[ST][RG][RL], bn[NT16][ST];
            if (!PF) {
                loadA(wk0 + CW * gc, av);
                loadB(wk0 + CW * gc, bv);
            } else if (gc + 1 < ng) {
                loadA(wk0 + CW * (gc + 1), an);
                loadB(wk0 + CW * (gc + 1), bn);
            }
#pragma unroll
            for (int st = 0; st < ST; ++st)
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int q = 0; q < RL; ++q)
#pragma unroll
                        for (int t = 0; t < NT16; ++t)
                            acc[g][q][t] = M::op(bv[t][st], av[st][g][q], acc[g][q][t]);
            if (PF) {
#pragma unroll
                for (int st = 0; st < ST; ++st)
#pragma unroll
                    for (int g = 0; g < RG; ++g)
#pragma unroll
                        for (int q = 0; q < RL; ++q) av[st][g][q] = an[st][g][q];
#pragma unroll
                for (int t = 0; t < NT16; ++t)
#pragma unroll
                    for (int st = 0; st < ST; ++st) bv[t][st] = bn[t][st];
            }
        }
    }

    nn_finish<T, NP, WK, TR, PG>(m, n, C, ldc, tile, s, nsl, part,
                                 reinterpret_cast<double*>(smem), [&](int pg, double* red) {
        const int t = pg / 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int pp = 16 * t + M::mrow(kk, r) - pg;
            if (pp >= 0 && pp < PG) {
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int q = 0; q < RL; ++q)
                        red[(w * PG + pp) * TR + 16 * RL * g + RL * rl + q] =
                            (double)acc[g][q][t][r];
            }
        }
    });
}

// --------------------------------------------------------------------------
// rowtile: O(m x nout) = X(m x kin) * Y(kin x nout), kin <= 4*KS <= 32,
// Y(ji, jo) = Y[ji * ys_in + jo * ys_out] (so B and B^T are both views).
//
// TSM2L (Design of TSM2L, Algorithm 6): a grid of fewer wavefronts than row
// tiles walks the horizontal tiles of A; each lane loads its 16-byte row
// runs of all kin columns once and B, held whole in registers, never leaves
// the chip, so C is written once and never re-read.  The same kernel gives
// dA = dC * B^T, where nout = k may be large: workgroups then also split the
// output columns and a wavefront reuses its X registers for every 16*NT16
// output columns of its range.
//
// On the matrix cores: O^T = Y^T * X^T with S[rl][kk] = Y(4 st + kk,
// col0 + 16 t + rl) and T[kk][rl] = X[row(rl, q), 4 st + kk]; lane l holds
// O[row(rl, q), col0 + 16 t + mrow(kk, r)] in acc[g][q][t][r] with
// row(rl, q) = row0 + 16*RL*g + RL*rl + q.
// --------------------------------------------------------------------------
template <typename T, int KS, int NT16, int RG, bool VEC, bool PF>
__global__ __launch_bounds__(256) void rowtile_kernel(
    int64_t m, int kin, int64_t nout, const T* __restrict__ X, int64_t ldx,
    const T* __restrict__ Y, int64_t ys_in, int64_t ys_out, T* __restrict__ O,
    int64_t ldo, int64_t cols_per_block) {
    typedef Mfma<T> M;
    typedef typename M::acc Acc;
    constexpr int RL = 16 / (int)sizeof(T);
    constexpr int TR = 16 * RL * RG;
    constexpr int WPB = 4;
    constexpr int CW = 16 * NT16;        // output columns per pass

    const int lane = threadIdx.x & (WAVE - 1);
    const int rl = lane & 15, kk = lane >> 4;
    const int w = threadIdx.x / WAVE;
    const int64_t cb0 = (int64_t)blockIdx.y * cols_per_block;
    const int64_t cb1 = (cb0 + cols_per_block < nout) ? cb0 + cols_per_block : nout;

    T yv[KS][NT16];
    auto loadY = [&](int64_t c0) {
#pragma unroll
        for (int st = 0; st < KS; ++st)
#pragma unroll
            for (int t = 0; t < NT16; ++t) {
                const int ji = 4 * st + kk;
                const int64_t jo = c0 + 16 * t + rl;
                yv[st][t] = (ji < kin && jo < cb1) ? Y[ji * ys_in + jo * ys_out] : T(0);
            }
    };
    const bool one_pass = (cb1 - cb0) <= CW;
    if (one_pass) loadY(cb0);

    auto loadX = [&](int64_t tile, T (&xv)[KS][RG][RL]) {
        const int64_t row0 = tile * TR;
        const bool full = (row0 + TR <= m);
#pragma unroll
        for (int st = 0; st < KS; ++st) {
            const int ji = 4 * st + kk;
#pragma unroll
            for (int g = 0; g < RG; ++g) {
                const int64_t r = row0 + 16 * RL * g + RL * rl;
                if (ji < kin)
                    load_run<T, RL, VEC>(X + r + ji * ldx, m - r, full, xv[st][g]);
                else
#pragma unroll
                    for (int q = 0; q < RL; ++q) xv[st][g][q] = T(0);
            }
        }
    };

    const int64_t ntiles = (m + TR - 1) / TR;
    const int64_t tstride = (int64_t)gridDim.x * WPB;
    int64_t tile = (int64_t)blockIdx.x * WPB + w;
    T xv[KS][RG][RL];
    if (tile < ntiles) loadX(tile, xv);
    for (; tile < ntiles; tile += tstride) {
        const int64_t row0 = tile * TR;
        const bool full = (row0 + TR <= m);
        // the next tile's rows are requested before this tile is multiplied
        T xn[KS][RG][RL];
        const bool more = tile + tstride < ntiles;
        if (PF && more) loadX(tile + tstride, xn);
        for (int64_t c0 = cb0; c0 < cb1; c0 += CW) {
            if (!one_pass) loadY(c0);
            Acc acc[RG][RL][NT16];
#pragma unroll
            for (int g = 0; g < RG; ++g)
#pragma unroll
                for (int q = 0; q < RL; ++q)
#pragma unroll
                    for (int t = 0; t < NT16; ++t) acc[g][q][t] = Acc{0, 0, 0, 0};
#pragma unroll
            for (int st = 0; st < KS; ++st)
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int q = 0; q < RL; ++q)
#pragma unroll
                        for (int t = 0; t < NT16; ++t)
                            acc[g][q][t] = M::op(yv[st][t], xv[st][g][q], acc[g][q][t]);
#pragma unroll
            for (int g = 0; g < RG; ++g) {
                const int64_t r = row0 + 16 * RL * g + RL * rl;
#pragma unroll
                for (int t = 0; t < NT16; ++t)
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const int64_t col = c0 + 16 * t + M::mrow(kk, rr);
                        if (col < cb1) {
                            T v[RL];
#pragma unroll
                            for (int q = 0; q < RL; ++q) v[q] = acc[g][q][t][rr];
                            store_run<T, RL, VEC>(O + r + col * ldo, m - r, full, v);
                        }
                    }
            }
        }
        if (more) {
            if (PF) {
#pragma unroll
                for (int st = 0; st < KS; ++st)
#pragma unroll
                    for (int g = 0; g < RG; ++g)
#pragma unroll
                        for (int q = 0; q < RL; ++q) xv[st][g][q] = xn[st][g][q];
            } else {
                loadX(tile + tstride, xv);
            }
        }
    }
}

// --------------------------------------------------------------------------
// tn: O(ncols x n) = X^T * Y with X (R x ncols) and Y (R x n) column-major:
// a reduction along the contiguous dimension.  TSM2R with a row-major A
// (X = A^T) and the gradient dB = A^T * dC.
//
// D = O tile: S[rl][kk] = X[r, c0 + rl], T[kk][rl] = Y[r, 16 t + rl] with the
// reduction index r = rb + RL*kk + q for step q, so lane l needs RL
// consecutive rows of ONE column for each operand.  Loading that directly
// makes every load instruction touch 16 columns with 64-byte pieces, which
// (measured) caps HBM reads near 60 %.  Instead each wavefront loads blocks
// of SR = 16*RL rows with the 4-columns-x-256-bytes pattern of the other
// kernels (lane (rl, kk) reads rows RL*rl .. of column 4 c + kk), stages
// them in its own padded LDS tile [column][row], and reads them back in the
// MFMA layout (16-byte LDS reads, four blocks of 4*RL rows per stage).  LDS operations of one
// wavefront execute in order, so no barrier is needed between the stage and
// the read-back.  Lane l holds O[c0 + mrow(kk, r), 16 t + rl] in acc[t][r].
// The WK wavefronts of a workgroup split the workgroup's slice of R, and
// workgroups split R again; partials are added in double precision in a
// fixed order (workgroup level here, across workgroups by
// split_reduce_kernel).
// --------------------------------------------------------------------------
template <typename T, int NT16, int G, bool VEC>
__global__ __launch_bounds__(256) void tn_kernel(
    int64_t R, int64_t ncols, int n, const T* __restrict__ X, int64_t ldx,
    const T* __restrict__ Y, int64_t ldy, T* __restrict__ O, int64_t ldo,
    int64_t rslice, double* __restrict__ part) {
    typedef Mfma<T> M;
    typedef typename M::acc Acc;
    constexpr int RL = 16 / (int)sizeof(T);
    constexpr int WK = 4;
    constexpr int SR = 16 * RL;                // rows per stage
    constexpr int SROW = SR + RL;              // padded LDS column (16 more bytes)
    constexpr int NC = 16 + 16 * NT16;         // staged columns: X tile, then Y tiles
    constexpr int NV = 4 * NT16;
    __shared__ __align__(16) T lds[WK][NC][SROW];
    __shared__ double red[WK][WAVE][NV];

    const int lane = threadIdx.x & (WAVE - 1);
    const int rl = lane & 15, kk = lane >> 4;
    const int w = threadIdx.x / WAVE;
    const int64_t ctile = blockIdx.x;
    const int64_t c0 = ctile * 16;
    const int s = blockIdx.y, nsl = gridDim.y;
    const int64_t sb0 = (int64_t)s * rslice;
    const int64_t sb1 = (sb0 + rslice < R) ? sb0 + rslice : R;
    const int64_t lw = rslice / WK;            // multiple of G * SR
    const int64_t wb0 = sb0 + w * lw;
    const int64_t wb1 = (wb0 + lw < sb1) ? wb0 + lw : sb1;
    T (*tile)[SROW] = lds[w];

    Acc acc[NT16];
#pragma unroll
    for (int t = 0; t < NT16; ++t) acc[t] = Acc{0, 0, 0, 0};

    // staged column sc: sc < 16 -> X column c0 + sc, else Y column sc - 16
    auto load = [&](int64_t rb, T (&v)[G][NC / 4][RL]) {
#pragma unroll
        for (int gs = 0; gs < G; ++gs) {
            const int64_t r = rb + gs * SR + RL * rl;
            const int64_t valid = wb1 - r;
            const bool full = valid >= RL;
#pragma unroll
            for (int cg = 0; cg < NC / 4; ++cg) {
                const int sc = 4 * cg + kk;
                const T* src;
                bool ok;
                if (sc < 16) {
                    src = X + r + (c0 + sc) * ldx;
                    ok = c0 + sc < ncols;
                } else {
                    src = Y + r + (int64_t)(sc - 16) * ldy;
                    ok = sc - 16 < n;
                }
                if (ok)
                    load_run<T, RL, VEC>(src, valid, full, v[gs][cg]);
                else
#pragma unroll
                    for (int q = 0; q < RL; ++q) v[gs][cg][q] = T(0);
            }
        }
    };

    if (wb1 > wb0) {
        const int64_t nit = (wb1 - wb0 + G * SR - 1) / (G * SR);
        T v[G][NC / 4][RL];
        load(wb0, v);
        for (int64_t it = 0; it < nit; ++it) {
            T vn[G][NC / 4][RL];
            if (it + 1 < nit) load(wb0 + (it + 1) * G * SR, vn);
#pragma unroll
            for (int gs = 0; gs < G; ++gs) {
                // stage: column 4 cg + kk, rows RL*rl .. RL*rl + RL - 1
#pragma unroll
                for (int cg = 0; cg < NC / 4; ++cg) {
                    typedef typename VecOf<T, RL>::type V;
                    V x;
#pragma unroll
                    for (int q = 0; q < RL; ++q) x[q] = v[gs][cg][q];
                    *reinterpret_cast<V*>(&tile[4 * cg + kk][RL * rl]) = x;
                }
                // read back in four blocks of 4*RL rows: X column rl and Y
                // columns 16 t + rl, rows 4*RL*h + RL*kk + q
                typedef typename VecOf<T, RL>::type V;
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const V xs = *reinterpret_cast<const V*>(&tile[rl][4 * RL * h + RL * kk]);
#pragma unroll
                    for (int t = 0; t < NT16; ++t) {
                        const V ys =
                            *reinterpret_cast<const V*>(&tile[16 + 16 * t + rl][4 * RL * h + RL * kk]);
#pragma unroll
                        for (int q = 0; q < RL; ++q) acc[t] = M::op(xs[q], ys[q], acc[t]);
                    }
                }
            }
#pragma unroll
            for (int gs = 0; gs < G; ++gs)
#pragma unroll
                for (int cg = 0; cg < NC / 4; ++cg)
#pragma unroll
                    for (int q = 0; q < RL; ++q) v[gs][cg][q] = vn[gs][cg][q];
        }
    }

    tn_finish<T, NT16, WK>(ncols, n, O, ldo, ctile, s, nsl, part, red, acc,
                           [](int kq, int r) { return Mfma<T>::mrow(kq, r); });
}

template <typename T>
__global__ void fill_zero_kernel(int64_t m, int64_t n, T* __restrict__ C, int64_t ldc) {
    const int64_t total = m * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % m, p = e / m;
        C[i + p * ldc] = T(0);
    }
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------
// Resident workgroups per CU of a kernel instance (queried once).
template <typename K>
static int occupancy(K kernel, int threads) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1)
        nb = 1;
    return nb;
}

static inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

struct NNInstance {
    const void* fn;
    int tile_rows;
    int chunk;        // columns per chunk of a wavefront
    int occ;          // resident workgroups per CU
    const char* name; // as profilers print the kernel
};

template <typename T, int NT16, int RG, int ST, bool VEC>
static NNInstance nn_instance() {
    static const int occ = occupancy(tsm2r_nn_kernel<T, NT16, RG, ST, 4, VEC>, 256);
    static char name[80];
    static const bool named =
        std::snprintf(name, sizeof name, "tsm2r_nn_kernel<%s, %d, %d, %d, 4, %s, %s>",
                      sizeof(T) == 8 ? "double" : "float", NT16, RG, ST, VEC ? "true" : "false",
                      TSM2X_NN_PREFETCH ? "true" : "false") > 0;
    (void)named;
    return NNInstance{(const void*)tsm2r_nn_kernel<T, NT16, RG, ST, 4, VEC>,
                      16 * (16 / (int)sizeof(T)) * RG, 4 * ST, occ, name};
}

// Two tile heights per type: 16*RL*2 rows with 16-column chunks, and twice
// the rows with 8-column chunks.  Both keep 8 KB of A in flight per wavefront.
template <bool VEC>
static bool nn_pick(int dtype, int np, bool tall, NNInstance* out) {
    if (dtype == DT_F64) {
        if (tall)
            *out = np <= 16 ? nn_instance<double, 1, 4, 2, VEC>() : nn_instance<double, 2, 4, 2, VEC>();
        else
            *out = np <= 16 ? nn_instance<double, 1, 2, 4, VEC>() : nn_instance<double, 2, 2, 4, VEC>();
        return true;
    }
    if (dtype == DT_F32) {
        if (tall)
            *out = np <= 16 ? nn_instance<float, 1, 4, 2, VEC>() : nn_instance<float, 2, 4, 2, VEC>();
        else
            *out = np <= 16 ? nn_instance<float, 1, 2, 4, VEC>() : nn_instance<float, 2, 2, 4, VEC>();
        return true;
    }
    return false;
}

static inline int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Grid of the TSM2R kernel.  Measured on gfx950, the streaming rate peaks when
// about 15/8 workgroups (7.5 wavefronts, 8 KB of A in flight each) are
// resident per CU: fewer leave HBM latency uncovered, more add concurrent
// streams without adding bandwidth, and a grid that leaves some CUs with one
// workgroup more than others runs at the pace of those CUs.  For each tile
// height the k split S is the one that brings tiles * S closest to that
// target; the tile height whose grid lands closer wins, ties going to fewer
// slices (longer streams per wavefront).
int plan_tsm2r(int64_t m, int64_t k, int64_t n, int dtype, int cus, bool vec, NNPlan* P) {
    // partial sums are stored at the kernel's padded width (16 or 32 columns)
    const int np = n <= 16 ? 16 : 32;
    const int es = dtype == DT_F64 ? 8 : 4;
    const int WK = 4;
    int64_t target = (int64_t)cus * 15 / 8;
    const char* ft = std::getenv("TSM2X_NN_TARGET");
    if (ft && *ft && std::strtoll(ft, nullptr, 10) > 0) target = std::strtoll(ft, nullptr, 10);
    const char* fs = std::getenv("TSM2X_NN_S");
    const int64_t s_force = (fs && *fs) ? std::strtoll(fs, nullptr, 10) : 0;
    const char* fh = std::getenv("TSM2X_NN_TALL");     // 0 or 1 forces a tile height
    const int64_t tall_force = (fh && *fh) ? std::strtoll(fh, nullptr, 10) : -1;

    bool found = false;
    double best_dev = 0;
    for (int tall = 0; tall < 2; ++tall) {
        if (tall_force >= 0 && tall != (int)tall_force) continue;
        NNInstance I{};
        if (!(vec ? nn_pick<true>(dtype, np, tall, &I) : nn_pick<false>(dtype, np, tall, &I)))
            return 1;
        const int64_t tiles = cdiv64(m, I.tile_rows);
        const int64_t slots = (int64_t)cus * I.occ;
        const int64_t tgt = target < slots ? target : slots;
        int64_t S = (tgt + tiles / 2) / tiles;                        // nearest integer
        const int64_t s_len = k / (WK * 64);                          // >= 64 columns per wave
        const int64_t s_cost = (k * es) / ((int64_t)np * 200);         // partials <= ~4 % of A
        if (S > s_len) S = s_len;
        if (S > s_cost) S = s_cost;
        if (S < 1) S = 1;
        if (s_force > 0) S = s_force;
        const int64_t gran = (int64_t)WK * I.chunk;
        int64_t ks = cdiv64(k, S);
        ks = cdiv64(ks, gran) * gran;
        S = cdiv64(k, ks);
        if (S < 1) S = 1;
        const int64_t W = tiles * S;
        const double dev = (double)(W > tgt ? W - tgt : tgt - W) / (double)tgt;
        // a later (taller) instance must be clearly better to replace the first
        if (!found || dev < best_dev - 0.02) {
            found = true;
            best_dev = dev;
            P->np = np;
            P->fn = I.fn;
            P->name = I.name;
            P->tiles = tiles;
            P->tile_rows = I.tile_rows;
            P->kslice = ks;
            P->S = (int)S;
            P->ws = S > 1 ? (size_t)tiles * S * np * I.tile_rows * 8 : 0;
        }
    }
    return found ? 0 : 1;
}

int launch_tsm2r_nn(const LaunchNN& L, int dtype, hipStream_t st) {
    int n32 = (int)L.n;
    // 16-byte loads of B's column runs need an aligned B with ldb*size % 16 == 0
    const int es = dtype == DT_F64 ? 8 : 4;
    int bvec = aligned16(L.B) && ((L.ldb * es) % 16 == 0);
    void* args[] = {(void*)&L.m,   (void*)&L.k,      (void*)&n32,    (void*)&L.A,
                    (void*)&L.lda, (void*)&L.B,      (void*)&L.ldb,  (void*)&L.C,
                    (void*)&L.ldc, (void*)&L.kslice, (void*)&L.part, (void*)&bvec};
    hipError_t e = hipLaunchKernel(L.fn, dim3((unsigned)L.tiles, (unsigned)L.S), dim3(256), args,
                                   0, st);
    if (e != hipSuccess) return 1;
    if (L.S > 1)
        return launch_split_reduce(dtype, L.tiles, L.S, L.np, L.tile_rows, L.m, (int)L.n, L.part,
                                   L.C, L.ldc, st);
    return 0;
}

template <typename T, int KS, int NT16, int RG, bool PF>
static int rowtile_launch_pf(const LaunchRT& L, bool vec, hipStream_t st) {
    // persistent grid: as many workgroups as fit at once (queried occupancy),
    // but no more than there are groups of 4 row tiles
    static const int occ_v = occupancy(rowtile_kernel<T, KS, NT16, RG, true, PF>, 256);
    static const int occ_s = occupancy(rowtile_kernel<T, KS, NT16, RG, false, PF>, 256);
    constexpr int64_t TR = 16 * (16 / (int64_t)sizeof(T)) * RG;
    const int64_t ntiles = (L.m + TR - 1) / TR;
    int64_t bx = (int64_t)L.cus * (vec ? occ_v : occ_s) / (L.blocks_y > 0 ? L.blocks_y : 1);
    const int64_t need = (ntiles + 3) / 4;
    if (bx > need) bx = need;
    if (L.blocks_x > 0 && bx > L.blocks_x) bx = L.blocks_x;
    if (bx < 1) bx = 1;
    dim3 grid((unsigned)bx, (unsigned)L.blocks_y), block(256);
    if (vec)
        hipLaunchKernelGGL((rowtile_kernel<T, KS, NT16, RG, true, PF>), grid, block, 0, st, L.m,
                           L.kin, L.nout, (const T*)L.X, L.ldx, (const T*)L.Y, L.ys_in, L.ys_out,
                           (T*)L.O, L.ldo, (int64_t)L.cols_per_block);
    else
        hipLaunchKernelGGL((rowtile_kernel<T, KS, NT16, RG, false, PF>), grid, block, 0, st, L.m,
                           L.kin, L.nout, (const T*)L.X, L.ldx, (const T*)L.Y, L.ys_in,
                           L.ys_out, (T*)L.O, L.ldo, (int64_t)L.cols_per_block);
    return 0;
}

template <typename T, int KS, int NT16, int RG>
static int rowtile_launch(const LaunchRT& L, bool vec, hipStream_t st) {
    static const char* e = std::getenv("TSM2X_RT_PF");
    const bool pf = e && *e == '1';   // measured: the extra waves beat the prefetch
    return pf ? rowtile_launch_pf<T, KS, NT16, RG, true>(L, vec, st)
              : rowtile_launch_pf<T, KS, NT16, RG, false>(L, vec, st);
}

template <typename T>
static int rowtile_dispatch(const LaunchRT& L, hipStream_t st) {
    const bool vec = aligned16(L.X) && aligned16(L.O) &&
                     ((L.ldx * (int64_t)sizeof(T)) % 16 == 0) &&
                     ((L.ldo * (int64_t)sizeof(T)) % 16 == 0);
    const bool wide = L.nout > 16;   // two 16-column tiles per pass
    switch (L.kp) {
        case 8: return wide ? rowtile_launch<T, 2, 2, 2>(L, vec, st) : rowtile_launch<T, 2, 1, 2>(L, vec, st);
        case 16: return wide ? rowtile_launch<T, 4, 2, 2>(L, vec, st) : rowtile_launch<T, 4, 1, 2>(L, vec, st);
        case 32: return wide ? rowtile_launch<T, 8, 2, 1>(L, vec, st) : rowtile_launch<T, 8, 1, 2>(L, vec, st);
    }
    return 1;
}

int launch_rowtile(const LaunchRT& L, int dtype, hipStream_t st) {
    if (dtype == DT_F64) return rowtile_dispatch<double>(L, st);
    if (dtype == DT_F32) return rowtile_dispatch<float>(L, st);
    return 1;
}

template <typename T, int NT16, int G>
static int tn_launch(const LaunchTN& L, bool vec, hipStream_t st) {
    dim3 grid((unsigned)L.groups, (unsigned)L.S), block(256);
    if (vec)
        hipLaunchKernelGGL((tn_kernel<T, NT16, G, true>), grid, block, 0, st, L.R, L.ncols,
                           (int)L.n, (const T*)L.X, L.ldx, (const T*)L.Y, L.ldy, (T*)L.O, L.ldo,
                           L.rslice, L.part);
    else
        hipLaunchKernelGGL((tn_kernel<T, NT16, G, false>), grid, block, 0, st, L.R, L.ncols,
                           (int)L.n, (const T*)L.X, L.ldx, (const T*)L.Y, L.ldy, (T*)L.O, L.ldo,
                           L.rslice, L.part);
    return 0;
}

template <typename T>
static int tn_dispatch(const LaunchTN& L, hipStream_t st) {
    const bool vec = aligned16(L.X) && aligned16(L.Y) &&
                     ((L.ldx * (int64_t)sizeof(T)) % 16 == 0) &&
                     ((L.ldy * (int64_t)sizeof(T)) % 16 == 0);
    // G stages of 16*RL rows per loop iteration (loads for the next iteration
    // are in flight while the current one is staged and multiplied)
    int rc = 1;
    if (L.rg == 4) rc = L.n <= 16 ? tn_launch<T, 1, 4>(L, vec, st) : tn_launch<T, 2, 4>(L, vec, st);
    else if (L.rg == 2) rc = L.n <= 16 ? tn_launch<T, 1, 2>(L, vec, st) : tn_launch<T, 2, 2>(L, vec, st);
    else rc = L.n <= 16 ? tn_launch<T, 1, 1>(L, vec, st) : tn_launch<T, 2, 1>(L, vec, st);
    if (rc || L.S <= 1) return rc;
    return launch_split_reduce(sizeof(T) == 8 ? DT_F64 : DT_F32, L.groups, L.S,
                               L.n <= 16 ? 16 : 32, 16, L.ncols, (int)L.n, L.part, L.O, L.ldo, st);
}

int launch_tn(const LaunchTN& L, int dtype, hipStream_t st) {
    if (dtype == DT_F64) return tn_dispatch<double>(L, st);
    if (dtype == DT_F32) return tn_dispatch<float>(L, st);
    return 1;
}

int launch_split_reduce(int dtype, int64_t groups, int S, int NP, int W, int64_t rows, int n,
                        const double* part, void* O, int64_t ldo, hipStream_t st) {
    const int64_t total = groups * NP * W;
    const bool wide = S >= 16;
    int64_t blocks = wide ? (total + 3) / 4 : (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    const dim3 g((unsigned)blocks), b(256);
    if (dtype == DT_F64) {
        if (wide)
            hipLaunchKernelGGL((split_reduce_kernel<double, true>), g, b, 0, st, groups, S, NP, W,
                               rows, n, part, (double*)O, ldo);
        else
            hipLaunchKernelGGL((split_reduce_kernel<double, false>), g, b, 0, st, groups, S, NP,
                               W, rows, n, part, (double*)O, ldo);
    } else {
        if (wide)
            hipLaunchKernelGGL((split_reduce_kernel<float, true>), g, b, 0, st, groups, S, NP, W,
                               rows, n, part, (float*)O, ldo);
        else
            hipLaunchKernelGGL((split_reduce_kernel<float, false>), g, b, 0, st, groups, S, NP, W,
                               rows, n, part, (float*)O, ldo);
    }
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

int launch_fill_zero(int64_t m, int64_t n, void* C, int64_t ldc, int dtype, hipStream_t st) {
    const int64_t total = m * n;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    if (dtype == DT_F64)
        hipLaunchKernelGGL(fill_zero_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, m, n,
                           (double*)C, ldc);
    else
        hipLaunchKernelGGL(fill_zero_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, m, n,
                           (float*)C, ldc);
    return 0;
}

}  // namespace tsm
