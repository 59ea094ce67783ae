// HIP kernels for gfx950 (MI355X): the TSM2L family and the reductions along
// the contiguous dimension.
//
//  rowtile   O = X*Y with X tall (m x kin, kin <= 32): each lane loads its
//            16-byte row runs of X once and produces the output columns from
//            a Y panel held in registers.  This is TSM2L (Algorithm 6: a grid
//            smaller than m walks the horizontal tiles of A) and also the
//            gradient dA = dC*B^T for both problem classes.
//
//  tn        O = X^T*Y with X (R x ncols) and Y (R x n) column-major, i.e. a
//            reduction along the contiguous dimension: TSM2R with a row-major
//            A, and the gradient dB = A^T*dC.  Loads stream 4 columns x 256
//            bytes per instruction and are re-read in MFMA order from a
//            wavefront-private LDS tile; wavefronts and workgroups split the
//            reduction, finished in double precision in a fixed order.
//
// Also the fixed-order sum of split partials and a zero fill.  The TSM2R
// kernel itself is in tsm2x_tsm2r.hip.
//            and finish it in double precision in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdlib>

#include "tsm2x_internal.h"
#include "tsm2x_device.h"

namespace tsm {

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
template <typename T, int KS, int NT16, int RG, bool VEC, bool NTS>
__global__ __launch_bounds__(256) void rowtile_kernel(
    int64_t m, int kin, int64_t nout, const T* __restrict__ X, int64_t ldx,
    const T* __restrict__ Y, int64_t ys_in, int64_t ys_out, T* __restrict__ O,
    int64_t ldo, int64_t cols_per_block, T beta) {
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
        const bool more = tile + tstride < ntiles;
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
                            if (beta != T(0)) {     // O is read only then
                                T o[RL];
                                load_run<T, RL, VEC>(O + r + col * ldo, m - r, full, o);
#pragma unroll
                                for (int q = 0; q < RL; ++q) v[q] = __builtin_fma(beta, o[q], v[q]);
                            }
                            store_run<T, RL, VEC, NTS>(O + r + col * ldo, m - r, full, v);
                        }
                    }
            }
        }
        if (more) {
            loadX(tile + tstride, xv);
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
template <typename T, int NT16, int G, int CT, bool VEC, bool YC>
__global__ __launch_bounds__(256) void tn_kernel(
    int64_t R, int64_t ncols, int n, const T* __restrict__ X, int64_t ldx,
    const T* __restrict__ Y, int64_t ldy, T* __restrict__ O, int64_t ldo,
    int64_t rslice, double* __restrict__ part, double beta, int pf) {
    typedef Mfma<T> M;
    typedef typename M::acc Acc;
    constexpr int RL = 16 / (int)sizeof(T);
    constexpr int WK = 4;
    constexpr int SR = 16 * RL;                // rows per stage
    constexpr int SROW = SR + RL;              // padded LDS column (16 more bytes)
    constexpr int NX = 16 * CT;                // staged X columns (CT output tiles)
    constexpr int NC = NX + 16 * NT16;         // then the Y columns
    constexpr int NV = 4 * NT16;
    __shared__ __align__(16) T lds[WK][NC][SROW];
    __shared__ double red[WK][WAVE][NV];

    const int lane = threadIdx.x & (WAVE - 1);
    const int rl = lane & 15, kk = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);   // wavefront-uniform
    const int64_t c0 = (int64_t)blockIdx.x * NX;
    const int s = blockIdx.y, nsl = gridDim.y;
    const int64_t sb0 = (int64_t)s * rslice;
    const int64_t sb1 = (sb0 + rslice < R) ? sb0 + rslice : R;
    const int64_t lw = rslice / WK;            // multiple of G * SR
    const int64_t wb0 = sb0 + w * lw;
    const int64_t wb1 = (wb0 + lw < sb1) ? wb0 + lw : sb1;
    T (*tile)[SROW] = lds[w];

    Acc acc[CT][NT16];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int t = 0; t < NT16; ++t) acc[ct][t] = Acc{0, 0, 0, 0};

    // staged column sc: sc < NX -> X column c0 + sc, else Y column sc - NX
    auto load = [&](int64_t rb, T (&v)[G][NC / 4][RL]) {
#pragma unroll
        for (int gs = 0; gs < G; ++gs) {
            const int64_t r = rb + gs * SR + RL * rl;
            const int64_t valid = wb1 - r;
            const bool full = valid >= RL;
#pragma unroll
            for (int cg = 0; cg < NC / 4; ++cg) {
                const int sc = 4 * cg + kk;
                if (cg < NX / 4) {
                    if (c0 + sc < ncols)
                        load_run<T, RL, VEC>(X + r + (c0 + sc) * ldx, valid, full, v[gs][cg]);
                    else
#pragma unroll
                        for (int q = 0; q < RL; ++q) v[gs][cg][q] = T(0);
                } else {
                    const T* src = Y + r + (int64_t)(sc - NX) * ldy;
                    if (YC && VEC && sc - NX < n && full) {
                        typedef typename VecOf<T, RL>::type V;
                        const V y = *reinterpret_cast<const V*>(src);
#pragma unroll
                        for (int q = 0; q < RL; ++q) v[gs][cg][q] = y[q];
                    } else if (sc - NX < n) {
                        load_run<T, RL, VEC>(src, valid, full, v[gs][cg]);
                    } else {
#pragma unroll
                        for (int q = 0; q < RL; ++q) v[gs][cg][q] = T(0);
                    }
                }
            }
        }
    };

    // stage the G stages of v and multiply; live: staged Y columns at or
    // beyond n are zeroed (the whole-step loads read column n - 1 there)
    auto stage_mul = [&](const T (&v)[G][NC / 4][RL], bool zero_dead) {
#pragma unroll
        for (int gs = 0; gs < G; ++gs) {
            // stage: column 4 cg + kk, rows RL*rl .. RL*rl + RL - 1
            wave_lds_fence();
#pragma unroll
            for (int cg = 0; cg < NC / 4; ++cg) {
                typedef typename VecOf<T, RL>::type V;
                const bool dead = zero_dead && cg >= NX / 4 && 4 * cg + kk - NX >= n;
                V x;
#pragma unroll
                for (int q = 0; q < RL; ++q) x[q] = dead ? T(0) : v[gs][cg][q];
                *reinterpret_cast<V*>(&tile[4 * cg + kk][RL * rl]) = x;
            }
            // read back in four blocks of 4*RL rows: X columns 16 ct + rl
            // and Y columns NX + 16 t + rl, rows 4*RL*h + RL*kk + q
            wave_lds_fence();
            typedef typename VecOf<T, RL>::type V;
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                V ys[NT16];
#pragma unroll
                for (int t = 0; t < NT16; ++t)
                    ys[t] = *reinterpret_cast<const V*>(&tile[NX + 16 * t + rl][4 * RL * h + RL * kk]);
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                    const V xs = *reinterpret_cast<const V*>(&tile[16 * ct + rl][4 * RL * h + RL * kk]);
#pragma unroll
                    for (int t = 0; t < NT16; ++t)
#pragma unroll
                        for (int q = 0; q < RL; ++q)
                            acc[ct][t] = M::op(xs[q], ys[t][q], acc[ct][t]);
                }
            }
        }
    };
    // whole steps: straight-line 16-byte loads (Y through the cache)
    auto load_full = [&](int64_t rb, T (&v)[G][NC / 4][RL]) {
        typedef typename VecOf<T, RL>::type V;
#pragma unroll
        for (int gs = 0; gs < G; ++gs) {
            const int64_t r = rb + gs * SR + RL * rl;
#pragma unroll
            for (int cg = 0; cg < NC / 4; ++cg) {
                const int sc = 4 * cg + kk;
                if (cg < NX / 4) {
                    load_run<T, RL, true>(X + r + (c0 + sc) * ldx, RL, true, v[gs][cg]);
                } else {
                    const int p = sc - NX < n ? sc - NX : n - 1;
                    const V y = *reinterpret_cast<const V*>(Y + r + (int64_t)p * ldy);
#pragma unroll
                    for (int q = 0; q < RL; ++q) v[gs][cg][q] = y[q];
                }
            }
        }
    };

    // pf and every step whole: the next step held in flight across the waits
    // for this one (the scheduling barriers keep its loads ahead of them;
    // the bounds branches of the general loop made those waits drain every
    // load).  Not with four stages per step, whose two steps do not fit the
    // registers.
    if (G <= 2 && pf && VEC && YC && wb1 > wb0 && c0 + NX <= ncols && (wb1 - wb0) % (G * SR) == 0) {
        const int64_t nit = (wb1 - wb0) / (G * SR);
        T va[G][NC / 4][RL], vb[G][NC / 4][RL];
        load_full(wb0, va);
        int64_t it = 0;
        for (; it + 2 < nit; it += 2) {
            load_full(wb0 + (it + 1) * G * SR, vb);
            __builtin_amdgcn_sched_barrier(0);
            stage_mul(va, true);
            load_full(wb0 + (it + 2) * G * SR, va);
            __builtin_amdgcn_sched_barrier(0);
            stage_mul(vb, true);
        }
        if (it + 1 < nit) {
            load_full(wb0 + (it + 1) * G * SR, vb);
            __builtin_amdgcn_sched_barrier(0);
            stage_mul(va, true);
            stage_mul(vb, true);
        } else {
            stage_mul(va, true);
        }
    } else if (wb1 > wb0) {
        const int64_t nit = (wb1 - wb0 + G * SR - 1) / (G * SR);
        T v[G][NC / 4][RL];
        load(wb0, v);
        for (int64_t it = 0; it < nit; ++it) {
            T vn[G][NC / 4][RL];
            if (it + 1 < nit) load(wb0 + (it + 1) * G * SR, vn);
            stage_mul(v, false);
#pragma unroll
            for (int gs = 0; gs < G; ++gs)
#pragma unroll
                for (int cg = 0; cg < NC / 4; ++cg)
#pragma unroll
                    for (int q = 0; q < RL; ++q) v[gs][cg][q] = vn[gs][cg][q];
        }
    }

    // one 16-column output tile at a time (global tile index blockIdx.x*CT + ct)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        if (ct > 0) __syncthreads();           // red is reused
        tn_finish<T, NT16, WK>(ncols, n, O, ldo, beta, (int64_t)blockIdx.x * CT + ct, s, nsl, part,
                               red, acc[ct], [](int kq, int r) { return Mfma<T>::mrow(kq, r); });
    }
}

// C := beta * C (zeros when beta == 0; C is then not read): the product of an
// empty k dimension.
template <typename T>
__global__ void fill_scale_kernel(int64_t m, int64_t n, T* __restrict__ C, int64_t ldc,
                                  T beta) {
    const int64_t total = m * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % m, p = e / m;
        C[i + p * ldc] = beta != T(0) ? beta * C[i + p * ldc] : T(0);
    }
}

// O (k x n, ld ldo) := transpose of Bt (n x k, ld ldb): a B given transposed,
// copied once into the workspace in the layout the TSM2R kernels read.
template <typename T>
__global__ void transpose_kernel(int64_t k, int64_t n, const T* __restrict__ Bt, int64_t ldb,
                                 T* __restrict__ O, int64_t ldo) {
    const int64_t total = k * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e % n, j = e / n;      // consecutive threads read along Bt's column
        O[j + p * ldo] = Bt[p + j * ldb];
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

template <typename T, int KS, int NT16, int RG, bool NTS>
static int rowtile_launch_st(const LaunchRT& L, bool vec, hipStream_t st) {
    // persistent grid: as many workgroups as fit at once (queried occupancy),
    // but no more than there are groups of 4 row tiles
    static const int occ_v = occupancy(rowtile_kernel<T, KS, NT16, RG, true, NTS>, 256);
    static const int occ_s = occupancy(rowtile_kernel<T, KS, NT16, RG, false, NTS>, 256);
    constexpr int64_t TR = 16 * (16 / (int64_t)sizeof(T)) * RG;
    const int64_t ntiles = (L.m + TR - 1) / TR;
    int64_t bx = (int64_t)L.cus * (vec ? occ_v : occ_s) / (L.blocks_y > 0 ? L.blocks_y : 1);
    const int64_t need = (ntiles + 3) / 4;
    if (bx > need) bx = need;
    if (L.blocks_x > 0 && bx > L.blocks_x) bx = L.blocks_x;
    if (bx < 1) bx = 1;
    dim3 grid((unsigned)bx, (unsigned)L.blocks_y), block(256);
    if (vec)
        TSM_LAUNCH((rowtile_kernel<T, KS, NT16, RG, true, NTS>), grid, block, 0, st, L.m,
                   L.kin, L.nout, (const T*)L.X, L.ldx, (const T*)L.Y, L.ys_in, L.ys_out,
                   (T*)L.O, L.ldo, (int64_t)L.cols_per_block, (T)L.beta);
    else
        TSM_LAUNCH((rowtile_kernel<T, KS, NT16, RG, false, NTS>), grid, block, 0, st, L.m,
                   L.kin, L.nout, (const T*)L.X, L.ldx, (const T*)L.Y, L.ys_in, L.ys_out,
                   (T*)L.O, L.ldo, (int64_t)L.cols_per_block, (T)L.beta);
    return 0;
}

// The stores of O are non-temporal (they fill whole cache lines: four columns
// x 256 bytes per wavefront instruction); TSM2X_RT_NTS=0 selects ordinary
// stores (measurement).  A next-tile register prefetch was measured and
// dropped: the extra waves it costs hid the latency better.
template <typename T, int KS, int NT16, int RG>
static int rowtile_launch(const LaunchRT& L, bool vec, hipStream_t st) {
    const char* e = std::getenv("TSM2X_RT_NTS");
    const bool nts = !(e && *e == '0');
    return nts ? rowtile_launch_st<T, KS, NT16, RG, true>(L, vec, st)
               : rowtile_launch_st<T, KS, NT16, RG, false>(L, vec, st);
}

template <typename T>
static int rowtile_dispatch(const LaunchRT& L, hipStream_t st) {
    const bool vec = aligned16(L.X) && aligned16(L.O) &&
                     ((L.ldx * (int64_t)sizeof(T)) % 16 == 0) &&
                     ((L.ldo * (int64_t)sizeof(T)) % 16 == 0);
    const bool wide = L.nout > 16;   // two 16-column tiles per pass
    switch (L.kp) {
        case 8: return wide ? rowtile_launch<T, 2, 2, 2>(L, vec, st) : rowtile_launch<T, 2, 1, 2>(L, vec, st);
        // k = 16 and 32 with n <= 16: one row group per lane (more waves per
        // SIMD) measured up to 16 % faster for float (k = 16) and 2.7 % on
        // average at k = 32, double the same or faster; for k = 8 and for the
        // wide instances with two groups it was slower
        case 16: return wide ? rowtile_launch<T, 4, 2, 2>(L, vec, st) : rowtile_launch<T, 4, 1, 1>(L, vec, st);
        case 32: return wide ? rowtile_launch<T, 8, 2, 1>(L, vec, st) : rowtile_launch<T, 8, 1, 1>(L, vec, st);
    }
    return 1;
}

int launch_rowtile(const LaunchRT& L, int dtype, hipStream_t st) {
    if (dtype == DT_F64) return rowtile_dispatch<double>(L, st);
    if (dtype == DT_F32) return rowtile_dispatch<float>(L, st);
    return 1;
}

template <typename T, int NT16, int G, int CT>
static int tn_launch(const LaunchTN& L, bool vec, hipStream_t st) {
    // L.groups 16-column tiles, a multiple of CT: CT of them per workgroup.
    // Y is read by every column group: cached loads when there are several
    // (YC), non-temporal ones when it is streamed once.
    const int64_t gx = L.groups / CT;
    dim3 grid((unsigned)gx, (unsigned)L.S), block(256);
    if (vec && gx > 1)
        TSM_LAUNCH((tn_kernel<T, NT16, G, CT, true, true>), grid, block, 0, st, L.R,
                           L.ncols, (int)L.n, (const T*)L.X, L.ldx, (const T*)L.Y, L.ldy, (T*)L.O,
                           L.ldo, L.rslice, L.part, L.beta, L.pf);
    else if (vec)
        TSM_LAUNCH((tn_kernel<T, NT16, G, CT, true, false>), grid, block, 0, st, L.R,
                           L.ncols, (int)L.n, (const T*)L.X, L.ldx, (const T*)L.Y, L.ldy, (T*)L.O,
                           L.ldo, L.rslice, L.part, L.beta, L.pf);
    else
        TSM_LAUNCH((tn_kernel<T, NT16, G, CT, false, false>), grid, block, 0, st, L.R,
                           L.ncols, (int)L.n, (const T*)L.X, L.ldx, (const T*)L.Y, L.ldy, (T*)L.O,
                           L.ldo, L.rslice, L.part, L.beta, L.pf);
    return 0;
}

template <typename T>
static int tn_dispatch(const LaunchTN& L, hipStream_t st) {
    const bool vec = aligned16(L.X) && aligned16(L.Y) &&
                     ((L.ldx * (int64_t)sizeof(T)) % 16 == 0) &&
                     ((L.ldy * (int64_t)sizeof(T)) % 16 == 0);
    // G stages of 16*RL rows per loop iteration (loads for the next iteration
    // are in flight while the current one is staged and multiplied); CT
    // 16-column output tiles per wavefront share each staged Y tile
    int rc = 1;
    const bool wide = L.n > 16;
    if (L.ct == 2) {
        rc = wide ? tn_launch<T, 2, 1, 2>(L, vec, st) : tn_launch<T, 1, 1, 2>(L, vec, st);
    } else if (L.rg == 4) {
        rc = wide ? tn_launch<T, 2, 4, 1>(L, vec, st) : tn_launch<T, 1, 4, 1>(L, vec, st);
    } else if (L.rg == 2) {
        rc = wide ? tn_launch<T, 2, 2, 1>(L, vec, st) : tn_launch<T, 1, 2, 1>(L, vec, st);
    } else {
        rc = wide ? tn_launch<T, 2, 1, 1>(L, vec, st) : tn_launch<T, 1, 1, 1>(L, vec, st);
    }
    if (rc || L.S <= 1) return rc;
    return launch_split_reduce(sizeof(T) == 8 ? DT_F64 : DT_F32, L.groups, L.S,
                               L.n <= 16 ? 16 : 32, 16, L.ncols, (int)L.n, L.part, L.O, L.ldo,
                               L.beta, st);
}

int launch_tn(const LaunchTN& L, int dtype, hipStream_t st) {
    if (dtype == DT_F64) return tn_dispatch<double>(L, st);
    if (dtype == DT_F32) return tn_dispatch<float>(L, st);
    return 1;
}

int launch_split_reduce(int dtype, int64_t groups, int S, int NP, int W, int64_t rows, int n,
                        const double* part, void* O, int64_t ldo, double beta, hipStream_t st) {
    const int64_t total = groups * NP * W;
    // a wavefront per output only where there are too few outputs to fill the
    // GPU with a thread each (2^18 outputs of 16 slices: the wavefront form's
    // lanes read 16 partials 2^21 bytes apart, and the precision-form TSM2R
    // at A 16384^2, n = 8 ran 14 % slower with 16 slices than with 15)
    const bool wide = S >= 16 && total < (int64_t)1 << 16;
    int64_t blocks = wide ? (total + 3) / 4 : (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    const dim3 g((unsigned)blocks), b(256);
    if (dtype == DT_F64) {
        if (wide)
            TSM_LAUNCH((split_reduce_kernel<double, true>), g, b, 0, st, groups, S, NP, W,
                               rows, n, part, (double*)O, ldo, beta);
        else
            TSM_LAUNCH((split_reduce_kernel<double, false>), g, b, 0, st, groups, S, NP,
                               W, rows, n, part, (double*)O, ldo, beta);
    } else {
        if (wide)
            TSM_LAUNCH((split_reduce_kernel<float, true>), g, b, 0, st, groups, S, NP, W,
                               rows, n, part, (float*)O, ldo, beta);
        else
            TSM_LAUNCH((split_reduce_kernel<float, false>), g, b, 0, st, groups, S, NP, W,
                               rows, n, part, (float*)O, ldo, beta);
    }
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

static dim3 flat_grid(int64_t total) {
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    return dim3((unsigned)blocks);
}

int launch_fill_scale(int64_t m, int64_t n, void* C, int64_t ldc, double beta, int dtype,
                      hipStream_t st) {
    const dim3 g = flat_grid(m * n);
    if (dtype == DT_F64)
        TSM_LAUNCH(fill_scale_kernel<double>, g, dim3(256), 0, st, m, n, (double*)C, ldc,
                           beta);
    else
        TSM_LAUNCH(fill_scale_kernel<float>, g, dim3(256), 0, st, m, n, (float*)C, ldc,
                           (float)beta);
    return 0;
}

int launch_transpose(int64_t k, int64_t n, const void* Bt, int64_t ldb, void* O, int64_t ldo,
                     int dtype, hipStream_t st) {
    const dim3 g = flat_grid(k * n);
    if (dtype == DT_F64)
        TSM_LAUNCH(transpose_kernel<double>, g, dim3(256), 0, st, k, n, (const double*)Bt,
                           ldb, (double*)O, ldo);
    else
        TSM_LAUNCH(transpose_kernel<float>, g, dim3(256), 0, st, k, n, (const float*)Bt,
                           ldb, (float*)O, ldo);
    return 0;
}

}  // namespace tsm
