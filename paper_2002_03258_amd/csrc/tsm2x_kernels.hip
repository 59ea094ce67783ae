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

#include "tsm2x_internal.h"

namespace tsm {

constexpr int WAVE = 64;

template <typename T, int N>
struct VecOf {
    typedef T type __attribute__((ext_vector_type(N)));
};

// RL consecutive elements starting at p: one 16-byte non-temporal load when
// the caller has checked alignment (VEC) and bounds (FULL); otherwise
// element-wise loads guarded by `valid` elements remaining.
template <typename T, int RL, bool VEC>
__device__ __forceinline__ void load_run(const T* __restrict__ p, int64_t valid,
                                         bool full, T (&out)[RL]) {
    if (VEC && full) {
        typedef typename VecOf<T, RL>::type V;
        V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
#pragma unroll
        for (int r = 0; r < RL; ++r) out[r] = v[r];
    } else {
#pragma unroll
        for (int r = 0; r < RL; ++r) out[r] = (r < valid) ? p[r] : T(0);
    }
}

template <typename T, int RL, bool VEC>
__device__ __forceinline__ void store_run(T* __restrict__ p, int64_t valid,
                                          bool full, const T (&v)[RL]) {
    if (VEC && full) {
        typedef typename VecOf<T, RL>::type V;
        V x;
#pragma unroll
        for (int r = 0; r < RL; ++r) x[r] = v[r];
        __builtin_nontemporal_store(x, reinterpret_cast<V*>(p));
    } else {
#pragma unroll
        for (int r = 0; r < RL; ++r)
            if (r < valid) p[r] = v[r];
    }
}

// Ticket protocol of the split reductions: every workgroup of a group
// publishes its double-precision partial, then takes a ticket; the one that
// draws the last ticket sums all partials in slice order and re-arms the
// counter for the next launch.
__device__ __forceinline__ bool take_last_ticket(unsigned* __restrict__ ticket,
                                                 int nslices) {
    __shared__ int s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned prev = atomicAdd(ticket, 1u);
        s_last = (prev == (unsigned)(nslices - 1)) ? 1 : 0;
    }
    __syncthreads();
    if (s_last) {
        __threadfence();
        return true;
    }
    return false;
}

__device__ __forceinline__ void rearm_ticket(unsigned* __restrict__ ticket) {
    if (threadIdx.x == 0) atomicExch(ticket, 0u);
}

// --------------------------------------------------------------------------
// tsm2r_nn
// --------------------------------------------------------------------------
template <typename T, int NP>
struct NNShape {
    static constexpr int RL = 16 / (int)sizeof(T);        // rows per lane
    static constexpr int TR = WAVE * RL;                  // rows per tile
    static constexpr int KC0 = 4096 / (NP * (int)sizeof(T));
    static constexpr int KC = KC0 < 64 ? KC0 : 64;        // B rows per chunk per wave
    static constexpr int PG0 = 16 / RL;                   // reduction column group
    static constexpr int PG = PG0 < NP ? PG0 : NP;
};

template <typename T, int NP, int WK, int U, bool VEC>
__global__ __launch_bounds__(WAVE * WK) void tsm2r_nn_kernel(
    int64_t m, int64_t k, int n, const T* __restrict__ A, int64_t lda,
    const T* __restrict__ B, int64_t ldb, T* __restrict__ C, int64_t ldc,
    int64_t kslice, double* __restrict__ part, unsigned* __restrict__ tickets) {
    typedef NNShape<T, NP> S_;
    constexpr int RL = S_::RL, TR = S_::TR, KC = S_::KC, PG = S_::PG;
    constexpr int NT = WAVE * WK;
    constexpr int VPT = (KC * NP) / WAVE;   // staged B values per thread
    static_assert((KC * NP) % WAVE == 0, "B chunk must split evenly");
    static_assert(2 * WK * KC * NP * (int)sizeof(T) <= 32768, "LDS budget");
    static_assert(WK * PG * TR * 8 <= 32768, "LDS budget");
    __shared__ __align__(16) unsigned char smem[32768];
    T* bst = reinterpret_cast<T*>(smem);   // [2][WK][KC][NP]

    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const int64_t tile = blockIdx.x;
    const int s = blockIdx.y, nsl = gridDim.y;
    const int64_t row0 = tile * TR;
    const int64_t lrow = row0 + (int64_t)lane * RL;
    const bool full = (row0 + TR <= m);
    const int64_t rvalid = m - lrow;   // rows this lane may touch (if < RL)
    const int64_t kb0 = (int64_t)s * kslice;
    const int64_t kb1 = (kb0 + kslice < k) ? kb0 + kslice : k;
    const int64_t lw = kslice / WK;
    const int64_t wk0 = kb0 + w * lw;
    const int64_t wk1 = (wk0 + lw < kb1) ? wk0 + lw : kb1;
    const int nchunks = (int)((lw + KC - 1) / KC);

    T acc[RL][NP];
#pragma unroll
    for (int r = 0; r < RL; ++r)
#pragma unroll
        for (int p = 0; p < NP; ++p) acc[r][p] = T(0);

    T breg[VPT];
    auto fetchB = [&](int c) {
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int v = threadIdx.x + i * NT;
            const int jj = v % KC, p = (v / KC) % NP, ww = v / (KC * NP);
            const int64_t wb = kb0 + ww * lw;
            const int64_t wend = (wb + lw < kb1) ? wb + lw : kb1;
            const int64_t j = wb + (int64_t)c * KC + jj;
            breg[i] = (p < n && j < wend) ? B[j + p * ldb] : T(0);
        }
    };
    auto storeB = [&](int buf) {
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int v = threadIdx.x + i * NT;
            const int jj = v % KC, p = (v / KC) % NP, ww = v / (KC * NP);
            bst[((buf * WK + ww) * KC + jj) * NP + p] = breg[i];
        }
    };

    // One column of A times one broadcast row of B (from LDS).
    auto fma_col = [&](const T (&a)[RL], const T* __restrict__ brow) {
        T b[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) b[p] = brow[p];
#pragma unroll
        for (int r = 0; r < RL; ++r)
#pragma unroll
            for (int p = 0; p < NP; ++p) acc[r][p] = __builtin_fma(a[r], b[p], acc[r][p]);
    };

    fetchB(0);
    storeB(0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunks) fetchB(c + 1);
        const int64_t c0 = wk0 + (int64_t)c * KC;
        const int64_t c1 = (c0 + KC < wk1) ? c0 + KC : wk1;
        if (c0 < c1) {
            const T* __restrict__ bs = bst + (buf * WK + w) * KC * NP;
            const T* __restrict__ Ap = A + lrow + c0 * lda;
            const int ncol = (int)(c1 - c0);
            const int ng = ncol / U;
            if (ng > 0) {
                T a[U][RL];
#pragma unroll
                for (int u = 0; u < U; ++u) load_run<T, RL, VEC>(Ap + u * lda, rvalid, full, a[u]);
                for (int g = 0; g < ng; ++g) {
                    T an[U][RL];
                    if (g + 1 < ng) {
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            load_run<T, RL, VEC>(Ap + ((g + 1) * U + u) * lda, rvalid, full, an[u]);
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) fma_col(a[u], bs + (g * U + u) * NP);
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int r = 0; r < RL; ++r) a[u][r] = an[u][r];
                }
            }
            for (int j = ng * U; j < ncol; ++j) {
                T a1[RL];
                load_run<T, RL, VEC>(Ap + j * lda, rvalid, full, a1);
                fma_col(a1, bs + j * NP);
            }
        }
        if (c + 1 < nchunks) storeB(buf ^ 1);
        __syncthreads();
    }

    // Sum the WK wavefronts' partials (double, wave order), PG columns at a time.
    double* red = reinterpret_cast<double*>(smem);   // [WK][PG][TR]
#pragma unroll
    for (int pg = 0; pg < NP; pg += PG) {
        if (pg < n) {
            __syncthreads();
#pragma unroll
            for (int pp = 0; pp < PG; ++pp)
#pragma unroll
                for (int r = 0; r < RL; ++r)
                    red[(w * PG + pp) * TR + lane * RL + r] = (double)acc[r][pg + pp];
            __syncthreads();
            for (int e = threadIdx.x; e < PG * TR; e += NT) {
                const int pp = e / TR, rr = e % TR;
                const int p = pg + pp;
                const int64_t row = row0 + rr;
                double v = red[pp * TR + rr];
#pragma unroll
                for (int ww = 1; ww < WK; ++ww) v += red[(ww * PG + pp) * TR + rr];
                if (p < n && row < m) {
                    if (nsl == 1)
                        C[row + p * ldc] = (T)v;
                    else
                        part[((tile * nsl + s) * NP + p) * TR + rr] = v;
                }
            }
        }
    }
    if (nsl == 1) return;
    if (!take_last_ticket(tickets + tile, nsl)) return;
    for (int e = threadIdx.x; e < n * TR; e += NT) {
        const int p = e / TR, rr = e % TR;
        const int64_t row = row0 + rr;
        if (row < m) {
            double v = 0.0;
            for (int s2 = 0; s2 < nsl; ++s2) v += part[((tile * nsl + s2) * NP + p) * TR + rr];
            C[row + p * ldc] = (T)v;
        }
    }
    rearm_ticket(tickets + tile);
}

// --------------------------------------------------------------------------
// rowtile: O(m x nout) = X(m x kin) * Y(kin x nout), kin <= KP <= 32.
// Y(ji, jo) = Y[ji * ys_in + jo * ys_out], so B and B^T are both views.
// --------------------------------------------------------------------------
template <typename T, int KP, int NC, bool VEC>
__global__ __launch_bounds__(256) void rowtile_kernel(
    int64_t m, int kin, int64_t nout, const T* __restrict__ X, int64_t ldx,
    const T* __restrict__ Y, int64_t ys_in, int64_t ys_out, T* __restrict__ O,
    int64_t ldo, int cols_per_block) {
    constexpr int RL = 16 / (int)sizeof(T);
    constexpr int TR = WAVE * RL;
    constexpr int WPB = 4;
    __shared__ __align__(16) T ys[(16384 / sizeof(T))];   // [cols_per_block][KP]

    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const int64_t colbase = (int64_t)blockIdx.y * cols_per_block;
    int ncb = cols_per_block;
    if (colbase + ncb > nout) ncb = (int)(nout - colbase);

    for (int e = threadIdx.x; e < cols_per_block * KP; e += 256) {
        const int jo = e / KP, ji = e % KP;
        const int64_t col = colbase + jo;
        ys[e] = (ji < kin && jo < ncb) ? Y[ji * ys_in + col * ys_out] : T(0);
    }
    __syncthreads();

    const int64_t ntiles = (m + TR - 1) / TR;
    for (int64_t tile = (int64_t)blockIdx.x * WPB + w; tile < ntiles;
         tile += (int64_t)gridDim.x * WPB) {
        const int64_t row0 = tile * TR;
        const int64_t lrow = row0 + (int64_t)lane * RL;
        const bool full = (row0 + TR <= m);
        const int64_t rvalid = m - lrow;
        T x[KP][RL];
#pragma unroll
        for (int ji = 0; ji < KP; ++ji) {
            if (ji < kin)
                load_run<T, RL, VEC>(X + lrow + ji * ldx, rvalid, full, x[ji]);
            else
#pragma unroll
                for (int r = 0; r < RL; ++r) x[ji][r] = T(0);
        }
        for (int jo = 0; jo < ncb; jo += NC) {
            T acc[NC][RL];
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) {
                const T* __restrict__ yr = ys + (jo + cc) * KP;
#pragma unroll
                for (int r = 0; r < RL; ++r) acc[cc][r] = T(0);
#pragma unroll
                for (int ji = 0; ji < KP; ++ji) {
                    const T b = yr[ji];
#pragma unroll
                    for (int r = 0; r < RL; ++r) acc[cc][r] = __builtin_fma(x[ji][r], b, acc[cc][r]);
                }
            }
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) {
                if (jo + cc < ncb)
                    store_run<T, RL, VEC>(O + lrow + (colbase + jo + cc) * ldo, rvalid, full, acc[cc]);
            }
        }
    }
}

// --------------------------------------------------------------------------
// tn: O(ncols x n) = X^T * Y, X (R x ncols), Y (R x n), both column-major.
// --------------------------------------------------------------------------
template <typename T, int NP, int J, bool VEC>
__global__ __launch_bounds__(256) void tn_kernel(
    int64_t R, int64_t ncols, int n, const T* __restrict__ X, int64_t ldx,
    const T* __restrict__ Y, int64_t ldy, T* __restrict__ O, int64_t ldo,
    int64_t rslice, double* __restrict__ part, unsigned* __restrict__ tickets) {
    constexpr int RL = 16 / (int)sizeof(T);
    constexpr int TR = WAVE * RL;
    constexpr int WPB = 4;
    constexpr int CPB = WPB * J;   // output rows (columns of X) per workgroup

    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const int64_t cgroup = blockIdx.x;
    const int64_t c0 = cgroup * CPB + (int64_t)w * J;
    const int s = blockIdx.y, nsl = gridDim.y;
    const int64_t rb0 = (int64_t)s * rslice;
    const int64_t rb1 = (rb0 + rslice < R) ? rb0 + rslice : R;

    T acc[J][NP];
#pragma unroll
    for (int c = 0; c < J; ++c)
#pragma unroll
        for (int p = 0; p < NP; ++p) acc[c][p] = T(0);

    for (int64_t r = rb0 + (int64_t)lane * RL; r < rb1 + (int64_t)lane * RL; r += TR) {
        // every lane runs the same trip count; lanes past rb1 load nothing
        const int64_t rv = rb1 - r;
        const bool full = rv >= RL;
        T y[NP][RL];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (p < n)
                load_run<T, RL, VEC>(Y + r + p * ldy, rv, full, y[p]);
            else
#pragma unroll
                for (int q = 0; q < RL; ++q) y[p][q] = T(0);
        }
#pragma unroll
        for (int c = 0; c < J; ++c) {
            T x[RL];
            if (c0 + c < ncols)
                load_run<T, RL, VEC>(X + r + (c0 + c) * ldx, rv, full, x);
            else
#pragma unroll
                for (int q = 0; q < RL; ++q) x[q] = T(0);
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int q = 0; q < RL; ++q) acc[c][p] = __builtin_fma(x[q], y[p][q], acc[c][p]);
        }
    }

    // Butterfly sum over the 64 lanes in double; lane 0's value is used.
    double tot[J][NP];
#pragma unroll
    for (int c = 0; c < J; ++c)
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            double v = (double)acc[c][p];
#pragma unroll
            for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
            tot[c][p] = v;
        }
    if (nsl == 1) {
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < J; ++c)
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    if (c0 + c < ncols && p < n) O[(c0 + c) + p * ldo] = (T)tot[c][p];
        }
        return;
    }
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < J; ++c)
#pragma unroll
            for (int p = 0; p < NP; ++p)
                part[((cgroup * nsl + s) * CPB + w * J + c) * NP + p] = tot[c][p];
    }
    if (!take_last_ticket(tickets + cgroup, nsl)) return;
    for (int e = threadIdx.x; e < CPB * NP; e += 256) {
        const int cc = e / NP, p = e % NP;
        const int64_t col = cgroup * CPB + cc;
        if (col < ncols && p < n) {
            double v = 0.0;
            for (int s2 = 0; s2 < nsl; ++s2) v += part[((cgroup * nsl + s2) * CPB + cc) * NP + p];
            O[col + p * ldo] = (T)v;
        }
    }
    rearm_ticket(tickets + cgroup);
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
static inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

template <typename T>
static int nn_dispatch(const LaunchNN& L, hipStream_t st) {
    const int np = L.np;
    const bool vec = aligned16(L.A) && ((L.lda * (int64_t)sizeof(T)) % 16 == 0);
    dim3 grid((unsigned)L.tiles, (unsigned)L.S), block(WAVE * 4);
#define TSM_NN(NPV, UV)                                                                           \
    if (np == NPV) {                                                                              \
        if (vec)                                                                                  \
            hipLaunchKernelGGL((tsm2r_nn_kernel<T, NPV, 4, UV, true>), grid, block, 0, st, L.m,    \
                               L.k, (int)L.n, (const T*)L.A, L.lda, (const T*)L.B, L.ldb,         \
                               (T*)L.C, L.ldc, L.kslice, L.part, L.tickets);                      \
        else                                                                                      \
            hipLaunchKernelGGL((tsm2r_nn_kernel<T, NPV, 4, UV, false>), grid, block, 0, st, L.m,   \
                               L.k, (int)L.n, (const T*)L.A, L.lda, (const T*)L.B, L.ldb,         \
                               (T*)L.C, L.ldc, L.kslice, L.part, L.tickets);                      \
        return 0;                                                                                 \
    }
    TSM_NN(1, 8)
    TSM_NN(2, 8)
    TSM_NN(4, 8)
    TSM_NN(8, 8)
    TSM_NN(16, 8)
    TSM_NN(32, 4)
#undef TSM_NN
    return 1;
}

int launch_tsm2r_nn(const LaunchNN& L, int dtype, hipStream_t st) {
    if (dtype == DT_F64) return nn_dispatch<double>(L, st);
    if (dtype == DT_F32) return nn_dispatch<float>(L, st);
    return 1;
}

template <typename T>
static int rowtile_dispatch(const LaunchRT& L, hipStream_t st) {
    const bool vec = aligned16(L.X) && aligned16(L.O) &&
                     ((L.ldx * (int64_t)sizeof(T)) % 16 == 0) &&
                     ((L.ldo * (int64_t)sizeof(T)) % 16 == 0);
    dim3 grid((unsigned)L.blocks_x, (unsigned)L.blocks_y), block(256);
#define TSM_RT(KPV, NCV)                                                                         \
    if (L.kp == KPV) {                                                                           \
        if (vec)                                                                                 \
            hipLaunchKernelGGL((rowtile_kernel<T, KPV, NCV, true>), grid, block, 0, st, L.m,      \
                               L.kin, L.nout, (const T*)L.X, L.ldx, (const T*)L.Y, L.ys_in,      \
                               L.ys_out, (T*)L.O, L.ldo, L.cols_per_block);                      \
        else                                                                                     \
            hipLaunchKernelGGL((rowtile_kernel<T, KPV, NCV, false>), grid, block, 0, st, L.m,     \
                               L.kin, L.nout, (const T*)L.X, L.ldx, (const T*)L.Y, L.ys_in,      \
                               L.ys_out, (T*)L.O, L.ldo, L.cols_per_block);                      \
        return 0;                                                                                \
    }
    TSM_RT(8, 8)
    TSM_RT(16, 8)
    TSM_RT(32, 4)
#undef TSM_RT
    return 1;
}

int launch_rowtile(const LaunchRT& L, int dtype, hipStream_t st) {
    if (dtype == DT_F64) return rowtile_dispatch<double>(L, st);
    if (dtype == DT_F32) return rowtile_dispatch<float>(L, st);
    return 1;
}

template <typename T>
static int tn_dispatch(const LaunchTN& L, hipStream_t st) {
    const bool vec = aligned16(L.X) && aligned16(L.Y) &&
                     ((L.ldx * (int64_t)sizeof(T)) % 16 == 0) &&
                     ((L.ldy * (int64_t)sizeof(T)) % 16 == 0);
    dim3 grid((unsigned)L.groups, (unsigned)L.S), block(256);
#define TSM_TN(NPV, JV)                                                                          \
    if (L.np == NPV) {                                                                           \
        if (vec)                                                                                 \
            hipLaunchKernelGGL((tn_kernel<T, NPV, JV, true>), grid, block, 0, st, L.R, L.ncols,   \
                               (int)L.n, (const T*)L.X, L.ldx, (const T*)L.Y, L.ldy, (T*)L.O,    \
                               L.ldo, L.rslice, L.part, L.tickets);                              \
        else                                                                                     \
            hipLaunchKernelGGL((tn_kernel<T, NPV, JV, false>), grid, block, 0, st, L.R, L.ncols,  \
                               (int)L.n, (const T*)L.X, L.ldx, (const T*)L.Y, L.ldy, (T*)L.O,    \
                               L.ldo, L.rslice, L.part, L.tickets);                              \
        return 0;                                                                                \
    }
    TSM_TN(1, TN_J(1))
    TSM_TN(2, TN_J(2))
    TSM_TN(4, TN_J(4))
    TSM_TN(8, TN_J(8))
    TSM_TN(16, TN_J(16))
    TSM_TN(32, TN_J(32))
#undef TSM_TN
    return 1;
}

int launch_tn(const LaunchTN& L, int dtype, hipStream_t st) {
    if (dtype == DT_F64) return tn_dispatch<double>(L, st);
    if (dtype == DT_F32) return tn_dispatch<float>(L, st);
    return 1;
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
