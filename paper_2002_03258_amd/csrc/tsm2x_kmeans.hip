// K-means assignment on the matrix cores.  K-means is the paper's first
// example of a tall-and-skinny GEMM user (Introduction): many points, few
// centroids.
//
// Points X (m x k, column-major: point i is row i) and centroids Mu (k x n,
// column-major: centroid c is column c).  For each point
//   label[i] = the smallest c with the smallest ||x_i - mu_c||^2,
//   dist[i]  = that squared distance (optional),
// reading X once per panel of centroids and writing only the labels and
// distances, never the m x n distance matrix.  The distance expands to
// ||x||^2 - 2 x.mu_c + ||mu_c||^2:
//  - the cross terms G = X * Mu are a TSM2L product on the 16x16x4 matrix
//    cores in the rowtile layout: Mu is the S operand
//    (S[rl][kk] = Mu[kc + 4 st + kk, c0 + 16 t + rl]), X enters through T as
//    the lane's 16-byte row runs, and lane l holds
//    G[row(rl, q), c0 + 16 t + mrow(kk, r)].  k is taken in chunks of 4*KS
//    columns, so any k works;
//  - ||mu_c||^2 comes from kmeans_norms_kernel (one value per centroid);
//  - ||x||^2 is summed from the same registers of X;
//  - the minimum over c of ||mu_c||^2 - 2 G[i, c] is taken within a lane
//    (its columns are visited in increasing c, so the first strict minimum
//    is the smallest index among equal values), then across the four lanes
//    (kk = 0..3) that hold the same rows: a reduce-scatter that leaves each
//    lane the result of RG*RL/4 of the RG*RL rows, which it stores.  NaN never
//    compares smaller; a row with no finite non-NaN value gets label 0 and a
//    NaN distance.
// More than 16*NT16 centroids are taken in panels with a running minimum
// (X is read once per panel).  A persistent grid walks the row tiles.
//
// Row-major X (ROWX: point i at X + i*ldx, its k values contiguous): a
// wavefront's tile is then one contiguous range, loaded in consecutive
// 16-byte pieces (1 KB per instruction) and written into a wavefront-private
// LDS tile [feature][point], from which each lane reads back the same
// registers as in the column-major case.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tsm2x_device.h"
#include "tsm2x_internal.h"

namespace tsm {

// a*b + c rounded once, in T
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__global__ void kmeans_norms_kernel(int k, int n, const T* __restrict__ Mu, int64_t ldm,
                                    T* __restrict__ mu2) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    T s = T(0);
    for (int j = 0; j < k; ++j) {
        const T v = Mu[j + (int64_t)c * ldm];
        s = fma_t(v, v, s);
    }
    mu2[c] = s;
}

// (v, c) replaces (bv, bc) when smaller, or equal with a smaller index
template <typename T>
__device__ __forceinline__ void take_min(T v, int c, T& bv, int& bc) {
    if (v < bv || (v == bv && c < bc)) {
        bv = v;
        bc = c;
    }
}

// Exchange between partner lanes by the gfx950 lane-swap instructions.
// S32: v_permlane32_swap, after which x = [x lanes 0-31, y lanes 0-31] and
// y = [x lanes 32-63, y lanes 32-63] (partner l ^ 32).  Otherwise
// v_permlane16_swap, which trades the odd 16-lane rows of x with the even
// rows of y (partner l ^ 16).
template <bool S32>
__device__ __forceinline__ void swap_u32(uint32_t& x, uint32_t& y) {
    if (S32) {
        const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
        x = r[0];
        y = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
        x = r[0];
        y = r[1];
    }
}
template <bool S32, typename V>
__device__ __forceinline__ void swap_lanes(V& x, V& y) {
    static_assert(sizeof(V) == 4 || sizeof(V) == 8, "32- or 64-bit values");
    if constexpr (sizeof(V) == 4) {
        uint32_t a = __builtin_bit_cast(uint32_t, x), b = __builtin_bit_cast(uint32_t, y);
        swap_u32<S32>(a, b);
        x = __builtin_bit_cast(V, a);
        y = __builtin_bit_cast(V, b);
    } else {
        uint2 a = __builtin_bit_cast(uint2, x), b = __builtin_bit_cast(uint2, y);
        swap_u32<S32>(a.x, b.x);
        swap_u32<S32>(a.y, b.y);
        x = __builtin_bit_cast(V, a);
        y = __builtin_bit_cast(V, b);
    }
}

// One step of the reduce-scatter over partner lanes (l ^ 32 for S32, else
// l ^ 16): of the 2H rows (v, c, x) each lane holds, the lower lane of a pair
// keeps rows 0 .. H-1 and the upper lane rows H .. 2H-1.  After swapping
// rows i and H + i, both values of the kept row are in each lane (the lower
// lane's first); they are combined into row i, so rows 0 .. H-1 of the
// arrays hold the kept half.
template <typename T, int H, bool S32>
__device__ __forceinline__ void scatter_step(T (&v)[2 * H], int (&c)[2 * H], T (&x)[2 * H]) {
#pragma unroll
    for (int i = 0; i < H; ++i) {
        swap_lanes<S32>(v[i], v[H + i]);
        swap_lanes<S32>(c[i], c[H + i]);
        swap_lanes<S32>(x[i], x[H + i]);
        take_min(v[H + i], c[H + i], v[i], c[i]);
        x[i] = x[i] + x[H + i];
    }
}

template <typename T, int KS, int NT16, int RG, bool VEC, bool RES, bool ROWX>
__global__ __launch_bounds__(256) void kmeans_assign_kernel(
    int64_t m, int k, int n, const T* __restrict__ X, int64_t ldx, const T* __restrict__ Mu,
    int64_t ldm, const T* __restrict__ mu2, int32_t* __restrict__ labels,
    T* __restrict__ dist) {
    typedef Mfma<T> M;
    typedef typename M::acc Acc;
    constexpr int RL = 16 / (int)sizeof(T);
    constexpr int TR = 16 * RL * RG;
    constexpr int R = RG * RL;          // rows of a lane: e = g * RL + q
    constexpr int WPB = 4;
    constexpr int CW = 16 * NT16;       // centroids per panel
    constexpr int KC = 4 * KS;          // columns of X per chunk
    constexpr int NONE = 0x7fffffff;
    static_assert(R % 4 == 0 && RL % (R / 4) == 0, "each lane of a row keeps whole rows");
    constexpr int NP = RG * KS;         // 16-byte pieces per lane and tile (either layout)
    constexpr int PPP = KC / RL;        // pieces per point of a chunk (ROWX)
    constexpr int SROW = TR + RL;       // padded LDS row (ROWX)
    __shared__ __align__(16) T lds[ROWX ? WPB : 1][ROWX ? KC : 1][ROWX ? SROW : 1];
    const T inf = __builtin_inf();

    const int lane = threadIdx.x & (WAVE - 1);
    const int rl = lane & 15, kk = lane >> 4;
    const int w = threadIdx.x / WAVE;
    typedef T Raw[NP][RL];

    T yv[KS][NT16], cn[NT16][4];
    auto loadY = [&](int kc, int c0) {
#pragma unroll
        for (int st = 0; st < KS; ++st)
#pragma unroll
            for (int t = 0; t < NT16; ++t) {
                const int j = kc + 4 * st + kk, c = c0 + 16 * t + rl;
                yv[st][t] = (j < k && c < n) ? Mu[j + (int64_t)c * ldm] : T(0);
            }
    };
    auto loadN = [&](int c0) {
#pragma unroll
        for (int t = 0; t < NT16; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = c0 + 16 * t + M::mrow(kk, r);
                cn[t][r] = c < n ? mu2[c] : T(__builtin_nan(""));   // never a minimum
            }
    };
    // fetch: this lane's pieces of a tile's chunk kc .. kc + KC - 1 of X.
    // Column-major: piece st*RG + g is rows RL*rl + q of block g, column
    // kc + 4 st + kk.  Row-major: piece i is the i-th of the lane's 16-byte
    // pieces in the tile's (point, feature) order.
    auto fetch = [&](int64_t tile, int kc, Raw& raw) {
        const int64_t row0 = tile * TR;
        const bool full = row0 + TR <= m;
        if (!ROWX) {
#pragma unroll
            for (int st = 0; st < KS; ++st) {
                const int j = kc + 4 * st + kk;
#pragma unroll
                for (int g = 0; g < RG; ++g) {
                    const int64_t r = row0 + 16 * RL * g + RL * rl;
                    if (j < k)
                        load_run<T, RL, VEC>(X + r + (int64_t)j * ldx, m - r, full,
                                             raw[st * RG + g]);
                    else
#pragma unroll
                        for (int q = 0; q < RL; ++q) raw[st * RG + g][q] = T(0);
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const int pc = lane + WAVE * i;
                const int p = pc / PPP, f0 = kc + (pc % PPP) * RL;
                const int64_t pt = row0 + p;
                const T* src = X + pt * ldx + f0;
                if (VEC && pt < m && f0 + RL <= k) {
                    typedef typename VecOf<T, RL>::type V;
                    const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(src));
#pragma unroll
                    for (int e = 0; e < RL; ++e) raw[i][e] = v[e];
                } else {
#pragma unroll
                    for (int e = 0; e < RL; ++e)
                        raw[i][e] = (pt < m && f0 + e < k) ? src[e] : T(0);
                }
            }
        }
    };
    // stage: the registers of the MFMA layout, xv[st][g][q] = X[row, kc + 4 st + kk]
    // with row = row0 + 16*RL*g + RL*rl + q
    auto stage = [&](const Raw& raw, T (&xv)[KS][RG][RL]) {
        if constexpr (!ROWX) {
#pragma unroll
            for (int st = 0; st < KS; ++st)
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int q = 0; q < RL; ++q) xv[st][g][q] = raw[st * RG + g][q];
            return;
        } else {
        T (*tl)[SROW] = lds[w];
        wave_lds_fence();
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int pc = lane + WAVE * i;
            const int p = pc / PPP, f = (pc % PPP) * RL;
#pragma unroll
            for (int e = 0; e < RL; ++e) tl[f + e][p] = raw[i][e];
        }
        wave_lds_fence();
        typedef typename VecOf<T, RL>::type V;
#pragma unroll
        for (int st = 0; st < KS; ++st)
#pragma unroll
            for (int g = 0; g < RG; ++g) {
                const V v = *reinterpret_cast<const V*>(&tl[4 * st + kk][16 * RL * g + RL * rl]);
#pragma unroll
                for (int q = 0; q < RL; ++q) xv[st][g][q] = v[q];
            }
        }
    };
    auto accumulate = [&](const T (&xv)[KS][RG][RL], Acc (&acc)[RG][RL][NT16], T (&x2)[R],
                          bool norms) {
        if (norms) {
#pragma unroll
            for (int st = 0; st < KS; ++st)
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int q = 0; q < RL; ++q)
                        x2[g * RL + q] = fma_t(xv[st][g][q], xv[st][g][q], x2[g * RL + q]);
        }
#pragma unroll
        for (int st = 0; st < KS; ++st)
#pragma unroll
            for (int g = 0; g < RG; ++g)
#pragma unroll
                for (int q = 0; q < RL; ++q)
#pragma unroll
                    for (int t = 0; t < NT16; ++t)
                        acc[g][q][t] = M::op(yv[st][t], xv[st][g][q], acc[g][q][t]);
    };
    // this lane's part of a panel, ||mu_c||^2 - 2 G[i, c], in increasing c
    // (mrow grows with r): the first strict minimum is the smallest index
    auto panel_min = [&](const Acc (&acc)[RG][RL][NT16], int c0, T (&bv)[R], int (&bc)[R]) {
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int q = 0; q < RL; ++q)
#pragma unroll
                for (int t = 0; t < NT16; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const T sv = fma_t(T(-2), (T)acc[g][q][t][r], cn[t][r]);
                        const bool lt = sv < bv[g * RL + q];
                        bv[g * RL + q] = lt ? sv : bv[g * RL + q];
                        bc[g * RL + q] = lt ? c0 + 16 * t + M::mrow(kk, r) : bc[g * RL + q];
                    }
    };
    // the four lanes of a row (rl, rl + 16, rl + 32, rl + 48): after the two
    // steps lane kk holds rows e = (kk >> 1) * R/2 + (kk & 1) * R/4 + i,
    // i < R/4 (e = g * RL + q: point row0 + 16*RL*g + RL*rl + q; the R/4
    // rows stay in one g because R/4 divides RL), and stores them
    auto finish = [&](int64_t tile, T (&bv)[R], int (&bc)[R], T (&x2)[R]) {
        const int64_t row0 = tile * TR;
        const bool full = row0 + TR <= m;
        scatter_step<T, R / 2, true>(bv, bc, x2);
        T v2[R / 2], x22[R / 2];
        int c2[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            v2[i] = bv[i];
            c2[i] = bc[i];
            x22[i] = x2[i];
        }
        scatter_step<T, R / 4, false>(v2, c2, x22);
        constexpr int NQ = R / 4;
        constexpr int HR = R / 2;
        const int e0 = (kk >> 1) * HR + (kk & 1) * NQ;
        const int64_t r = row0 + 16 * RL * (e0 / RL) + RL * rl + e0 % RL;
        int32_t lab[NQ];
        T d[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const bool none = c2[i] == NONE;
            lab[i] = none ? 0 : c2[i];
            const T v = x22[i] + v2[i];
            d[i] = none ? T(__builtin_nan("")) : (v < T(0) ? T(0) : v);
        }
        store_run<int32_t, NQ, VEC, false>(labels + r, m - r, full, lab);
        if (dist) store_run<T, NQ, VEC, false>(dist + r, m - r, full, d);
    };
    auto init = [&](T (&bv)[R], int (&bc)[R], T (&x2)[R]) {
#pragma unroll
        for (int e = 0; e < R; ++e) {
            bv[e] = inf;
            bc[e] = NONE;
            x2[e] = T(0);
        }
    };

    const int64_t ntiles = (m + TR - 1) / TR;
    const int64_t stride = (int64_t)gridDim.x * WPB;
    int64_t tile = (int64_t)blockIdx.x * WPB + w;
    if (RES) {
        loadY(0, 0);
        loadN(0);
        Raw cur;
        if (tile < ntiles) fetch(tile, 0, cur);
        for (; tile < ntiles; tile += stride) {
            const bool more = tile + stride < ntiles;
            Raw nxt;
            if (more) fetch(tile + stride, 0, nxt);
            T xv[KS][RG][RL];
            stage(cur, xv);
            T bv[R], x2[R];
            int bc[R];
            init(bv, bc, x2);
            Acc acc[RG][RL][NT16];
#pragma unroll
            for (int g = 0; g < RG; ++g)
#pragma unroll
                for (int q = 0; q < RL; ++q)
#pragma unroll
                    for (int t = 0; t < NT16; ++t) acc[g][q][t] = Acc{0, 0, 0, 0};
            accumulate(xv, acc, x2, true);
            panel_min(acc, 0, bv, bc);
            finish(tile, bv, bc, x2);
            if (more) {
#pragma unroll
                for (int i = 0; i < NP; ++i)
#pragma unroll
                    for (int e = 0; e < RL; ++e) cur[i][e] = nxt[i][e];
            }
        }
        return;
    }
    for (; tile < ntiles; tile += stride) {
        T bv[R], x2[R];
        int bc[R];
        init(bv, bc, x2);
        for (int c0 = 0; c0 < n; c0 += CW) {
            loadN(c0);
            Acc acc[RG][RL][NT16];
#pragma unroll
            for (int g = 0; g < RG; ++g)
#pragma unroll
                for (int q = 0; q < RL; ++q)
#pragma unroll
                    for (int t = 0; t < NT16; ++t) acc[g][q][t] = Acc{0, 0, 0, 0};
            for (int kc = 0; kc < k; kc += KC) {
                loadY(kc, c0);
                Raw raw;
                fetch(tile, kc, raw);
                T xv[KS][RG][RL];
                stage(raw, xv);
                accumulate(xv, acc, x2, c0 == 0);
            }
            panel_min(acc, c0, bv, bc);
        }
        finish(tile, bv, bc, x2);
    }
}

template <typename K>
static int km_occupancy(K kernel) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, 0) != hipSuccess || nb < 1)
        nb = 1;
    return nb;
}

template <typename T, int KS, int NT16, bool RES, bool ROWX>
static int km_launch(const LaunchKM& L, hipStream_t st) {
    // row groups per lane: one for float (64-point wave tiles) keeps the
    // registers at four waves per SIMD, which measured 10 % faster on
    // row-major points than two groups at two waves; double needs two so
    // that each of the four lanes of a row keeps at least one row
    constexpr int RG = sizeof(T) == 4 ? 1 : 2;
    constexpr int64_t TR = 16 * (16 / (int64_t)sizeof(T)) * RG;
    static const int occ = km_occupancy(kmeans_assign_kernel<T, KS, NT16, RG, true, RES, ROWX>);
    const int64_t ntiles = (L.m + TR - 1) / TR;
    int64_t bx = (int64_t)L.cus * occ;
    const int64_t need = (ntiles + 3) / 4;
    if (bx > need) bx = need;
    if (bx < 1) bx = 1;
    const unsigned nb = (unsigned)((L.n + 255) / 256);
    TSM_LAUNCH(kmeans_norms_kernel<T>, dim3(nb), dim3(256), 0, st, (int)L.k, (int)L.n,
                       (const T*)L.Mu, L.ldm, (T*)L.mu2);
    if (hipGetLastError() != hipSuccess) return 1;
    // 16-byte runs of X (row-major: the last piece of a point whose k values
    // end inside it is read element-wise) and of the outputs
    const int es = (int)sizeof(T);
    const bool vec = ((uintptr_t)L.X & 15u) == 0 && (L.ldx * es) % 16 == 0 &&
                     ((uintptr_t)L.labels & 15u) == 0 && ((uintptr_t)L.dist & 15u) == 0;
    dim3 g((unsigned)bx), b(256);
    if (vec)
        TSM_LAUNCH((kmeans_assign_kernel<T, KS, NT16, RG, true, RES, ROWX>), g, b, 0, st, L.m,
                           (int)L.k, (int)L.n, (const T*)L.X, L.ldx, (const T*)L.Mu, L.ldm,
                           (const T*)L.mu2, L.labels, (T*)L.dist);
    else
        TSM_LAUNCH((kmeans_assign_kernel<T, KS, NT16, RG, false, RES, ROWX>), g, b, 0, st, L.m,
                           (int)L.k, (int)L.n, (const T*)L.X, L.ldx, (const T*)L.Mu, L.ldm,
                           (const T*)L.mu2, L.labels, (T*)L.dist);
    return hipGetLastError() != hipSuccess;
}

template <typename T, int KS, int NT16>
static int km_res(const LaunchKM& L, hipStream_t st) {
    const bool res = L.k <= 4 * KS && L.n <= 16 * NT16;
    if (L.x_rowmajor)
        return res ? km_launch<T, KS, NT16, true, true>(L, st)
                   : km_launch<T, KS, NT16, false, true>(L, st);
    return res ? km_launch<T, KS, NT16, true, false>(L, st)
               : km_launch<T, KS, NT16, false, false>(L, st);
}

template <typename T>
static int km_dispatch(const LaunchKM& L, hipStream_t st) {
    const bool wide = L.n > 16;
    if (L.k <= 8) return wide ? km_res<T, 2, 2>(L, st) : km_res<T, 2, 1>(L, st);
    if (L.k <= 16) return wide ? km_res<T, 4, 2>(L, st) : km_res<T, 4, 1>(L, st);
    return wide ? km_res<T, 8, 2>(L, st) : km_res<T, 8, 1>(L, st);
}

int launch_kmeans_assign(const LaunchKM& L, int dtype, hipStream_t st) {
    if (dtype == DT_F64) return km_dispatch<double>(L, st);
    if (dtype == DT_F32) return km_dispatch<float>(L, st);
    return 1;
}

}  // namespace tsm
