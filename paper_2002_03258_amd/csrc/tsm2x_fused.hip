// Fused backward of a TSM2L product C = A*B (A m x k, B k x n, k, n <= 32;
// A plain, or the 16-bit planes of the precision form with float B, dC):
// one pass over the rows reads A and dC once and produces
//   dA = dC * B^T   (written row tile by row tile, a TSM2L product with B^T)
//   dB = A^T * dC   (accumulated in registers, reduced in double at the end)
// instead of two passes (dC, dA) + (A, dC).
//
// Per wavefront and 16*RL*RG-row tile, on the 16x16x4 matrix cores:
//  dA part (as rowtile): S[rl][kk] = B[16 t + rl, 4 st + kk] held in
//    registers, T[kk][rl] = dC[row(rl, q), 4 st + kk]; lane l gets
//    dA[row(rl, q), 16 t + mrow(kk, r)].
//  dB part (as tn): the tile's rows r = rb + RL*kk + q in steps of 4*RL,
//    S[rl][kk] = A[r, 16 ta + rl], T[kk][rl] = dC[r, 16 tb + rl]; lane l
//    accumulates dB[16 ta + mrow(kk, r), 16 tb + rl].
// A and dC are loaded once, in the 4-columns-x-256-bytes pattern; the dB
// part re-reads them from a wavefront-private LDS tile in its own layout.
// HBM sees A, dC and dA once each.  A persistent grid walks the row tiles;
// each workgroup leaves a double partial of dB, summed in workgroup order by
// split_reduce_kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tsm2x_device.h"
#include "tsm2x_half.h"
#include "tsm2x_internal.h"

namespace tsm {

// AF < 0: A holds T.  AF = FMT_BF16 / FMT_F16 (T = float): A is the 16-bit hi
// plane and, with ASPLIT, Alo the lo plane.  A only feeds dB, which is staged
// through LDS, so a lane loads 8 rows of a column (one 16-byte run per plane)
// and writes them, widened to float (hi + lo is exact in float), into the
// staged block they belong to.
template <typename T, int NTK, int NTN, int RG, bool VEC, int AF, bool ASPLIT>
__global__ __launch_bounds__(256) void tsm2l_bwd_kernel(
    int64_t m, int k, int n, const void* __restrict__ Av, const uint16_t* __restrict__ Alo,
    int64_t lda, const T* __restrict__ B, int64_t ldb, const T* __restrict__ dC, int64_t lddc,
    T* __restrict__ dA, int64_t ldda, double* __restrict__ part) {
    typedef Mfma<T> M;
    typedef typename M::acc Acc;
    typedef typename VecOf<T, 16 / sizeof(T)>::type V;
    constexpr int RL = 16 / (int)sizeof(T);
    constexpr int TR = 16 * RL * RG;
    constexpr int WPB = 4;
    constexpr int KSN = 4 * NTN;        // steps of 4 over n (dA part, dC columns)
    constexpr int KSK = 4 * NTK;        // steps of 4 over k (A columns)
    constexpr int NB = NTK * NTN;       // dB tiles
    constexpr int KP = 16 * NTK, NP = 16 * NTN;
    constexpr int SR = 16 * RL;         // rows per staged block
    constexpr int SROW = SR + RL;       // padded LDS column
    __shared__ __align__(16) T lds[WPB][KP + NP][SROW];
    __shared__ double red[WPB][WAVE][4 * NB];

    const int lane = threadIdx.x & (WAVE - 1);
    const int rl = lane & 15, kk = lane >> 4;
    const int w = threadIdx.x / WAVE;
    T (*tile)[SROW] = lds[w];
    static_assert(AF < 0 || (sizeof(T) == 4 && RL == 4), "16-bit A with float operands");

    // 16-bit A: rows r .. r + 7 of column c, one 16-byte run per plane
    auto loadA16 = [&](int64_t r, int c, bool full, uint32_t (&d)[2][4]) {
        const int64_t off = r + (int64_t)c * lda;
#pragma unroll
        for (int pl = 0; pl < (ASPLIT ? 2 : 1); ++pl) {
            const uint16_t* h = (pl == 0 ? (const uint16_t*)Av : Alo) + off;
            if (VEC && full) {
                const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(h));
#pragma unroll
                for (int e = 0; e < 4; ++e) d[pl][e] = v[e];
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t x0 = (2 * e < m - r) ? h[2 * e] : 0u;
                    const uint32_t x1 = (2 * e + 1 < m - r) ? h[2 * e + 1] : 0u;
                    d[pl][e] = x0 | (x1 << 16);
                }
            }
        }
    };

    // B^T as the S operand of the dA part: yv[st][t] = B[16 t + rl, 4 st + kk]
    T yv[KSN][NTK];
#pragma unroll
    for (int st = 0; st < KSN; ++st)
#pragma unroll
        for (int t = 0; t < NTK; ++t) {
            const int j = 16 * t + rl, p = 4 * st + kk;
            yv[st][t] = (j < k && p < n) ? B[j + (int64_t)p * ldb] : T(0);
        }

    Acc accb[NTK][NTN];
#pragma unroll
    for (int a = 0; a < NTK; ++a)
#pragma unroll
        for (int b = 0; b < NTN; ++b) accb[a][b] = Acc{0, 0, 0, 0};

    const int64_t ntiles = (m + TR - 1) / TR;
    for (int64_t tile_i = (int64_t)blockIdx.x * WPB + w; tile_i < ntiles;
         tile_i += (int64_t)gridDim.x * WPB) {
        const int64_t row0 = tile_i * TR;
        const bool full = (row0 + TR <= m);
        // rows RL*rl + q of each 16*RL-row block g, columns 4 st + kk: the
        // 4-columns-x-256-bytes load pattern, for dC and for A
        T xv[KSN][RG][RL], xa[AF < 0 ? KSK : 1][RG][RL];
        // 16-bit A: lane rl holds rows 8 rl .. 8 rl + 7 of the tile, i.e. rows
        // 8 (rl % 8) .. of staged block rl / 8
        uint32_t x16[AF < 0 ? 1 : KSK][2][4];
        if (AF >= 0) {
            const int64_t r = row0 + 8 * rl;
#pragma unroll
            for (int st = 0; st < KSK; ++st) {
                const int c = 4 * st + kk;
                if (c < k)
                    loadA16(r, c, full, x16[AF < 0 ? 0 : st]);
                else
#pragma unroll
                    for (int pl = 0; pl < 2; ++pl)
#pragma unroll
                        for (int e = 0; e < 4; ++e) x16[AF < 0 ? 0 : st][pl][e] = 0u;
            }
        }
#pragma unroll
        for (int g = 0; g < RG; ++g) {
            const int64_t r = row0 + SR * g + RL * rl;
#pragma unroll
            for (int st = 0; st < KSN; ++st) {
                const int p = 4 * st + kk;
                if (p < n)
                    load_run<T, RL, VEC>(dC + r + p * lddc, m - r, full, xv[st][g]);
                else
#pragma unroll
                    for (int q = 0; q < RL; ++q) xv[st][g][q] = T(0);
            }
            if (AF < 0) {
#pragma unroll
                for (int st = 0; st < KSK; ++st) {
                    const int c = 4 * st + kk;
                    if (c < k)
                        load_run<T, RL, VEC>((const T*)Av + r + (int64_t)c * lda, m - r, full,
                                             xa[AF < 0 ? st : 0][g]);
                    else
#pragma unroll
                        for (int q = 0; q < RL; ++q) xa[AF < 0 ? st : 0][g][q] = T(0);
                }
            }
        }
        // ---- dA = dC * B^T for this tile
        Acc acca[RG][RL][NTK];
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int q = 0; q < RL; ++q)
#pragma unroll
                for (int t = 0; t < NTK; ++t) acca[g][q][t] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int st = 0; st < KSN; ++st)
#pragma unroll
            for (int g = 0; g < RG; ++g)
#pragma unroll
                for (int q = 0; q < RL; ++q)
#pragma unroll
                    for (int t = 0; t < NTK; ++t)
                        acca[g][q][t] = M::op(yv[st][t], xv[st][g][q], acca[g][q][t]);
#pragma unroll
        for (int g = 0; g < RG; ++g) {
            const int64_t r = row0 + SR * g + RL * rl;
#pragma unroll
            for (int t = 0; t < NTK; ++t)
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int col = 16 * t + M::mrow(kk, rr);
                    if (col < k) {
                        T v[RL];
#pragma unroll
                        for (int q = 0; q < RL; ++q) v[q] = acca[g][q][t][rr];
                        store_run<T, RL, VEC>(dA + r + (int64_t)col * ldda, m - r, full, v);
                    }
                }
        }
        // ---- dB += A^T * dC over the same rows: stage each 16*RL-row block
        // in this wavefront's LDS tile [column][row] (A columns, then dC
        // columns) and read it back with the reduction index on kk
#pragma unroll
        for (int g = 0; g < RG; ++g) {
            wave_lds_fence();
            if (AF < 0) {
#pragma unroll
                for (int st = 0; st < KSK; ++st) {
                    V x;
#pragma unroll
                    for (int q = 0; q < RL; ++q) x[q] = xa[AF < 0 ? st : 0][g][q];
                    *reinterpret_cast<V*>(&tile[4 * st + kk][RL * rl]) = x;
                }
            } else if ((rl >> 3) == g) {
                // widen this lane's 8 rows (hi + lo is exact in float)
#pragma unroll
                for (int st = 0; st < KSK; ++st) {
                    V x0, x1;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t(&d)[2][4] = x16[AF < 0 ? 0 : st];
                        float a0 = half_val<(AF < 0 ? 0 : AF)>(d[0][q >> 1], q & 1);
                        float a1 = half_val<(AF < 0 ? 0 : AF)>(d[0][2 + (q >> 1)], q & 1);
                        if (ASPLIT) {
                            a0 += half_val<(AF < 0 ? 0 : AF)>(d[1][q >> 1], q & 1);
                            a1 += half_val<(AF < 0 ? 0 : AF)>(d[1][2 + (q >> 1)], q & 1);
                        }
                        x0[q] = (T)a0;
                        x1[q] = (T)a1;
                    }
                    *reinterpret_cast<V*>(&tile[4 * st + kk][8 * (rl & 7)]) = x0;
                    *reinterpret_cast<V*>(&tile[4 * st + kk][8 * (rl & 7) + 4]) = x1;
                }
            }
#pragma unroll
            for (int st = 0; st < KSN; ++st) {
                V x;
#pragma unroll
                for (int q = 0; q < RL; ++q) x[q] = xv[st][g][q];
                *reinterpret_cast<V*>(&tile[KP + 4 * st + kk][RL * rl]) = x;
            }
            wave_lds_fence();
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                V xs[NTK], ys[NTN];
#pragma unroll
                for (int a = 0; a < NTK; ++a)
                    xs[a] = *reinterpret_cast<const V*>(&tile[16 * a + rl][4 * RL * h + RL * kk]);
#pragma unroll
                for (int b = 0; b < NTN; ++b)
                    ys[b] = *reinterpret_cast<const V*>(&tile[KP + 16 * b + rl][4 * RL * h + RL * kk]);
#pragma unroll
                for (int q = 0; q < RL; ++q)
#pragma unroll
                    for (int a = 0; a < NTK; ++a)
#pragma unroll
                        for (int b = 0; b < NTN; ++b)
                            accb[a][b] = M::op(xs[a][q], ys[b][q], accb[a][b]);
            }
        }
    }

    // workgroup sum of dB in wave order; one partial per workgroup:
    // part[blk][p][c] with c = 16 a + mrow(kk, r), p = 16 b + rl
#pragma unroll
    for (int a = 0; a < NTK; ++a)
#pragma unroll
        for (int b = 0; b < NTN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[w][lane][(a * NTN + b) * 4 + r] = (double)accb[a][b][r];
    __syncthreads();
    constexpr int NV = 4 * NB;
    for (int e = threadIdx.x; e < WAVE * NV; e += 256) {
        const int ln = e / NV, vi = e % NV;
        double v = red[0][ln][vi];
#pragma unroll
        for (int ww = 1; ww < WPB; ++ww) v += red[ww][ln][vi];
        const int ab = vi / 4, r = vi % 4;
        const int a = ab / NTN, b = ab % NTN;
        const int c = 16 * a + M::mrow(ln >> 4, r);
        const int p = 16 * b + (ln & 15);
        part[((int64_t)blockIdx.x * NP + p) * KP + c] = v;
    }
}

template <typename K>
static int fused_occupancy(K kernel) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, 0) != hipSuccess || nb < 1)
        nb = 1;
    return nb;
}

template <typename T, int NTK, int NTN, int AF, bool ASPLIT>
static int bwd_launch(const LaunchBwd& L, int64_t* blocks_out, hipStream_t st, bool plan_only) {
    constexpr int RG = 2;
    constexpr int64_t TR = 16 * (16 / (int64_t)sizeof(T)) * RG;
    static const int occ = fused_occupancy(tsm2l_bwd_kernel<T, NTK, NTN, RG, true, AF, ASPLIT>);
    const int64_t ntiles = (L.m + TR - 1) / TR;
    int64_t bx = (int64_t)L.cus * occ;
    const int64_t need = (ntiles + 3) / 4;
    if (bx > need) bx = need;
    if (bx < 1) bx = 1;
    *blocks_out = bx;
    if (plan_only) return 0;
    // A: 16-byte runs of T, or of the 16-bit planes
    const bool avec = AF < 0 ? ((uintptr_t)L.A & 15u) == 0 && (L.lda * (int64_t)sizeof(T)) % 16 == 0
                             : ((uintptr_t)L.A & 15u) == 0 && L.lda % 8 == 0;
    const bool vec = avec && ((uintptr_t)L.dC & 15u) == 0 && ((uintptr_t)L.dA & 15u) == 0 &&
                     (L.lddc * (int64_t)sizeof(T)) % 16 == 0 &&
                     (L.ldda * (int64_t)sizeof(T)) % 16 == 0;
    const uint16_t* alo = ASPLIT ? (const uint16_t*)L.A + L.lda * L.k : nullptr;
    dim3 g((unsigned)bx), b(256);
    if (vec)
        TSM_LAUNCH((tsm2l_bwd_kernel<T, NTK, NTN, RG, true, AF, ASPLIT>), g, b, 0, st,
                           L.m, (int)L.k, (int)L.n, L.A, alo, L.lda, (const T*)L.B, L.ldb,
                           (const T*)L.dC, L.lddc, (T*)L.dA, L.ldda, L.part);
    else
        TSM_LAUNCH((tsm2l_bwd_kernel<T, NTK, NTN, RG, false, AF, ASPLIT>), g, b, 0, st,
                           L.m, (int)L.k, (int)L.n, L.A, alo, L.lda, (const T*)L.B, L.ldb,
                           (const T*)L.dC, L.lddc, (T*)L.dA, L.ldda, L.part);
    if (hipGetLastError() != hipSuccess) return 1;
    return launch_split_reduce(sizeof(T) == 8 ? DT_F64 : DT_F32, 1, (int)bx, 16 * NTN, 16 * NTK,
                               L.k, (int)L.n, L.part, L.dB, L.lddb, 0.0, st);
}

template <typename T, int AF, bool ASPLIT>
static int bwd_dispatch(const LaunchBwd& L, int64_t* blocks, hipStream_t st, bool plan_only) {
    if (L.k <= 16)
        return L.n <= 16 ? bwd_launch<T, 1, 1, AF, ASPLIT>(L, blocks, st, plan_only)
                         : bwd_launch<T, 1, 2, AF, ASPLIT>(L, blocks, st, plan_only);
    return L.n <= 16 ? bwd_launch<T, 2, 1, AF, ASPLIT>(L, blocks, st, plan_only)
                     : bwd_launch<T, 2, 2, AF, ASPLIT>(L, blocks, st, plan_only);
}

int launch_tsm2l_bwd(const LaunchBwd& L, int dtype, int64_t* blocks, hipStream_t st,
                     bool plan_only) {
    switch (dtype) {
        case DT_F64: return bwd_dispatch<double, -1, false>(L, blocks, st, plan_only);
        case DT_F32: return bwd_dispatch<float, -1, false>(L, blocks, st, plan_only);
        case DT_BF16: return bwd_dispatch<float, FMT_BF16, false>(L, blocks, st, plan_only);
        case DT_BF16_SPLIT: return bwd_dispatch<float, FMT_BF16, true>(L, blocks, st, plan_only);
        case DT_F16: return bwd_dispatch<float, FMT_F16, false>(L, blocks, st, plan_only);
        case DT_F16_SPLIT: return bwd_dispatch<float, FMT_F16, true>(L, blocks, st, plan_only);
    }
    return 1;
}

}  // namespace tsm
