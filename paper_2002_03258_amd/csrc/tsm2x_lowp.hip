// Low-precision storage form of A for TSM2R on gfx950.
//
//  split_kernel   hi = RNE(a), lo = RNE(a - hi) for a float matrix A, written
//                 as bfloat16 or binary16 planes (a - hi is exact in float).
//
//  tsm2r_lp       C = A*B with A given by its hi plane (single form) or its
//                 hi and lo planes (split form, value hi + lo), B and C float.
//                 The bulk arithmetic runs on the 16x16x32 bf16/f16 matrix
//                 cores with float accumulation; the per-workgroup and
//                 cross-workgroup sums are double, as in the float kernels.
//
// Dataflow (same outer-product form as the float TSM2R kernel): C^T = B^T*A^T
// with the MFMA "S" operand a 16 x 32 block of B^T and the "T" operand a
// 32 x 16 block of A^T.  The T operand wants, per lane, eight consecutive
// k values of ONE row, but a column-major A is contiguous along rows; a lane
// therefore loads 16 bytes (8 rows) from each of 8 columns j0 + 8*kk + i,
// and transposes that 8 x 8 block of 16-bit values in registers (one byte
// permute per output dword) so that MFMA instance q gets row 8*rl + q.
// Every element of A is still loaded exactly once with 16-byte loads.
//
// B is float; once per call it is split into bf16/f16 terms B1 + B2 + B3
// (b1 = RNE(b), b2 = RNE(b - b1), b3 = RNE(b - b1 - b2), each difference
// exact in float) by split_b_kernel, which writes them to the workspace
// already packed as the MFMA "S" operand: every row tile re-reads B, and the
// terms are then one cached 16-byte load per lane and term instead of a split
// in every chunk of every tile.  Three terms reproduce a float B (bf16:
// |b - b1 - b2 - b3| <= 2^-24 |b|; binary16 keeps 11 bits per term).  Products
// kept:
//   single:  hi*(B1 + B2 + B3)
//   split:   hi*(B1 + B2 + B3) + lo*(B1 + B2)
// The split form drops lo*B3 only: |lo| <= 2^-8 |a| and |B3| <= 2^-16 |b| for
// bf16 (2^-11 and 2^-22 for binary16), so it is below 2^-24 |a||b|.  Against
// the stored values hi (+ lo) the arithmetic error is then that of float
// accumulation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdlib>
#include <type_traits>

#include "tsm2x_device.h"
#include "tsm2x_half.h"
#include "tsm2x_internal.h"

namespace tsm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <int FMT>
__device__ __forceinline__ f32x4 mfma32(u32x4 s, u32x4 t, f32x4 d) {
    if (FMT == FMT_BF16)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, s),
                                                       __builtin_bit_cast(bf16x8, t), d, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, s),
                                                  __builtin_bit_cast(f16x8, t), d, 0, 0, 0);
}

// Eight floats as three bf16 terms t1 + t2 + t3, packed two per dword
// (value 2d in the low half of dword d): t1 = RNE(y), t2 = RNE(y - t1),
// t3 = RNE(y - t1 - t2), each difference exact in float (the same terms as
// the split of B; the hardware conversion rounds to nearest even).
__device__ __forceinline__ void bf16_terms8(const float (&y)[8], u32x4& t1, u32x4& t2, u32x4& t3) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    auto pk = [](float a, float b) {
        const bf16x2 v = {(__bf16)a, (__bf16)b};
        return __builtin_bit_cast(uint32_t, v);
    };
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const float a = y[2 * d], b = y[2 * d + 1];
        const uint32_t p1 = pk(a, b);
        const float ra = a - __uint_as_float(p1 << 16);
        const float rb = b - __uint_as_float(p1 & 0xffff0000u);
        const uint32_t p2 = pk(ra, rb);
        const float sa = ra - __uint_as_float(p2 << 16);
        const float sb = rb - __uint_as_float(p2 & 0xffff0000u);
        t1[d] = p1;
        t2[d] = p2;
        t3[d] = pk(sa, sb);
    }
}

// --------------------------------------------------------------------------
// split
// --------------------------------------------------------------------------
template <int FMT, bool LO, bool VEC>
__global__ __launch_bounds__(256) void split_kernel(int64_t m, int64_t k,
                                                    const float* __restrict__ A, int64_t lda,
                                                    uint16_t* __restrict__ hi,
                                                    uint16_t* __restrict__ lo, int64_t ldh) {
    const int64_t chunks = (m + 7) / 8;
    const int64_t total = chunks * k;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / chunks, i0 = (e % chunks) * 8;
        const float* src = A + i0 + j * lda;
        const int64_t valid = m - i0;
        float a[8];
        if (VEC && valid >= 8) {
            const f32x4 v0 = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(src));
            const f32x4 v1 = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(src) + 1);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = v0[q];
                a[4 + q] = v1[q];
            }
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) a[q] = q < valid ? src[q] : 0.f;
        }
        uint32_t h[8], l[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            h[q] = rne16<FMT>(a[q]);
            const float hv = val16<FMT>(h[q]);
            // a - hi is exact; a non-finite hi (overflow, NaN) is carried on
            l[q] = rne16<FMT>(__builtin_isfinite(hv) ? a[q] - hv : hv);
        }
        uint16_t* dh = hi + i0 + j * ldh;
        uint16_t* dl = LO ? lo + i0 + j * ldh : nullptr;
        if (VEC && valid >= 8) {
            u32x4 vh, vl;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                vh[d] = h[2 * d] | (h[2 * d + 1] << 16);
                vl[d] = l[2 * d] | (l[2 * d + 1] << 16);
            }
            __builtin_nontemporal_store(vh, reinterpret_cast<u32x4*>(dh));
            if (LO) __builtin_nontemporal_store(vl, reinterpret_cast<u32x4*>(dl));
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q < valid) {
                    dh[q] = (uint16_t)h[q];
                    if (LO) dl[q] = (uint16_t)l[q];
                }
        }
    }
}

// --------------------------------------------------------------------------
// tsm2r_lp
// --------------------------------------------------------------------------
// 8 consecutive 16-bit values as 4 dwords (value 2d in the low half of d).
template <bool VEC>
__device__ __forceinline__ void load8h(const uint16_t* __restrict__ p, int64_t valid, bool full,
                                       uint32_t (&d)[4]) {
    if (VEC && full) {
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
#pragma unroll
        for (int e = 0; e < 4; ++e) d[e] = v[e];
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t x0 = (2 * e < valid) ? p[2 * e] : 0u;
            const uint32_t x1 = (2 * e + 1 < valid) ? p[2 * e + 1] : 0u;
            d[e] = x0 | (x1 << 16);
        }
    }
}

// Bit patterns of the NBT terms of eight float values, packed two per dword
// (value 2e in the low half of dword e): the MFMA operand layout.
template <int FMT, int NBT>
__device__ __forceinline__ void split_terms8(const float (&v)[8], u32x4 (&out)[NBT]) {
    uint32_t h[NBT][8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        float res = v[i];
#pragma unroll
        for (int c = 0; c < NBT; ++c) {
            h[c][i] = rne16<FMT>(res);
            res = res - val16<FMT>(h[c][i]);
        }
    }
#pragma unroll
    for (int c = 0; c < NBT; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) out[c][e] = h[c][2 * e] | (h[c][2 * e + 1] << 16);
}

// B (k x n, B(j, p) = B[j*bsj + p*bsp]) as the packed S operand of
// tsm2r_lp: for 32-row chunk c of B, 16-column group t and term e, the u32x4
// of lane (rl, kk) holds rows 32 c + 8 kk .. 32 c + 8 kk + 7 of column
// 16 t + rl (zero beyond k or n), at Bt[((c * nt16 + t) * LP_BTERMS + e) * 64
// + lane].  One thread per (c, t, lane).
constexpr int LP_BTERMS = 3;

template <int FMT>
__global__ __launch_bounds__(256) void split_b_kernel(int64_t k, int n, const float* __restrict__ B,
                                                      int64_t bsj, int64_t bsp, int nt16,
                                                      u32x4* __restrict__ Bt) {
    const int64_t chunks = (k + 31) / 32;
    const int64_t total = chunks * nt16 * WAVE;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(e % WAVE);
        const int64_t ct = e / WAVE;
        const int t = (int)(ct % nt16);
        const int64_t c = ct / nt16;
        const int rl = lane & 15, kk = lane >> 4;
        const int p = 16 * t + rl;
        const int64_t jb = 32 * c + 8 * kk;
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (p < n && jb + i < k) ? B[(jb + i) * bsj + p * bsp] : 0.f;
        u32x4 out[LP_BTERMS];
        split_terms8<FMT, LP_BTERMS>(v, out);
#pragma unroll
        for (int q = 0; q < LP_BTERMS; ++q) Bt[(ct * LP_BTERMS + q) * WAVE + lane] = out[q];
    }
}

// RS false: the WK wavefronts of a workgroup share one 128-row tile and split
// its k slice in WK parts, summed in the finish.  RS true: they take WK
// adjacent 128-row tiles over the whole k slice, so that a workgroup reads
// WK x 256 contiguous bytes of every column it visits (longer runs per column
// at a time read faster: measured 6.47 -> 6.84 TB/s for the bare pattern),
// and each wavefront's sums are final for its rows.  PF (with RS): the next
// chunk's loads in flight while this one is multiplied.
template <int FMT, int NT16, bool SPLIT, int WK, bool VEC, bool RS, bool PF, int U>
__global__ __launch_bounds__(WAVE * WK) void tsm2r_lp_kernel(
    int64_t m, int64_t k, int n, const uint16_t* __restrict__ Ah,
    const uint16_t* __restrict__ Al, int64_t lda, const u32x4* __restrict__ Bt,
    float* __restrict__ C, int64_t ldc, int64_t kslice, double* __restrict__ part,
    double beta) {
    constexpr int TR = 128;              // a wavefront's tile: 16 lanes x 8 rows
    constexpr int TRW = RS ? WK * TR : TR;   // the workgroup's rows
    constexpr int NP = 16 * NT16;
    constexpr int PG = 4;
    constexpr int NPL = SPLIT ? 2 : 1;   // planes
    constexpr int NBT = LP_BTERMS;       // B terms
    __shared__ __align__(16) unsigned char smem[WK * PG * TR * 8];

    const int lane = threadIdx.x & (WAVE - 1);
    const int rl = lane & 15, kk = lane >> 4;
    const int w = threadIdx.x / WAVE;
    const int64_t tile = blockIdx.x;
    const int s = blockIdx.y, nsl = gridDim.y;
    const int64_t row0 = tile * TRW + (RS ? w * TR : 0);
    const int64_t r = row0 + 8 * rl;     // this lane's 8 rows
    const bool full = (row0 + TR <= m);
    const int64_t kb0 = (int64_t)s * kslice;
    const int64_t kb1 = (kb0 + kslice < k) ? kb0 + kslice : k;
    const int64_t lw = RS ? kslice : kslice / WK;
    const int64_t wk0 = kb0 + (RS ? 0 : w * lw);
    const int64_t wk1 = (wk0 + lw < kb1) ? wk0 + lw : kb1;

    f32x4 acc[8][NT16];
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int t = 0; t < NT16; ++t) acc[q][t] = f32x4{0.f, 0.f, 0.f, 0.f};

    // raw[pl][i][d]: plane pl, column j0 + 8 kk + i, rows r + 2d, r + 2d + 1
    // a whole chunk of a full tile (wavefront-uniform): 16-byte loads
    // without per-lane bounds
    auto loadA_full = [&](int64_t j0, uint32_t (&raw)[NPL][8][4]) {
        const int64_t off = r + (j0 + 8 * kk) * lda;
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) {
            const uint16_t* p = (pl == 0 ? Ah : Al) + off;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
#pragma unroll
                for (int d = 0; d < 4; ++d) raw[pl][i][d] = v[d];
                p += lda;
            }
        }
    };
    auto loadA = [&](int64_t j0, uint32_t (&raw)[NPL][8][4]) {
        if (VEC && full && j0 + 32 <= wk1) {
            loadA_full(j0, raw);
            return;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t j = j0 + 8 * kk + i;
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl) {
                const uint16_t* P = pl == 0 ? Ah : Al;
                if (j < wk1)
                    load8h<VEC>(P + r + j * lda, m - r, full, raw[pl][i]);
                else
#pragma unroll
                    for (int d = 0; d < 4; ++d) raw[pl][i][d] = 0u;
            }
        }
    };
    // the packed B terms of the chunk at j0 (a multiple of 32): cached loads,
    // every row tile reads them
    auto loadBt = [&](int64_t j0, u32x4 (&bt)[NT16][NBT]) {
        const int64_t c = j0 / 32;
#pragma unroll
        for (int t = 0; t < NT16; ++t)
#pragma unroll
            for (int e = 0; e < NBT; ++e) bt[t][e] = Bt[((c * NT16 + t) * NBT + e) * WAVE + lane];
    };

    // the products of the chunk at j0 whose A is in raw
    auto chunk = [&](const uint32_t (&raw)[NPL][8][4], const u32x4 (&bt)[NT16][NBT]) {
        // 8 x 8 transpose of each plane: instance q gets row r + q
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            u32x4 tq[NPL];
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t lo = raw[pl][2 * e][q / 2];
                    const uint32_t hi = raw[pl][2 * e + 1][q / 2];
                    tq[pl][e] = (q & 1) ? ((lo >> 16) | (hi & 0xffff0000u))
                                        : ((lo & 0xffffu) | (hi << 16));
                }
#pragma unroll
            for (int t = 0; t < NT16; ++t) {
#pragma unroll
                for (int c = 0; c < NBT; ++c) acc[q][t] = mfma32<FMT>(bt[t][c], tq[0], acc[q][t]);
                if (SPLIT) {
                    acc[q][t] = mfma32<FMT>(bt[t][0], tq[NPL - 1], acc[q][t]);
                    acc[q][t] = mfma32<FMT>(bt[t][1], tq[NPL - 1], acc[q][t]);
                }
            }
        }
    };

    // PF: a register prefetch of the next chunk, held in flight across the
    // waits for this one.  It doubles the loads a wavefront has outstanding
    // (32 KB per wavefront for the split form) at the cost of occupancy (one
    // wavefront per SIMD for the split form), and with one workgroup per CU
    // it measured 6-10 % faster than the row split alone at A 32768^2 and
    // 16384^2.  Without the scheduling barriers the compiler sank the next
    // chunk's loads below the waits and it gained nothing.
    if (wk1 > wk0 && row0 < m) {
        const int ng = (int)((wk1 - wk0 + 31) / 32);
        if (!PF || !(VEC && full && (wk1 - wk0) % (32 * U) == 0)) {
            for (int g = 0; g < ng; ++g) {
                uint32_t raw[NPL][8][4];
                u32x4 bt[NT16][NBT];
                loadA(wk0 + 32 * g, raw);
                loadBt(wk0 + 32 * g, bt);
                chunk(raw, bt);
            }
        } else {
            // every chunk whole: the next step in flight while this one is
            // multiplied, in straight-line code (no bounds branches, so the
            // waits for this step's operands leave the next step's loads
            // outstanding); its B terms are loaded before its A for the same
            // reason.  A step is U chunks: the single form takes two, so
            // that a wavefront has as many bytes in flight as the split form.
            uint32_t ra[U][NPL][8][4], rb[U][NPL][8][4];
            u32x4 ba[U][NT16][NBT], bb[U][NT16][NBT];
            auto load_step = [&](int64_t j0, uint32_t (&r)[U][NPL][8][4], u32x4 (&b)[U][NT16][NBT]) {
#pragma unroll
                for (int u = 0; u < U; ++u) loadBt(j0 + 32 * u, b[u]);
#pragma unroll
                for (int u = 0; u < U; ++u) loadA_full(j0 + 32 * u, r[u]);
            };
            auto mul_step = [&](const uint32_t (&r)[U][NPL][8][4], const u32x4 (&b)[U][NT16][NBT]) {
#pragma unroll
                for (int u = 0; u < U; ++u) chunk(r[u], b[u]);
            };
            const int ns = (int)((wk1 - wk0) / (32 * U));
            load_step(wk0, ra, ba);
            int g = 0;
            // (the scheduling barriers keep the next step's loads ahead of
            // the waits for this one: two steps in flight per wavefront)
            for (; g + 2 < ns; g += 2) {
                load_step(wk0 + 32 * U * (g + 1), rb, bb);
                __builtin_amdgcn_sched_barrier(0);
                mul_step(ra, ba);
                load_step(wk0 + 32 * U * (g + 2), ra, ba);
                __builtin_amdgcn_sched_barrier(0);
                mul_step(rb, bb);
            }
            if (g + 1 < ns) {
                load_step(wk0 + 32 * U * (g + 1), rb, bb);
                __builtin_amdgcn_sched_barrier(0);
                mul_step(ra, ba);
                mul_step(rb, bb);
            } else {
                mul_step(ra, ba);
            }
        }
    }

    // lane holds C[r + q, 16 t + 4 kk + rr] in acc[q][t][rr]
    nn_finish<float, NP, WK, TRW, PG, RS ? 1 : WK>(
        m, n, C, ldc, beta, tile, s, nsl, part, reinterpret_cast<double*>(smem),
        [&](int pg, double* red) {
            const int t = pg / 16;
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int pp = 16 * t + Mfma<float>::mrow(kk, rr) - pg;
                if (pp >= 0 && pp < PG) {
                    double* dst = RS ? red + pp * TRW + w * TR : red + (w * PG + pp) * TR;
#pragma unroll
                    for (int q = 0; q < 8; ++q) dst[8 * rl + q] = (double)acc[q][t][rr];
                }
            }
        });
}

// Value of row q (0..7) of a lane's 16-byte run of each plane: hi, or hi + lo.
// hi + lo is exact in float: lo rounds a - hi at or above a's last bit, so
// the sum stays on a's 24-bit grid.
template <int FMT, int NPL>
__device__ __forceinline__ float plane_val(const uint32_t (&raw)[NPL][4], int q) {
    float a = half_val<FMT>(raw[0][q >> 1], q & 1);
    if (NPL == 2) a += half_val<FMT>(raw[NPL - 1][q >> 1], q & 1);
    return a;
}

// --------------------------------------------------------------------------
// tsm2l_lp: C = A*B with A tall (m x k, k <= 32) in the low-precision form,
// B (k x n, n <= 32) and C float.  TSM2L (Algorithm 6) carries few flops per
// byte (2*n per element of A), so the planes are widened to float in
// registers and the float 16x16x4 matrix cores do the products, with B kept
// in float.  A lane's 16-byte load is 8 rows of one column: element q is the
// T operand of MFMA instance q as it stands, S is a 16 x 4 block of B^T held
// in registers for the whole kernel.  A persistent grid walks 128-row tiles;
// the next tile's planes (16 VGPRs per plane) are in flight while the
// current one is multiplied and stored.
// --------------------------------------------------------------------------
// waves per SIMD the instances are compiled for (the most that fit without spills)
template <int KS, int NT16>
constexpr int lp_l_waves() { return (NT16 == 1 && KS <= 4) ? 3 : (KS * NT16 <= 8 ? 2 : 1); }

template <int FMT, int KS, int NT16, bool SPLIT, bool VEC>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(lp_l_waves<KS, NT16>(), 8))) void tsm2l_lp_kernel(
    int64_t m, int k, int n, const uint16_t* __restrict__ Ah, const uint16_t* __restrict__ Al,
    int64_t lda, const float* __restrict__ B, int64_t bsj, int64_t bsp, float beta,
    float* __restrict__ C, int64_t ldc) {
    typedef Mfma<float> M;
    constexpr int RL = 8;                // rows per 16-byte run of 16-bit values
    constexpr int TR = 16 * RL;
    constexpr int WPB = 4;
    constexpr int NPL = SPLIT ? 2 : 1;
    const int lane = threadIdx.x & (WAVE - 1);
    const int rl = lane & 15, kk = lane >> 4;
    const int w = threadIdx.x / WAVE;

    // S operand: B[4 st + kk, 16 t + rl]
    float bv[KS][NT16];
#pragma unroll
    for (int st = 0; st < KS; ++st)
#pragma unroll
        for (int t = 0; t < NT16; ++t) {
            const int j = 4 * st + kk, p = 16 * t + rl;
            bv[st][t] = (j < k && p < n) ? B[j * bsj + (int64_t)p * bsp] : 0.f;
        }

    auto load = [&](int64_t tile, uint32_t (&raw)[KS][NPL][4]) {
        const int64_t r = tile * TR + RL * rl;
        const bool full = tile * TR + TR <= m;
#pragma unroll
        for (int st = 0; st < KS; ++st) {
            const int j = 4 * st + kk;
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl) {
                const uint16_t* P = pl == 0 ? Ah : Al;
                if (j < k)
                    load8h<VEC>(P + r + (int64_t)j * lda, m - r, full, raw[st][pl]);
                else
#pragma unroll
                    for (int d = 0; d < 4; ++d) raw[st][pl][d] = 0u;
            }
        }
    };

    const int64_t ntiles = (m + TR - 1) / TR;
    const int64_t tstride = (int64_t)gridDim.x * WPB;
    int64_t tile = (int64_t)blockIdx.x * WPB + w;
    uint32_t raw[KS][NPL][4];
    if (tile < ntiles) load(tile, raw);
    for (; tile < ntiles; tile += tstride) {
        const int64_t r = tile * TR + RL * rl;
        const bool full = tile * TR + TR <= m;
        const bool more = tile + tstride < ntiles;
        uint32_t rn[KS][NPL][4];
        if (more) load(tile + tstride, rn);
        f32x4 acc[RL][NT16];
#pragma unroll
        for (int q = 0; q < RL; ++q)
#pragma unroll
            for (int t = 0; t < NT16; ++t) acc[q][t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < KS; ++st)
#pragma unroll
            for (int q = 0; q < RL; ++q) {
                const float a = plane_val<FMT, NPL>(raw[st], q);
#pragma unroll
                for (int t = 0; t < NT16; ++t) acc[q][t] = M::op(bv[st][t], a, acc[q][t]);
            }
        // acc[q][t][rr] = C[r + q, 16 t + mrow(kk, rr)]: 8 rows of a column
#pragma unroll
        for (int t = 0; t < NT16; ++t)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int col = 16 * t + M::mrow(kk, rr);
                if (col < n) {
                    float v0[4], v1[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        v0[q] = acc[q][t][rr];
                        v1[q] = acc[4 + q][t][rr];
                    }
                    float* c = C + r + (int64_t)col * ldc;
                    if (beta != 0.f) {
                        float o0[4], o1[4];
                        load_run<float, 4, VEC>(c, m - r, full, o0);
                        load_run<float, 4, VEC>(c + 4, m - r - 4, full, o1);
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            v0[q] = __builtin_fmaf(beta, o0[q], v0[q]);
                            v1[q] = __builtin_fmaf(beta, o1[q], v1[q]);
                        }
                    }
                    // the two stores fill alternate 16-byte halves of the lines
                    store_run<float, 4, VEC, false>(c, m - r, full, v0);
                    store_run<float, 4, VEC, false>(c + 4, m - r - 4, full, v1);
                }
            }
        if (more) {
#pragma unroll
            for (int st = 0; st < KS; ++st)
#pragma unroll
                for (int pl = 0; pl < NPL; ++pl)
#pragma unroll
                    for (int d = 0; d < 4; ++d) raw[st][pl][d] = rn[st][pl][d];
        }
    }
}

// --------------------------------------------------------------------------
// tn_lp: O(ncols x n) = X^T * Y with X (R x ncols) in the low-precision form
// and Y (R x n) float: the gradient dB = A^T * dC of the low-precision form.
// As tn_kernel: per wavefront step of 128 rows, a lane loads 8 rows of one X
// column per plane (16 bytes, four columns per load instruction), widens X
// to float and stages it in a wavefront-private LDS tile; it reads back X
// column 16 ct + rl, 4 consecutive rows at a time, as the S operand of the
// float 16x16x4 matrix cores.  The T operand, Y columns 16 t + rl at the
// same rows, is either staged the same way (YD false: 4 rows of one column
// twice per lane, when one column group streams Y from HBM once) or loaded
// straight in operand order (YD: Y is small and every column group re-reads
// it, so the loads hit L2 and need no LDS; CT output tiles per workgroup then
// share each Y word).  Reduction across wavefronts and workgroups as in
// tn_kernel.
//
// bfloat16 planes with Y direct (MX; the split form for n <= 16) run on the
// 16x16x32 bf16 matrix cores instead: X is staged in LDS as loaded (16-bit,
// no widening) and read back as the S operand (lane (rl, kk): column
// 16 ct + rl, 8 consecutive rows 32 blk + 8 kk ..), Y is loaded in the
// matching T operand order (column 16 t + rl, the same 8 rows) and split
// into three bf16 terms in registers, and each 32-row block takes
// hi*(Y1 + Y2 + Y3) (+ lo*(Y1 + Y2)), the products the TSM2R form keeps:
// three (five) matrix-core instructions where the float path takes eight,
// and no widening.  Products of 16-bit values are exact in float, so the
// error against the stored values is that of float accumulation, as on the
// float path.  Whole wavefronts load straight-line; ragged ones (rows, X
// columns, unaligned Y) take the same step with bounds-checked loads.
// Y columns beyond n read column n - 1; their output columns are never
// stored.  With four output tiles per workgroup the split form's 16-bit
// tiles take 136 KB of LDS: one workgroup per CU.  For n > 16 (YT) Y's
// terms are split once per call into the workspace, packed in the operand
// order, and the step loads them instead of splitting Y in registers.
// --------------------------------------------------------------------------
// (YT instances run one workgroup per CU, held there by their LDS: their
// registers need not leave room for a second wavefront per SIMD)
template <int FMT, int NT16, int CT, bool SPLIT, bool VEC, bool YC, bool YD, bool YT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(YT ? 1 : 2, 8))) void tn_lp_kernel(
    int64_t R, int64_t ncols, int n, const uint16_t* __restrict__ Xh,
    const uint16_t* __restrict__ Xl, int64_t ldx, const float* __restrict__ Y, int64_t ldy,
    float* __restrict__ O, int64_t ldo, int64_t rslice, double* __restrict__ part,
    const u32x4* __restrict__ Yt, int pf) {
    typedef Mfma<float> M;
    constexpr int WK = 4;
    constexpr int SR = 128;                    // rows per step
    constexpr int SROW = SR + 4;               // padded LDS column (16 more bytes)
    constexpr int NX = 16 * CT;                // staged X columns (CT output tiles)
    constexpr int NC = NX + (YD ? 0 : 16 * NT16);   // then the staged Y columns
    constexpr int XG = 4 * CT;                 // X column groups of 4
    constexpr int YG = 4 * NT16;               // Y column groups of 4 (staged Y)
    constexpr int NB = SR / 16;                // 16-row blocks per step
    constexpr int NPL = SPLIT ? 2 : 1;
    // bfloat16 planes with Y direct run on the 16-bit matrix cores (MX): all
    // of their wavefronts, whole or ragged.  The split form with n > 16 does
    // so only with Y's terms packed once per call (YT): with the split of Y
    // in registers its step does not fit, and it keeps the float path
    constexpr bool MX = FMT == FMT_BF16 && YD && (!SPLIT || NT16 == 1 || YT);
    static_assert(!YT || (FMT == FMT_BF16 && YD), "packed Y terms feed the bf16 matrix cores");
    constexpr int SROW16 = SR + 8;             // padded 16-bit LDS column (16 more bytes)
    __shared__ __align__(16) float lds[WK][MX ? 1 : NC][SROW];
    __shared__ __align__(16) uint16_t lds16[WK][MX ? NPL : 1][MX ? NX : 1][SROW16];
    __shared__ double red[WK][WAVE][4 * NT16];

    const int lane = threadIdx.x & (WAVE - 1);
    const int rl = lane & 15, kk = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);   // wavefront-uniform
    const int64_t c0 = (int64_t)blockIdx.x * NX;
    const int s = blockIdx.y, nsl = gridDim.y;
    const int64_t sb0 = (int64_t)s * rslice;
    const int64_t sb1 = (sb0 + rslice < R) ? sb0 + rslice : R;
    const int64_t lw = rslice / WK;            // multiple of SR
    const int64_t wb0 = sb0 + w * lw;
    const int64_t wb1 = (wb0 + lw < sb1) ? wb0 + lw : sb1;
    float (*tile)[SROW] = lds[w];
    uint16_t (*tile16)[MX ? NX : 1][SROW16] = lds16[w];

    f32x4 acc[CT][NT16];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int t = 0; t < NT16; ++t) acc[ct][t] = f32x4{0.f, 0.f, 0.f, 0.f};

    // Y words a lane holds per step: staged (YD false), rows 64 h + 4 rl of
    // column 4 cg + kk; direct (YD), the MFMA operand itself, rows
    // 16 hb + 4 kk of column 16 t + rl (Y is small and re-read by every column
    // group, so these loads hit L2; nothing of Y goes through LDS)
    constexpr int YW = YD ? NB * NT16 : 2 * YG;
    auto loadY = [&](int64_t rb, float (&yv)[YW][4]) {
#pragma unroll
        for (int yi = 0; yi < YW; ++yi) {
            // staged: yi = h * YG + cg; direct: yi = hb * NT16 + t
            const int64_t r = YD ? rb + 16 * (yi / NT16) + 4 * kk : rb + 64 * (yi / YG) + 4 * rl;
            const int p = YD ? 16 * (yi % NT16) + rl : 4 * (yi % YG) + kk;
            const int64_t valid = wb1 - r;
            const bool full = valid >= 4;
            if (YC && VEC && p < n && full) {
                // Y re-read by every column group: through the cache
                const f32x4 y = *reinterpret_cast<const f32x4*>(Y + r + (int64_t)p * ldy);
#pragma unroll
                for (int q = 0; q < 4; ++q) yv[yi][q] = y[q];
            } else if (p < n)
                load_run<float, 4, VEC>(Y + r + (int64_t)p * ldy, valid, full, yv[yi]);
            else
#pragma unroll
                for (int q = 0; q < 4; ++q) yv[yi][q] = 0.f;
        }
    };
    // X (and staged Y) of a step are loaded one step ahead; direct Y is loaded
    // at the start of its own step (its registers would cost a wavefront)
    auto loadX = [&](int64_t rb, uint32_t (&xv)[XG][NPL][4]) {
        {
            const int64_t r = rb + 8 * rl;
            const int64_t valid = wb1 - r;
            const bool full = valid >= 8;
#pragma unroll
            for (int cg = 0; cg < XG; ++cg) {
                const int64_t c = c0 + 4 * cg + kk;
#pragma unroll
                for (int pl = 0; pl < NPL; ++pl) {
                    const uint16_t* P = pl == 0 ? Xh : Xl;
                    if (c < ncols)
                        load8h<VEC>(P + r + c * ldx, valid, full, xv[cg][pl]);
                    else
#pragma unroll
                        for (int d = 0; d < 4; ++d) xv[cg][pl][d] = 0u;
                }
            }
        }
    };

    // stage X (and staged Y) of a step and multiply
    auto step = [&](const uint32_t (&xv)[XG][NPL][4], const float (&yv)[YW][4]) {
        // stage: X column 4 cg + kk rows 8 rl .. 8 rl + 7 (widened),
        //        Y column NX + 4 cg + kk rows 64 h + 4 rl .. 64 h + 4 rl + 3
        wave_lds_fence();
#pragma unroll
        for (int cg = 0; cg < XG; ++cg) {
            f32x4 x0, x1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                x0[q] = plane_val<FMT, NPL>(xv[cg], q);
                x1[q] = plane_val<FMT, NPL>(xv[cg], 4 + q);
            }
            *reinterpret_cast<f32x4*>(&tile[4 * cg + kk][8 * rl]) = x0;
            *reinterpret_cast<f32x4*>(&tile[4 * cg + kk][8 * rl + 4]) = x1;
        }
        if (!YD) {
#pragma unroll
            for (int yi = 0; yi < YW; ++yi) {
                f32x4 y;
#pragma unroll
                for (int q = 0; q < 4; ++q) y[q] = yv[yi][q];
                *reinterpret_cast<f32x4*>(&tile[NX + 4 * (yi % YG) + kk][64 * (yi / YG) + 4 * rl]) = y;
            }
        }
        // read back 16-row blocks: rows 16 hb + 4 kk + q; each Y block
        // serves the CT output tiles
        wave_lds_fence();
#pragma unroll
        for (int hb = 0; hb < NB; ++hb) {
            f32x4 ys[NT16];
#pragma unroll
            for (int t = 0; t < NT16; ++t) {
                if (YD) {
                    const bool live = 16 * t + rl < n;
#pragma unroll
                    for (int q = 0; q < 4; ++q) ys[t][q] = live ? yv[hb * NT16 + t][q] : 0.f;
                } else {
                    ys[t] = *reinterpret_cast<const f32x4*>(&tile[NX + 16 * t + rl][16 * hb + 4 * kk]);
                }
            }
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const f32x4 xs = *reinterpret_cast<const f32x4*>(&tile[16 * ct + rl][16 * hb + 4 * kk]);
#pragma unroll
                for (int t = 0; t < NT16; ++t)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[ct][t] = M::op(xs[q], ys[t][q], acc[ct][t]);
            }
        }
    };

    // pf and every step whole (rows and columns in range, 16-byte loads, Y
    // direct): straight-line loads, the next step's X kept in flight across
    // the waits for this step's operands (the scheduling barriers stop the
    // compiler from sinking those loads below the waits).
    const bool whole = !MX && pf && VEC && YC && YD && c0 + NX <= ncols && (wb1 - wb0) % SR == 0;
    // MX: the same whole-wavefront test without pf (pf only picks one or two
    // steps in flight, with the same arithmetic); ragged wavefronts take the
    // MX step too, with bounds-checked loads
    const bool mx_whole = MX && VEC && YC && c0 + NX <= ncols && (wb1 - wb0) % SR == 0;
    // two steps in flight need two X steps in registers: not with four split tiles
    constexpr bool MX_TWO = MX && !(SPLIT && CT >= 4);
    auto loadX_full = [&](int64_t rb, uint32_t (&xv)[XG][NPL][4]) {
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) {
            const uint16_t* P = (pl == 0 ? Xh : Xl) + rb + 8 * rl + (c0 + kk) * ldx;
#pragma unroll
            for (int cg = 0; cg < XG; ++cg) {
                const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(P + 4 * cg * ldx));
#pragma unroll
                for (int d = 0; d < 4; ++d) xv[cg][pl][d] = v[d];
            }
        }
    };
    // columns p >= n load column n - 1 (in range); the step zeroes them
    auto loadY_full = [&](int64_t rb, float (&yv)[YW][4]) {
#pragma unroll
        for (int yi = 0; yi < YW; ++yi) {
            const int p = 16 * (yi % NT16) + rl;
            const int pc = p < n ? p : n - 1;
            const f32x4 y = *reinterpret_cast<const f32x4*>(Y + rb + 16 * (yi / NT16) + 4 * kk +
                                                            (int64_t)pc * ldy);
#pragma unroll
            for (int q = 0; q < 4; ++q) yv[yi][q] = y[q];
        }
    };

    // MX: Y rows rb + 32 blk + 8 kk .. + 7 of column 16 t + rl (n - 1 beyond n)
    // YT: the three bf16 terms of Y, split once per call (split_b_kernel on
    // Y), packed in the operand order: 32-row block b, column group t, term
    // e at Yt[((b * NT16 + t) * 3 + e) * 64 + lane], zero beyond R and n
    typedef typename std::conditional<YT, u32x4[4][NT16][3], f32x4[4][NT16][2]>::type YBuf;
    const int64_t nblk = (R + 31) / 32;
    auto loadY_mx = [&](int64_t rb, YBuf& ym) {
        if constexpr (YT) {
#pragma unroll
            for (int blk = 0; blk < 4; ++blk)
#pragma unroll
                for (int t = 0; t < NT16; ++t)
#pragma unroll
                    for (int e = 0; e < 3; ++e)
                        ym[blk][t][e] = Yt[(((rb >> 5) + blk) * NT16 + t) * 3 * WAVE + e * WAVE + lane];
        } else {
#pragma unroll
            for (int blk = 0; blk < 4; ++blk)
#pragma unroll
                for (int t = 0; t < NT16; ++t) {
                    const int p = 16 * t + rl;
                    const int pc = p < n ? p : n - 1;
                    const f32x4* src = reinterpret_cast<const f32x4*>(Y + rb + 32 * blk + 8 * kk +
                                                                      (int64_t)pc * ldy);
                    ym[blk][t][0] = src[0];
                    ym[blk][t][1] = src[1];
                }
        }
    };
    // the same rows with bounds: rows at or beyond wb1 and columns beyond n
    // are zero (ragged wavefronts, unaligned Y)
    auto loadY_mx_gen = [&](int64_t rb, YBuf& ym) {
        if constexpr (YT) {
            // X rows at or beyond wb1 are zero; blocks beyond R are not read
#pragma unroll
            for (int blk = 0; blk < 4; ++blk)
#pragma unroll
                for (int t = 0; t < NT16; ++t)
#pragma unroll
                    for (int e = 0; e < 3; ++e) {
                        const int64_t b = (rb >> 5) + blk;
                        ym[blk][t][e] = b < nblk ? Yt[(b * NT16 + t) * 3 * WAVE + e * WAVE + lane]
                                                 : u32x4{0u, 0u, 0u, 0u};
                    }
        } else {
#pragma unroll
            for (int blk = 0; blk < 4; ++blk)
#pragma unroll
                for (int t = 0; t < NT16; ++t) {
                    const int p = 16 * t + rl;
                    const int64_t r = rb + 32 * blk + 8 * kk;
                    const int64_t valid = wb1 - r;
                    float v0[4], v1[4];
                    if (p < n) {
                        load_run<float, 4, VEC>(Y + r + (int64_t)p * ldy, valid, valid >= 4, v0);
                        load_run<float, 4, VEC>(Y + r + 4 + (int64_t)p * ldy, valid - 4, valid >= 8,
                                                v1);
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) v0[q] = v1[q] = 0.f;
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        ym[blk][t][0][q] = v0[q];
                        ym[blk][t][1][q] = v1[q];
                    }
                }
        }
    };
    // products kept: hi*(Y1 + Y2 + Y3) (+ lo*(Y1 + Y2)), as in tsm2r_lp
    auto step_mx = [&](const uint32_t (&xv)[XG][NPL][4], const YBuf& ym) {
        wave_lds_fence();
#pragma unroll
        for (int cg = 0; cg < XG; ++cg)
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl)
                *reinterpret_cast<u32x4*>(&tile16[pl][4 * cg + kk][8 * rl]) =
                    u32x4{xv[cg][pl][0], xv[cg][pl][1], xv[cg][pl][2], xv[cg][pl][3]};
        wave_lds_fence();
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
            u32x4 y1[NT16], y2[NT16], y3[NT16];
#pragma unroll
            for (int t = 0; t < NT16; ++t) {
                if constexpr (YT) {
                    y1[t] = ym[blk][t][0];
                    y2[t] = ym[blk][t][1];
                    y3[t] = ym[blk][t][2];
                } else {
                    float y[8];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        y[q] = ym[blk][t][0][q];
                        y[4 + q] = ym[blk][t][1][q];
                    }
                    bf16_terms8(y, y1[t], y2[t], y3[t]);
                }
            }
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                u32x4 xs[NPL];
#pragma unroll
                for (int pl = 0; pl < NPL; ++pl)
                    xs[pl] = *reinterpret_cast<const u32x4*>(&tile16[pl][16 * ct + rl][32 * blk + 8 * kk]);
#pragma unroll
                for (int t = 0; t < NT16; ++t) {
                    acc[ct][t] = mfma32<FMT_BF16>(xs[0], y1[t], acc[ct][t]);
                    acc[ct][t] = mfma32<FMT_BF16>(xs[0], y2[t], acc[ct][t]);
                    acc[ct][t] = mfma32<FMT_BF16>(xs[0], y3[t], acc[ct][t]);
                    if (SPLIT) {
                        acc[ct][t] = mfma32<FMT_BF16>(xs[NPL - 1], y1[t], acc[ct][t]);
                        acc[ct][t] = mfma32<FMT_BF16>(xs[NPL - 1], y2[t], acc[ct][t]);
                    }
                }
            }
        }
    };

    if (MX && wb1 > wb0 && mx_whole) {
        const int64_t nit = (wb1 - wb0) / SR;
        uint32_t xa[XG][NPL][4], xb[XG][NPL][4];
        YBuf ym;
        if (!MX_TWO || !pf) {
            // one step at a time, no conditional loads (measured faster for
            // n <= 8, where the step is short)
            for (int64_t it = 0; it < nit; ++it) {
                loadX_full(wb0 + it * SR, xa);
                loadY_mx(wb0 + it * SR, ym);
                step_mx(xa, ym);
            }
        } else {
            // two steps per iteration, the next step's X in flight (as below)
            loadX_full(wb0, xa);
            int64_t it = 0;
            for (; it + 2 < nit; it += 2) {
                loadY_mx(wb0 + it * SR, ym);
                loadX_full(wb0 + (it + 1) * SR, xb);
                __builtin_amdgcn_sched_barrier(0);
                step_mx(xa, ym);
                loadY_mx(wb0 + (it + 1) * SR, ym);
                loadX_full(wb0 + (it + 2) * SR, xa);
                __builtin_amdgcn_sched_barrier(0);
                step_mx(xb, ym);
            }
            loadY_mx(wb0 + it * SR, ym);
            if (it + 1 < nit) {
                loadX_full(wb0 + (it + 1) * SR, xb);
                step_mx(xa, ym);
                loadY_mx(wb0 + (it + 1) * SR, ym);
                step_mx(xb, ym);
            } else {
                step_mx(xa, ym);
            }
        }
    } else if (MX && wb1 > wb0) {
        // ragged or unaligned: one step at a time, loads bounds-checked
        const int64_t nit = (wb1 - wb0 + SR - 1) / SR;
        for (int64_t it = 0; it < nit; ++it) {
            uint32_t xv[XG][NPL][4];
            YBuf ym;
            loadX(wb0 + it * SR, xv);
            loadY_mx_gen(wb0 + it * SR, ym);
            step_mx(xv, ym);
        }
    } else if (!MX && wb1 > wb0 && whole) {
        // two steps per iteration with no conditional loads inside (a load
        // issued on one path only makes the waits after the join count it
        // as absent, and they then wait for everything)
        const int64_t nit = (wb1 - wb0) / SR;
        uint32_t xa[XG][NPL][4], xb[XG][NPL][4];
        float yv[YW][4];
        loadX_full(wb0, xa);
        int64_t it = 0;
        for (; it + 2 < nit; it += 2) {
            loadY_full(wb0 + it * SR, yv);
            loadX_full(wb0 + (it + 1) * SR, xb);
            __builtin_amdgcn_sched_barrier(0);
            step(xa, yv);
            loadY_full(wb0 + (it + 1) * SR, yv);
            loadX_full(wb0 + (it + 2) * SR, xa);
            __builtin_amdgcn_sched_barrier(0);
            step(xb, yv);
        }
        loadY_full(wb0 + it * SR, yv);
        if (it + 1 < nit) {
            loadX_full(wb0 + (it + 1) * SR, xb);
            step(xa, yv);
            loadY_full(wb0 + (it + 1) * SR, yv);
            step(xb, yv);
        } else {
            step(xa, yv);
        }
    } else if (!MX && wb1 > wb0) {
        const int64_t nit = (wb1 - wb0 + SR - 1) / SR;
        uint32_t xv[XG][NPL][4];
        float yv[YW][4];
        loadX(wb0, xv);
        if (!YD) loadY(wb0, yv);
        for (int64_t it = 0; it < nit; ++it) {
            uint32_t xn[XG][NPL][4];
            float yn[YW][4];
            if (YD) loadY(wb0 + it * SR, yv);
            if (it + 1 < nit) {
                loadX(wb0 + (it + 1) * SR, xn);
                if (!YD) loadY(wb0 + (it + 1) * SR, yn);
            }
            step(xv, yv);
#pragma unroll
            for (int cg = 0; cg < XG; ++cg)
#pragma unroll
                for (int pl = 0; pl < NPL; ++pl)
#pragma unroll
                    for (int d = 0; d < 4; ++d) xv[cg][pl][d] = xn[cg][pl][d];
            if (!YD) {
#pragma unroll
                for (int yi = 0; yi < YW; ++yi)
#pragma unroll
                    for (int q = 0; q < 4; ++q) yv[yi][q] = yn[yi][q];
            }
        }
    }

    // one 16-column output tile at a time (global tile index blockIdx.x*CT + ct)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        if (ct > 0) __syncthreads();           // red is reused
        tn_finish<float, NT16, WK>(ncols, n, O, ldo, 0.0, (int64_t)blockIdx.x * CT + ct, s, nsl,
                                   part, red, acc[ct],
                                   [](int kq, int r) { return Mfma<float>::mrow(kq, r); });
    }
}

// --------------------------------------------------------------------------
// plans and launches
// --------------------------------------------------------------------------
template <typename K>
static int lp_occupancy(K kernel) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, 0) != hipSuccess || nb < 1)
        nb = 1;
    return nb;
}

template <int FMT, int NT16, bool SPLIT, bool VEC, bool RS, bool PF, int U>
static const void* lp_fn(int* occ) {
    static const int o = lp_occupancy(tsm2r_lp_kernel<FMT, NT16, SPLIT, 4, VEC, RS, PF, U>);
    *occ = o;
    return (const void*)tsm2r_lp_kernel<FMT, NT16, SPLIT, 4, VEC, RS, PF, U>;
}

// the split form steps one 32-column chunk at a time; the single form SU
template <int FMT, bool VEC, bool RS, bool PF, int SU>
static const void* lp_pick_f(bool split, int nt16, int* occ) {
    if (split)
        return nt16 == 1 ? lp_fn<FMT, 1, true, VEC, RS, PF, 1>(occ) : lp_fn<FMT, 2, true, VEC, RS, PF, 1>(occ);
    return nt16 == 1 ? lp_fn<FMT, 1, false, VEC, RS, PF, SU>(occ) : lp_fn<FMT, 2, false, VEC, RS, PF, SU>(occ);
}

// variant 0: wavefronts split k; 1: row split; 2: row split with the next
// step in flight (single form: two chunks per step); 3: as 2 with one chunk
// per step for the single form
template <bool VEC>
static const void* lp_pick(int fmt, bool split, int nt16, int var, int* occ) {
    if (fmt == FMT_BF16) {
        if (var == 0) return lp_pick_f<FMT_BF16, VEC, false, false, 1>(split, nt16, occ);
        if (var == 1) return lp_pick_f<FMT_BF16, VEC, true, false, 1>(split, nt16, occ);
        if (var == 3) return lp_pick_f<FMT_BF16, VEC, true, true, 1>(split, nt16, occ);
        return lp_pick_f<FMT_BF16, VEC, true, true, 2>(split, nt16, occ);
    }
    if (var == 0) return lp_pick_f<FMT_F16, VEC, false, false, 1>(split, nt16, occ);
    if (var == 1) return lp_pick_f<FMT_F16, VEC, true, false, 1>(split, nt16, occ);
    if (var == 3) return lp_pick_f<FMT_F16, VEC, true, true, 1>(split, nt16, occ);
    return lp_pick_f<FMT_F16, VEC, true, true, 2>(split, nt16, occ);
}

static inline int64_t cdiv_lp(int64_t a, int64_t b) { return (a + b - 1) / b; }

int plan_tsm2r_lp(int64_t m, int64_t k, int64_t n, int dtype, int cus, bool vec, NNPlan* P) {
    const int fmt = (dtype == DT_BF16 || dtype == DT_BF16_SPLIT) ? FMT_BF16 : FMT_F16;
    const bool split = dtype == DT_BF16_SPLIT || dtype == DT_F16_SPLIT;
    const int nt16 = n <= 16 ? 1 : 2;
    // the workgroup's wavefronts on adjacent row tiles, each with its next
    // chunk in flight (see tsm2r_lp_kernel); TSM2X_LP_RS=0 selects the k
    // split among them, 1 the row split without the prefetch (measurement
    // only)
    const char* frs = std::getenv("TSM2X_LP_RS");
    int var = (frs && *frs) ? (int)std::strtol(frs, nullptr, 10) : 2;
    if (var < 0 || var > 3) var = 2;
    if (!vec && var >= 2) var = 1;      // the prefetch needs 16-byte loads of the planes
    const bool rs = var != 0;
    int occ = 1;
    P->fn = vec ? lp_pick<true>(fmt, split, nt16, var, &occ) : lp_pick<false>(fmt, split, nt16, var, &occ);
    const int WK = 4, TR = rs ? WK * 128 : 128;
    P->np = 16 * nt16;
    P->tile_rows = TR;
    P->tiles = cdiv_lp(m, TR);
    // with the prefetch: one workgroup per CU, never more (A 32768^2 and
    // 16384^2, n = 8..32: 256 workgroups beat 192 by 6-12 % and 288-320 by
    // 20-30 %, as the CUs holding a second workgroup finish last); without
    // it, as for the float kernel, about 15/8 resident workgroups per CU
    const int64_t slots = (int64_t)cus * occ;
    int64_t S;
    if (var >= 2) {
        S = cus / P->tiles;
    } else {
        int64_t tgt = (int64_t)cus * 15 / 8;
        if (tgt > slots) tgt = slots;
        S = (tgt + P->tiles / 2) / P->tiles;
    }
    const int64_t s_len = k / (rs ? 64 : WK * 64);
    // the float kernel's cap on the partials' traffic, for both forms (the
    // single form, half the bytes of A, measured 11 % faster at A 16384^2,
    // n = 8 with the 15 slices it allows than with 10)
    const int64_t s_cost = (k * 4) / ((int64_t)P->np * 200);
    if (S > s_len) S = s_len;
    if (S > s_cost) S = s_cost;
    if (S < 1) S = 1;
    const char* fs = std::getenv("TSM2X_LP_S");
    if (fs && *fs && std::strtoll(fs, nullptr, 10) > 0) S = std::strtoll(fs, nullptr, 10);
    const int64_t gran = rs ? 32 : (int64_t)WK * 32;
    int64_t ks = cdiv_lp(k, S);
    ks = cdiv_lp(ks, gran) * gran;
    P->kslice = ks;
    P->S = (int)cdiv_lp(k, ks);
    if (P->S < 1) P->S = 1;
    P->ws = P->S > 1 ? (size_t)P->tiles * P->S * P->np * TR * 8 : 0;
    return 0;
}

int launch_tsm2r_lp(const LaunchNN& L, int dtype, hipStream_t st) {
    const bool split = dtype == DT_BF16_SPLIT || dtype == DT_F16_SPLIT;
    const uint16_t* ah = (const uint16_t*)L.A;
    const uint16_t* al = split ? ah + L.lda * L.k : nullptr;
    int n32 = (int)L.n;
    double beta = L.beta;
    // L.B: B's terms packed by launch_split_b
    void* args[] = {(void*)&L.m,   (void*)&L.k,      (void*)&n32,    (void*)&ah,
                    (void*)&al,    (void*)&L.lda,    (void*)&L.B,    (void*)&L.C,
                    (void*)&L.ldc, (void*)&L.kslice, (void*)&L.part, (void*)&beta};
    hipError_t e;
    {
        LaunchTimer timer(L.fn, st);
        e = hipLaunchKernel(L.fn, dim3((unsigned)L.tiles, (unsigned)L.S), dim3(256), args, 0, st);
    }
    if (e != hipSuccess) return 1;
    if (L.S > 1)
        return launch_split_reduce(DT_F32, L.tiles, L.S, L.np, L.tile_rows, L.m, (int)L.n, L.part,
                                   L.C, L.ldc, L.beta, st);
    return 0;
}

size_t lp_bterms_bytes(int64_t k, int64_t n) {
    return (size_t)((k + 31) / 32) * (n <= 16 ? 1 : 2) * LP_BTERMS * WAVE * sizeof(u32x4);
}

int launch_split_b(int64_t k, int64_t n, const float* B, int64_t bsj, int64_t bsp, int dtype,
                   void* out, hipStream_t st) {
    const int nt16 = n <= 16 ? 1 : 2;
    const int64_t total = (k + 31) / 32 * nt16 * WAVE;
    int64_t blocks = cdiv_lp(total, 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    const bool bf = dtype == DT_BF16 || dtype == DT_BF16_SPLIT;
    if (bf)
        TSM_LAUNCH(split_b_kernel<FMT_BF16>, dim3((unsigned)blocks), dim3(256), 0, st, k, (int)n, B,
                   bsj, bsp, nt16, (u32x4*)out);
    else
        TSM_LAUNCH(split_b_kernel<FMT_F16>, dim3((unsigned)blocks), dim3(256), 0, st, k, (int)n, B,
                   bsj, bsp, nt16, (u32x4*)out);
    return 0;
}

template <int FMT, int KS, int NT16, bool SPLIT>
static void tsm2l_lp_go(int64_t m, int k, int n, const uint16_t* ah, const uint16_t* al,
                        int64_t lda, const float* B, int64_t bsj, int64_t bsp, float beta,
                        float* C, int64_t ldc, bool vec, int cus, hipStream_t st) {
    // k <= 16: one 128-row tile per wavefront (measured faster); k = 32: a
    // persistent grid of as many workgroups as fit at once, each wavefront
    // prefetching its next tile.  Never more than there are groups of 4 tiles.
    static const int occ_v = lp_occupancy(tsm2l_lp_kernel<FMT, KS, NT16, SPLIT, true>);
    static const int occ_s = lp_occupancy(tsm2l_lp_kernel<FMT, KS, NT16, SPLIT, false>);
    int64_t blocks = KS <= 4 ? INT64_MAX : (int64_t)cus * (vec ? occ_v : occ_s);
    const char* fb = std::getenv("TSM2X_RT_BLOCKS");
    if (fb && *fb && std::strtoll(fb, nullptr, 10) > 0) blocks = std::strtoll(fb, nullptr, 10);
    const int64_t need = cdiv_lp(cdiv_lp(m, 128), 4);
    if (blocks > need) blocks = need;
    if (blocks > 0x7fffffff) blocks = 0x7fffffff;
    if (blocks < 1) blocks = 1;
    dim3 g((unsigned)blocks), b(256);
    if (vec)
        TSM_LAUNCH((tsm2l_lp_kernel<FMT, KS, NT16, SPLIT, true>), g, b, 0, st, m, k, n, ah,
                           al, lda, B, bsj, bsp, beta, C, ldc);
    else
        TSM_LAUNCH((tsm2l_lp_kernel<FMT, KS, NT16, SPLIT, false>), g, b, 0, st, m, k, n,
                           ah, al, lda, B, bsj, bsp, beta, C, ldc);
}

template <int FMT, bool SPLIT>
static void tsm2l_lp_ks(int64_t m, int k, int n, const uint16_t* ah, const uint16_t* al,
                        int64_t lda, const float* B, int64_t bsj, int64_t bsp, float beta,
                        float* C, int64_t ldc, bool vec, int cus, hipStream_t st) {
#define TSM_L(KS, NT)                                                                          \
    tsm2l_lp_go<FMT, KS, NT, SPLIT>(m, k, n, ah, al, lda, B, bsj, bsp, beta, C, ldc, vec, cus, \
                                    st);                                                        \
    return
    if (k <= 8) { if (n <= 16) { TSM_L(2, 1); } TSM_L(2, 2); }
    if (k <= 16) { if (n <= 16) { TSM_L(4, 1); } TSM_L(4, 2); }
    if (n <= 16) { TSM_L(8, 1); }
    TSM_L(8, 2);
#undef TSM_L
}

int launch_tsm2l_lp(int64_t m, int64_t k, int64_t n, const void* A, int64_t lda, const float* B,
                    int64_t bsj, int64_t bsp, float beta, float* C, int64_t ldc, int dtype,
                    int cus, hipStream_t st) {
    const int fmt = (dtype == DT_BF16 || dtype == DT_BF16_SPLIT) ? FMT_BF16 : FMT_F16;
    const bool split = dtype == DT_BF16_SPLIT || dtype == DT_F16_SPLIT;
    const bool vec = ((uintptr_t)A & 15u) == 0 && (lda % 8) == 0 && ((uintptr_t)C & 15u) == 0 &&
                     (ldc % 4) == 0;
    const uint16_t* ah = (const uint16_t*)A;
    const uint16_t* al = split ? ah + lda * k : nullptr;
    const int ki = (int)k, ni = (int)n;
    if (fmt == FMT_BF16) {
        if (split)
            tsm2l_lp_ks<FMT_BF16, true>(m, ki, ni, ah, al, lda, B, bsj, bsp, beta, C, ldc, vec, cus, st);
        else
            tsm2l_lp_ks<FMT_BF16, false>(m, ki, ni, ah, al, lda, B, bsj, bsp, beta, C, ldc, vec, cus, st);
    } else {
        if (split)
            tsm2l_lp_ks<FMT_F16, true>(m, ki, ni, ah, al, lda, B, bsj, bsp, beta, C, ldc, vec, cus, st);
        else
            tsm2l_lp_ks<FMT_F16, false>(m, ki, ni, ah, al, lda, B, bsj, bsp, beta, C, ldc, vec, cus, st);
    }
    return 0;
}

static int launch_tn_lp_main(const LaunchTN& L, int dtype, hipStream_t st) {
    const int fmt = (dtype == DT_BF16 || dtype == DT_BF16_SPLIT) ? FMT_BF16 : FMT_F16;
    const bool split = dtype == DT_BF16_SPLIT || dtype == DT_F16_SPLIT;
    const bool vec = ((uintptr_t)L.X & 15u) == 0 && (L.ldx % 8) == 0 &&
                     ((uintptr_t)L.Y & 15u) == 0 && (L.ldy % 4) == 0;
    const uint16_t* xh = (const uint16_t*)L.X;
    const uint16_t* xl = split ? xh + L.ldx * L.ncols : nullptr;
    // L.groups 16-column tiles, a multiple of L.ct: L.ct of them per workgroup
    const int64_t gx = L.groups / L.ct;
    dim3 g((unsigned)gx, (unsigned)L.S), b(256);
    const int ni = (int)L.n;
    // Y is re-read by every column group: cached loads when there are several
    const bool yc = gx > 1;
    const u32x4* yt = (const u32x4*)L.yt;
#define TSM_T(F, NT, CT, SP, YD, ...)                                                              \
    {                                                                                               \
        if (vec && yc)                                                                              \
            TSM_LAUNCH((tn_lp_kernel<F, NT, CT, SP, true, true, YD, ##__VA_ARGS__>), g, b, 0, st,   \
                       L.R, L.ncols, ni, xh, xl, L.ldx, (const float*)L.Y, L.ldy, (float*)L.O,      \
                       L.ldo, L.rslice, L.part, yt, pf);                                            \
        else if (vec)                                                                               \
            TSM_LAUNCH((tn_lp_kernel<F, NT, CT, SP, true, false, YD, ##__VA_ARGS__>), g, b, 0, st,  \
                       L.R, L.ncols, ni, xh, xl, L.ldx, (const float*)L.Y, L.ldy, (float*)L.O,      \
                       L.ldo, L.rslice, L.part, yt, pf);                                            \
        else                                                                                        \
            TSM_LAUNCH((tn_lp_kernel<F, NT, CT, SP, false, false, YD, ##__VA_ARGS__>), g, b, 0, st, \
                       L.R, L.ncols, ni, xh, xl, L.ldx, (const float*)L.Y, L.ldy, (float*)L.O,      \
                       L.ldo, L.rslice, L.part, yt, pf);                                            \
        return 0;                                                                                   \
    }
    // Y straight from L2 when several column groups re-read it (measured,
    // bf16 split, 16384^2, n = 8: 4.9 TB/s staged, 5.2 direct, 5.85 direct
    // with two tiles per workgroup); staged through LDS when one group
    // streams it from HBM once (2^23 x 16: 5.15 staged, 4.06 direct).  Two
    // output tiles per workgroup always take Y direct (staged, they need
    // 101 KB of LDS per workgroup).  TSM2X_TN_YD=0/1 overrides (measurement).
    const int pf = L.pf;
    const char* yde = std::getenv("TSM2X_TN_YD");
    const bool yd = (yde && *yde) ? *yde == '1' : yc;
#define TSM_T2(F, SP)                                                                     \
    {                                                                                     \
        if (L.ct == 2) {                                                                  \
            if (L.n <= 16) TSM_T(F, 1, 2, SP, true) else TSM_T(F, 2, 2, SP, true)         \
        } else if (yd) {                                                                  \
            if (L.n <= 16) TSM_T(F, 1, 1, SP, true) else TSM_T(F, 2, 1, SP, true)         \
        } else {                                                                          \
            if (L.n <= 16) TSM_T(F, 1, 1, SP, false) else TSM_T(F, 2, 1, SP, false)       \
        }                                                                                 \
    }
    if (fmt == FMT_BF16) {
        if (yt) {
            // Y split once into packed terms: four tiles per workgroup, n > 16
            if (L.ct != 4 || L.n <= 16) return 1;
            if (split) TSM_T(FMT_BF16, 2, 4, true, true, true) else TSM_T(FMT_BF16, 2, 4, false, true, true)
        }
        if (L.ct == 4 && L.n <= 16) {
            if (split) TSM_T(FMT_BF16, 1, 4, true, true) else TSM_T(FMT_BF16, 1, 4, false, true)
        }
        if (split) TSM_T2(FMT_BF16, true) else TSM_T2(FMT_BF16, false)
    } else {
        if (split) TSM_T2(FMT_F16, true) else TSM_T2(FMT_F16, false)
    }
#undef TSM_T2
#undef TSM_T
    return 1;
}

int launch_tn_lp(const LaunchTN& L, int dtype, hipStream_t st) {
    if (L.yt) {
        // Y's bf16 terms in the operand order, as for B in tsm2r_lp (rows
        // of Y are the reduction index here: Y(j, p) = Y[j + p*ldy])
        if (launch_split_b(L.R, L.n, (const float*)L.Y, 1, L.ldy, dtype, (void*)L.yt, st)) return 1;
    }
    const int rc = launch_tn_lp_main(L, dtype, st);
    if (rc || L.S <= 1) return rc;
    return launch_split_reduce(DT_F32, L.groups, L.S, L.n <= 16 ? 16 : 32, 16, L.ncols, (int)L.n,
                               L.part, L.O, L.ldo, 0.0, st);
}

int launch_split(int64_t m, int64_t k, const float* A, int64_t lda, void* hi, void* lo,
                 int64_t ldh, int fmt, hipStream_t st) {
    const bool vec = ((uintptr_t)A & 15u) == 0 && (lda % 4) == 0 && ((uintptr_t)hi & 15u) == 0 &&
                     (!lo || ((uintptr_t)lo & 15u) == 0) && (ldh % 8) == 0;
    const int64_t total = cdiv_lp(m, 8) * k;
    int64_t blocks = cdiv_lp(total, 256);
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    dim3 g((unsigned)blocks), b(256);
    uint16_t* h = (uint16_t*)hi;
    uint16_t* l = (uint16_t*)lo;
#define TSM_SPLIT(F, LO, V) \
    TSM_LAUNCH((split_kernel<F, LO, V>), g, b, 0, st, m, k, A, lda, h, l, ldh)
    if (fmt == FMT_BF16) {
        if (lo) { if (vec) TSM_SPLIT(FMT_BF16, true, true); else TSM_SPLIT(FMT_BF16, true, false); }
        else { if (vec) TSM_SPLIT(FMT_BF16, false, true); else TSM_SPLIT(FMT_BF16, false, false); }
    } else {
        if (lo) { if (vec) TSM_SPLIT(FMT_F16, true, true); else TSM_SPLIT(FMT_F16, true, false); }
        else { if (vec) TSM_SPLIT(FMT_F16, false, true); else TSM_SPLIT(FMT_F16, false, false); }
    }
#undef TSM_SPLIT
    return 0;
}

}  // namespace tsm
