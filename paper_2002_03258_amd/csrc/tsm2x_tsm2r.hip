// TSM2R on gfx950 (MI355X): C = A*B with column-major A (m x k, k large) and
// B (k x n), n <= 32.  The kernel, its instances and the grid planner.
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
// multiplied (the prefetching of Algorithm 4); where every chunk is whole
// and the host asks for it (pf), in straight-line code that keeps those
// loads outstanding across the waits for the current chunk.  Lane l ends up with
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
    int64_t kslice, double* __restrict__ part, int bvec, int pf, double beta) {
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
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);   // wavefront-uniform
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

    auto mul = [&](const T (&av)[ST][RG][RL], const T (&bv)[NT16][ST]) {
#pragma unroll
        for (int st = 0; st < ST; ++st)
#pragma unroll
            for (int g = 0; g < RG; ++g)
#pragma unroll
                for (int q = 0; q < RL; ++q)
#pragma unroll
                    for (int t = 0; t < NT16; ++t)
                        acc[g][q][t] = M::op(bv[t][st], av[st][g][q], acc[g][q][t]);
    };
    // a whole chunk of a full tile: straight-line 16-byte loads; B columns
    // p >= n read column n - 1 (in range) and are zeroed after the wait
    auto loadA_full = [&](int64_t j0, T (&av)[ST][RG][RL]) {
        const T* base = A + row0 + RL * rl + (j0 + ST * kk) * lda;
#pragma unroll
        for (int st = 0; st < ST; ++st)
#pragma unroll
            for (int g = 0; g < RG; ++g)
                load_run<T, RL, true>(base + st * lda + 16 * RL * g, RL, true, av[st][g]);
    };
    auto loadB_full = [&](int64_t j0, T (&bv)[NT16][ST]) {
        typedef typename VecOf<T, BW>::type V;
#pragma unroll
        for (int t = 0; t < NT16; ++t) {
            const int p = 16 * t + rl;
            const T* __restrict__ src = B + j0 + ST * kk + (int64_t)(p < n ? p : n - 1) * ldb;
#pragma unroll
            for (int h = 0; h < ST / BW; ++h) {
                const V v = *reinterpret_cast<const V*>(src + h * BW);
#pragma unroll
                for (int e = 0; e < BW; ++e) bv[t][h * BW + e] = v[e];
            }
        }
    };
    auto mul_live = [&](const T (&av)[ST][RG][RL], const T (&bv)[NT16][ST]) {
        T bz[NT16][ST];
#pragma unroll
        for (int t = 0; t < NT16; ++t)
#pragma unroll
            for (int st = 0; st < ST; ++st) bz[t][st] = 16 * t + rl < n ? bv[t][st] : T(0);
        mul(av, bz);
    };

    // Every chunk whole: the next chunk held in flight across the waits for
    // this one (the scheduling barriers stop the compiler from sinking its
    // loads below them; with the bounds branches of the general loop, the
    // waits after each join counted nothing as in flight and drained every
    // load).  Not for the tall tiles (RG = 4), whose two chunks do not fit
    // the register budget.
    if (PF && RG <= 2 && VEC && pf && full && bvec && wk1 > wk0 && (wk1 - wk0) % CW == 0) {
        const int ng = (int)((wk1 - wk0) / CW);
        T aa[ST][RG][RL], ab[ST][RG][RL], ba[NT16][ST], bb[NT16][ST];
        loadB_full(wk0, ba);
        loadA_full(wk0, aa);
        int gc = 0;
        for (; gc + 2 < ng; gc += 2) {
            loadB_full(wk0 + CW * (gc + 1), bb);
            loadA_full(wk0 + CW * (gc + 1), ab);
            __builtin_amdgcn_sched_barrier(0);
            mul_live(aa, ba);
            loadB_full(wk0 + CW * (gc + 2), ba);
            loadA_full(wk0 + CW * (gc + 2), aa);
            __builtin_amdgcn_sched_barrier(0);
            mul_live(ab, bb);
        }
        if (gc + 1 < ng) {
            loadB_full(wk0 + CW * (gc + 1), bb);
            loadA_full(wk0 + CW * (gc + 1), ab);
            __builtin_amdgcn_sched_barrier(0);
            mul_live(aa, ba);
            mul_live(ab, bb);
        } else {
            mul_live(aa, ba);
        }
    } else if (wk1 > wk0) {
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
            mul(av, bv);
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

    nn_finish<T, NP, WK, TR, PG>(m, n, C, ldc, beta, tile, s, nsl, part,
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
// slices (longer streams per wavefront).  A pin from the caller (an
// autotuner) replaces either choice.
//
// With the next chunk held in flight (tsm2r_nn_kernel, pf) one workgroup per
// CU streams faster than 15/8 without it: where the shorter tiles can fill
// 7/8 to all of the CUs exactly once (tiles * S in [7/8, 1] x CUs), that plan
// is taken (A 10240^2 to 30720^2, n = 2..32: 0 to +14 %; grids of 320 on 256
// CUs, two rounds with a third of the CUs holding two, lost 14-24 %, and are
// never formed).  pf is also on for n > 16 and FP32 with n <= 4, with any
// grid (tsm2r_nn_kernel).
static int nn_pf(int64_t n, int dtype, int tall, int64_t W, int cus) {
    if (tall) return 0;
    if (n > 16 || (dtype == DT_F32 && n <= 4)) return 1;
    return (W <= cus && 8 * W >= 7 * (int64_t)cus) ? 1 : 0;
}

int plan_tsm2r(int64_t m, int64_t k, int64_t n, int dtype, int cus, bool vec, NNPlan* P,
               const NNPin* pin) {
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
    int64_t tall_force = (fh && *fh) ? std::strtoll(fh, nullptr, 10) : -1;
    int64_t s_pin = s_force;
    if (pin && pin->S > 0) s_pin = pin->S;
    if (pin && pin->tall >= 0) tall_force = pin->tall;

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
        if (s_pin > 0) S = s_pin;
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
            P->tall = tall;
            P->occ = I.occ;
        }
    }
    if (!found) return 1;
    // one workgroup per CU with the prefetch, unless the caller or an
    // override fixed the plan (the prefetch needs 16-byte loads of A)
    const bool free_plan = vec && s_pin <= 0 && tall_force < 0 && !(ft && *ft);
    if (free_plan) {
        NNInstance I{};
        if (nn_pick<true>(dtype, np, false, &I)) {
            const int64_t tiles = cdiv64(m, I.tile_rows);
            int64_t S = cus / tiles;
            const int64_t s_len = k / (WK * 64);
            const int64_t s_cost = (k * es) / ((int64_t)np * 200);
            if (S > s_len) S = s_len;
            if (S > s_cost) S = s_cost;
            if (S < 1) S = 1;
            const int64_t gran = (int64_t)WK * I.chunk;
            int64_t ks = cdiv64(k, S);
            ks = cdiv64(ks, gran) * gran;
            S = cdiv64(k, ks);
            const int64_t W = tiles * S;
            if (W <= cus && 8 * W >= 7 * (int64_t)cus && I.occ >= 1) {
                P->fn = I.fn;
                P->name = I.name;
                P->tiles = tiles;
                P->tile_rows = I.tile_rows;
                P->kslice = ks;
                P->S = (int)S;
                P->ws = S > 1 ? (size_t)tiles * S * np * I.tile_rows * 8 : 0;
                P->tall = 0;
                P->occ = I.occ;
            }
        }
    }
    P->pf = vec ? nn_pf(n, dtype, P->tall, P->tiles * P->S, cus) : 0;
    return 0;
}

int launch_tsm2r_nn(const LaunchNN& L, int dtype, hipStream_t st) {
    int n32 = (int)L.n;
    // 16-byte loads of B's column runs need an aligned B with ldb*size % 16 == 0
    const int es = dtype == DT_F64 ? 8 : 4;
    int bvec = aligned16(L.B) && ((L.ldb * es) % 16 == 0);
    // the next chunk held in flight (see tsm2r_nn_kernel) where it measured
    // faster (the plan's choice, plan_tsm2r): one workgroup per CU; n > 16,
    // where the matrix cores' share of a chunk is largest, +15-25 % (FP32 at
    // 32768^2, n = 32: 5.1 -> 6.0 TB/s); FP32 with n <= 4, +2-9 %; with the
    // 15/8 grid and n = 8, 16 it measured -5..+1 %.  TSM2X_NN_PF=0/1
    // overrides (measurement).
    const char* pfe = std::getenv("TSM2X_NN_PF");
    int pf = (pfe && *pfe) ? (int)std::strtol(pfe, nullptr, 10) : L.pf;
    double beta = L.beta;
    void* args[] = {(void*)&L.m,   (void*)&L.k,      (void*)&n32,    (void*)&L.A,
                    (void*)&L.lda, (void*)&L.B,      (void*)&L.ldb,  (void*)&L.C,
                    (void*)&L.ldc, (void*)&L.kslice, (void*)&L.part, (void*)&bvec,
                    (void*)&pf,    (void*)&beta};
    hipError_t e;
    {
        LaunchTimer timer(L.fn, st);
        e = hipLaunchKernel(L.fn, dim3((unsigned)L.tiles, (unsigned)L.S), dim3(256), args, 0, st);
    }
    if (e != hipSuccess) return 1;
    if (L.S > 1)
        return launch_split_reduce(dtype, L.tiles, L.S, L.np, L.tile_rows, L.m, (int)L.n, L.part,
                                   L.C, L.ldc, L.beta, st);
    return 0;
}

}  // namespace tsm
