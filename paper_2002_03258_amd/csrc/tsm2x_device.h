// Device-side building blocks shared by the gfx950 kernels: 16-byte runs,
// the 16x16x4 matrix-core step, the workgroup-level finish of the split
// reductions and the ordered sum of split partials.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsm {

constexpr int WAVE = 64;

// Orders this wavefront's LDS stores and loads around a hand-over of staged
// data between its lanes.  The compiler sees one lane's accesses only: where
// it can prove that a lane's own store and later load touch different
// addresses (the lane reads what other lanes wrote), it may move the load
// above the store, or reuse a load from an earlier tile, and the lane then
// reads stale LDS.  The fence forbids that reordering; at wavefront scope it
// emits no instruction (a wavefront's LDS operations complete in order).
// Used before a tile is staged (its previous contents have been read) and
// before the staged tile is read back.
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

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

// The store counterpart; NT = false for ordinary stores (a wavefront whose
// 16-byte stores leave gaps that a second instruction fills: non-temporal
// stores of such half-filled lines reach HBM as separate partial writes).
template <typename T, int RL, bool VEC, bool NT = true>
__device__ __forceinline__ void store_run(T* __restrict__ p, int64_t valid,
                                          bool full, const T (&v)[RL]) {
    if (VEC && full) {
        typedef typename VecOf<T, RL>::type V;
        V x;
#pragma unroll
        for (int r = 0; r < RL; ++r) x[r] = v[r];
        if (NT)
            __builtin_nontemporal_store(x, reinterpret_cast<V*>(p));
        else
            *reinterpret_cast<V*>(p) = x;
    } else {
#pragma unroll
        for (int r = 0; r < RL; ++r)
            if (r < valid) p[r] = v[r];
    }
}

// --------------------------------------------------------------------------
// Matrix-core building block shared by the kernels below.
//
// A 16x16x4 MFMA computes D[16x16] += S[16x4] * T[4x16] with lane l
// (rl = l % 16, kk = l / 16) supplying S[rl][kk] and T[kk][rl] and holding
// D[mrow(kk, r)][rl] in its accumulator element r = 0..3, where
// mrow = 4*kk + r for the float variant and kk + 4*r for the double one.
// The tall operand is always fed through T: lane l loads 16 bytes = RL
// consecutive rows RL*rl + q (q < RL) of one column and hands element q to
// MFMA instance q, so every element of the tall operand is loaded once, with
// 16-byte loads, and each instance covers 16 rows strided by RL.
// --------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
    typedef f32x4 acc;
    static __device__ __forceinline__ int mrow(int kk, int r) { return 4 * kk + r; }
    static __device__ __forceinline__ acc op(float s, float t, acc d) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(s, t, d, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    typedef f64x4 acc;
    static __device__ __forceinline__ int mrow(int kk, int r) { return kk + 4 * r; }
    static __device__ __forceinline__ acc op(double s, double t, acc d) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(s, t, d, 0, 0, 0);
    }
};

// An output element: v, or v + beta * (old value) when beta != 0 (the old
// value is read only then), added in double and rounded once to T.
template <typename T>
__device__ __forceinline__ T beta_out(double v, double beta, const T* p) {
    return (T)(beta != 0.0 ? v + beta * (double)*p : v);
}

// Sum of NSUM wavefronts' partials (double, wavefront order) for one row
// tile of TR rows of a workgroup of WK wavefronts.  With one k slice the
// result is the output; otherwise it is this workgroup's partial,
// part[((tile * nsl + s) * NP + p) * TR + row], and a second kernel
// (split_reduce_kernel) adds the slices in order.  `red` is LDS scratch of
// [NSUM][PG][TR] doubles; put(pg, red) stores this wavefront's values of
// columns pg .. pg+PG-1 (NSUM = WK: every wavefront all TR rows, summed;
// NSUM = 1: each wavefront its own rows of the tile).  C := beta*C + sum (C is
// read only if beta != 0).
template <typename T, int NP, int WK, int TR, int PG, int NSUM = WK, typename Put>
__device__ __forceinline__ void nn_finish(int64_t m, int n, T* __restrict__ C, int64_t ldc,
                                          double beta, int64_t tile, int s, int nsl,
                                          double* __restrict__ part, double* red, Put&& put) {
    constexpr int NT = WAVE * WK;
    const int64_t row0 = tile * TR;
#pragma unroll
    for (int pg = 0; pg < NP; pg += PG) {
        if (pg < n) {
            __syncthreads();
            put(pg, red);
            __syncthreads();
            for (int e = threadIdx.x; e < PG * TR; e += NT) {
                const int pp = e / TR, rr = e % TR;
                const int p = pg + pp;
                const int64_t row = row0 + rr;
                double v = red[pp * TR + rr];
#pragma unroll
                for (int ww = 1; ww < NSUM; ++ww) v += red[(ww * PG + pp) * TR + rr];
                if (p < n && row < m) {
                    if (nsl == 1)
                        C[row + p * ldc] = beta_out(v, beta, C + row + p * ldc);
                    else
                        part[((tile * nsl + s) * NP + p) * TR + rr] = v;
                }
            }
        }
    }
}

// The same for the column tiles of the tn kernels: acc[t][r] of lane l is
// O[c0 + mrow(l/16, r), 16 t + l%16]; partials go to
// part[((ctile * nsl + s) * NP + p) * 16 + c].
template <typename T, int NT16, int WK, typename Acc, typename MRow>
__device__ __forceinline__ void tn_finish(int64_t ncols, int n, T* __restrict__ O, int64_t ldo,
                                          double beta, int64_t ctile, int s, int nsl,
                                          double* __restrict__ part, double (*red)[WAVE][4 * NT16],
                                          const Acc (&acc)[NT16], MRow mrow) {
    constexpr int NV = 4 * NT16;
    constexpr int NP = 16 * NT16;
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
#pragma unroll
    for (int t = 0; t < NT16; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[w][lane][4 * t + r] = (double)acc[t][r];
    __syncthreads();
    for (int e = threadIdx.x; e < WAVE * NV; e += WAVE * WK) {
        const int ln = e / NV, vi = e % NV;
        double v = red[0][ln][vi];
#pragma unroll
        for (int ww = 1; ww < WK; ++ww) v += red[ww][ln][vi];
        const int t = vi / 4, r = vi % 4;
        const int c = mrow(ln >> 4, r);
        const int64_t col = ctile * 16 + c;
        const int p = 16 * t + (ln & 15);
        if (nsl == 1) {
            if (col < ncols && p < n) O[col + p * ldo] = beta_out(v, beta, O + col + p * ldo);
        } else {
            part[((ctile * nsl + s) * NP + p) * 16 + c] = v;
        }
    }
}

// Ordered sum of split partials: O[g*W + r, p] = beta * O[g*W + r, p] + sum
// over s of part[((g * S + s) * NP + p) * W + r], for rows g*W + r < rows and
// p < n (O is read only if beta != 0).
// One thread per output when S is small.  For many slices one wavefront
// per output: lane l adds slices l, l+64, ... in order, then a butterfly in a
// fixed pattern combines the lanes, so the result does not depend on timing.
template <typename T, bool WIDE>
__global__ __launch_bounds__(256) void split_reduce_kernel(int64_t groups, int S, int NP, int W,
                                                           int64_t rows, int n,
                                                           const double* __restrict__ part,
                                                           T* __restrict__ O, int64_t ldo,
                                                           double beta) {
    const int64_t E = (int64_t)NP * W;
    const int64_t total = groups * E;
    if (!WIDE) {
        for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
             idx += (int64_t)gridDim.x * blockDim.x) {
            const int64_t g = idx / E, e = idx % E;
            const int p = (int)(e / W), r = (int)(e % W);
            const int64_t row = g * W + r;
            if (p < n && row < rows) {
                double v = 0.0;
                for (int s = 0; s < S; ++s) v += part[(g * S + s) * E + e];
                O[row + p * ldo] = beta_out(v, beta, O + row + p * ldo);
            }
        }
    } else {
        const int lane = threadIdx.x & (WAVE - 1);
        const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / WAVE;
        const int64_t nw = (int64_t)gridDim.x * blockDim.x / WAVE;
        for (int64_t idx = wid; idx < total; idx += nw) {
            const int64_t g = idx / E, e = idx % E;
            const int p = (int)(e / W), r = (int)(e % W);
            const int64_t row = g * W + r;
            if (p < n && row < rows) {     // uniform across the wavefront
                double v = 0.0;
                for (int s = lane; s < S; s += WAVE) v += part[(g * S + s) * E + e];
#pragma unroll
                for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
                if (lane == 0) O[row + p * ldo] = beta_out(v, beta, O + row + p * ldo);
            }
        }
    }
}

}  // namespace tsm
