// Device-side building blocks shared by the gfx950 kernels: 16-byte runs,
// the ticketed split-reduction protocol, the 16x16x4 matrix-core step and
// the row-tile finish of the TSM2R kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Sum of the WK wavefronts' double partials for one row tile and, when the k
// range is split across workgroups, the ticketed final sum.  `red` is LDS
// scratch of [WK][PG][TR] doubles; put(pg, red) stores this wavefront's
// values of columns pg .. pg+PG-1.
template <typename T, int NP, int WK, int TR, int PG, typename Put>
__device__ __forceinline__ void nn_finish(int64_t m, int n, T* __restrict__ C, int64_t ldc,
                                          int64_t tile, int s, int nsl,
                                          double* __restrict__ part,
                                          unsigned* __restrict__ tickets, double* red,
                                          Put&& put) {
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

}  // namespace tsm
