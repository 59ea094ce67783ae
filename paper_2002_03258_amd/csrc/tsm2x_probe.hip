// Bandwidth probes (measurement support; no product uses them): the HBM
// ceilings the products are compared with, measured with the products' own
// load and store forms.
//
//  probe_stream_kernel  linear streams of 16-byte non-temporal accesses, each
//                       wavefront moving one 4 KB piece per iteration of a
//                       grid-stride loop: read only, copy, or write only.
//  probe_tiles_kernel   the access pattern of the TSM2L kernel (rowtile)
//                       without its arithmetic: a persistent grid walks row
//                       tiles, each lane loading 16-byte runs of the kin
//                       input columns (4 columns x 256 bytes per wavefront
//                       instruction) and storing 16-byte runs of the nout
//                       output columns in the rowtile order.  With a second
//                       input (TWO), the pattern of the fused TSM2L backward:
//                       two inputs of kin columns read, one output written,
//                       in its taller tiles.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tsm2x.h"
#include "tsm2x_device.h"
#include "tsm2x_internal.h"

namespace tsm {

typedef uint32_t u32x4p __attribute__((ext_vector_type(4)));

// KIND 0: read src (the xor of every word is compared with a value it never
// takes in practice, so the loads cannot be dropped; a match writes one word
// of dst); 1: copy src to dst; 2: write a pattern to dst.
template <int KIND>
__global__ __launch_bounds__(256) void probe_stream_kernel(const u32x4p* __restrict__ src,
                                                           u32x4p* __restrict__ dst,
                                                           int64_t nvec) {
    constexpr int U = 4;                          // 16-byte accesses per lane per piece
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / WAVE;
    uint32_t acc = 0;
    for (int64_t base = wave * (U * WAVE); base < nvec; base += nwaves * (U * WAVE)) {
        u32x4p v[U];
        if (KIND != 2) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = base + u * WAVE + lane;
                v[u] = i < nvec ? __builtin_nontemporal_load(src + i) : u32x4p{0, 0, 0, 0};
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t x = (uint32_t)(base + u * WAVE + lane);
                v[u] = u32x4p{x, x ^ 1u, x ^ 2u, x ^ 3u};
            }
        }
        if (KIND == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = base + u * WAVE + lane;
                if (i < nvec) __builtin_nontemporal_store(v[u], dst + i);
            }
        }
    }
    if (KIND == 0 && acc == 0x5bd1e995u && lane == 0) dst[0] = u32x4p{acc, 0, 0, 0};
}

// Output column c = 16 t + mrow(kk, rr) of a row tile receives input column
// 4 ((4 t + rr) % KS) + kk of the same rows (of X, or of X + Y with TWO): a
// fixed column mapping, so that every store depends on a load; only the
// bytes moved matter.
template <typename T, int KS, int NT16, int RG, bool VEC, bool TWO>
__global__ __launch_bounds__(256) void probe_tiles_kernel(int64_t m, int kin, int nout,
                                                          const T* __restrict__ X, int64_t ldx,
                                                          const T* __restrict__ Y, int64_t ldy,
                                                          T* __restrict__ O, int64_t ldo) {
    typedef Mfma<T> M;
    constexpr int RL = 16 / (int)sizeof(T);
    constexpr int TR = 16 * RL * RG;
    constexpr int WPB = 4;
    const int lane = threadIdx.x & (WAVE - 1);
    const int rl = lane & 15, kk = lane >> 4;
    const int w = threadIdx.x / WAVE;
    const int64_t ntiles = (m + TR - 1) / TR;
    const int64_t tstride = (int64_t)gridDim.x * WPB;
    for (int64_t tile = (int64_t)blockIdx.x * WPB + w; tile < ntiles; tile += tstride) {
        const int64_t row0 = tile * TR;
        const bool full = row0 + TR <= m;
        T xv[KS][RG][RL], yv[TWO ? KS : 1][RG][RL];
#pragma unroll
        for (int st = 0; st < KS; ++st) {
            const int ji = 4 * st + kk;
#pragma unroll
            for (int g = 0; g < RG; ++g) {
                const int64_t r = row0 + 16 * RL * g + RL * rl;
                if (ji < kin) {
                    load_run<T, RL, VEC>(X + r + ji * ldx, m - r, full, xv[st][g]);
                    if (TWO) load_run<T, RL, VEC>(Y + r + ji * ldy, m - r, full, yv[TWO ? st : 0][g]);
                } else {
#pragma unroll
                    for (int q = 0; q < RL; ++q) xv[st][g][q] = yv[TWO ? st : 0][g][q] = T(0);
                }
            }
        }
        if (TWO) {
#pragma unroll
            for (int st = 0; st < KS; ++st)
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int q = 0; q < RL; ++q) xv[st][g][q] += yv[TWO ? st : 0][g][q];
        }
#pragma unroll
        for (int g = 0; g < RG; ++g) {
            const int64_t r = row0 + 16 * RL * g + RL * rl;
#pragma unroll
            for (int t = 0; t < NT16; ++t)
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int col = 16 * t + M::mrow(kk, rr);
                    if (col < nout) store_run<T, RL, VEC>(O + r + col * ldo, m - r, full,
                                                          xv[(4 * t + rr) % KS][g]);
                }
        }
    }
}

template <typename K>
static int probe_occupancy(K kernel) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, 0) != hipSuccess || nb < 1)
        nb = 1;
    return nb;
}

template <typename T, int KS, int NT16, int RG, bool TWO>
static void probe_tiles_go(int64_t m, int kin, int nout, const void* X, int64_t ldx,
                           const void* Y, int64_t ldy, void* O, int64_t ldo, int64_t blocks,
                           int cus, hipStream_t st) {
    const bool vec = ((uintptr_t)X & 15u) == 0 && ((uintptr_t)O & 15u) == 0 &&
                     (ldx * (int64_t)sizeof(T)) % 16 == 0 && (ldo * (int64_t)sizeof(T)) % 16 == 0 &&
                     (!TWO || (((uintptr_t)Y & 15u) == 0 && (ldy * (int64_t)sizeof(T)) % 16 == 0));
    static const int occ = probe_occupancy(probe_tiles_kernel<T, KS, NT16, RG, true, TWO>);
    constexpr int64_t TR = 16 * (16 / (int64_t)sizeof(T)) * RG;
    const int64_t need = ((m + TR - 1) / TR + 3) / 4;
    int64_t bx = blocks > 0 ? blocks : (int64_t)cus * occ;
    if (bx > need) bx = need;
    if (bx > 0x7fffffff) bx = 0x7fffffff;
    if (bx < 1) bx = 1;
    if (vec)
        TSM_LAUNCH((probe_tiles_kernel<T, KS, NT16, RG, true, TWO>), dim3((unsigned)bx), dim3(256), 0,
                   st, m, kin, nout, (const T*)X, ldx, (const T*)Y, ldy, (T*)O, ldo);
    else
        TSM_LAUNCH((probe_tiles_kernel<T, KS, NT16, RG, false, TWO>), dim3((unsigned)bx), dim3(256),
                   0, st, m, kin, nout, (const T*)X, ldx, (const T*)Y, ldy, (T*)O, ldo);
}

// the row groups per lane of the rowtile instance for (kin, nout); with two
// inputs those of the fused backward (two groups)
template <typename T>
static void probe_tiles_pick(int64_t m, int kin, int nout, const void* X, int64_t ldx,
                             const void* Y, int64_t ldy, void* O, int64_t ldo, int64_t blocks,
                             int cus, hipStream_t st) {
    const bool wide = nout > 16;
#define TSM_P(KS, NT, RG)                                                                          \
    {                                                                                              \
        if (Y) probe_tiles_go<T, KS, NT, 2, true>(m, kin, nout, X, ldx, Y, ldy, O, ldo, blocks,   \
                                                   cus, st);                                        \
        else probe_tiles_go<T, KS, NT, RG, false>(m, kin, nout, X, ldx, Y, ldy, O, ldo, blocks,   \
                                                   cus, st);                                        \
        return;                                                                                    \
    }
    if (kin <= 8) {
        if (wide) TSM_P(2, 2, 2) else TSM_P(2, 1, 2)
    } else if (kin <= 16) {
        if (wide) TSM_P(4, 2, 2) else TSM_P(4, 1, 1)
    } else {
        if (wide) TSM_P(8, 2, 1) else TSM_P(8, 1, 1)
    }
#undef TSM_P
}

}  // namespace tsm

using namespace tsm;

extern "C" {

int tsm2x_probe_stream(int kind, const void* src, void* dst, int64_t bytes, int64_t blocks,
                       void* stream) {
    if (kind < 0 || kind > 2) return -1;
    if (kind != 2 && (!src || ((uintptr_t)src & 15u))) return -2;
    if (!dst || ((uintptr_t)dst & 15u)) return -3;
    if (bytes < 0 || bytes % 16) return -4;
    if (blocks < 0 || blocks > 0x7fffffff) return -5;
    if (bytes == 0) return TSM_SUCCESS;
    const int64_t nvec = bytes / 16;
    const int64_t pieces = (nvec + 4 * WAVE - 1) / (4 * WAVE);     // 4 KB per wavefront
    int64_t bx = blocks > 0 ? blocks : 65536;
    if (bx > (pieces + 3) / 4) bx = (pieces + 3) / 4;
    if (bx < 1) bx = 1;
    hipStream_t st = (hipStream_t)stream;
    const dim3 g((unsigned)bx), b(256);
    const u32x4p* s = (const u32x4p*)src;
    u32x4p* d = (u32x4p*)dst;
    if (kind == 0) TSM_LAUNCH(probe_stream_kernel<0>, g, b, 0, st, s, d, nvec);
    else if (kind == 1) TSM_LAUNCH(probe_stream_kernel<1>, g, b, 0, st, s, d, nvec);
    else TSM_LAUNCH(probe_stream_kernel<2>, g, b, 0, st, s, d, nvec);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? TSM_SUCCESS : TSM_ERR_HIP;
}

int tsm2x_probe_tiles(int64_t m, int kin, int nout, const void* X, int64_t ldx, const void* Y,
                      int64_t ldy, void* O, int64_t ldo, int dtype, int64_t blocks, void* stream) {
    if (m < 0) return -1;
    if (kin < 1 || kin > 32) return -2;
    if (nout < 1 || nout > 32) return -3;
    if (!X && m > 0) return -4;
    if (ldx < (m > 1 ? m : 1)) return -5;
    if (Y && ldy < (m > 1 ? m : 1)) return -7;
    if (!O && m > 0) return -8;
    if (ldo < (m > 1 ? m : 1)) return -9;
    if (dtype != TSM_F64 && dtype != TSM_F32) return -10;
    if (blocks < 0) return -11;
    if (m == 0) return TSM_SUCCESS;
    int cus = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 256;
    hipStream_t st = (hipStream_t)stream;
    if (dtype == TSM_F64)
        probe_tiles_pick<double>(m, kin, nout, X, ldx, Y, ldy, O, ldo, blocks, cus, st);
    else
        probe_tiles_pick<float>(m, kin, nout, X, ldx, Y, ldy, O, ldo, blocks, cus, st);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? TSM_SUCCESS : TSM_ERR_HIP;
}

}  // extern "C"
