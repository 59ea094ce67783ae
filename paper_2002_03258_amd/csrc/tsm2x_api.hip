// C ABI of the tall-and-skinny product library (declared in include/tsm2x.h):
// argument checking (host only, before any HIP call), launch planning,
// workspace management and dispatch to the gfx950 kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/tsm2x.h"
#include "tsm2x_internal.h"

using namespace tsm;

namespace {

thread_local std::string g_last_hip;

int hip_fail(hipError_t e, const char* what) {
    g_last_hip = std::string(what) + ": " + hipGetErrorString(e);
    return TSM_ERR_HIP;
}

int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return TSM_SUCCESS;
}

struct DevState {
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int cus = 0;
};
std::mutex g_mu;
std::vector<DevState> g_dev;

DevState* dev_state(int* dev_out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    if (dev_out) *dev_out = dev;
    if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
    return &g_dev[dev];
}

int cu_count() {
    std::lock_guard<std::mutex> lk(g_mu);
    DevState* d = dev_state(nullptr);
    if (!d) return 256;
    if (d->cus == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess || v <= 0)
            v = 256;
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            v = 256;
        d->cus = v > 0 ? v : 256;
    }
    return d->cus;
}

int64_t env_int(const char* name, int64_t dflt) {
    const char* s = std::getenv(name);
    if (!s || !*s) return dflt;
    return std::strtoll(s, nullptr, 10);
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool valid_dtype(int dt) { return dt >= TSM_F64 && dt <= TSM_F16_SPLIT; }
bool plain_dtype(int dt) { return dt == TSM_F64 || dt == TSM_F32; }
int esize(int dt) { return dt == TSM_F64 ? 8 : 4; }

bool vec_ok(const void* p, int64_t ld, int es) {
    return ((uintptr_t)p & 15u) == 0 && ((ld * es) % 16) == 0;
}

int pow2_ge(int64_t n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

// ------------------------------------------------------------- plans
// TSM2R plans pinned by the caller, per (m, k, n, dtype); shared by all devices
typedef std::tuple<int64_t, int64_t, int64_t, int> PinKey;
std::mutex g_pin_mu;
std::map<PinKey, NNPin> g_pins;

NNPin pin_of(int64_t m, int64_t k, int64_t n, int dtype) {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    auto it = g_pins.find(PinKey(m, k, n, dtype));
    return it == g_pins.end() ? NNPin{0, -1} : it->second;
}

int plan_nn(int64_t m, int64_t k, int64_t n, int dtype, int cus, bool vec, NNPlan* P) {
    const NNPin pin = pin_of(m, k, n, dtype);
    return plan_tsm2r(m, k, n, dtype, cus, vec, P, &pin);
}

struct RTPlan {
    int kp;
    int64_t cpb;
    int64_t bx, by;
};

// rowtile: a wavefront owns 16*RL*RG rows; one pass covers up to 32 output
// columns.  For nout <= 32 a persistent grid of about 8 workgroups per CU
// walks the row tiles; wider outputs are also split into column ranges.
RTPlan plan_rowtile(int64_t m, int64_t kin, int64_t nout, int dt, int cus) {
    RTPlan P{};
    const int es = esize(dt);
    const int RL = 16 / es;
    P.kp = kin <= 8 ? 8 : (kin <= 16 ? 16 : 32);
    // row groups per lane of the instance rowtile_dispatch launches
    const int RG = P.kp == 8 ? 2 : (P.kp == 16 && nout > 16 ? 2 : 1);
    const int64_t TR = 16 * RL * RG;
    const int64_t ntiles = cdiv(m, TR);
    const int64_t wblocks = cdiv(ntiles, 4);
    // nout <= 32 (TSM2L): the persistent grid is capped by occupancy at launch.
    // Wide outputs (dA of TSM2R, write-bound): one workgroup per CU, each
    // wavefront keeping one row tile for a long column range.  Measured: the
    // fewer column ranges are written at once, the closer together in time
    // each column's row tiles are written (256 workgroups: FP32 6.0 TB/s;
    // 1024: 4.9 TB/s)
    const int64_t cap = env_int("TSM2X_RT_BLOCKS", (int64_t)cus * (nout > 32 ? 1 : 4));
    if (nout <= 32) {
        P.cpb = nout;
        P.by = 1;
    } else {
        // enough column ranges to fill the machine, each a multiple of 32
        int64_t by = cdiv(cap, wblocks);
        if (by < 1) by = 1;
        int64_t cpb = cdiv(nout, by);
        cpb = cdiv(cpb, 32) * 32;
        if (cpb < 32) cpb = 32;
        P.cpb = cpb;
        P.by = cdiv(nout, cpb);
    }
    int64_t bx = wblocks;
    int64_t lim = cap / P.by;
    if (lim < 1) lim = 1;
    if (bx > lim) bx = lim;
    if (bx < 1) bx = 1;
    P.bx = bx;
    return P;
}

struct TNPlan {
    int64_t groups;         // 16-column output tiles (a multiple of ct)
    int S;
    int64_t rslice;
    int rg;
    int ct;                 // output tiles per workgroup
    int pf;                 // 16-bit forms: the next step's X held in flight
    bool yt;                // bf16 planes, n > 16: Y split once into packed terms
    size_t yt_off;          // their offset in the workspace
    size_t ws;
};

// tn: one workgroup per ct 16-row output tiles (columns of X) and slice of
// R; the WK = 4 wavefronts split the slice.
TNPlan plan_tn(int64_t R, int64_t ncols, int64_t n, int dt, int cus) {
    TNPlan P{};
    // output tiles per workgroup: two share each Y tile when there are
    // several column groups (Y is then re-read by every group).  The 16-bit
    // forms take Y straight from L2 then (staged in LDS too, two tiles needed
    // one workgroup per CU).  With n > 16 two tiles fit one workgroup per CU
    // only; with the next step in flight they still beat one tile (A 16384^2
    // and 32768^2, n = 24, 32: split 3.4-4.2 -> 4.4-4.9 TB/s, single
    // 2.0-2.6 -> 2.5-3.1; without the prefetch one tile was faster)
    // bfloat16 planes with n <= 16 and more than four tiles: four tiles per
    // workgroup and one workgroup per CU on the 16-bit matrix cores
    // (tn_lp_kernel, MX; A 16384^2, n = 8: split 5.8 -> 6.6 TB/s, single
    // 5.4 -> 6.5 in the access-pattern probe of this grid)
    // For n > 16 the four tiles take Y's bf16 terms split once per call into
    // the workspace (their registers would not hold the split in the step;
    // A 16384^2, n = 32: split 4.4 -> 5.3 TB/s, single 3.4 -> 4.7), while
    // Y's terms stay below 256 MB (192 bytes per row: R up to 1.4 M).
    const bool bf = dt == DT_BF16 || dt == DT_BF16_SPLIT;
    const size_t yt_bytes = lp_bterms_bytes(R, n);
    const bool four = bf && cdiv(ncols, 16) > 4 && (n <= 16 || yt_bytes <= ((size_t)256 << 20));
    const int ct_dflt = four ? 4 : 2;
    P.ct = ncols > 16 ? (int)env_int("TSM2X_TN_CT", ct_dflt) : 1;
    if (P.ct == 4 && !bf) P.ct = 2;
    if (P.ct != 1 && P.ct != 2 && P.ct != 4) P.ct = 1;
    // rows per wavefront loop iteration: G stages of 16*RL rows for the
    // float kernels (one stage with two output tiles), 128 for the 16-bit form
    P.rg = P.ct >= 2 ? 1 : (int)env_int("TSM2X_TN_G", 2);
    if (P.rg != 1 && P.rg != 2 && P.rg != 4) P.rg = 2;
    const int64_t RB = plain_dtype(dt) ? 16 * (16 / esize(dt)) * P.rg : 128;
    const int NT16 = n <= 16 ? 1 : 2;
    P.groups = cdiv(cdiv(ncols, 16), P.ct) * P.ct;
    const int64_t target = env_int("TSM2X_TN_TARGET_BLOCKS", (int64_t)cus * (P.ct == 4 ? 1 : 2));
    int64_t S = cdiv(target, P.groups / P.ct);
    const int64_t s_len = R / (RB * 4 * 8);   // >= 8 steps per wavefront
    if (S > s_len) S = s_len;
    if (S < 1) S = 1;
    int64_t rs = cdiv(R, S);
    rs = cdiv(rs, RB * 4) * (RB * 4);
    P.rslice = rs;
    P.S = (int)cdiv(R, rs);
    if (P.S < 1) P.S = 1;
    P.ws = P.S > 1 ? (size_t)P.groups * P.S * 256 * NT16 * 8 : 0;
    P.yt = P.ct == 4 && n > 16;
    if (P.yt) {
        P.yt_off = (P.ws + 255) / 256 * 256;
        P.ws = P.yt_off + yt_bytes;
    }
    // The next step held in flight (tn_kernel, tn_lp_kernel), where it
    // measured faster.  Float forms: for n > 16, +48-66 % (A 16384^2 to
    // 32768^2: 3.0-3.3 -> 4.5-5.3 TB/s); for n <= 16 from -18 % to +6 %, so
    // not there.  16-bit single form: always (n = 8 and 16: 3.8-4.2 -> 4.8-5.7
    // TB/s) and for n > 16 (above).  16-bit split form with n <= 16, whose
    // steps move twice the bytes: only when the grid holds more than two
    // workgroups per CU (at A 16384^2, n = 8, one round of 512 workgroups:
    // 5.80 TB/s without, 5.21 with; at 32768^2, four rounds: 6.34 -> 6.51
    // (n = 8), 5.89 -> 6.17 (n = 16)).  bfloat16 planes with several column
    // groups run on the bf16 matrix cores (tn_lp_kernel, MX): with four tiles
    // the single form takes two steps (probe, A 16384^2, n = 8: 6.6 TB/s
    // against 5.8 with one; packed dC terms, n = 32: 4.7 against 3.8) and the
    // split form one (two do not fit its registers); with two tiles (an
    // override) one step for n <= 8 (5.5 against 4.9 TB/s).
    const bool split = dt == DT_BF16_SPLIT || dt == DT_F16_SPLIT;
    const bool mx = bf && (!split || n <= 16 || P.yt) && P.groups / P.ct > 1;
    const bool pf = plain_dtype(dt) ? n > 16
                    : mx            ? P.ct == 4 || n > 8
                                    : !split || n > 16 || (P.groups / P.ct) * P.S > 2 * (int64_t)cus;
    P.pf = (int)env_int("TSM2X_TN_PF", pf ? 1 : 0);
    return P;
}

// Workspace: caller's (checked) or the library's grow-only per-device buffer.
int get_ws(size_t need, void* user, size_t user_bytes, void** out) {
    *out = nullptr;
    if (need == 0) return TSM_SUCCESS;
    if (user) {
        if (user_bytes < need || ((uintptr_t)user & 255u)) return TSM_ERR_WORKSPACE;
        *out = user;
        return TSM_SUCCESS;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    DevState* d = dev_state(nullptr);
    if (!d) return hip_fail(hipErrorInvalidDevice, "hipGetDevice");
    if (d->ws_bytes < need) {
        if (d->ws) {
            hipError_t e = hipFree(d->ws);
            d->ws = nullptr;
            d->ws_bytes = 0;
            if (e != hipSuccess) return hip_fail(e, "hipFree(workspace)");
        }
        size_t bytes = need < ((size_t)1 << 20) ? ((size_t)1 << 20) : need;
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            g_last_hip = std::string("hipMalloc(workspace): ") + hipGetErrorString(e);
            return TSM_ERR_ALLOC;
        }
        d->ws = p;
        d->ws_bytes = bytes;
    }
    *out = d->ws;
    return TSM_SUCCESS;
}

// Validation of (m, k, n, A, lda, B, ldb, C, ldc, dtype) for C = A*B with
// column-major (or, for `rowA`, row-major) A.  `base` is the position of m.
int check_mm(int base, int64_t m, int64_t k, int64_t n, const void* A, int64_t lda,
             const void* B, int64_t ldb, const void* C, int64_t ldc, int dtype, bool rowA) {
    if (m < 0) return -(base + 0);
    if (k < 0) return -(base + 1);
    if (n < 0) return -(base + 2);
    if (!A && m > 0 && k > 0) return -(base + 3);
    const int64_t mina = rowA ? (k > 1 ? k : 1) : (m > 1 ? m : 1);
    if (lda < mina) return -(base + 4);
    if (!B && k > 0 && n > 0) return -(base + 5);
    if (ldb < (k > 1 ? k : 1)) return -(base + 6);
    if (!C && m > 0 && n > 0) return -(base + 7);
    if (ldc < (m > 1 ? m : 1)) return -(base + 8);
    if (!valid_dtype(dtype)) return -(base + 9);
    return TSM_SUCCESS;
}

// Validation for the extended product entry points; argument positions
// 1 transA, 2 transB, 3 m, 4 k, 5 n, 6 A, 7 lda, 8 B, 9 ldb, 10 beta, 11 C,
// 12 ldc, 13 dtype.
int check_ex(int transA, int transB, int64_t m, int64_t k, int64_t n, const void* A,
             int64_t lda, const void* B, int64_t ldb, const void* C, int64_t ldc, int dtype) {
    if (transA != 0 && transA != 1) return -1;
    if (transB != 0 && transB != 1) return -2;
    if (m < 0) return -3;
    if (k < 0) return -4;
    if (n < 0) return -5;
    if (!A && m > 0 && k > 0) return -6;
    const int64_t mina = transA ? k : m;
    if (lda < (mina > 1 ? mina : 1)) return -7;
    if (!B && k > 0 && n > 0) return -8;
    const int64_t minb = transB ? n : k;
    if (ldb < (minb > 1 ? minb : 1)) return -9;
    if (!C && m > 0 && n > 0) return -11;
    if (ldc < (m > 1 ? m : 1)) return -12;
    if (!valid_dtype(dtype)) return -13;
    return TSM_SUCCESS;
}

// Leading dimension of the column-major copy of a transposed B (k x n), kept
// a multiple of 16 bytes so the kernels' 16-byte B loads apply.
int64_t bt_ld(int64_t k, int ce) { return cdiv(k, 16 / ce) * (16 / ce); }

// Bytes of split partials of a TSM2R-kernel product of at most 32 columns,
// for the kernel instance the call launches (`vec`: 16-byte loads of A).
size_t tsm2r_part(int transA, int64_t m, int64_t k, int64_t n, int dtype, bool vec) {
    const int cus = cu_count();
    if (!plain_dtype(dtype)) {
        NNPlan P{};
        plan_tsm2r_lp(m, k, n, dtype, cus, vec, &P);
        return P.ws;
    }
    if (transA) return plan_tn(k, m, n, dtype, cus).ws;
    NNPlan P{};
    return plan_nn(m, k, n, dtype, cus, vec, &P) ? 0 : P.ws;
}

// Workspace of a TSM2R-kernel product of at most 32 columns: the split
// partials, then room for B when it is given transposed (plain types) or for
// B's packed 16-bit terms (precision form, B read in either order).
size_t tsm2r_ws(int transA, int64_t m, int64_t k, int64_t n, int dtype, bool transB, bool vec) {
    const size_t part = align256(tsm2r_part(transA, m, k, n, dtype, vec));
    if (!plain_dtype(dtype)) return part + lp_bterms_bytes(k, n);
    const int ce = esize(dtype);
    return part + (transB ? (size_t)bt_ld(k, ce) * n * ce : 0);
}

// The most any plan of the call can need (the query does not know A's
// alignment, which picks the kernel instance).
size_t tsm2r_ws_max(int transA, int64_t m, int64_t k, int64_t n, int dtype, bool transB) {
    const size_t a = tsm2r_ws(transA, m, k, n, dtype, transB, true);
    const size_t b = tsm2r_ws(transA, m, k, n, dtype, transB, false);
    return a > b ? a : b;
}

// C := beta*C + op(A)*op(B) on validated arguments.  `lform` asks for the TSM2L
// kernels (all of B on chip); they need a column-major A and k <= 32, other
// shapes run on the TSM2R kernels, which are correct for any k.  n > 32 is
// done in panels of 32 columns of B and C, A being read once per panel.
int product(bool lform, int transA, int transB, int64_t m, int64_t k, int64_t n, const void* A,
            int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc,
            int dtype, void* ws, size_t ws_bytes, hipStream_t st) {
    if (transA && !plain_dtype(dtype)) return TSM_ERR_UNSUPPORTED;   // planes are column-major
    if (m == 0 || n == 0) return TSM_SUCCESS;
    const int ce = plain_dtype(dtype) ? esize(dtype) : 4;             // element size of B, C
    const int cdt = plain_dtype(dtype) ? dtype : TSM_F32;
    if (k == 0) {
        launch_fill_scale(m, n, C, ldc, beta, cdt, st);
        return check_launch("fill_scale_kernel");
    }
    if (n > 32) {
        for (int64_t p0 = 0; p0 < n; p0 += 32) {
            const int64_t np = n - p0 < 32 ? n - p0 : 32;
            const char* Bp = (const char*)B + (transB ? p0 : p0 * ldb) * ce;
            char* Cp = (char*)C + p0 * ldc * ce;
            int rc = product(lform, transA, transB, m, k, np, A, lda, Bp, ldb, beta, Cp, ldc,
                             dtype, ws, ws_bytes, st);
            if (rc) return rc;
        }
        return TSM_SUCCESS;
    }
    const int cus = cu_count();
    if (lform && !transA && k <= 32) {
        // B(j, p) at B[j*bsj + p*bsp]: both orders of B are plain strides here
        const int64_t bsj = transB ? ldb : 1, bsp = transB ? 1 : ldb;
        if (!plain_dtype(dtype)) {
            launch_tsm2l_lp(m, k, n, A, lda, (const float*)B, bsj, bsp, (float)beta, (float*)C,
                            ldc, dtype, cus, st);
            return check_launch("tsm2l_lp_kernel");
        }
        RTPlan P = plan_rowtile(m, k, n, dtype, cus);
        LaunchRT L{};
        L.m = m; L.kin = (int)k; L.nout = n; L.X = A; L.ldx = lda; L.Y = B; L.ys_in = bsj;
        L.ys_out = bsp; L.O = C; L.ldo = ldc; L.kp = P.kp; L.cols_per_block = (int)P.cpb;
        L.blocks_x = P.bx; L.blocks_y = P.by; L.cus = cus; L.beta = beta;
        if (launch_rowtile(L, dtype, st)) return TSM_ERR_UNSUPPORTED;
        return check_launch("rowtile_kernel");
    }
    // TSM2R kernels; workspace = [split partials][B copied column-major, or
    // B's packed 16-bit terms for the precision form]
    const bool avec = vec_ok(A, lda, plain_dtype(dtype) ? esize(dtype) : 2);
    void* w = nullptr;
    int rc = get_ws(tsm2r_ws(transA, m, k, n, dtype, transB, avec), ws, ws_bytes, &w);
    if (rc) return rc;
    if (!plain_dtype(dtype)) {
        // A: 16-bit hi plane (and lo plane lda*k elements after it); B, C float
        NNPlan P{};
        plan_tsm2r_lp(m, k, n, dtype, cus, avec, &P);
        void* bt = (char*)w + align256(P.ws);
        launch_split_b(k, n, (const float*)B, transB ? ldb : 1, transB ? 1 : ldb, dtype, bt, st);
        rc = check_launch("split_b_kernel");
        if (rc) return rc;
        LaunchNN L{};
        L.fn = P.fn;
        L.m = m; L.k = k; L.n = n; L.A = A; L.lda = lda; L.B = bt; L.ldb = 0; L.C = C;
        L.ldc = ldc; L.np = P.np; L.tile_rows = P.tile_rows; L.tiles = P.tiles; L.S = P.S;
        L.kslice = P.kslice; L.beta = beta;
        if (P.S > 1) L.part = (double*)w;
        launch_tsm2r_lp(L, dtype, st);
        return check_launch("tsm2r_lp_kernel");
    }
    const void* Bk = B;
    int64_t ldbk = ldb;
    if (transB) {
        void* bc = (char*)w + align256(tsm2r_part(transA, m, k, n, dtype, avec));
        launch_transpose(k, n, B, ldb, bc, bt_ld(k, ce), cdt, st);
        rc = check_launch("transpose_kernel");
        if (rc) return rc;
        Bk = bc;
        ldbk = bt_ld(k, ce);
    }
    if (transA) {
        // A given transposed is the column-major k x m matrix X = A^T (ld lda):
        // C = X^T * B, a reduction along the contiguous dimension.
        TNPlan P = plan_tn(k, m, n, dtype, cus);
        LaunchTN L{};
        L.R = k; L.ncols = m; L.n = n;
        L.X = A; L.ldx = lda; L.Y = Bk; L.ldy = ldbk; L.O = C; L.ldo = ldc;
        L.groups = P.groups; L.S = P.S; L.rslice = P.rslice; L.rg = P.rg; L.ct = P.ct;
        L.pf = P.pf;
        L.beta = beta;
        if (P.S > 1) L.part = (double*)w;
        if (launch_tn(L, dtype, st)) return TSM_ERR_UNSUPPORTED;
        return check_launch("tn_kernel");
    }
    NNPlan P{};
    if (plan_nn(m, k, n, dtype, cus, vec_ok(A, lda, esize(dtype)), &P)) return TSM_ERR_UNSUPPORTED;
    LaunchNN L{};
    L.fn = P.fn;
    L.m = m; L.k = k; L.n = n; L.A = A; L.lda = lda; L.B = Bk; L.ldb = ldbk; L.C = C; L.ldc = ldc;
    L.np = P.np; L.tile_rows = P.tile_rows; L.tiles = P.tiles; L.S = P.S; L.kslice = P.kslice;
    L.beta = beta;
    L.pf = P.pf;
    if (P.S > 1) L.part = (double*)w;
    if (launch_tsm2r_nn(L, dtype, st)) return TSM_ERR_UNSUPPORTED;
    return check_launch("tsm2r_nn_kernel");
}

}  // namespace

extern "C" {

int tsm2r_ex(int transA, int transB, int64_t m, int64_t k, int64_t n, const void* A,
             int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc,
             int dtype, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_ex(transA, transB, m, k, n, A, lda, B, ldb, C, ldc, dtype);
    if (rc) return rc;
    return product(false, transA, transB, m, k, n, A, lda, B, ldb, beta, C, ldc, dtype, ws,
                   ws_bytes, (hipStream_t)stream);
}

int tsm2l_ex(int transA, int transB, int64_t m, int64_t k, int64_t n, const void* A,
             int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc,
             int dtype, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_ex(transA, transB, m, k, n, A, lda, B, ldb, C, ldc, dtype);
    if (rc) return rc;
    return product(true, transA, transB, m, k, n, A, lda, B, ldb, beta, C, ldc, dtype, ws,
                   ws_bytes, (hipStream_t)stream);
}

int tsm2x_gemm(int transA, int transB, int64_t m, int64_t k, int64_t n, const void* A,
               int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc,
               int dtype, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_ex(transA, transB, m, k, n, A, lda, B, ldb, C, ldc, dtype);
    if (rc) return rc;
    // the paper's two shape classes: a tall-and-skinny A (k small, all of B on
    // chip) goes to TSM2L, a large A to TSM2R
    const bool lform = transA == 0 && k <= 32;
    return product(lform, transA, transB, m, k, n, A, lda, B, ldb, beta, C, ldc, dtype, ws,
                   ws_bytes, (hipStream_t)stream);
}

int tsm2r(int64_t m, int64_t k, int64_t n, const void* A, int64_t lda, const void* B,
          int64_t ldb, void* C, int64_t ldc, int dtype, void* stream) {
    int rc = check_mm(1, m, k, n, A, lda, B, ldb, C, ldc, dtype, false);
    if (rc) return rc;
    return product(false, 0, 0, m, k, n, A, lda, B, ldb, 0.0, C, ldc, dtype, nullptr, 0,
                   (hipStream_t)stream);
}

int tsm2l(int64_t m, int64_t k, int64_t n, const void* A, int64_t lda, const void* B,
          int64_t ldb, void* C, int64_t ldc, int dtype, void* stream) {
    int rc = check_mm(1, m, k, n, A, lda, B, ldb, C, ldc, dtype, false);
    if (rc) return rc;
    return product(true, 0, 0, m, k, n, A, lda, B, ldb, 0.0, C, ldc, dtype, nullptr, 0,
                   (hipStream_t)stream);
}

int tsm_grad_a(int64_t m, int64_t k, int64_t n, const void* dC, int64_t lddc, const void* B,
               int64_t ldb, void* dA, int64_t ldda, int dtype, void* stream) {
    if (m < 0) return -1;
    if (k < 0) return -2;
    if (n < 0) return -3;
    if (!dC && m > 0 && n > 0) return -4;
    if (lddc < (m > 1 ? m : 1)) return -5;
    if (!B && k > 0 && n > 0) return -6;
    if (ldb < (k > 1 ? k : 1)) return -7;
    if (!dA && m > 0 && k > 0) return -8;
    if (ldda < (m > 1 ? m : 1)) return -9;
    if (!valid_dtype(dtype)) return -10;
    if (n > 32 || !plain_dtype(dtype)) return TSM_ERR_UNSUPPORTED;
    if (m == 0 || k == 0) return TSM_SUCCESS;
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        launch_fill_scale(m, k, dA, ldda, 0.0, dtype, st);
        return check_launch("fill_scale_kernel");
    }
    // dA = dC * B^T: X = dC (m x n), Y(p, j) = B[j + p*ldb].
    RTPlan P = plan_rowtile(m, n, k, dtype, cu_count());
    LaunchRT L{};
    L.m = m; L.kin = (int)n; L.nout = k; L.X = dC; L.ldx = lddc; L.Y = B; L.ys_in = ldb;
    L.ys_out = 1; L.O = dA; L.ldo = ldda; L.kp = P.kp; L.cols_per_block = (int)P.cpb;
    L.blocks_x = P.bx; L.blocks_y = P.by; L.cus = cu_count();
    if (launch_rowtile(L, dtype, st)) return TSM_ERR_UNSUPPORTED;
    return check_launch("rowtile_kernel");
}

int tsm_grad_b(int64_t m, int64_t k, int64_t n, const void* A, int64_t lda, const void* dC,
               int64_t lddc, void* dB, int64_t lddb, int dtype, void* ws, size_t ws_bytes,
               void* stream) {
    if (m < 0) return -1;
    if (k < 0) return -2;
    if (n < 0) return -3;
    if (!A && m > 0 && k > 0) return -4;
    if (lda < (m > 1 ? m : 1)) return -5;
    if (!dC && m > 0 && n > 0) return -6;
    if (lddc < (m > 1 ? m : 1)) return -7;
    if (!dB && k > 0 && n > 0) return -8;
    if (lddb < (k > 1 ? k : 1)) return -9;
    if (!valid_dtype(dtype)) return -10;
    if (n > 32) return TSM_ERR_UNSUPPORTED;
    if (k == 0 || n == 0) return TSM_SUCCESS;
    hipStream_t st = (hipStream_t)stream;
    if (m == 0) {
        launch_fill_scale(k, n, dB, lddb, 0.0, plain_dtype(dtype) ? dtype : TSM_F32, st);
        return check_launch("fill_scale_kernel");
    }
    // dB = A^T * dC: X = A (R = m rows, k columns), Y = dC.
    TNPlan P = plan_tn(m, k, n, dtype, cu_count());
    void* w = nullptr;
    int rc = get_ws(P.ws, ws, ws_bytes, &w);
    if (rc) return rc;
    LaunchTN L{};
    L.R = m; L.ncols = k; L.n = n; L.X = A; L.ldx = lda; L.Y = dC; L.ldy = lddc; L.O = dB;
    L.ldo = lddb; L.groups = P.groups; L.S = P.S; L.rslice = P.rslice; L.rg = P.rg; L.ct = P.ct;
    L.pf = P.pf;
    if (P.S > 1) L.part = (double*)w;
    if (P.yt) L.yt = (char*)w + P.yt_off;
    if (!plain_dtype(dtype)) {
        if (launch_tn_lp(L, dtype, st)) return TSM_ERR_UNSUPPORTED;
        return check_launch("tn_lp_kernel");
    }
    if (launch_tn(L, dtype, st)) return TSM_ERR_UNSUPPORTED;
    return check_launch("tn_kernel");
}

}  // extern "C"

// Scratch of the allocation-free fused backward: room for the dB partials
// of 2048 workgroups of the widest instance (32 x 32 doubles each), i.e. a
// persistent grid of 8 resident workgroups on each of 256 compute units.
// Every device holds its own copy for the life of the process.  Host code
// never passes `scratch` itself (on the host the name is only a stand-in);
// it uses the per-device address hipGetSymbolAddress returns.
static constexpr size_t kBwdScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) double scratch[kBwdScratchBytes / sizeof(double)];

namespace {

// Argument checks of tsm2l_backward (positions 1..14).
int check_bwd(int64_t m, int64_t k, int64_t n, const void* A, int64_t lda, const void* B,
              int64_t ldb, const void* dC, int64_t lddc, const void* dA, int64_t ldda,
              const void* dB, int64_t lddb, int dtype) {
    if (m < 0) return -1;
    if (k < 0) return -2;
    if (n < 0) return -3;
    if (!A && m > 0 && k > 0) return -4;
    if (lda < (m > 1 ? m : 1)) return -5;
    if (!B && k > 0 && n > 0) return -6;
    if (ldb < (k > 1 ? k : 1)) return -7;
    if (!dC && m > 0 && n > 0) return -8;
    if (lddc < (m > 1 ? m : 1)) return -9;
    if (!dA && m > 0 && k > 0) return -10;
    if (ldda < (m > 1 ? m : 1)) return -11;
    if (!dB && k > 0 && n > 0) return -12;
    if (lddb < (k > 1 ? k : 1)) return -13;
    if (!valid_dtype(dtype)) return -14;
    if (k > 32 || n > 32) return TSM_ERR_UNSUPPORTED;
    return TSM_SUCCESS;
}

// The fused backward on checked arguments; `part` supplies the dB partials
// (one k x n double block per workgroup): part(need) returns the buffer for
// `need` bytes, or null with *rc set.
template <typename PartFn>
int run_bwd(int64_t m, int64_t k, int64_t n, const void* A, int64_t lda, const void* B,
            int64_t ldb, const void* dC, int64_t lddc, void* dA, int64_t ldda, void* dB,
            int64_t lddb, int dtype, hipStream_t st, PartFn part) {
    if (k == 0) return TSM_SUCCESS;
    const int odt = plain_dtype(dtype) ? dtype : TSM_F32;      // B, dC, dA, dB
    if (m == 0 || n == 0) {
        // dA (m x k) is zero when n == 0; dB (k x n) is zero when m == 0
        if (m > 0) launch_fill_scale(m, k, dA, ldda, 0.0, odt, st);
        if (n > 0) launch_fill_scale(k, n, dB, lddb, 0.0, odt, st);
        return check_launch("fill_scale_kernel");
    }
    LaunchBwd L{};
    L.m = m; L.k = k; L.n = n; L.A = A; L.lda = lda; L.B = B; L.ldb = ldb; L.dC = dC;
    L.lddc = lddc; L.dA = dA; L.ldda = ldda; L.dB = dB; L.lddb = lddb; L.cus = cu_count();
    int64_t blocks = 0;
    launch_tsm2l_bwd(L, dtype, &blocks, st, true);
    const size_t need = (size_t)blocks * (k <= 16 ? 16 : 32) * (n <= 16 ? 16 : 32) * 8;
    int rc = TSM_SUCCESS;
    L.part = (double*)part(need, &rc);
    if (rc) return rc;
    launch_tsm2l_bwd(L, dtype, &blocks, st, false);
    return check_launch("tsm2l_bwd_kernel");
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// This device's scratch address (looked up once per device, with the device
// current); null with *rc set on failure.
void* scratch_ptr(int* rc) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *rc = hip_fail(e, "hipGetDevice");
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        g_last_hip = "scratch: device index beyond the supported 64 devices";
        *rc = TSM_ERR_UNSUPPORTED;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *rc = hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                           "hipGetSymbolAddress(scratch)");
            return nullptr;
        }
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" {

int tsm2l_backward_noalloc(int64_t m, int64_t k, int64_t n, const void* A, int64_t lda,
                           const void* B, int64_t ldb, const void* dC, int64_t lddc, void* dA,
                           int64_t ldda, void* dB, int64_t lddb, int dtype, void* stream) {
    int rc = check_bwd(m, k, n, A, lda, B, ldb, dC, lddc, dA, ldda, dB, lddb, dtype);
    if (rc) return rc;
    return run_bwd(m, k, n, A, lda, B, ldb, dC, lddc, dA, ldda, dB, lddb, dtype,
                   (hipStream_t)stream, [](size_t need, int* prc) -> void* {
                       if (need > kBwdScratchBytes) {
                           g_last_hip = "tsm2l_backward_noalloc: the dB partials need " +
                                        std::to_string(need) + " bytes, beyond the " +
                                        std::to_string(kBwdScratchBytes) + "-byte scratch";
                           *prc = TSM_ERR_WORKSPACE;
                           return nullptr;
                       }
                       return scratch_ptr(prc);
                   });
}

int tsm2l_backward(int64_t m, int64_t k, int64_t n, const void* A, int64_t lda, const void* B,
                   int64_t ldb, const void* dC, int64_t lddc, void* dA, int64_t ldda, void* dB,
                   int64_t lddb, int dtype, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_bwd(m, k, n, A, lda, B, ldb, dC, lddc, dA, ldda, dB, lddb, dtype);
    if (rc) return rc;
    return run_bwd(m, k, n, A, lda, B, ldb, dC, lddc, dA, ldda, dB, lddb, dtype,
                   (hipStream_t)stream, [&](size_t need, int* prc) -> void* {
                       void* w = nullptr;
                       *prc = get_ws(need, ws, ws_bytes, &w);
                       return w;
                   });
}

int tsm2x_split(int64_t m, int64_t k, const float* A, int64_t lda, void* hi, void* lo,
                int64_t ldh, int fmt, void* stream) {
    if (m < 0) return -1;
    if (k < 0) return -2;
    if (!A && m > 0 && k > 0) return -3;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (!hi && m > 0 && k > 0) return -5;
    if (ldh < (m > 1 ? m : 1)) return -7;
    if (fmt != 0 && fmt != 1) return -8;
    if (m == 0 || k == 0) return TSM_SUCCESS;
    launch_split(m, k, A, lda, hi, lo, ldh, fmt, (hipStream_t)stream);
    return check_launch("split_kernel");
}

int tsm_kmeans_assign(int64_t m, int64_t k, int64_t n, const void* X, int64_t ldx,
                      int x_rowmajor, const void* Mu, int64_t ldm, int32_t* labels, void* dist,
                      int dtype, void* ws, size_t ws_bytes, void* stream) {
    if (m < 0) return -1;
    if (k < 1 || k > INT32_MAX) return -2;
    if (n < 1 || n > INT32_MAX) return -3;
    if (!X && m > 0) return -4;
    if (x_rowmajor != 0 && x_rowmajor != 1) return -6;
    if (ldx < (x_rowmajor ? k : (m > 1 ? m : 1))) return -5;
    if (!Mu) return -7;
    if (ldm < k) return -8;
    if (!labels && m > 0) return -9;
    if (!plain_dtype(dtype)) return -11;
    if (m == 0) return TSM_SUCCESS;
    void* w = nullptr;
    int rc = get_ws(align256((size_t)n * esize(dtype)), ws, ws_bytes, &w);
    if (rc) return rc;
    LaunchKM L{};
    L.m = m; L.k = k; L.n = n; L.X = X; L.ldx = ldx; L.x_rowmajor = x_rowmajor; L.Mu = Mu;
    L.ldm = ldm; L.mu2 = w;
    L.labels = labels; L.dist = dist; L.cus = cu_count();
    if (launch_kmeans_assign(L, dtype, (hipStream_t)stream)) {
        g_last_hip = "kmeans_assign_kernel: launch failed";
        return TSM_ERR_HIP;
    }
    return TSM_SUCCESS;
}

size_t tsm2x_workspace_size(int op, int64_t m, int64_t k, int64_t n, int dtype) {
    if (op == TSM_OP_KMEANS)
        return (m >= 0 && k >= 1 && n >= 1 && plain_dtype(dtype)) ? align256((size_t)n * esize(dtype)) : 0;
    if (m <= 0 || k <= 0 || n <= 0 || !valid_dtype(dtype)) return 0;
    const int64_t np = n < 32 ? n : 32;      // panels of 32 columns reuse one workspace
    // products: enough for a B given transposed as well
    switch (op) {
        case TSM_OP_TSM2R: return tsm2r_ws_max(0, m, k, np, dtype, true);
        case TSM_OP_TSM2R_ROWMAJOR: return plain_dtype(dtype) ? tsm2r_ws_max(1, m, k, np, dtype, true) : 0;
        case TSM_OP_TSM2L: return k <= 32 ? 0 : tsm2r_ws_max(0, m, k, np, dtype, true);
        case TSM_OP_GRAD_B: return n <= 32 ? plan_tn(m, k, n, dtype, cu_count()).ws : 0;
        default: return 0;
    }
}

const char* tsm2x_kernel_name(int op, int64_t m, int64_t k, int64_t n, int dtype) {
    if (op != TSM_OP_TSM2R || m <= 0 || k <= 0 || n <= 0 || n > 32 || !plain_dtype(dtype))
        return nullptr;
    NNPlan P{};
    return plan_nn(m, k, n, dtype, cu_count(), true, &P) ? nullptr : P.name;
}

int tsm2x_tsm2r_plan(int64_t m, int64_t k, int64_t n, int dtype, int* slices, int* tall,
                     int64_t* tiles, int* tile_rows, int* occupancy, int* cus) {
    if (m <= 0) return -1;
    if (k <= 0) return -2;
    if (n <= 0 || n > 32) return -3;
    if (!plain_dtype(dtype)) return -4;
    const int c = cu_count();
    NNPlan P{};
    if (plan_nn(m, k, n, dtype, c, true, &P)) return TSM_ERR_UNSUPPORTED;
    if (slices) *slices = P.S;
    if (tall) *tall = P.tall;
    if (tiles) *tiles = P.tiles;
    if (tile_rows) *tile_rows = P.tile_rows;
    if (occupancy) *occupancy = P.occ;
    if (cus) *cus = c;
    return TSM_SUCCESS;
}

int tsm2x_tsm2r_pin(int64_t m, int64_t k, int64_t n, int dtype, int slices, int tall) {
    if (m <= 0) return -1;
    if (k <= 0) return -2;
    if (n <= 0 || n > 32) return -3;
    if (!plain_dtype(dtype)) return -4;
    if (slices < 0 || slices > k) return -5;
    if (tall < -1 || tall > 1) return -6;
    std::lock_guard<std::mutex> lk(g_pin_mu);
    if (slices == 0 && tall == -1)
        g_pins.erase(PinKey(m, k, n, dtype));
    else
        g_pins[PinKey(m, k, n, dtype)] = NNPin{slices, tall};
    return TSM_SUCCESS;
}

const char* tsm2x_error_string(int code) {
    if (code < 0) return "invalid argument (the code is minus its 1-based position)";
    switch (code) {
        case TSM_SUCCESS: return "success";
        case TSM_ERR_UNSUPPORTED: return "shape or storage type outside the supported range";
        case TSM_ERR_HIP: return "a HIP runtime call failed (see tsm2x_last_hip_error)";
        case TSM_ERR_WORKSPACE: return "workspace too small or not 256-byte aligned";
        case TSM_ERR_ALLOC: return "could not allocate the library workspace";
        default: return "unknown error code";
    }
}

const char* tsm2x_last_hip_error(void) { return g_last_hip.c_str(); }

int tsm2x_version(void) { return 100; }

void tsm2x_finalize(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (size_t d = 0; d < g_dev.size(); ++d) {
        if (g_dev[d].ws) {
            (void)hipSetDevice((int)d);
            (void)hipFree(g_dev[d].ws);
            g_dev[d].ws = nullptr;
            g_dev[d].ws_bytes = 0;
        }
    }
    (void)hipSetDevice(cur);
}

}  // extern "C"
