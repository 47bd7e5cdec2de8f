/*
 * C ABI of libebv.so (declared in include/ebv.h): argument checks, workspace
 * layout and the order of launches.  All arithmetic happens in the kernels
 * of ebv_kernels.hip.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/ebv.h"
#include "ebv_internal.hpp"
#include "ebv_pairing.h"

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct DeviceInfo {
    bool checked = false;
    bool ok = false;
    int cus = 0;
};

std::mutex g_mu;
std::vector<DeviceInfo> g_dev;

int current_device_info(DeviceInfo &out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return EBV_ERR_NO_DEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_dev.size() <= dev)
        g_dev.resize(dev + 1);
    DeviceInfo &d = g_dev[dev];
    if (!d.checked) {
        hipDeviceProp_t p;
        d.checked = true;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) {
            d.ok = std::strncmp(p.gcnArchName, "gfx950", 6) == 0;
            d.cus = p.multiProcessorCount;
        }
    }
    out = d;
    return d.ok ? EBV_OK : EBV_ERR_NO_DEVICE;
}

int hip_status(hipError_t e) { return e == hipSuccess ? EBV_OK : EBV_ERR_HIP; }


/* Workspace of the multi-workgroup triangular solves: status word, ticket
 * counter, solved-blocks counter. */
/* Multi-workgroup triangular solves: status, ticket and solved-block
 * counters, then the exchange buffer of the solved rows. */
size_t trsv_ctl_bytes() { return align_up(sizeof(int) * 3); }
size_t trsv_ws_bytes(int64_t n, size_t elem) { return trsv_ctl_bytes() + ebv::trsv_xb_bytes(elem, n); }


/* Mixed precision (dense): [trsv ints][diagonal tile][conv int][rbits u64[nrhs]]
 * [bbits u64[nrhs]][A32 n*n floats][R32 n*nrhs floats][R64 n*nrhs doubles] */
struct MixedLayout {
    size_t trsv, dtile, xb, conv, rbits, bbits, a32, r32, r64, total;
    MixedLayout(int64_t n, int64_t nrhs)
    {
        trsv = 0; /* the factor's control words 0..2 serve the solves */
        dtile = 0;
        xb = ebv::factor_ws_bytes(sizeof(float), n);
        conv = xb + ebv::trsv_xb_bytes(sizeof(float), n);
        rbits = conv + kAlign;
        bbits = rbits + align_up(8 * (size_t)nrhs);
        a32 = bbits + align_up(8 * (size_t)nrhs);
        r32 = a32 + align_up(4 * (size_t)n * (size_t)n);
        r64 = r32 + align_up(4 * (size_t)n * (size_t)nrhs);
        total = r64 + align_up(8 * (size_t)n * (size_t)nrhs);
    }
};

/* Batched: [status, queue] then (mixed) W floats[totA], R32 floats[totB], X doubles[totB]. */
struct BatchedLayout {
    size_t hdr, w, r32, x, total;
    BatchedLayout(int64_t totA, int64_t totB, bool mixed)
    {
        hdr = 0;
        w = kAlign;
        if (!mixed) {
            r32 = x = total = w;
            return;
        }
        r32 = w + align_up(4 * (size_t)totA);
        x = r32 + align_up(4 * (size_t)totB);
        total = x + align_up(8 * (size_t)totB);
    }
};

bool ws_ok(const void *ws, size_t have, size_t need)
{
    if (need == 0)
        return true;
    return ws != nullptr && have >= need && ((uintptr_t)ws % kAlign) == 0;
}

ebv::DenseTuning g_tuning{0, 1, 3, 1024};

} /* namespace */

extern "C" {

int ebv_version(void) { return 100; }

const char *ebv_status_string(int status)
{
    if (status < 0)
        return "invalid argument";
    switch (status) {
    case EBV_OK: return "success";
    case EBV_ERR_HIP: return "HIP runtime error";
    case EBV_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case EBV_ERR_UNSUPPORTED: return "arguments outside what this build supports";
    case EBV_ERR_NOT_CONVERGED: return "refinement did not converge";
    case EBV_ERR_NO_DEVICE: return "no gfx950 device is current";
    default: return "unknown status";
    }
}

int ebv_init(void)
{
    DeviceInfo d;
    return current_device_info(d);
}

size_t ebv_workspace_status_offset(void) { return 0; }

size_t ebv_workspace_size(int op, ebv_dtype dtype, int64_t n, int64_t nrhs, int64_t batch)
{
    if (n < 0 || nrhs < 0 || batch < 0)
        return 0;
    switch (op) {
    case EBV_OP_FACTOR:
        return batch <= 1 ? ebv::factor_ws_bytes(dtype == EBV_F32 ? sizeof(float) : sizeof(double), n) : 0;
    case EBV_OP_BAND:
        return 0;
    case EBV_OP_SOLVE:
    case EBV_OP_ADJOINT:
        return batch <= 1 ? trsv_ws_bytes(n, dtype == EBV_F32 ? sizeof(float) : sizeof(double)) : 0;
    case EBV_OP_BATCHED:
        return BatchedLayout(n, nrhs, false).total;
    case EBV_OP_BATCHED_MIXED:
        return BatchedLayout(n, nrhs, true).total;
    case EBV_OP_MIXED:
        return MixedLayout(n, nrhs).total;
    case EBV_OP_FACTOR_SOLVE:
    {
        const size_t elem = dtype == EBV_F32 ? sizeof(float) : sizeof(double);
        return ebv::factor_ws_bytes(elem, n) + ebv::trsv_xb_bytes(elem, n);
    }
    default:
        return 0;
    }
}

int ebv_set_dense_tuning(int small_update_below, int lookahead, int defer_group, int defer_above)
{
    if (small_update_below < 0)
        return -1;
    if (lookahead != 0 && lookahead != 1)
        return -2;
    if (defer_group < 1 || defer_group > 4)
        return -3;
    if (defer_above < 0)
        return -4;
    g_tuning.small_update_below = small_update_below;
    g_tuning.lookahead = lookahead;
    g_tuning.defer_group = defer_group;
    g_tuning.defer_above = defer_above;
    return EBV_OK;
}

int ebv_profile_update_enable(int max_launches)
{
    if (max_launches < 0)
        return -1;
    return ebv::profile_update_enable(max_launches) == 0 ? EBV_OK : EBV_ERR_HIP;
}

int ebv_profile_update_read(double *ms_total, int64_t *launches, double *flops_total)
{
    if (!ms_total)
        return -1;
    if (!launches)
        return -2;
    if (!flops_total)
        return -3;
    return ebv::profile_update_read(ms_total, launches, flops_total) == 0 ? EBV_OK : EBV_ERR_HIP;
}

int ebv_lu_factor(ebv_dtype dtype, int64_t n, void *A, int64_t lda, int64_t batch, int64_t strideA, int32_t *info,
                  void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -1;
    if (n < 0 || n > INT32_MAX)
        return -2;
    if (n > 0 && batch > 0 && A == nullptr)
        return -3;
    if (lda < std::max<int64_t>(1, n))
        return -4;
    if (batch < 0)
        return -5;
    if (batch > 1 && strideA < n * lda)
        return -6;
    if (n == 0 || batch == 0)
        return EBV_OK;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    hipError_t e;
    if (batch == 1) {
        if (!ws_ok(ws, ws_bytes, ebv::factor_ws_bytes(dtype == EBV_F32 ? sizeof(float) : sizeof(double), n)))
            return EBV_ERR_WORKSPACE;
        e = dtype == EBV_F64 ? ebv::dense_factor<double>((double *)A, lda, (int)n, info, ws, g_tuning, stream)
                             : ebv::dense_factor<float>((float *)A, lda, (int)n, info, ws, g_tuning, stream);
    } else {
        e = dtype == EBV_F64 ? ebv::batch_factor<double>((double *)A, lda, (int)n, batch, strideA, info, stream)
                             : ebv::batch_factor<float>((float *)A, lda, (int)n, batch, strideA, info, stream);
    }
    return hip_status(e);
}

int ebv_lu_solve(ebv_dtype dtype, int64_t n, int64_t nrhs, const void *LU, int64_t lda, void *B, int64_t ldb,
                 int64_t batch, int64_t strideLU, int64_t strideB, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -1;
    if (n < 0 || n > INT32_MAX)
        return -2;
    if (nrhs < 0 || nrhs > INT32_MAX)
        return -3;
    const bool work = n > 0 && nrhs > 0 && batch > 0;
    if (work && LU == nullptr)
        return -4;
    if (lda < std::max<int64_t>(1, n))
        return -5;
    if (work && B == nullptr)
        return -6;
    if (ldb < std::max<int64_t>(1, nrhs))
        return -7;
    if (batch < 0)
        return -8;
    if (batch > 1 && strideLU < n * lda)
        return -9;
    if (batch > 1 && strideB < n * ldb)
        return -10;
    if (!work)
        return EBV_OK;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    hipError_t e = hipSuccess;
    if (batch == 1) {
        const size_t elem = dtype == EBV_F32 ? sizeof(float) : sizeof(double);
        if (!ws_ok(ws, ws_bytes, trsv_ws_bytes(n, elem)))
            return EBV_ERR_WORKSPACE;
        int *wsi = (int *)ws;
        void *xb = (char *)ws + trsv_ctl_bytes();
        if ((e = ebv::fill_i32(wsi, 1, 0, stream)) != hipSuccess)
            return EBV_ERR_HIP;
        if (dtype == EBV_F64) {
            e = ebv::dense_trsv<double>(0, (const double *)LU, lda, (int)n, (double *)B, ldb, (int)nrhs, wsi,
                                        (double *)xb, nullptr, stream);
            if (e == hipSuccess)
                e = ebv::dense_trsv<double>(1, (const double *)LU, lda, (int)n, (double *)B, ldb, (int)nrhs, wsi,
                                            (double *)xb, nullptr, stream);
        } else {
            e = ebv::dense_trsv<float>(0, (const float *)LU, lda, (int)n, (float *)B, ldb, (int)nrhs, wsi,
                                       (float *)xb, nullptr, stream);
            if (e == hipSuccess)
                e = ebv::dense_trsv<float>(1, (const float *)LU, lda, (int)n, (float *)B, ldb, (int)nrhs, wsi,
                                           (float *)xb, nullptr, stream);
        }
    } else {
        e = dtype == EBV_F64
                ? ebv::batch_solve<double>(false, (const double *)LU, lda, (int)n, strideLU, (double *)B, ldb, strideB, (int)nrhs, batch, stream)
                : ebv::batch_solve<float>(false, (const float *)LU, lda, (int)n, strideLU, (float *)B, ldb, strideB, (int)nrhs, batch, stream);
    }
    return hip_status(e);
}

int ebv_lu_factor_solve(ebv_dtype dtype, int64_t n, int64_t nrhs, void *A, int64_t lda, void *B, int64_t ldb,
                        int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -1;
    if (n < 0 || n > INT32_MAX)
        return -2;
    if (nrhs < 0 || nrhs > INT32_MAX)
        return -3;
    if (n > 0 && A == nullptr)
        return -4;
    if (lda < std::max<int64_t>(1, n))
        return -5;
    if (n > 0 && nrhs > 0 && B == nullptr)
        return -6;
    if (ldb < std::max<int64_t>(1, nrhs))
        return -7;
    if (n == 0)
        return EBV_OK;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    const size_t elem = dtype == EBV_F32 ? sizeof(float) : sizeof(double);
    if (!ws_ok(ws, ws_bytes, ebv::factor_ws_bytes(elem, n) + ebv::trsv_xb_bytes(elem, n)))
        return EBV_ERR_WORKSPACE;
    const int ni = (int)n, nr = (int)nrhs;
    const hipError_t e = dtype == EBV_F64
                             ? ebv::factor_solve<double>((double *)A, lda, ni, info, ws, g_tuning, stream, (double *)B,
                                                         ldb, nr)
                             : ebv::factor_solve<float>((float *)A, lda, ni, info, ws, g_tuning, stream, (float *)B,
                                                        ldb, nr);
    return hip_status(e);
}

int ebv_lu_factor_band(int64_t n, int64_t kl, int64_t ku, double *AB, int64_t ldab, int32_t *info, hipStream_t stream)
{
    if (n < 0 || n > INT32_MAX)
        return -1;
    if (kl < 0)
        return -2;
    if (ku < 0)
        return -3;
    if (n > 0 && AB == nullptr)
        return -4;
    if (ldab < kl + ku + 1)
        return -5;
    if (kl > 64 || ku > 64)
        return EBV_ERR_UNSUPPORTED;
    if (n == 0)
        return EBV_OK;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    return hip_status(ebv::band_factor(AB, ldab, (int)n, (int)kl, (int)ku, info, stream));
}

int ebv_lu_solve_band(int64_t n, int64_t kl, int64_t ku, int64_t nrhs, const double *AB, int64_t ldab, double *B,
                      int64_t ldb, hipStream_t stream)
{
    if (n < 0 || n > INT32_MAX)
        return -1;
    if (kl < 0)
        return -2;
    if (ku < 0)
        return -3;
    if (nrhs < 0 || nrhs > INT32_MAX)
        return -4;
    const bool work = n > 0 && nrhs > 0;
    if (work && AB == nullptr)
        return -5;
    if (ldab < kl + ku + 1)
        return -6;
    if (work && B == nullptr)
        return -7;
    if (ldb < std::max<int64_t>(1, nrhs))
        return -8;
    if (kl > 64 || ku > 64)
        return EBV_ERR_UNSUPPORTED;
    if (!work)
        return EBV_OK;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    return hip_status(ebv::band_solve(AB, ldab, (int)n, (int)kl, (int)ku, B, ldb, (int)nrhs, stream));
}

int ebv_batched_order(int64_t count, const int32_t *n_host, int32_t *order_host)
{
    if (count < 0 || count > INT32_MAX)
        return -1;
    if (count > 0 && n_host == nullptr)
        return -2;
    if (count > 0 && order_host == nullptr)
        return -3;
    std::vector<int32_t> idx((size_t)count);
    std::iota(idx.begin(), idx.end(), 0);
    /* costliest first (n^3), ties by index so the order is deterministic */
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
        const double ca = (double)n_host[a] * n_host[a] * n_host[a];
        const double cb = (double)n_host[b] * n_host[b] * n_host[b];
        return ca > cb;
    });
    for (int64_t r = 0; r < count; ++r)
        order_host[r] = idx[(size_t)ebv_batch_slot((int)r, (int)count)];
    return EBV_OK;
}

int ebv_lu_factor_batched(ebv_dtype dtype, int64_t count, const int32_t *n, const int64_t *offA, void *A,
                          int64_t totA, const int64_t *offB, void *B, int64_t totB, const int32_t *order,
                          int32_t *info, int mixed, int32_t max_iter, double tol, int32_t *iters, int32_t wg_per_cu,
                          void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -1;
    if (count < 0 || count > INT32_MAX)
        return -2;
    const bool work = count > 0;
    if (work && n == nullptr)
        return -3;
    if (work && offA == nullptr)
        return -4;
    if (work && A == nullptr)
        return -5;
    if (totA < 0)
        return -6;
    if (work && B != nullptr && offB == nullptr)
        return -7;
    if (work && mixed && B == nullptr)
        return -8;
    if (totB < 0)
        return -9;
    if (mixed != 0 && mixed != 1)
        return -12;
    if (mixed && dtype != EBV_F64)
        return -1;
    if (mixed && max_iter < 0)
        return -13;
    if (mixed && !(tol >= 0.0))
        return -14;
    if (wg_per_cu < 0 || wg_per_cu > 8)
        return -16;
    if (!work)
        return EBV_OK;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    const BatchedLayout lay(totA, totB, mixed != 0);
    if (!ws_ok(ws, ws_bytes, lay.total))
        return EBV_ERR_WORKSPACE;
    DeviceInfo d;
    current_device_info(d);
    const int grid = std::max(1, d.cus * (wg_per_cu ? wg_per_cu : 2));
    char *w = (char *)ws;
    int *hdr = (int *)(w + lay.hdr);
    hipError_t e = ebv::fill_i32(hdr, 2, 0, stream);
    if (e != hipSuccess)
        return EBV_ERR_HIP;
    if (!mixed) {
        e = dtype == EBV_F64
                ? ebv::batched_run<double>((int)count, n, offA, (double *)A, offB, (double *)B, order, info, hdr + 1, grid, stream)
                : ebv::batched_run<float>((int)count, n, offA, (float *)A, offB, (float *)B, order, info, hdr + 1, grid, stream);
    } else {
        e = ebv::batched_mixed_run((int)count, n, offA, (const double *)A, offB, (double *)B, order, info, hdr + 1,
                                   (float *)(w + lay.w), (float *)(w + lay.r32), (double *)(w + lay.x), max_iter, tol,
                                   iters, grid, stream);
    }
    return hip_status(e);
}

int ebv_lu_solve_adjoint(ebv_dtype dtype, int64_t n, int64_t nrhs, const void *LU, int64_t lda, const void *X,
                         int64_t ldx, void *Bbar, int64_t ldb, void *Abar, int64_t ldabar, int64_t batch,
                         int64_t strideLU, int64_t strideX, int64_t strideB, int64_t strideAbar, void *ws,
                         size_t ws_bytes, hipStream_t stream)
{
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -1;
    if (n < 0 || n > INT32_MAX)
        return -2;
    if (nrhs < 0 || nrhs > INT32_MAX)
        return -3;
    const bool work = n > 0 && nrhs > 0 && batch > 0;
    if (work && LU == nullptr)
        return -4;
    if (lda < std::max<int64_t>(1, n))
        return -5;
    if (work && Abar != nullptr && X == nullptr)
        return -6;
    if (ldx < std::max<int64_t>(1, nrhs))
        return -7;
    if (work && Bbar == nullptr)
        return -8;
    if (ldb < std::max<int64_t>(1, nrhs))
        return -9;
    if (Abar != nullptr && ldabar < std::max<int64_t>(1, n))
        return -11;
    if (batch < 0)
        return -12;
    if (batch > 1 && strideLU < n * lda)
        return -13;
    if (batch > 1 && X != nullptr && strideX < n * ldx)
        return -14;
    if (batch > 1 && strideB < n * ldb)
        return -15;
    if (batch > 1 && Abar != nullptr && strideAbar < n * ldabar)
        return -16;
    if (!work)
        return EBV_OK;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    hipError_t e = hipSuccess;
    const bool f64 = dtype == EBV_F64;
    if (batch == 1) {
        if (!ws_ok(ws, ws_bytes, trsv_ws_bytes(n, f64 ? sizeof(double) : sizeof(float))))
            return EBV_ERR_WORKSPACE;
        int *wsi = (int *)ws;
        void *xb = (char *)ws + trsv_ctl_bytes();
        if ((e = ebv::fill_i32(wsi, 1, 0, stream)) != hipSuccess)
            return EBV_ERR_HIP;
        if (f64) {
            e = ebv::dense_trsv<double>(2, (const double *)LU, lda, (int)n, (double *)Bbar, ldb, (int)nrhs, wsi,
                                        (double *)xb, nullptr, stream);
            if (e == hipSuccess)
                e = ebv::dense_trsv<double>(3, (const double *)LU, lda, (int)n, (double *)Bbar, ldb, (int)nrhs, wsi,
                                            (double *)xb, nullptr, stream);
        } else {
            e = ebv::dense_trsv<float>(2, (const float *)LU, lda, (int)n, (float *)Bbar, ldb, (int)nrhs, wsi,
                                       (float *)xb, nullptr, stream);
            if (e == hipSuccess)
                e = ebv::dense_trsv<float>(3, (const float *)LU, lda, (int)n, (float *)Bbar, ldb, (int)nrhs, wsi,
                                           (float *)xb, nullptr, stream);
        }
    } else {
        e = f64 ? ebv::batch_solve<double>(true, (const double *)LU, lda, (int)n, strideLU, (double *)Bbar, ldb, strideB, (int)nrhs, batch, stream)
                : ebv::batch_solve<float>(true, (const float *)LU, lda, (int)n, strideLU, (float *)Bbar, ldb, strideB, (int)nrhs, batch, stream);
    }
    if (e != hipSuccess)
        return EBV_ERR_HIP;
    if (Abar != nullptr) {
        e = f64 ? ebv::outer_neg<double>((int)n, (int)nrhs, (const double *)Bbar, ldb, strideB, (const double *)X, ldx, strideX,
                                         (double *)Abar, ldabar, strideAbar, batch, stream)
                : ebv::outer_neg<float>((int)n, (int)nrhs, (const float *)Bbar, ldb, strideB, (const float *)X, ldx, strideX,
                                        (float *)Abar, ldabar, strideAbar, batch, stream);
    }
    return hip_status(e);
}

int ebv_lu_solve_mixed(int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B, int64_t ldb, double *X,
                       int64_t ldx, int32_t max_iter, double tol, int32_t *iters, double *relres, int32_t *info,
                       void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (n < 0 || n > INT32_MAX)
        return -1;
    if (nrhs < 0 || nrhs > 64)
        return -2;
    const bool work = n > 0 && nrhs > 0;
    if (work && A == nullptr)
        return -3;
    if (lda < std::max<int64_t>(1, n))
        return -4;
    if (work && B == nullptr)
        return -5;
    if (ldb < std::max<int64_t>(1, nrhs))
        return -6;
    if (work && X == nullptr)
        return -7;
    if (ldx < std::max<int64_t>(1, nrhs))
        return -8;
    if (max_iter < 0)
        return -9;
    if (!(tol >= 0.0))
        return -10;
    if (!work)
        return EBV_OK;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    const MixedLayout lay(n, nrhs);
    if (!ws_ok(ws, ws_bytes, lay.total))
        return EBV_ERR_WORKSPACE;
    char *w = (char *)ws;
    int *wsi = (int *)(w + lay.trsv);
    int *conv = (int *)(w + lay.conv);
    unsigned long long *rbits = (unsigned long long *)(w + lay.rbits);
    unsigned long long *bbits = (unsigned long long *)(w + lay.bbits);
    float *A32 = (float *)(w + lay.a32);
    float *XB = (float *)(w + lay.xb);
    float *R32 = (float *)(w + lay.r32);
    double *R64 = (double *)(w + lay.r64);
    const int ni = (int)n, nr = (int)nrhs;
    hipError_t e;
#define EBV_TRY(x)                                                                                                     \
    do {                                                                                                               \
        if ((e = (x)) != hipSuccess)                                                                                   \
            return EBV_ERR_HIP;                                                                                        \
    } while (0)
    EBV_TRY(ebv::fill_i32(wsi, 1, 0, stream));
    EBV_TRY(ebv::fill_i32(conv, 1, 0, stream));
    EBV_TRY(ebv::fill_i32((int *)rbits, 2 * nrhs, 0, stream));
    EBV_TRY(ebv::fill_i32((int *)bbits, 2 * nrhs, 0, stream));
    if (iters)
        EBV_TRY(ebv::fill_i32(iters, nrhs, -1, stream));
    EBV_TRY((ebv::convert<double, float>(ni, ni, A, lda, A32, n, nullptr, stream)));
    EBV_TRY(ebv::dense_factor<float>(A32, n, ni, info, (void *)(w + lay.dtile), g_tuning, stream));
    EBV_TRY(ebv::mixed_colmax(ni, nr, B, ldb, bbits, stream));
    EBV_TRY((ebv::convert<double, float>(ni, nr, B, ldb, R32, nrhs, nullptr, stream)));
    for (int it = 0; it <= max_iter; ++it) {
        EBV_TRY(ebv::dense_trsv<float>(0, A32, n, ni, R32, nrhs, nr, wsi, XB, conv, stream));
        EBV_TRY(ebv::dense_trsv<float>(1, A32, n, ni, R32, nrhs, nr, wsi, XB, conv, stream));
        EBV_TRY(ebv::mixed_xupdate(ni, nr, X, ldx, R32, nrhs, it == 0, conv, stream));
        EBV_TRY(ebv::mixed_residual(ni, nr, A, lda, B, ldb, X, ldx, R64, nrhs, rbits, conv, stream));
        EBV_TRY(ebv::mixed_check(nr, rbits, bbits, tol, it, iters, relres, conv, stream));
        if (it < max_iter)
            EBV_TRY((ebv::convert<double, float>(ni, nr, R64, nrhs, R32, nrhs, conv, stream)));
    }
#undef EBV_TRY
    return EBV_OK;
}

} /* extern "C" */
