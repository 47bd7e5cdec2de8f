/*
 * C ABI of libebv.so (declared in include/ebv.h): argument checks, workspace
 * layout and the order of launches.  All arithmetic happens in the kernels
 * of ebv_kernels.hip.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/ebv.h"
#include "ebv_internal.hpp"
#include "ebv_pairing.h"

/* Workspace of ebv_lu_factor_solve_noalloc: a file-scope device array, one
 * copy per device, sized for the factor + solve of the largest system that
 * entry point accepts (FP64, whose elements are the larger).  In host code
 * the name is a host-side stand-in, never a device address: the address of
 * each device's copy is looked up once per device (device_scratch) and only
 * that address reaches the kernels. */
constexpr int64_t kNoAllocMaxN = 16384;
constexpr size_t kScratchBytes =
    ebv::factor_ws_bytes(sizeof(double), kNoAllocMaxN) + ebv::trsv_xb_bytes(sizeof(double), kNoAllocMaxN);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct DeviceInfo {
    bool checked = false;
    bool ok = false;
    int cus = 0;
    void *scratch = nullptr;     /* this device's copy of `scratch` */
    hipError_t scratch_err = hipErrorUnknown;
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
        /* this device is current: the address of its copy of the array */
        if (d.ok) {
            void *ptr = nullptr;
            d.scratch_err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            d.scratch = d.scratch_err == hipSuccess ? ptr : nullptr;
        }
    }
    out = d;
    return d.ok ? EBV_OK : EBV_ERR_NO_DEVICE;
}

int hip_status(hipError_t e) { return e == hipSuccess ? EBV_OK : EBV_ERR_HIP; }


/* Multi-workgroup triangular solves: status, ticket and solved-block
 * counters, then the exchange buffer of the solved rows. */
size_t trsv_ctl_bytes() { return align_up(sizeof(int) * ebv::kCtlHead); }
size_t trsv_ws_bytes(int64_t n, size_t elem) { return trsv_ctl_bytes() + ebv::trsv_xb_bytes(elem, n); }


/* Mixed precision (dense): [factor workspace: control words + diagonal
 * tile][exchange rows][conv int, margin u64][rbits u64[nrhs]][xbits u64[nrhs]]
 * [A32 n*n floats][R32 n*nrhs floats][R64 n*nrhs doubles] */
struct MixedLayout {
    size_t trsv, dtile, xb, conv, mbits, rbits, xbits, a32, r32, r64, total;
    MixedLayout(int64_t n, int64_t nrhs)
    {
        trsv = 0; /* the factor's first control words serve the solves */
        dtile = 0;
        xb = ebv::factor_ws_bytes(sizeof(float), n);
        conv = xb + ebv::trsv_xb_bytes(sizeof(float), n);
        mbits = conv + 8;
        rbits = conv + kAlign;
        xbits = rbits + align_up(8 * (size_t)nrhs);
        a32 = xbits + align_up(8 * (size_t)nrhs);
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

/* Tuned schedule of the ragged batch, per form (0: FP64, 1: FP32, 2: FP32
 * factor + FP64 refinement). */
struct BatchedTuning {
    int wg_per_cu = 2;
    int order = EBV_ORDER_EBV;
};

constexpr unsigned kMagic = 0xEB7C0DE5u;

bool parse_int(const char *v, long lo, long hi, int &out)
{
    char *end = nullptr;
    const long x = std::strtol(v, &end, 10);
    if (end == v || *end != '\0' || x < lo || x > hi)
        return false;
    out = (int)x;
    return true;
}

} /* namespace */

/* Library handle: the tuning of the single-system factor and of the ragged
 * batch, and the measurement hook's events.  It owns no device memory; the
 * events are created on the device current when the hook is enabled. */
/* Ordering events of the transfer pipeline on one device: per slot, the
 * inputs are on the device (in), the slot's factor + solve is done (done),
 * the slot's result has left the device (out). */
struct PipelineEvents {
    int device = -1;
    hipEvent_t in[2] = {nullptr, nullptr}, done[2] = {nullptr, nullptr}, out[2] = {nullptr, nullptr};
};

struct ebv_ctx {
    unsigned magic = kMagic;
    ebv::DenseTuning dense{0, 1, 3, 1024, 0, 4};
    BatchedTuning batched[3];
    ebv::UpdateProfile prof;
    std::vector<PipelineEvents> pipe; /* created on first use per device */
};

namespace {

bool handle_ok(const ebv_ctx *h) { return h != nullptr && h->magic == kMagic; }

int batched_slot(ebv_dtype dtype, int mixed) { return mixed ? 2 : (dtype == EBV_F32 ? 1 : 0); }

/* One "key value" line of a tuning table. */
int apply_tuning(ebv_ctx &c, const std::string &key, const std::string &val)
{
    const char *v = val.c_str();
    ebv::DenseTuning &d = c.dense;
    if (key == "dense.small_update_below")
        return parse_int(v, 0, 1L << 30, d.small_update_below) ? EBV_OK : EBV_ERR_TUNING_FILE;
    if (key == "dense.lookahead")
        return parse_int(v, 0, 1, d.lookahead) ? EBV_OK : EBV_ERR_TUNING_FILE;
    if (key == "dense.defer_group")
        return parse_int(v, 1, 4, d.defer_group) ? EBV_OK : EBV_ERR_TUNING_FILE;
    if (key == "dense.f32.defer_group")
        return parse_int(v, 1, 4, d.defer_group_f32) ? EBV_OK : EBV_ERR_TUNING_FILE;
    if (key == "dense.defer_above")
        return parse_int(v, 0, 1L << 30, d.defer_above) ? EBV_OK : EBV_ERR_TUNING_FILE;
    static const char *forms[3] = {"batched.f64.", "batched.f32.", "batched.mixed."};
    for (int f = 0; f < 3; ++f) {
        const std::string pre = forms[f];
        if (key.compare(0, pre.size(), pre) != 0)
            continue;
        const std::string k = key.substr(pre.size());
        if (k == "wg_per_cu")
            return parse_int(v, 1, 8, c.batched[f].wg_per_cu) ? EBV_OK : EBV_ERR_TUNING_FILE;
        if (k == "order") {
            if (val == "ebv")
                c.batched[f].order = EBV_ORDER_EBV;
            else if (val == "index")
                c.batched[f].order = EBV_ORDER_INDEX;
            else if (val == "longest")
                c.batched[f].order = EBV_ORDER_LONGEST_FIRST;
            else
                return EBV_ERR_TUNING_FILE;
            return EBV_OK;
        }
        return EBV_ERR_TUNING_FILE;
    }
    return EBV_ERR_TUNING_FILE;
}

int load_tuning_file(ebv_ctx &c, const char *path)
{
    FILE *f = std::fopen(path, "r");
    if (!f)
        return EBV_ERR_TUNING_FILE;
    ebv_ctx tmp;
    tmp.dense = c.dense;
    for (int i = 0; i < 3; ++i)
        tmp.batched[i] = c.batched[i];
    char line[512];
    int st = EBV_OK;
    while (st == EBV_OK && std::fgets(line, sizeof line, f)) {
        std::string ln(line);
        const size_t hash = ln.find('#');
        if (hash != std::string::npos)
            ln.resize(hash);
        const char *ws = " \t\r\n";
        const size_t a = ln.find_first_not_of(ws);
        if (a == std::string::npos)
            continue;
        const size_t b = ln.find_first_of(ws, a);
        if (b == std::string::npos) {
            st = EBV_ERR_TUNING_FILE;
            break;
        }
        const size_t c2 = ln.find_first_not_of(ws, b);
        const size_t d = c2 == std::string::npos ? std::string::npos : ln.find_first_of(ws, c2);
        if (c2 == std::string::npos || (d != std::string::npos && ln.find_first_not_of(ws, d) != std::string::npos)) {
            st = EBV_ERR_TUNING_FILE;
            break;
        }
        st = apply_tuning(tmp, ln.substr(a, b - a), ln.substr(c2, d == std::string::npos ? std::string::npos : d - c2));
    }
    std::fclose(f);
    if (st == EBV_OK) { /* all or nothing */
        c.dense = tmp.dense;
        for (int i = 0; i < 3; ++i)
            c.batched[i] = tmp.batched[i];
    }
    return st;
}

} /* namespace */

extern "C" {

int ebv_version(void) { return 200; }

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
    case EBV_ERR_TUNING_FILE: return "tuning table unreadable or malformed";
    case EBV_ERR_NO_MEMORY: return "host allocation failed";
    case EBV_ERR_TOO_LARGE: return "system larger than the static scratch of the allocation-free entry point";
    default: return "unknown status";
    }
}

int ebv_init(void)
{
    DeviceInfo d;
    return current_device_info(d);
}

int ebv_create(ebv_handle *h)
{
    if (!h)
        return -1;
    *h = nullptr;
    ebv_ctx *c = new (std::nothrow) ebv_ctx;
    if (!c)
        return EBV_ERR_NO_MEMORY;
    const char *path = std::getenv("EBV_TUNING_FILE");
    if (path && *path) {
        const int st = load_tuning_file(*c, path);
        if (st != EBV_OK) {
            delete c;
            return st;
        }
    }
    *h = c;
    return EBV_OK;
}

int ebv_destroy(ebv_handle h)
{
    if (!h)
        return EBV_OK;
    if (!handle_ok(h))
        return -1;
    (void)ebv::profile_update_enable(h->prof, 0);
    for (auto &pe : h->pipe)
        for (int k = 0; k < 2; ++k)
            for (hipEvent_t e : {pe.in[k], pe.done[k], pe.out[k]})
                if (e)
                    (void)hipEventDestroy(e);
    h->magic = 0;
    delete h;
    return EBV_OK;
}

int ebv_load_tuning(ebv_handle h, const char *path)
{
    if (!handle_ok(h))
        return -1;
    if (!path)
        return -2;
    return load_tuning_file(*h, path);
}

size_t ebv_workspace_status_offset(void) { return 0; }

size_t ebv_workspace_size(int op, ebv_dtype dtype, int64_t n, int64_t nrhs, int64_t batch)
{
    if (n < 0 || nrhs < 0 || batch < 0)
        return 0;
    const size_t elem = dtype == EBV_F32 ? sizeof(float) : sizeof(double);
    switch (op) {
    case EBV_OP_FACTOR:
        return batch <= 1 ? ebv::factor_ws_bytes(elem, n) : 0;
    case EBV_OP_BAND:
        return 0;
    case EBV_OP_SOLVE:
    case EBV_OP_ADJOINT:
        return batch <= 1 ? trsv_ws_bytes(n, elem) : 0;
    case EBV_OP_BATCHED:
        return BatchedLayout(n, nrhs, false).total;
    case EBV_OP_BATCHED_MIXED:
        return BatchedLayout(n, nrhs, true).total;
    case EBV_OP_MIXED:
        return MixedLayout(n, nrhs).total;
    case EBV_OP_FACTOR_SOLVE:
        return ebv::factor_ws_bytes(elem, n) + ebv::trsv_xb_bytes(elem, n);
    case EBV_OP_INVERSE:
        return align_up((size_t)((n + 63) / 64) * 64 * 64 * elem);
    case EBV_OP_BAND_SOLVE: /* per 64-row block: two inverses, two band tiles */
        return align_up((size_t)((n + 63) / 64) * 4 * 64 * 64 * sizeof(double));
    default:
        return 0;
    }
}

int ebv_set_dense_tuning(ebv_handle h, int small_update_below, int lookahead, int defer_group, int defer_above)
{
    if (!handle_ok(h))
        return -1;
    if (small_update_below < 0)
        return -2;
    if (lookahead != 0 && lookahead != 1)
        return -3;
    if (defer_group < 1 || defer_group > 4)
        return -4;
    if (defer_above < 0)
        return -5;
    h->dense.small_update_below = small_update_below;
    h->dense.lookahead = lookahead;
    h->dense.defer_group = defer_group;
    h->dense.defer_above = defer_above;
    return EBV_OK;
}

int ebv_set_batched_tuning(ebv_handle h, ebv_dtype dtype, int mixed, int wg_per_cu, int order)
{
    if (!handle_ok(h))
        return -1;
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -2;
    if (mixed != 0 && mixed != 1)
        return -3;
    if (wg_per_cu < 1 || wg_per_cu > 8)
        return -4;
    if (order < EBV_ORDER_EBV || order > EBV_ORDER_LONGEST_FIRST)
        return -5;
    BatchedTuning &b = h->batched[batched_slot(dtype, mixed)];
    b.wg_per_cu = wg_per_cu;
    b.order = order;
    return EBV_OK;
}

int ebv_get_batched_tuning(ebv_handle h, ebv_dtype dtype, int mixed, int *wg_per_cu, int *order)
{
    if (!handle_ok(h))
        return -1;
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -2;
    if (mixed != 0 && mixed != 1)
        return -3;
    if (!wg_per_cu)
        return -4;
    if (!order)
        return -5;
    const BatchedTuning &b = h->batched[batched_slot(dtype, mixed)];
    *wg_per_cu = b.wg_per_cu;
    *order = b.order;
    return EBV_OK;
}

int ebv_set_wait_limit(ebv_handle h, int64_t spins)
{
    if (!handle_ok(h))
        return -1;
    if (spins < 0)
        return -2;
    h->dense.wait_limit = spins;
    return EBV_OK;
}

int ebv_profile_update_enable(ebv_handle h, int max_launches)
{
    if (!handle_ok(h))
        return -1;
    if (max_launches < 0)
        return -2;
    return ebv::profile_update_enable(h->prof, max_launches) == 0 ? EBV_OK : EBV_ERR_HIP;
}

int ebv_profile_update_read(ebv_handle h, double *ms_total, int64_t *launches, double *flops_total)
{
    if (!handle_ok(h))
        return -1;
    if (!ms_total)
        return -2;
    if (!launches)
        return -3;
    if (!flops_total)
        return -4;
    return ebv::profile_update_read(h->prof, ms_total, launches, flops_total) == 0 ? EBV_OK : EBV_ERR_HIP;
}

int ebv_lu_factor(ebv_handle h, ebv_dtype dtype, int64_t n, void *A, int64_t lda, int64_t batch, int64_t strideA,
                  int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!handle_ok(h))
        return -1;
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -2;
    if (n < 0 || n > INT32_MAX)
        return -3;
    if (n > 0 && batch > 0 && A == nullptr)
        return -4;
    if (lda < std::max<int64_t>(1, n))
        return -5;
    if (batch < 0)
        return -6;
    if (batch > 1 && strideA < n * lda)
        return -7;
    if (n == 0 || batch == 0)
        return EBV_OK;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    hipError_t e;
    if (batch == 1) {
        if (!ws_ok(ws, ws_bytes, ebv::factor_ws_bytes(dtype == EBV_F32 ? sizeof(float) : sizeof(double), n)))
            return EBV_ERR_WORKSPACE;
        e = dtype == EBV_F64 ? ebv::dense_factor<double>((double *)A, lda, (int)n, info, ws, h->dense, &h->prof, stream)
                             : ebv::dense_factor<float>((float *)A, lda, (int)n, info, ws, h->dense, &h->prof, stream);
        if (e == hipSuccess)
            e = ebv::fold_status((const int *)ws, info, stream);
    } else {
        /* one system per workgroup: its elements are addressed with 32-bit
         * byte offsets */
        const int64_t elem = dtype == EBV_F32 ? (int64_t)sizeof(float) : (int64_t)sizeof(double);
        if (n * lda * elem >= ebv::kWgMaxSystemBytes)
            return EBV_ERR_UNSUPPORTED;
        e = dtype == EBV_F64 ? ebv::batch_factor<double>((double *)A, lda, (int)n, batch, strideA, info, stream)
                             : ebv::batch_factor<float>((float *)A, lda, (int)n, batch, strideA, info, stream);
    }
    return hip_status(e);
}

int ebv_lu_solve(ebv_handle h, ebv_dtype dtype, int64_t n, int64_t nrhs, const void *LU, int64_t lda, void *B,
                 int64_t ldb, int64_t batch, int64_t strideLU, int64_t strideB, int32_t *info, void *ws,
                 size_t ws_bytes, hipStream_t stream)
{
    if (!handle_ok(h))
        return -1;
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -2;
    if (n < 0 || n > INT32_MAX)
        return -3;
    if (nrhs < 0 || nrhs > INT32_MAX)
        return -4;
    const bool work = n > 0 && nrhs > 0 && batch > 0;
    if (work && LU == nullptr)
        return -5;
    if (lda < std::max<int64_t>(1, n))
        return -6;
    if (work && B == nullptr)
        return -7;
    if (ldb < std::max<int64_t>(1, nrhs))
        return -8;
    if (batch < 0)
        return -9;
    if (batch > 1 && strideLU < n * lda)
        return -10;
    if (batch > 1 && strideB < n * ldb)
        return -11;
    if (!work)
        return EBV_OK;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    hipError_t e = hipSuccess;
    if (info && (e = ebv::fill_i32(info, batch, 0, stream)) != hipSuccess)
        return EBV_ERR_HIP;
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
                                        (double *)xb, nullptr, info, stream, false, h->dense.wait_limit);
            if (e == hipSuccess)
                e = ebv::dense_trsv<double>(1, (const double *)LU, lda, (int)n, (double *)B, ldb, (int)nrhs, wsi,
                                            (double *)xb, nullptr, info, stream, false, h->dense.wait_limit);
        } else {
            e = ebv::dense_trsv<float>(0, (const float *)LU, lda, (int)n, (float *)B, ldb, (int)nrhs, wsi,
                                       (float *)xb, nullptr, info, stream, false, h->dense.wait_limit);
            if (e == hipSuccess)
                e = ebv::dense_trsv<float>(1, (const float *)LU, lda, (int)n, (float *)B, ldb, (int)nrhs, wsi,
                                           (float *)xb, nullptr, info, stream, false, h->dense.wait_limit);
        }
    } else {
        e = dtype == EBV_F64
                ? ebv::batch_solve<double>(false, (const double *)LU, lda, (int)n, strideLU, (double *)B, ldb, strideB, (int)nrhs, batch, stream)
                : ebv::batch_solve<float>(false, (const float *)LU, lda, (int)n, strideLU, (float *)B, ldb, strideB, (int)nrhs, batch, stream);
    }
    return hip_status(e);
}

int ebv_lu_factor_solve(ebv_handle h, ebv_dtype dtype, int64_t n, int64_t nrhs, void *A, int64_t lda, void *B,
                        int64_t ldb, int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!handle_ok(h))
        return -1;
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -2;
    if (n < 0 || n > INT32_MAX)
        return -3;
    if (nrhs < 0 || nrhs > INT32_MAX)
        return -4;
    if (n > 0 && A == nullptr)
        return -5;
    if (lda < std::max<int64_t>(1, n))
        return -6;
    if (n > 0 && nrhs > 0 && B == nullptr)
        return -7;
    if (ldb < std::max<int64_t>(1, nrhs))
        return -8;
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
                             ? ebv::factor_solve<double>((double *)A, lda, ni, info, ws, h->dense, &h->prof, stream,
                                                         (double *)B, ldb, nr)
                             : ebv::factor_solve<float>((float *)A, lda, ni, info, ws, h->dense, &h->prof, stream,
                                                        (float *)B, ldb, nr);
    return hip_status(e);
}

size_t ebv_noalloc_scratch_bytes(void) { return kScratchBytes; }

int64_t ebv_noalloc_max_n(void) { return kNoAllocMaxN; }

int ebv_lu_factor_solve_noalloc(ebv_handle h, ebv_dtype dtype, int64_t n, int64_t nrhs, void *A, int64_t lda,
                                void *B, int64_t ldb, int32_t *info, hipStream_t stream)
{
    if (!handle_ok(h))
        return -1;
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -2;
    if (n < 0)
        return -3;
    if (n > kNoAllocMaxN)
        return EBV_ERR_TOO_LARGE;
    if (nrhs < 0 || nrhs > INT32_MAX)
        return -4;
    if (n > 0 && A == nullptr)
        return -5;
    if (lda < std::max<int64_t>(1, n))
        return -6;
    if (n > 0 && nrhs > 0 && B == nullptr)
        return -7;
    if (ldb < std::max<int64_t>(1, nrhs))
        return -8;
    if (n == 0)
        return EBV_OK;
    DeviceInfo d;
    int st = current_device_info(d);
    if (st != EBV_OK)
        return st;
    if (d.scratch == nullptr)
        return EBV_ERR_HIP;
    /* the same launches as ebv_lu_factor_solve; its first launch clears the
     * control words and marks the exchange rows, so nothing left in the
     * array by an earlier call is read */
    const int ni = (int)n, nr = (int)nrhs;
    const hipError_t e = dtype == EBV_F64
                             ? ebv::factor_solve<double>((double *)A, lda, ni, info, d.scratch, h->dense, &h->prof,
                                                         stream, (double *)B, ldb, nr)
                             : ebv::factor_solve<float>((float *)A, lda, ni, info, d.scratch, h->dense, &h->prof,
                                                        stream, (float *)B, ldb, nr);
    return hip_status(e);
}

int ebv_lu_inverse(ebv_handle h, ebv_dtype dtype, int64_t n, const void *LU, int64_t lda, void *Ainv, int64_t ldai,
                   void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!handle_ok(h))
        return -1;
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -2;
    if (n < 0 || n > INT32_MAX)
        return -3;
    if (n > 0 && LU == nullptr)
        return -4;
    if (lda < std::max<int64_t>(1, n))
        return -5;
    if (n > 0 && Ainv == nullptr)
        return -6;
    if (ldai < std::max<int64_t>(1, n))
        return -7;
    if (n == 0)
        return EBV_OK;
    const size_t elem = dtype == EBV_F32 ? sizeof(float) : sizeof(double);
    /* the result must not overlap the factors it is computed from */
    const char *lu0 = (const char *)LU, *lu1 = lu0 + ((n - 1) * lda + n) * elem;
    const char *x0 = (const char *)Ainv, *x1 = x0 + ((n - 1) * ldai + n) * elem;
    if (x0 < lu1 && lu0 < x1)
        return -6;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    if (!ws_ok(ws, ws_bytes, ebv_workspace_size(EBV_OP_INVERSE, dtype, n, 0, 1)))
        return EBV_ERR_WORKSPACE;
    const hipError_t e = dtype == EBV_F64 ? ebv::lu_inverse<double>((const double *)LU, lda, (int)n, (double *)Ainv,
                                                                    ldai, (double *)ws, stream)
                                          : ebv::lu_inverse<float>((const float *)LU, lda, (int)n, (float *)Ainv, ldai,
                                                                   (float *)ws, stream);
    return hip_status(e);
}

int ebv_pipeline_factor_solve(ebv_handle h, ebv_dtype dtype, int64_t count, int64_t n, int64_t nrhs,
                              void *const *A_host, void *const *B_host, void *const *dA, void *const *dB,
                              int32_t *info, void *ws, size_t ws_bytes, hipStream_t compute, hipStream_t copy_in,
                              hipStream_t copy_out)
{
    if (!handle_ok(h))
        return -1;
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -2;
    if (count < 0)
        return -3;
    if (n < 0 || n > INT32_MAX)
        return -4;
    if (nrhs < 0 || nrhs > INT32_MAX)
        return -5;
    if (count == 0 || n == 0)
        return EBV_OK;
    if (!A_host)
        return -6;
    if (nrhs > 0 && !B_host)
        return -7;
    for (int64_t s = 0; s < count; ++s) {
        if (!A_host[s])
            return -6;
        if (nrhs > 0 && !B_host[s])
            return -7;
    }
    if (!dA || !dA[0] || (count > 1 && !dA[1]))
        return -8;
    if (nrhs > 0 && (!dB || !dB[0] || (count > 1 && !dB[1])))
        return -9;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    const size_t elem = dtype == EBV_F32 ? sizeof(float) : sizeof(double);
    if (!ws_ok(ws, ws_bytes, ebv::factor_ws_bytes(elem, n) + ebv::trsv_xb_bytes(elem, n)))
        return EBV_ERR_WORKSPACE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return EBV_ERR_HIP;
    PipelineEvents *pe = nullptr;
    for (auto &p : h->pipe)
        if (p.device == dev)
            pe = &p;
    if (!pe) {
        PipelineEvents p;
        p.device = dev;
        for (int k = 0; k < 2; ++k)
            for (hipEvent_t *e : {&p.in[k], &p.done[k], &p.out[k]})
                if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess)
                    return EBV_ERR_HIP;
        h->pipe.push_back(p);
        pe = &h->pipe.back();
    }
    const size_t abytes = (size_t)n * (size_t)n * elem, bbytes = (size_t)n * (size_t)nrhs * elem;
    hipError_t e = hipSuccess;
    /* system s uses slot k = s % 2; its upload waits until slot k's previous
     * system (s - 2) is factored (dA) and its result downloaded (dB) */
    for (int64_t s = 0; s < count && e == hipSuccess; ++s) {
        const int k = (int)(s & 1);
        if (s >= 2) {
            e = hipStreamWaitEvent(copy_in, pe->done[k], 0);
            if (e == hipSuccess)
                e = hipStreamWaitEvent(copy_in, pe->out[k], 0);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(dA[k], A_host[s], abytes, hipMemcpyHostToDevice, copy_in);
        if (e == hipSuccess && nrhs > 0)
            e = hipMemcpyAsync(dB[k], B_host[s], bbytes, hipMemcpyHostToDevice, copy_in);
        if (e == hipSuccess)
            e = hipEventRecord(pe->in[k], copy_in);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(compute, pe->in[k], 0);
        if (e == hipSuccess) {
            int32_t *inf = info ? info + s : nullptr;
            e = dtype == EBV_F64
                    ? (nrhs > 0 ? ebv::factor_solve<double>((double *)dA[k], n, (int)n, inf, ws, h->dense, &h->prof,
                                                            compute, (double *)dB[k], nrhs, (int)nrhs)
                                : ebv::dense_factor<double>((double *)dA[k], n, (int)n, inf, ws, h->dense, &h->prof,
                                                            compute))
                    : (nrhs > 0 ? ebv::factor_solve<float>((float *)dA[k], n, (int)n, inf, ws, h->dense, &h->prof,
                                                           compute, (float *)dB[k], nrhs, (int)nrhs)
                                : ebv::dense_factor<float>((float *)dA[k], n, (int)n, inf, ws, h->dense, &h->prof,
                                                           compute));
        }
        if (e == hipSuccess && nrhs == 0 && info)
            e = ebv::fold_status((const int *)ws, info + s, compute);
        if (e == hipSuccess)
            e = hipEventRecord(pe->done[k], compute);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(copy_out, pe->done[k], 0);
        /* the result goes back: X (or, factor only, the factors) */
        if (e == hipSuccess)
            e = nrhs > 0 ? hipMemcpyAsync(B_host[s], dB[k], bbytes, hipMemcpyDeviceToHost, copy_out)
                         : hipMemcpyAsync(A_host[s], dA[k], abytes, hipMemcpyDeviceToHost, copy_out);
        if (e == hipSuccess)
            e = hipEventRecord(pe->out[k], copy_out);
    }
    return hip_status(e);
}

/* Block envelope of a skyline profile (host arrays): -1 when f or g is out of
 * range (f[i] > i, g[j] > j or negative) or n exceeds the tiled envelope's
 * limit, else 0 and the plan with its tile count. */
static int skyline_plan(int64_t n, const int32_t *f, const int32_t *g, ebv::SkyPlan &pl, int64_t &ntiles)
{
    if (n > (int64_t)ebv::kSkyMaxBlocks * 64)
        return -1;
    pl.n = (int)n;
    pl.nt = (int)((n + 63) / 64);
    for (int b = 0; b < pl.nt; ++b) {
        pl.F[b] = (int16_t)b;
        pl.G[b] = (int16_t)b;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (f[i] < 0 || f[i] > i || g[i] < 0 || g[i] > i)
            return -1;
        const int b = (int)(i / 64);
        pl.F[b] = (int16_t)std::min<int>(pl.F[b], f[i] / 64);
        pl.G[b] = (int16_t)std::min<int>(pl.G[b], g[i] / 64);
    }
    pl.LTo[0] = 0;
    pl.UTo[0] = 0;
    for (int b = 0; b < pl.nt; ++b) {
        pl.LTo[b + 1] = pl.LTo[b] + (b - pl.F[b] + 1);
        pl.UTo[b + 1] = pl.UTo[b] + (b - pl.G[b]);
    }
    ntiles = (int64_t)pl.LTo[pl.nt] + pl.UTo[pl.nt];
    return 0;
}

/* Entries of the strictly lower envelope (the length of AL). */
static int64_t skyline_lower_entries(int64_t n, const int32_t *f)
{
    int64_t e = 0;
    for (int64_t i = 0; i < n; ++i)
        e += i - f[i];
    return e;
}

/* The envelope tiles, one inverse pack per diagonal tile (the factor uses
 * the first for the current step, the solve all of them), then the factor's
 * control words (status, a ticket and a flag per block step). */
static size_t skyline_tiles_bytes(int nb, int64_t ntiles)
{
    return align_up((size_t)(ntiles + nb) * 64 * 64 * sizeof(double));
}
static size_t skyline_ws_bytes(int nb, int64_t ntiles)
{
    return skyline_tiles_bytes(nb, ntiles) + align_up(sizeof(int) * (size_t)(ebv::kCtlHead + 2 * nb));
}

size_t ebv_skyline_workspace_size(int64_t n, const int32_t *f_host, const int32_t *g_host)
{
    if (n <= 0 || !f_host || !g_host)
        return 0;
    ebv::SkyPlan pl;
    int64_t nt = 0;
    if (skyline_plan(n, f_host, g_host, pl, nt) != 0)
        return 0;
    return skyline_ws_bytes(pl.nt, nt);
}

int ebv_lu_factor_skyline(ebv_handle h, int64_t n, const int32_t *f_host, const int32_t *g_host, const int32_t *f,
                          const int64_t *rp, double *AL, const int32_t *g, const int64_t *cp, double *AU,
                          int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!handle_ok(h))
        return -1;
    if (n < 0)
        return -2;
    if (n == 0)
        return EBV_OK;
    if (!f_host)
        return -3;
    if (!g_host)
        return -4;
    ebv::SkyPlan pl;
    int64_t nt = 0;
    if (skyline_plan(n, f_host, g_host, pl, nt) != 0)
        return n > (int64_t)ebv::kSkyMaxBlocks * 64 ? EBV_ERR_UNSUPPORTED : -3;
    /* AL may be NULL when the lower envelope is empty (f[i] = i for all i) */
    if (!f || !rp || (!AL && skyline_lower_entries(n, f_host) > 0))
        return !f ? -5 : (!rp ? -6 : -7);
    if (!g || !cp || !AU)
        return !g ? -8 : (!cp ? -9 : -10);
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    if (!ws_ok(ws, ws_bytes, skyline_ws_bytes(pl.nt, nt)))
        return EBV_ERR_WORKSPACE;
    double *tiles = (double *)ws;
    int *ctl = (int *)((char *)ws + skyline_tiles_bytes(pl.nt, nt));
    const long wlim = h->dense.wait_limit > 0 ? (long)h->dense.wait_limit : 1L << 24;
    hipError_t e = ebv::skyline_pack(pl, f, rp, AL, g, cp, AU, tiles, false, stream);
    if (e == hipSuccess)
        e = ebv::skyline_factor(pl, tiles, tiles + nt * 64 * 64, ctl, info, wlim, stream);
    if (e == hipSuccess)
        e = ebv::skyline_pack(pl, f, rp, AL, g, cp, AU, tiles, true, stream);
    return hip_status(e);
}

int ebv_lu_solve_skyline(ebv_handle h, int64_t n, int64_t nrhs, const int32_t *f_host, const int32_t *g_host,
                         const int32_t *f, const int64_t *rp, const double *AL, const int32_t *g, const int64_t *cp,
                         const double *AU, double *B, int64_t ldb, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!handle_ok(h))
        return -1;
    if (n < 0)
        return -2;
    if (nrhs < 0 || nrhs > INT32_MAX)
        return -3;
    if (n == 0 || nrhs == 0)
        return EBV_OK;
    if (!f_host)
        return -4;
    if (!g_host)
        return -5;
    ebv::SkyPlan pl;
    int64_t nt = 0;
    if (skyline_plan(n, f_host, g_host, pl, nt) != 0)
        return n > (int64_t)ebv::kSkyMaxBlocks * 64 ? EBV_ERR_UNSUPPORTED : -4;
    if (!f || !rp || (!AL && skyline_lower_entries(n, f_host) > 0))
        return !f ? -6 : (!rp ? -7 : -8);
    if (!g || !cp || !AU)
        return !g ? -9 : (!cp ? -10 : -11);
    if (!B)
        return -12;
    if (ldb < nrhs)
        return -13;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    if (!ws_ok(ws, ws_bytes, skyline_ws_bytes(pl.nt, nt)))
        return EBV_ERR_WORKSPACE;
    double *tiles = (double *)ws;
    hipError_t e = ebv::skyline_pack(pl, f, rp, const_cast<double *>(AL), g, cp, const_cast<double *>(AU), tiles,
                                     false, stream);
    if (e == hipSuccess)
        e = ebv::skyline_solve(pl, tiles, tiles + nt * 64 * 64, B, ldb, (int)nrhs, stream);
    return hip_status(e);
}

int ebv_lu_factor_band(ebv_handle h, int64_t n, int64_t kl, int64_t ku, double *AB, int64_t ldab, int32_t *info,
                       void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!handle_ok(h))
        return -1;
    if (n < 0 || n > INT32_MAX)
        return -2;
    if (kl < 0)
        return -3;
    if (ku < 0)
        return -4;
    if (n > 0 && AB == nullptr)
        return -5;
    if (ldab < kl + ku + 1)
        return -6;
    if (kl > 64 || ku > 64)
        return EBV_ERR_UNSUPPORTED;
    if (n == 0)
        return EBV_OK;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    if (!ws_ok(ws, ws_bytes, ebv_workspace_size(EBV_OP_BAND, EBV_F64, n, 0, 1)))
        return EBV_ERR_WORKSPACE;
    return hip_status(ebv::band_factor(AB, ldab, (int)n, (int)kl, (int)ku, info, stream));
}

int ebv_lu_solve_band(ebv_handle h, int64_t n, int64_t kl, int64_t ku, int64_t nrhs, const double *AB, int64_t ldab,
                      double *B, int64_t ldb, int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!handle_ok(h))
        return -1;
    if (n < 0 || n > INT32_MAX)
        return -2;
    if (kl < 0)
        return -3;
    if (ku < 0)
        return -4;
    if (nrhs < 0 || nrhs > INT32_MAX)
        return -5;
    const bool work = n > 0 && nrhs > 0;
    if (work && AB == nullptr)
        return -6;
    if (ldab < kl + ku + 1)
        return -7;
    if (work && B == nullptr)
        return -8;
    if (ldb < std::max<int64_t>(1, nrhs))
        return -9;
    if (kl > 64 || ku > 64)
        return EBV_ERR_UNSUPPORTED;
    if (!work)
        return EBV_OK;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    if (!ws_ok(ws, ws_bytes, ebv_workspace_size(EBV_OP_BAND_SOLVE, EBV_F64, n, nrhs, 1)))
        return EBV_ERR_WORKSPACE;
    hipError_t e = hipSuccess;
    if (info && (e = ebv::fill_i32(info, 1, 0, stream)) != hipSuccess)
        return EBV_ERR_HIP;
    return hip_status(
        ebv::band_solve(AB, ldab, (int)n, (int)kl, (int)ku, B, ldb, (int)nrhs, static_cast<double *>(ws), stream));
}

int ebv_batched_order(int policy, int64_t count, const int32_t *n_host, int32_t *order_host)
{
    if (policy < EBV_ORDER_EBV || policy > EBV_ORDER_LONGEST_FIRST)
        return -1;
    if (count < 0 || count > INT32_MAX)
        return -2;
    if (count > 0 && n_host == nullptr)
        return -3;
    if (count > 0 && order_host == nullptr)
        return -4;
    std::vector<int32_t> idx((size_t)count);
    std::iota(idx.begin(), idx.end(), 0);
    if (policy == EBV_ORDER_INDEX) {
        std::copy(idx.begin(), idx.end(), order_host);
        return EBV_OK;
    }
    /* costliest first (n^3), ties by index so the order is deterministic */
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
        const double ca = (double)n_host[a] * n_host[a] * n_host[a];
        const double cb = (double)n_host[b] * n_host[b] * n_host[b];
        return ca > cb;
    });
    for (int64_t r = 0; r < count; ++r)
        order_host[r] = policy == EBV_ORDER_EBV ? idx[(size_t)ebv_batch_slot((int)r, (int)count)] : idx[(size_t)r];
    return EBV_OK;
}

int ebv_lu_factor_batched(ebv_handle h, ebv_dtype dtype, int64_t count, const int32_t *n, const int64_t *offA,
                          void *A, int64_t totA, const int64_t *offB, void *B, int64_t totB, const int32_t *order,
                          int32_t *info, int mixed, int32_t max_iter, double tol, int32_t *iters, int32_t wg_per_cu,
                          void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!handle_ok(h))
        return -1;
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -2;
    if (count < 0 || count > INT32_MAX)
        return -3;
    const bool work = count > 0;
    if (work && n == nullptr)
        return -4;
    if (work && offA == nullptr)
        return -5;
    if (work && A == nullptr)
        return -6;
    if (totA < 0)
        return -7;
    if (work && B != nullptr && offB == nullptr)
        return -8;
    if (work && mixed && B == nullptr)
        return -9;
    if (totB < 0)
        return -10;
    if (mixed != 0 && mixed != 1)
        return -13;
    if (mixed && dtype != EBV_F64)
        return -2;
    if (mixed && max_iter < 0)
        return -14;
    if (mixed && !(tol >= 0.0))
        return -15;
    if (wg_per_cu < 0 || wg_per_cu > 8)
        return -17;
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
    const int wpc = wg_per_cu ? wg_per_cu : h->batched[batched_slot(dtype, mixed)].wg_per_cu;
    const int grid = std::max(1, d.cus * wpc);
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

int ebv_lu_solve_adjoint(ebv_handle h, ebv_dtype dtype, int64_t n, int64_t nrhs, const void *LU, int64_t lda,
                         const void *X, int64_t ldx, void *Bbar, int64_t ldb, void *Abar, int64_t ldabar,
                         int64_t batch, int64_t strideLU, int64_t strideX, int64_t strideB, int64_t strideAbar,
                         int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!handle_ok(h))
        return -1;
    if (dtype != EBV_F64 && dtype != EBV_F32)
        return -2;
    if (n < 0 || n > INT32_MAX)
        return -3;
    if (nrhs < 0 || nrhs > INT32_MAX)
        return -4;
    const bool work = n > 0 && nrhs > 0 && batch > 0;
    if (work && LU == nullptr)
        return -5;
    if (lda < std::max<int64_t>(1, n))
        return -6;
    if (work && Abar != nullptr && X == nullptr)
        return -7;
    if (ldx < std::max<int64_t>(1, nrhs))
        return -8;
    if (work && Bbar == nullptr)
        return -9;
    if (ldb < std::max<int64_t>(1, nrhs))
        return -10;
    if (Abar != nullptr && ldabar < std::max<int64_t>(1, n))
        return -12;
    if (batch < 0)
        return -13;
    if (batch > 1 && strideLU < n * lda)
        return -14;
    if (batch > 1 && X != nullptr && strideX < n * ldx)
        return -15;
    if (batch > 1 && strideB < n * ldb)
        return -16;
    if (batch > 1 && Abar != nullptr && strideAbar < n * ldabar)
        return -17;
    if (!work)
        return EBV_OK;
    int st = ebv_init();
    if (st != EBV_OK)
        return st;
    hipError_t e = hipSuccess;
    const bool f64 = dtype == EBV_F64;
    if (info && (e = ebv::fill_i32(info, batch, 0, stream)) != hipSuccess)
        return EBV_ERR_HIP;
    if (batch == 1) {
        if (!ws_ok(ws, ws_bytes, trsv_ws_bytes(n, f64 ? sizeof(double) : sizeof(float))))
            return EBV_ERR_WORKSPACE;
        int *wsi = (int *)ws;
        void *xb = (char *)ws + trsv_ctl_bytes();
        if ((e = ebv::fill_i32(wsi, 1, 0, stream)) != hipSuccess)
            return EBV_ERR_HIP;
        if (f64) {
            e = ebv::dense_trsv<double>(2, (const double *)LU, lda, (int)n, (double *)Bbar, ldb, (int)nrhs, wsi,
                                        (double *)xb, nullptr, info, stream, false, h->dense.wait_limit);
            if (e == hipSuccess)
                e = ebv::dense_trsv<double>(3, (const double *)LU, lda, (int)n, (double *)Bbar, ldb, (int)nrhs, wsi,
                                            (double *)xb, nullptr, info, stream, false, h->dense.wait_limit);
        } else {
            e = ebv::dense_trsv<float>(2, (const float *)LU, lda, (int)n, (float *)Bbar, ldb, (int)nrhs, wsi,
                                       (float *)xb, nullptr, info, stream, false, h->dense.wait_limit);
            if (e == hipSuccess)
                e = ebv::dense_trsv<float>(3, (const float *)LU, lda, (int)n, (float *)Bbar, ldb, (int)nrhs, wsi,
                                           (float *)xb, nullptr, info, stream, false, h->dense.wait_limit);
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

int ebv_lu_solve_mixed(ebv_handle h, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
                       int64_t ldb, double *X, int64_t ldx, int32_t max_iter, double tol, int32_t *iters, double *ferr,
                       int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!handle_ok(h))
        return -1;
    if (n < 0 || n > INT32_MAX)
        return -2;
    if (nrhs < 0 || nrhs > 64)
        return -3;
    const bool work = n > 0 && nrhs > 0;
    if (work && A == nullptr)
        return -4;
    if (lda < std::max<int64_t>(1, n))
        return -5;
    if (work && B == nullptr)
        return -6;
    if (ldb < std::max<int64_t>(1, nrhs))
        return -7;
    if (work && X == nullptr)
        return -8;
    if (ldx < std::max<int64_t>(1, nrhs))
        return -9;
    if (max_iter < 0)
        return -10;
    if (!(tol >= 0.0))
        return -11;
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
    unsigned long long *mbits = (unsigned long long *)(w + lay.mbits);
    unsigned long long *rbits = (unsigned long long *)(w + lay.rbits);
    unsigned long long *xbits = (unsigned long long *)(w + lay.xbits);
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
    EBV_TRY(ebv::fill_u64(mbits, 1, 0x7FF0000000000000ull, stream)); /* +inf */
    EBV_TRY(ebv::fill_u64(rbits, nrhs, 0, stream));
    EBV_TRY(ebv::fill_u64(xbits, nrhs, 0, stream));
    if (iters)
        EBV_TRY(ebv::fill_i32(iters, nrhs, -1, stream));
    EBV_TRY(ebv::convert_margin(ni, A, lda, A32, n, mbits, stream));
    EBV_TRY(ebv::dense_factor<float>(A32, n, ni, info, (void *)(w + lay.dtile), h->dense, nullptr, stream));
    EBV_TRY((ebv::convert<double, float>(ni, nr, B, ldb, R32, nrhs, nullptr, stream)));
    for (int it = 0; it <= max_iter; ++it) {
        EBV_TRY(ebv::dense_trsv<float>(0, A32, n, ni, R32, nrhs, nr, wsi, XB, conv, nullptr, stream, false, h->dense.wait_limit));
        EBV_TRY(ebv::dense_trsv<float>(1, A32, n, ni, R32, nrhs, nr, wsi, XB, conv, nullptr, stream, false, h->dense.wait_limit));
        EBV_TRY(ebv::mixed_xupdate(ni, nr, X, ldx, R32, nrhs, it == 0, xbits, conv, stream));
        EBV_TRY(ebv::mixed_residual(ni, nr, A, lda, B, ldb, X, ldx, R64, nrhs, rbits, conv, stream));
        EBV_TRY(ebv::mixed_check(nr, rbits, xbits, mbits, tol, it, iters, ferr, conv, stream));
        if (it < max_iter)
            EBV_TRY((ebv::convert<double, float>(ni, nr, R64, nrhs, R32, nrhs, conv, stream)));
    }
    EBV_TRY(ebv::fold_status(wsi, info, stream));
#undef EBV_TRY
    return EBV_OK;
}

} /* extern "C" */
