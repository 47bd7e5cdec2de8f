/* Launchers shared between the kernels (ebv_kernels.hip) and the C ABI (ebv_api.cpp). */
#ifndef EBV_INTERNAL_HPP
#define EBV_INTERNAL_HPP

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace ebv {

struct DenseTuning {
    int small_update_below; /* trailing size at or below which 64-row update tiles are used */
    int lookahead;          /* 1: one launch per block step (k_step); 0: panel + update launches */
    int defer_group;        /* look-ahead: column classes G; a class is updated every G-th step (1..4) */
    int defer_above;        /* ... while the region past the panel is larger than this */
};

/* Workspace of the single-system factor: first the control words -- the
 * status word, two words of the triangular-solve chain that may follow on
 * the same workspace, and per block step s the words 3 + 2s (ticket
 * counter) and 4 + 2s (the diagonal tile's ready flag) -- then the factored
 * diagonal tile's pack for the panel solves (64 x 64 elements). */
inline size_t factor_ctl_bytes(int64_t n)
{
    const int64_t nb = (n + 63) / 64;
    return (sizeof(int) * (size_t)(3 + 2 * nb) + 255) / 256 * 256;
}
inline size_t factor_pg_bytes(size_t elem) { return (64 * 64 * elem + 255) / 256 * 256; }
inline size_t factor_ws_bytes(size_t elem, int64_t n) { return factor_ctl_bytes(n) + factor_pg_bytes(elem); }

/* Exchange buffer of the multi-workgroup triangular solve: the solved rows
 * (n rounded up to 64, 16 columns), then the partial sums of the helper
 * workgroups (kTrsvHelpers per 64-row block, 64 x 16 each). */
constexpr int kTrsvHelpers = 2;
inline size_t trsv_xb_bytes(size_t elem, int64_t n)
{
    const int64_t nb = (n + 63) / 64;
    return ((size_t)(kTrsvHelpers + 1) * nb * 64 * 16 * elem + 255) / 256 * 256;
}

hipError_t fill_i32(int *p, int64_t count, int value, hipStream_t st);

int profile_update_enable(int max_launches);
int profile_update_read(double *ms_total, int64_t *launches, double *flops_total);

/* Single-system factor; prefilled: info and the control words were cleared
 * by the caller on the same stream. */
template <typename T>
hipError_t dense_factor(T *A, int64_t lda, int n, int32_t *info, void *ws, const DenseTuning &tun, hipStream_t st,
                        T *B = nullptr, int64_t ldb = 0, int nrhs = 0, bool prefilled = false);
/* Factor + backward substitution on a workspace of factor_ws_bytes followed
 * by trsv_xb_bytes (B riding along in the factor). */
template <typename T>
hipError_t factor_solve(T *A, int64_t lda, int n, int32_t *info, void *ws, const DenseTuning &tun, hipStream_t st,
                        T *B, int64_t ldb, int nrhs);
/* Multi-workgroup triangular solve: wsi = status, ticket counter, solved
 * counter (3 ints); xb = exchange buffer of trsv_xb_bytes(sizeof(T), n);
 * prefilled: the counters are zero and xb is marked for the first launch. */
template <typename T>
hipError_t dense_trsv(int mode, const T *LU, int64_t lda, int n, T *B, int64_t ldb, int nrhs, int *wsi, T *xb,
                      const int *skip, hipStream_t st, bool prefilled = false);
template <typename T>
hipError_t batch_factor(T *A, int64_t lda, int n, int64_t batch, int64_t strideA, int32_t *info, hipStream_t st);
template <typename T>
hipError_t batch_solve(bool adjoint, const T *LU, int64_t lda, int n, int64_t strideLU, T *B, int64_t ldb,
                       int64_t strideB, int nrhs, int64_t batch, hipStream_t st);
template <typename T>
hipError_t batched_run(int count, const int *ns, const int64_t *offA, T *A, const int64_t *offB, T *B,
                       const int *order, int32_t *info, int *queue, int grid, hipStream_t st);
hipError_t batched_mixed_run(int count, const int *ns, const int64_t *offA, const double *A, const int64_t *offB,
                             double *B, const int *order, int32_t *info, int *queue, float *W, float *R32,
                             double *X, int max_iter, double tol, int32_t *iters, int grid, hipStream_t st);
hipError_t band_factor(double *AB, int64_t ldab, int n, int kl, int ku, int32_t *info, hipStream_t st);
hipError_t band_solve(const double *AB, int64_t ldab, int n, int kl, int ku, double *B, int64_t ldb, int nrhs,
                      hipStream_t st);
template <typename T>
hipError_t outer_neg(int n, int nrhs, const T *Bb, int64_t ldb, int64_t strideB, const T *X, int64_t ldx,
                     int64_t strideX, T *Abar, int64_t ldabar, int64_t strideAbar, int64_t batch, hipStream_t st);
template <typename TI, typename TO>
hipError_t convert(int rows, int cols, const TI *S, int64_t lds, TO *D, int64_t ldd, const int *skip, hipStream_t st);
hipError_t mixed_colmax(int n, int nrhs, const double *B, int64_t ldb, unsigned long long *bits, hipStream_t st);
hipError_t mixed_residual(int n, int nrhs, const double *A, int64_t lda, const double *B, int64_t ldb, const double *X,
                          int64_t ldx, double *R, int64_t ldr, unsigned long long *bits, const int *skip, hipStream_t st);
hipError_t mixed_check(int nrhs, unsigned long long *rbits, const unsigned long long *bbits, double tol, int it,
                       int32_t *iters, double *relres, int *conv, hipStream_t st);
hipError_t mixed_xupdate(int n, int nrhs, double *X, int64_t ldx, const float *D, int64_t ldd, int first,
                         const int *skip, hipStream_t st);

} /* namespace ebv */

#endif
