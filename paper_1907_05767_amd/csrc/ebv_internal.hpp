/* Launchers shared between the kernels (ebv_kernels.hip) and the C ABI (ebv_api.cpp). */
#ifndef EBV_INTERNAL_HPP
#define EBV_INTERNAL_HPP

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <vector>

namespace ebv {

/* Event brackets around the block-step launches of the single-system
 * factor (owned by a library handle): created up front, one pair per launch
 * up to their number, with each launch's algorithmic flop count. */
struct UpdateProfile {
    std::vector<hipEvent_t> ev;
    std::vector<double> flops;
    int used = 0;
};
int profile_update_enable(UpdateProfile &p, int max_launches);
int profile_update_read(UpdateProfile &p, double *ms_total, int64_t *launches, double *flops_total);

struct DenseTuning {
    int small_update_below; /* trailing size at or below which 64-row update tiles are used */
    int lookahead;          /* 1: one launch per block step (k_step); 0: panel + update launches */
    int defer_group;        /* look-ahead: column classes G; a class is updated every G-th step (1..4) */
    int defer_above;        /* ... while the region past the panel is larger than this */
    long long wait_limit;   /* spins before a bounded wait gives up (0: the defaults) */
    int defer_group_f32;    /* defer_group of the FP32 factor (1..4) */
};

/* Control words at the head of every multi-workgroup workspace: the status
 * word (bounded waits that give up OR 1 into it, a launch that finds its
 * ticket counter not reset ORs 2), then the triangular solve's ticket and
 * solved-blocks counters. */
constexpr int kCtlHead = 3;

/* Systems factored by a single workgroup (uniform and ragged batches) are
 * addressed with 32-bit byte offsets: n * lda * sizeof(element) must stay
 * below this. */
constexpr int64_t kWgMaxSystemBytes = int64_t(1) << 31;

/* Workspace of the single-system factor: first the control words -- the
 * kCtlHead words above, then per block step s the words kCtlHead + 2s
 * (ticket counter) and kCtlHead + 1 + 2s (the diagonal tile's ready flag)
 * -- then the factored diagonal tile's pack for the panel solves (64 x 64
 * elements). */
constexpr size_t factor_ctl_bytes(int64_t n)
{
    const int64_t nb = (n + 63) / 64;
    return (sizeof(int) * (size_t)(kCtlHead + 2 * nb) + 255) / 256 * 256;
}
constexpr size_t factor_pg_bytes(size_t elem) { return (64 * 64 * elem + 255) / 256 * 256; }
constexpr size_t factor_ws_bytes(size_t elem, int64_t n) { return factor_ctl_bytes(n) + factor_pg_bytes(elem); }

/* Exchange buffer of the multi-workgroup triangular solve: the solved rows
 * (n rounded up to 64, 16 columns), then the partial sums of the helper
 * workgroups (kTrsvHelpers per 64-row block, 64 x 16 each). */
constexpr int kTrsvHelpers = 2;
constexpr size_t trsv_xb_bytes(size_t elem, int64_t n)
{
    const int64_t nb = (n + 63) / 64;
    return ((size_t)(kTrsvHelpers + 1) * nb * 64 * 16 * elem + 255) / 256 * 256;
}

/* Explicit inverse from the factors: P receives the inverse packs of the
 * diagonal tiles (ceil(n/64) * 64 * 64 elements), X (n x n, pitch ldx) the
 * inverse. */
template <typename T>
hipError_t lu_inverse(const T *LU, int64_t lda, int n, T *X, int64_t ldx, T *P, hipStream_t st);

/* Block envelope of a skyline (profile) system, at 64 x 64 tile granularity:
 * block row I holds its lower tiles J = F[I] .. I (the diagonal tile last),
 * block column J its upper tiles I = G[J] .. J-1, packed 64 x 64 (pitch 64)
 * at tile indices LTo[I] + (J - F[I]) and LTo[nt] + UTo[J] + (I - G[J]) of
 * the tile array.  Passed to the kernels by value. */
constexpr int kSkyMaxBlocks = 256; /* n <= 16384 */
struct SkyPlan {
    int n, nt;
    int16_t F[kSkyMaxBlocks], G[kSkyMaxBlocks];
    int32_t LTo[kSkyMaxBlocks + 1], UTo[kSkyMaxBlocks + 1];
};
/* Pack the skyline arrays into the tiles (unpack = false) or the tiles back
 * into them (only entries inside the envelope are written). */
hipError_t skyline_pack(const SkyPlan &pl, const int32_t *f, const int64_t *rp, double *AL, const int32_t *g,
                        const int64_t *cp, double *AU, double *tiles, bool unpack, hipStream_t st);
/* P: 64 x 64 doubles of workspace for the diagonal tile's inverse pack; ctl:
 * kCtlHead + 2 nt ints of control words (cleared here); wlim: spins before a
 * bounded wait gives up (its status then lands in info as -status). */
hipError_t skyline_factor(const SkyPlan &pl, double *tiles, double *P, int *ctl, int32_t *info, long wlim,
                          hipStream_t st);
/* P: nt packs of 64 x 64 doubles (the diagonal tiles' inverses, overwritten). */
hipError_t skyline_solve(const SkyPlan &pl, const double *tiles, double *P, double *B, int64_t ldb, int nrhs,
                         hipStream_t st);

hipError_t fill_i32(int *p, int64_t count, int value, hipStream_t st);
/* info = -status when the workspace's status word is nonzero (one thread). */
hipError_t fold_status(const int *status, int32_t *info, hipStream_t st);

/* Single-system factor; prefilled: info and the control words were cleared
 * by the caller on the same stream. */
template <typename T>
hipError_t dense_factor(T *A, int64_t lda, int n, int32_t *info, void *ws, const DenseTuning &tun, UpdateProfile *prof,
                        hipStream_t st, T *B = nullptr, int64_t ldb = 0, int nrhs = 0, bool prefilled = false);
/* Factor + backward substitution on a workspace of factor_ws_bytes followed
 * by trsv_xb_bytes (B riding along in the factor). */
template <typename T>
hipError_t factor_solve(T *A, int64_t lda, int n, int32_t *info, void *ws, const DenseTuning &tun, UpdateProfile *prof,
                        hipStream_t st, T *B, int64_t ldb, int nrhs);
/* Multi-workgroup triangular solve: wsi = status, ticket counter, solved
 * counter (kCtlHead ints); xb = exchange buffer of trsv_xb_bytes(sizeof(T), n);
 * prefilled: the counters are zero and xb is marked for the first launch;
 * info (or NULL): receives -status at the end of each launch when the status
 * word is nonzero. */
template <typename T>
hipError_t dense_trsv(int mode, const T *LU, int64_t lda, int n, T *B, int64_t ldb, int nrhs, int *wsi, T *xb,
                      const int *skip, int32_t *info, hipStream_t st, bool prefilled = false,
                      long long wait_limit = 0);
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
                      double *P, hipStream_t st);
template <typename T>
hipError_t outer_neg(int n, int nrhs, const T *Bb, int64_t ldb, int64_t strideB, const T *X, int64_t ldx,
                     int64_t strideX, T *Abar, int64_t ldabar, int64_t strideAbar, int64_t batch, hipStream_t st);
template <typename TI, typename TO>
hipError_t convert(int rows, int cols, const TI *S, int64_t lds, TO *D, int64_t ldd, const int *skip, hipStream_t st);
/* Mixed precision.  convert_margin: D = float(A) (n x n) and the strict
 * diagonal-dominance margin min_i (|a_ii| - sum_{j != i} |a_ij|), clamped at
 * 0, into *mbits as the bits of a non-negative double (atomic minimum; the
 * word starts at the bits of +inf).  Non-negative doubles order like their
 * bit patterns, which every *bits word below relies on. */
hipError_t convert_margin(int n, const double *A, int64_t lda, float *D, int64_t ldd, unsigned long long *mbits,
                          hipStream_t st);
/* R = B - A X and max_i |r_ic| into rbits[c]. */
hipError_t mixed_residual(int n, int nrhs, const double *A, int64_t lda, const double *B, int64_t ldb, const double *X,
                          int64_t ldx, double *R, int64_t ldr, unsigned long long *rbits, const int *skip, hipStream_t st);
/* Stopping test after refinement step `it`: column c has converged when its
 * forward-error bound max_i|r_ic| / (margin * max_i|x_ic|) <= tol; every
 * column's bound goes to ferr[c]. */
hipError_t mixed_check(int nrhs, unsigned long long *rbits, unsigned long long *xbits, const unsigned long long *mbits,
                       double tol, int it, int32_t *iters, double *ferr, int *conv, hipStream_t st);
/* X (+)= D, and max_i |x_ic| of the result into xbits[c]. */
hipError_t mixed_xupdate(int n, int nrhs, double *X, int64_t ldx, const float *D, int64_t ldd, int first,
                         unsigned long long *xbits, const int *skip, hipStream_t st);
hipError_t fill_u64(unsigned long long *p, int64_t count, unsigned long long value, hipStream_t st);

} /* namespace ebv */

#endif
