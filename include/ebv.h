/*
 * ebv.h -- C ABI of libebv.so: no-pivot Doolittle LU and triangular solves for
 * diagonally dominant systems AX = B on AMD MI355X (gfx950), after Hashemi,
 * Lahooti and Shirani, "Equal bi-Vectorized (EbV) method to high performance
 * on GPU" (arXiv:1907.05767).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are row-major: a_ij is at A[i*lda + j], lda >= n.  Right-hand
 *   sides are n x nrhs row-major: b_ic at B[i*ldb + c], ldb >= nrhs.
 * - Every array argument is a DEVICE pointer unless its comment says "host".
 *   The caller allocates and owns all memory; the library never allocates or
 *   frees device memory, never synchronizes the stream and never reads device
 *   memory on the host, so calls may be captured into a hipGraph.
 * - All work is enqueued on `stream` (0 = the null stream) in call order.
 * - Return value: EBV_OK (0); -i when argument i (1-based) is invalid, checked
 *   on the host before anything is enqueued; or a positive EBV_ERR_* code.
 * - Numerical breakdown is reported per system in a DEVICE int32 `info`
 *   (may be NULL): 0 ok, k > 0 when the pivot of elimination step k (1-based)
 *   was exactly zero.  Strict diagonal dominance (the paper's Eq. 2) guarantees
 *   nonzero pivots and is a documented precondition, not checked.  After a
 *   zero pivot the contents of the factor are unspecified.
 * - Workspace: entry points that take (ws, ws_bytes) need at least
 *   ebv_workspace_size(...) bytes of device memory, 256-byte aligned.  Its
 *   contents need no initialization and are clobbered.  Two calls that run
 *   concurrently must not share a workspace.
 * - n = 0, nrhs = 0 or batch = 0 return EBV_OK without enqueuing work.
 */
#ifndef EBV_H
#define EBV_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { EBV_F64 = 0, EBV_F32 = 1 } ebv_dtype;

enum {
    EBV_OK = 0,
    EBV_ERR_HIP = 1,           /* a HIP runtime call failed (launch, attribute query) */
    EBV_ERR_WORKSPACE = 2,     /* ws is NULL, too small or misaligned */
    EBV_ERR_UNSUPPORTED = 3,   /* valid arguments outside what this build implements */
    EBV_ERR_NOT_CONVERGED = 4, /* reserved for host-side reporting of refinement */
    EBV_ERR_NO_DEVICE = 5      /* no gfx950 device is current */
};

/* Operation codes for ebv_workspace_size. */
enum {
    EBV_OP_FACTOR = 0,
    EBV_OP_SOLVE = 1,
    EBV_OP_BATCHED = 2,
    EBV_OP_ADJOINT = 3,
    EBV_OP_MIXED = 4,
    EBV_OP_BAND = 5,
    EBV_OP_BATCHED_MIXED = 6,
    EBV_OP_FACTOR_SOLVE = 7
};

/* Library version (major*100 + minor). */
int ebv_version(void);

/* Human-readable text for a status code (static storage). */
const char *ebv_status_string(int status);

/* Queries the current device once per device and checks that it is gfx950.
 * Called implicitly by every entry point; returns EBV_ERR_NO_DEVICE otherwise. */
int ebv_init(void);

/* Device-side error word of a workspace: kernels that wait on other
 * workgroups give up after a bounded spin and OR 1 into this word.  Returns
 * the byte offset of that int32 inside any workspace (always 0). */
size_t ebv_workspace_status_offset(void);

/* Bytes of workspace an operation needs (0 when it needs none).
 *   op     EBV_OP_*; dtype the factor precision; n, nrhs the system size;
 *   batch  number of systems.  For EBV_OP_BATCHED and EBV_OP_BATCHED_MIXED
 *          pass the total element counts of the packed A and B in n and nrhs
 *          (totA, totB of ebv_lu_factor_batched) and the system count in batch. */
size_t ebv_workspace_size(int op, ebv_dtype dtype, int64_t n, int64_t nrhs, int64_t batch);

/* Tuning of the single-system factor (ebv_lu_factor with batch = 1 and
 * ebv_lu_factor_solve).  small_update_below: look-ahead update tiles are
 * 128 x 64 while the trailing block is larger than this, else 64 x 64
 * (default 0; the launch-per-phase scheme uses 128 x 128 and 64 x 64).
 * lookahead: 1 (default) runs one launch per 64-wide block step, in which
 * the next diagonal tile and panel are formed while the trailing update of
 * the current step runs; 0 runs the panel and the update as separate
 * launches.  defer_group G (1..4, default 3) and defer_above (default
 * 1024), look-ahead only: while the trailing block is larger than
 * defer_above, block column J is brought up to date only in every G-th
 * launch (those with (s + 1) mod G = J mod G) with K = 64 G, so the trailing
 * block is read and written once per G steps and each launch updates about
 * 1/G of it; G = 1 updates everything in every launch.  All settings give the
 * same factor up to rounding order.  Returns -i for an invalid argument i.
 * Process-wide; not thread-safe against concurrent calls. */
int ebv_set_dense_tuning(int small_update_below, int lookahead, int defer_group, int defer_above);

/* Measurement of the trailing-update kernel of the single-system factor.
 * ebv_profile_update_enable(m): create 2*m events up front (on the current
 * device); each later update launch of ebv_lu_factor (batch = 1) is then
 * bracketed by an event pair on its stream, up to m launches; m = 0 turns
 * this off and destroys the events.  ebv_profile_update_read synchronizes
 * on the recorded events and returns (and resets) the summed elapsed
 * milliseconds, the number of launches and their summed algorithmic flops
 * (2 * m^2 * kw per launch for an m x m trailing block and panel width kw).
 * Host pointers; -i for a NULL argument i. */
int ebv_profile_update_enable(int max_launches);
int ebv_profile_update_read(double *ms_total, int64_t *launches, double *flops_total);

/*
 * ebv_lu_factor -- Doolittle LU without pivoting, in place (paper Eq. 3, the
 * elimination step of Eq. 6-a/6-c, the work split of Eq. 7).
 *   A      (in/out) batch matrices n x n, system b at A + b*strideA elements;
 *          on exit the strictly lower part holds L (unit diagonal implied)
 *          and the upper part holds U.
 *   lda    >= max(1, n); strideA >= n*lda when batch > 1.
 *   info   device int32[batch] or NULL.
 *   dtype  EBV_F64 (double*) or EBV_F32 (float*).
 *   ws     ebv_workspace_size(EBV_OP_FACTOR, ...) bytes when batch = 1: launch
 *          control words first (the status word at offset 0, then
 *          4*(2 + 2*ceil(n/64)) bytes, the whole rounded up to 256 bytes),
 *          then the current diagonal tile's pack for the panel solves
 *          (64*64 elements); none when batch > 1 (ws may then be NULL).
 * Single systems (batch = 1) use a multi-workgroup blocked factorization;
 * batch > 1 factors one system per workgroup.
 */
int ebv_lu_factor(ebv_dtype dtype, int64_t n, void *A, int64_t lda, int64_t batch,
                  int64_t strideA, int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * ebv_lu_solve -- solve L Y = B by forward substitution, then U X = Y by
 * backward substitution (paper Eq. 1), with the factors from ebv_lu_factor.
 *   LU     (in) factors, lda as above.   B (in/out) right-hand sides -> X.
 *   strideLU, strideB: element strides between systems when batch > 1.
 *   ws     ebv_workspace_size(EBV_OP_SOLVE, dtype, n, nrhs, batch) bytes when
 *          batch = 1: three int32 control words padded to 256 bytes, then
 *          the exchange rows of the solved blocks (ceil(n/64)*64 x 16
 *          elements) and the partial sums of the helper workgroups
 *          (2 * ceil(n/64) blocks of 64 x 16 elements); none when batch > 1.
 */
int ebv_lu_solve(ebv_dtype dtype, int64_t n, int64_t nrhs, const void *LU, int64_t lda,
                 void *B, int64_t ldb, int64_t batch, int64_t strideLU, int64_t strideB,
                 void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * ebv_lu_factor_solve -- factor one system and solve it (Eq. 1 with the
 * factorization of Eq. 3/6): A is overwritten by L\U exactly as by
 * ebv_lu_factor, and B (n x nrhs, ldb >= nrhs) by X.  The forward
 * substitution L Y = B is carried out inside the factorization, B riding
 * along as extra columns of the elimination (each block step applies L_kk^{-1}
 * and the rank-64 update to them as well); the backward substitution
 * U X = Y follows.  Results agree with ebv_lu_factor + ebv_lu_solve up to
 * rounding order.
 *   info   device int32 or NULL, as for ebv_lu_factor.
 *   ws     ebv_workspace_size(EBV_OP_FACTOR_SOLVE, dtype, n, nrhs, 1) bytes:
 *          the factor's layout (the backward substitution uses control
 *          words 0..2), then the exchange rows of the solved blocks
 *          (ceil(n/64)*64 x 16 elements) and the partial sums of the
 *          helper workgroups (2 * ceil(n/64) blocks of 64 x 16 elements).
 */
int ebv_lu_factor_solve(ebv_dtype dtype, int64_t n, int64_t nrhs, void *A, int64_t lda, void *B, int64_t ldb,
                        int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * ebv_lu_factor_band / ebv_lu_solve_band -- the same factorization and solves
 * restricted to a band matrix with kl sub- and ku super-diagonals (FP64).
 * Without pivoting the factors keep the band, so they overwrite it in place.
 * Storage is row-wise: a_ij at AB[i*ldab + (j - i + kl)], ldab >= kl+ku+1.
 * Slots that fall outside the matrix are ignored.  This build supports
 * 0 <= kl, ku <= 64 (EBV_ERR_UNSUPPORTED otherwise).
 */
int ebv_lu_factor_band(int64_t n, int64_t kl, int64_t ku, double *AB, int64_t ldab,
                       int32_t *info, hipStream_t stream);
int ebv_lu_solve_band(int64_t n, int64_t kl, int64_t ku, int64_t nrhs, const double *AB,
                      int64_t ldab, double *B, int64_t ldb, hipStream_t stream);

/*
 * ebv_lu_factor_batched -- factor and solve `count` independent systems of
 * uneven size in one persistent launch (Eq. 1 and Eq. 6 per system; the EbV
 * pairing of the paper's equalization applied to whole systems through
 * `order`).
 *   n      device int32[count]: sizes (n_s >= 0).
 *   offA   device int64[count]: element offset of system s in A (lda = n_s).
 *   totA   elements of A (>= max_s offA[s] + n_s^2); sizes the workspace.
 *   offB   device int64[count]: element offset of system s in B (n_s x 1).
 *   totB   elements of B (>= max_s offB[s] + n_s).
 *   B      may be NULL when mixed == 0: factor only.
 *   order  device int32[count] or NULL: the order in which workgroups take
 *          systems; ebv_batched_order() computes the EbV order (largest with
 *          smallest).  NULL takes systems in index order.
 *   mixed  0: factor in `dtype` in place in A and solve in place in B.
 *          1: (dtype must be EBV_F64, B non-NULL) factor a float copy of each
 *          system in the workspace, keep A unchanged, and refine X (returned
 *          in B) in double until max_i |b - A x|_i <= tol * max_i |b_i| or
 *          max_iter corrections; iters (device int32[count] or NULL) receives
 *          the correction count per system, -1 when not converged.
 *   info   device int32[count] or NULL.
 *   wg_per_cu  workgroups per compute unit in the persistent grid (0 = 2).
 */
int ebv_lu_factor_batched(ebv_dtype dtype, int64_t count, const int32_t *n, const int64_t *offA,
                          void *A, int64_t totA, const int64_t *offB, void *B, int64_t totB,
                          const int32_t *order, int32_t *info, int mixed, int32_t max_iter,
                          double tol, int32_t *iters, int32_t wg_per_cu, void *ws, size_t ws_bytes,
                          hipStream_t stream);

/* EbV batch schedule on the host: order_host[r] = index of the system taken
 * r-th, pairing the costliest remaining system (by n^3) with the cheapest.
 *   n_host, order_host: HOST int32[count]. */
int ebv_batched_order(int64_t count, const int32_t *n_host, int32_t *order_host);

/*
 * ebv_lu_solve_adjoint -- reverse-mode derivative of X = A^{-1} B reusing the
 * factors: Bbar = A^{-T} Xbar (U^T Z = Xbar, then L^T Bbar = Z) and, when
 * Abar != NULL, Abar = -Bbar X^T.
 *   LU (in) factors from ebv_lu_factor; X (in) the solution, ldx >= nrhs;
 *   Bbar (in: Xbar, out: Bbar), ldb >= nrhs; Abar (out) n x n, ldabar >= n.
 *   Strides are element offsets between systems when batch > 1.
 */
int ebv_lu_solve_adjoint(ebv_dtype dtype, int64_t n, int64_t nrhs, const void *LU, int64_t lda,
                         const void *X, int64_t ldx, void *Bbar, int64_t ldb, void *Abar,
                         int64_t ldabar, int64_t batch, int64_t strideLU, int64_t strideX,
                         int64_t strideB, int64_t strideAbar, void *ws, size_t ws_bytes,
                         hipStream_t stream);

/*
 * ebv_lu_solve_mixed -- mixed-precision solve of one dense system: factor a
 * float copy of A (kept in the workspace), solve in float, then refine in
 * double: R = B - A X, stop when max_i |r_ic| / max_i |b_ic| <= tol for every
 * column c, else X += solve_float(R), at most max_iter corrections.
 *   A, B (in, unchanged) double; X (out) double n x nrhs, ldx >= nrhs.
 *   iters  device int32[nrhs] or NULL: corrections used per column (-1 when
 *          not converged after max_iter).
 *   relres device double[nrhs] or NULL: final max_i|r_ic| / max_i|b_ic|.
 *   info   device int32 or NULL: zero pivot of the float factor.
 * The refinement loop is a fixed sequence of launches whose kernels exit
 * early once the device-side test has passed, so the call never synchronizes.
 */
int ebv_lu_solve_mixed(int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
                       int64_t ldb, double *X, int64_t ldx, int32_t max_iter, double tol,
                       int32_t *iters, double *relres, int32_t *info, void *ws, size_t ws_bytes,
                       hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* EBV_H */
