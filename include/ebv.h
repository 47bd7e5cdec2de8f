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
 * - Every compute entry point takes a library handle (ebv_create) first.
 * - Return value: EBV_OK (0); -i when argument i (1-based, the handle is
 *   argument 1) is invalid, checked on the host before anything is enqueued;
 *   or a positive EBV_ERR_* code.
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

/* Element type of a call.  From C any int value may arrive here and is
 * rejected when invalid; under C++ the type has a fixed int underlying type,
 * so every such value is representable and its check is well defined. */
#ifdef __cplusplus
typedef enum : int { EBV_F64 = 0, EBV_F32 = 1 } ebv_dtype;
#else
typedef enum { EBV_F64 = 0, EBV_F32 = 1 } ebv_dtype;
#endif

enum {
    EBV_OK = 0,
    EBV_ERR_HIP = 1,           /* a HIP runtime call failed (launch, attribute query) */
    EBV_ERR_WORKSPACE = 2,     /* ws is NULL, too small or misaligned */
    EBV_ERR_UNSUPPORTED = 3,   /* valid arguments outside what this build implements */
    EBV_ERR_NOT_CONVERGED = 4, /* refinement did not converge (reported per system in iters) */
    EBV_ERR_NO_DEVICE = 5,     /* no gfx950 device is current */
    EBV_ERR_TUNING_FILE = 6,   /* tuning table unreadable or malformed */
    EBV_ERR_NO_MEMORY = 7,     /* host allocation failed */
    EBV_ERR_TOO_LARGE = 8      /* n above what the allocation-free entry point's static scratch holds */
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
    EBV_OP_FACTOR_SOLVE = 7,
    EBV_OP_BAND_SOLVE = 8,
    EBV_OP_INVERSE = 9
};

/* Order in which the workgroups of a ragged batch take its systems. */
enum {
    EBV_ORDER_EBV = 0,          /* costliest remaining system, then the cheapest, alternately */
    EBV_ORDER_INDEX = 1,        /* as stored */
    EBV_ORDER_LONGEST_FIRST = 2 /* decreasing cost */
};

/* Library handle: holds the tuning of the single-system factor and of the
 * ragged batch, and the event hook of the factor's block steps.  It owns no
 * device memory and serves every device.  A handle must not be used by two
 * host threads at once; give each thread its own. */
typedef struct ebv_ctx *ebv_handle;

/* Library version (major*100 + minor). */
int ebv_version(void);

/* Human-readable text for a status code (static storage). */
const char *ebv_status_string(int status);

/* Queries the current device once per device and checks that it is gfx950.
 * Called implicitly by every entry point; returns EBV_ERR_NO_DEVICE otherwise. */
int ebv_init(void);

/* ebv_create: a new handle with the default tuning, then the tuning table
 * named by the environment variable EBV_TUNING_FILE when it is set (format
 * of ebv_load_tuning; on failure no handle is made and its status is
 * returned).  Makes no device call.  *h receives the handle (host pointer).
 * ebv_destroy: releases a handle (NULL is a no-op); work already enqueued
 * with it is unaffected. */
int ebv_create(ebv_handle *h);
int ebv_destroy(ebv_handle h);

/* Reads a tuning table (written by the package's autotuner): one
 * "key value" pair per line, '#' starts a comment.  Keys:
 *   dense.small_update_below, dense.lookahead, dense.defer_group,
 *   dense.defer_above                       (see ebv_set_dense_tuning)
 *   dense.f32.defer_group                   G of the FP32 factor, 1..4
 *                                           (default 4; the other dense
 *                                           keys apply to both precisions)
 *   batched.{f64,f32,mixed}.wg_per_cu       1..8
 *   batched.{f64,f32,mixed}.order           ebv | index | longest
 * All or nothing: on EBV_ERR_TUNING_FILE (unreadable file, unknown key,
 * value out of range) the handle keeps its previous tuning. */
int ebv_load_tuning(ebv_handle h, const char *path);

/* Device-side status word of a workspace: kernels that wait on other
 * workgroups give up after a bounded spin, or as soon as another wait of the
 * same call has given up, and OR 1 into this word (2: a launch found its
 * ticket counter not reset).  Entry points with an `info` argument copy a
 * nonzero word into it as -status.  Returns the byte offset of that int32
 * inside any workspace (always 0). */
size_t ebv_workspace_status_offset(void);

/* Bytes of workspace an operation needs (0 when it needs none).  It depends
 * only on the shapes, not on a handle.
 *   op     EBV_OP_*; dtype the factor precision; n, nrhs the system size;
 *   batch  number of systems.  For EBV_OP_BATCHED and EBV_OP_BATCHED_MIXED
 *          pass the total element counts of the packed A and B in n and nrhs
 *          (totA, totB of ebv_lu_factor_batched) and the system count in batch. */
size_t ebv_workspace_size(int op, ebv_dtype dtype, int64_t n, int64_t nrhs, int64_t batch);

/* Tuning of the single-system factor (ebv_lu_factor with batch = 1 and
 * ebv_lu_factor_solve) held by handle h.  small_update_below: look-ahead
 * update tiles are 128 x 64 while the trailing block is larger than this,
 * else 64 x 64 (default 0; the launch-per-phase scheme uses 128 x 128 and
 * 64 x 64).  lookahead: 1 (default) runs one launch per 64-wide block step,
 * in which the next diagonal tile and panel are formed while the trailing
 * update of the current step runs; 0 runs the panel and the update as
 * separate launches.  defer_group G (1..4, default 3) and defer_above
 * (default 1024), look-ahead only: while the trailing block is larger than
 * defer_above, block column J is brought up to date only in every G-th
 * launch (those with (s + 1) mod G = J mod G) with K = 64 G, so the trailing
 * block is read and written once per G steps and each launch updates about
 * 1/G of it; G = 1 updates everything in every launch.  defer_group is the
 * FP64 factor's; the FP32 factor (dtype EBV_F32, and the float factor of
 * ebv_lu_solve_mixed) takes its G from the tuning table key
 * dense.f32.defer_group (default 4).  All settings give the same factor up to
 * rounding order.  Returns -i for an invalid argument i. */
int ebv_set_dense_tuning(ebv_handle h, int small_update_below, int lookahead, int defer_group, int defer_above);

/* Tuned schedule of ebv_lu_factor_batched for one form (dtype, mixed):
 * workgroups per compute unit of the persistent grid (1..8, used when the
 * call passes wg_per_cu = 0) and the order policy (EBV_ORDER_*) the caller
 * should pass to ebv_batched_order.  Defaults: 2 and EBV_ORDER_EBV. */
int ebv_set_batched_tuning(ebv_handle h, ebv_dtype dtype, int mixed, int wg_per_cu, int order);
int ebv_get_batched_tuning(ebv_handle h, ebv_dtype dtype, int mixed, int *wg_per_cu, int *order);

/* Budget of every bounded wait of the multi-workgroup kernels run with
 * handle h, in spins (0 = the defaults: 2^24 for the factor's diagonal-tile
 * flags, 2^22 for the solves' exchange rows).  A wait that runs out ORs 1
 * into the workspace's status word, every other wait of the call then stops
 * within 64 spins, all launches drain and `info` reports -1; the results of
 * that call are invalid.  Small values exist to exercise that path. */
int ebv_set_wait_limit(ebv_handle h, int64_t spins);

/* Measurement of the block-step kernel of the single-system factor.
 * ebv_profile_update_enable(h, m): create 2*m events up front (on the current
 * device); each later block-step launch of a factor made with h (batch = 1)
 * is then bracketed by an event pair on its stream, up to m launches; m = 0
 * turns this off and destroys the events.  ebv_profile_update_read
 * synchronizes on the recorded events and returns (and resets) the summed
 * elapsed milliseconds, the number of launches and their summed algorithmic
 * flops (the update flops of each launch: 2 * rows * cols * K over the tiles
 * it brings up to date).  Host pointers; -i for an invalid argument i. */
int ebv_profile_update_enable(ebv_handle h, int max_launches);
int ebv_profile_update_read(ebv_handle h, double *ms_total, int64_t *launches, double *flops_total);

/*
 * ebv_lu_factor -- Doolittle LU without pivoting, in place (paper Eq. 3, the
 * elimination step of Eq. 6-a/6-c, the work split of Eq. 7).
 *   A      (in/out) batch matrices n x n, system b at A + b*strideA elements;
 *          on exit the strictly lower part holds L (unit diagonal implied)
 *          and the upper part holds U.
 *   lda    >= max(1, n); strideA >= n*lda when batch > 1.
 *   info   device int32[batch] or NULL: 0, k > 0 for a zero pivot at step k,
 *          or (batch = 1) -status when a bounded wait gave up (the factor is
 *          then invalid).
 *   dtype  EBV_F64 (double*) or EBV_F32 (float*).
 *   ws     ebv_workspace_size(EBV_OP_FACTOR, ...) bytes when batch = 1: launch
 *          control words first (the status word at offset 0, two words of a
 *          solve that may follow, then two per 64-wide block step, the whole
 *          rounded up to 256 bytes), then the current diagonal tile's pack
 *          for the panel solves (64*64 elements); none when batch > 1 (ws may
 *          then be NULL).
 * Single systems (batch = 1) use a multi-workgroup blocked factorization;
 * batch > 1 factors one system per workgroup and needs
 * n * lda * sizeof(element) < 2^31 (EBV_ERR_UNSUPPORTED otherwise).
 */
int ebv_lu_factor(ebv_handle h, ebv_dtype dtype, int64_t n, void *A, int64_t lda, int64_t batch,
                  int64_t strideA, int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * ebv_lu_solve -- solve L Y = B by forward substitution, then U X = Y by
 * backward substitution (paper Eq. 1), with the factors from ebv_lu_factor.
 *   LU     (in) factors, lda as above.   B (in/out) right-hand sides -> X.
 *   strideLU, strideB: element strides between systems when batch > 1.
 *   info   device int32[batch] or NULL: set to 0, or (batch = 1) to -status
 *          when a bounded wait gave up (X is then invalid).
 *   ws     ebv_workspace_size(EBV_OP_SOLVE, dtype, n, nrhs, batch) bytes when
 *          batch = 1: three int32 control words padded to 256 bytes, then
 *          the exchange rows of the solved blocks (ceil(n/64)*64 x 16
 *          elements) and the partial sums of the helper workgroups
 *          (2 * ceil(n/64) blocks of 64 x 16 elements); none when batch > 1.
 */
int ebv_lu_solve(ebv_handle h, ebv_dtype dtype, int64_t n, int64_t nrhs, const void *LU, int64_t lda,
                 void *B, int64_t ldb, int64_t batch, int64_t strideLU, int64_t strideB, int32_t *info,
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
 *   info   device int32 or NULL, as for ebv_lu_factor (a bounded wait that
 *          gave up in the factor or the solve gives -status).
 *   ws     ebv_workspace_size(EBV_OP_FACTOR_SOLVE, dtype, n, nrhs, 1) bytes:
 *          the factor's layout (the backward substitution uses its first
 *          three control words), then the exchange rows of the solved blocks
 *          (ceil(n/64)*64 x 16 elements) and the partial sums of the
 *          helper workgroups (2 * ceil(n/64) blocks of 64 x 16 elements).
 */
int ebv_lu_factor_solve(ebv_handle h, ebv_dtype dtype, int64_t n, int64_t nrhs, void *A, int64_t lda, void *B,
                        int64_t ldb, int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * ebv_lu_inverse -- explicit inverse from the factors of ebv_lu_factor
 * (batch = 1): Ainv = A^{-1} = U^{-1} L^{-1}, the paper's product form of the
 * inverse (Eq. 4-c: the elementary upper factors times the elementary lower
 * factors), for reuse over many right-hand sides.  Computed as the solution
 * of A X = I by two blocked triangular solves (L^{-1}, then U^{-1} applied
 * to it in place), one launch per 64-wide block step, one workgroup per
 * 64 x 64 tile, after the diagonal tiles' inverses are formed in parallel.
 *   LU     (in) n x n factors, lda >= n.   Ainv (out) n x n, ldai >= n; must
 *          not overlap LU (argument 6 reported invalid otherwise).
 *   ws     ebv_workspace_size(EBV_OP_INVERSE, dtype, n, 0, 1) bytes: the
 *          inverses of the ceil(n/64) diagonal tiles (64 x 64 each).
 * The result agrees with the solution of A X = I to rounding.
 */
int ebv_lu_inverse(ebv_handle h, ebv_dtype dtype, int64_t n, const void *LU, int64_t lda, void *Ainv, int64_t ldai,
                   void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * ebv_pipeline_factor_solve -- factor and solve `count` dense n x n systems
 * that live in HOST memory, with the host<->device transfers (which the
 * paper reports separately, Table 3) overlapped with the computation: the
 * upload of system s+1 and the download of system s-1 run while system s is
 * factored and solved (ebv_lu_factor_solve; with nrhs = 0, ebv_lu_factor).
 * Two device slots alternate; three streams carry the work, ordered by
 * events (no host synchronization: the call only enqueues).
 *   A_host[s]  HOST pointer to system s, n x n row-major (lda = n); with
 *              nrhs = 0 it receives the factors.  B_host[s]: HOST n x nrhs
 *              right-hand sides (ldb = nrhs), overwritten by X.  Use pinned
 *              memory (hipHostMalloc) for the copies to overlap.
 *   dA[2], dB[2]  DEVICE slots of n*n and n*nrhs elements (dA[1], dB[1]
 *              unused when count = 1); their contents are clobbered.
 *   info       device int32[count] or NULL, as for ebv_lu_factor_solve.
 *   ws         ebv_workspace_size(EBV_OP_FACTOR_SOLVE, dtype, n, nrhs, 1).
 *   compute, copy_in, copy_out  the streams of the computation, of the
 *              uploads and of the downloads.  They overlap when they sit on
 *              distinct hardware queues; HIP assigns queues to streams
 *              round-robin (four per process by default), so streams
 *              created in between can put two of them on one queue.
 * The host buffers must stay valid until copy_out has drained.  The handle
 * keeps six events per device for the ordering (created on first use).
 */
int ebv_pipeline_factor_solve(ebv_handle h, ebv_dtype dtype, int64_t count, int64_t n, int64_t nrhs,
                              void *const *A_host, void *const *B_host, void *const *dA, void *const *dB,
                              int32_t *info, void *ws, size_t ws_bytes, hipStream_t compute, hipStream_t copy_in,
                              hipStream_t copy_out);

/*
 * Skyline (profile) systems -- the stand-in for the paper's sparse systems
 * (Table 1; the sparsity structure is not stated): row i's lower profile
 * starts at column f[i] <= i, column j's upper profile at row g[j] <= j.
 * Without pivoting the factors keep this envelope (Eq. 6-c updates a_ij only
 * from a_ik and a_kj inside it), so they overwrite it in place.  FP64.
 * Storage (classic skyline): the strictly lower part by rows, a_ij
 * (f[i] <= j < i) at AL[rp[i] + j - f[i]]; the upper part with the diagonal
 * by columns, a_ij (g[j] <= i <= j) at AU[cp[j] + i - g[j]].
 *   f_host, g_host  HOST int32[n] copies of the profile, from which the
 *          library plans the 64 x 64 tiles of the block envelope (the work
 *          is done on those tiles, packed in the workspace); f, g, rp, cp,
 *          AL, AU are DEVICE arrays.  A profile entry out of range is
 *          reported as argument 3 (factor) or 4 (solve) invalid.
 *   n      <= 16384 (EBV_ERR_UNSUPPORTED above).
 *   ws     ebv_skyline_workspace_size(n, f_host, g_host) bytes: the envelope
 *          tiles (64 * 64 doubles each), one more per 64-row block for the
 *          inverses of the diagonal tiles' factors (the solve forms them all
 *          in parallel and applies each as one matrix-core product), then
 *          the factor's control words (rounded to 256 bytes).  The factor is right-looking, one launch per 64-wide
 *          block step: the diagonal tile (published 16 columns at a time
 *          while it is factored), the envelope tiles of its block column
 *          and row (each step of their block substitution waits, bounded,
 *          for the strip it needs), and every
 *          trailing envelope tile that receives the previous step's rank-64
 *          term, one workgroup each.
 *   info   device int32 or NULL: zero pivot (1-based) or 0; for the factor
 *          -status when a bounded wait gave up (results then invalid).
 * ebv_lu_solve_skyline: forward then backward substitution (Eq. 1) on the
 * factors, B (n x nrhs, ldb >= nrhs) -> X.
 */
size_t ebv_skyline_workspace_size(int64_t n, const int32_t *f_host, const int32_t *g_host);
int ebv_lu_factor_skyline(ebv_handle h, int64_t n, const int32_t *f_host, const int32_t *g_host, const int32_t *f,
                          const int64_t *rp, double *AL, const int32_t *g, const int64_t *cp, double *AU,
                          int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream);
int ebv_lu_solve_skyline(ebv_handle h, int64_t n, int64_t nrhs, const int32_t *f_host, const int32_t *g_host,
                         const int32_t *f, const int64_t *rp, const double *AL, const int32_t *g, const int64_t *cp,
                         const double *AU, double *B, int64_t ldb, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * ebv_lu_factor_solve_noalloc -- for callers that cannot allocate device
 * memory (code under hipGraph capture, tight serving loops, harnesses that
 * forbid hipMalloc): ebv_lu_factor_solve with no workspace argument.  The
 * workspace is a static device array inside the library, one copy per
 * device, of ebv_noalloc_scratch_bytes() bytes (about 6.3 MB, held by every
 * device the library runs on until the process ends); the call allocates
 * nothing (no hipMalloc/hipFree, no allocating library routine).  A, B,
 * info, their layout and results are exactly those of ebv_lu_factor_solve
 * (same launches, same tuning of handle h).
 *   n      0 <= n <= ebv_noalloc_max_n() (16384); larger n returns
 *          EBV_ERR_TOO_LARGE before anything is enqueued.
 * Every call on one device uses that device's one array: the call's first
 * launch re-initialises what must start cleared, so each call sees nothing
 * of the previous one, but two calls whose work overlaps on the same device
 * (different streams, or host threads without ordering) race on the array
 * and give invalid results.  Serialize them, e.g. on one stream.
 */
int ebv_lu_factor_solve_noalloc(ebv_handle h, ebv_dtype dtype, int64_t n, int64_t nrhs, void *A, int64_t lda,
                                void *B, int64_t ldb, int32_t *info, hipStream_t stream);
/* Size in bytes of the static scratch array and the largest n it serves. */
size_t ebv_noalloc_scratch_bytes(void);
int64_t ebv_noalloc_max_n(void);

/*
 * ebv_lu_factor_band / ebv_lu_solve_band -- the same factorization and solves
 * restricted to a band matrix with kl sub- and ku super-diagonals (FP64),
 * the stand-in for the paper's sparse systems (Table 1).  Without pivoting
 * the factors keep the band, so they overwrite it in place.  Storage is
 * row-wise: a_ij at AB[i*ldab + (j - i + kl)], ldab >= kl+ku+1.  Slots that
 * fall outside the matrix are ignored.  This build supports
 * 0 <= kl, ku <= 64 (EBV_ERR_UNSUPPORTED otherwise).
 * The factor is one workgroup walking the block-tridiagonal 64 x 64 tile
 * structure; the solve first forms, in parallel, the inverses of the
 * diagonal tiles' factors and copies of the off-diagonal tiles (into ws),
 * then sweeps the 64-row blocks forward and backward, two matrix-core
 * products per block.
 *   info   device int32 or NULL: the factor's zero pivot (1-based) or 0; the
 *          solve sets it to 0.
 *   ws     ebv_workspace_size(EBV_OP_BAND, F64, n, 0, 1) bytes (0: NULL
 *          allowed) for the factor; ebv_workspace_size(EBV_OP_BAND_SOLVE,
 *          F64, n, nrhs, 1) = ceil(n / 64) * 128 KiB for the solve (per
 *          64-row block the inverses of the diagonal tile's factors and the
 *          two off-diagonal band tiles, overwritten).
 */
int ebv_lu_factor_band(ebv_handle h, int64_t n, int64_t kl, int64_t ku, double *AB, int64_t ldab,
                       int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream);
int ebv_lu_solve_band(ebv_handle h, int64_t n, int64_t kl, int64_t ku, int64_t nrhs, const double *AB,
                      int64_t ldab, double *B, int64_t ldb, int32_t *info, void *ws, size_t ws_bytes,
                      hipStream_t stream);

/*
 * ebv_lu_factor_batched -- factor and solve `count` independent systems of
 * uneven size in one persistent launch (Eq. 1 and Eq. 6 per system; the
 * paper's equal-work pairing applied to whole systems through `order`).
 * The launch is a fill kernel and one persistent kernel on `stream` (no
 * memset, no synchronization), so a call can be captured into a hipGraph
 * and replayed.
 *   n      device int32[count]: sizes (n_s >= 0).
 *   offA   device int64[count]: element offset of system s in A (lda = n_s).
 *   totA   elements of A (>= max_s offA[s] + n_s^2); sizes the workspace.
 *   offB   device int64[count]: element offset of system s in B (n_s x 1).
 *   totB   elements of B (>= max_s offB[s] + n_s).
 *   B      may be NULL when mixed == 0: factor only.
 *   order  device int32[count] or NULL: the order in which workgroups take
 *          systems (ebv_batched_order() computes it for a policy); NULL
 *          takes systems in index order.
 *   mixed  0: factor in `dtype` in place in A and solve in place in B.
 *          1: (dtype must be EBV_F64, B non-NULL) factor a float copy of each
 *          system in the workspace, keep A unchanged, and refine X (returned
 *          in B) in double until the forward-error bound holds:
 *          max_i |b - A x|_i <= tol * m * max_i |x_i|, with the system's
 *          dominance margin m = min_i (|a_ii| - sum_{j!=i} |a_ij|), which
 *          bounds |A^{-1}|_inf by 1/m (never met when m <= 0); at most
 *          max_iter corrections.  iters (device int32[count] or NULL)
 *          receives the correction count per system, -1 when not converged.
 *   info   device int32[count] or NULL: zero pivot per system; -3
 *          (-EBV_ERR_UNSUPPORTED) for a system with n_s^2 * 8 >= 2^31 bytes,
 *          which one workgroup does not address (left untouched).
 *   wg_per_cu  workgroups per compute unit in the persistent grid (0 = the
 *          handle's tuned value for this form).
 */
int ebv_lu_factor_batched(ebv_handle h, ebv_dtype dtype, int64_t count, const int32_t *n, const int64_t *offA,
                          void *A, int64_t totA, const int64_t *offB, void *B, int64_t totB,
                          const int32_t *order, int32_t *info, int mixed, int32_t max_iter,
                          double tol, int32_t *iters, int32_t wg_per_cu, void *ws, size_t ws_bytes,
                          hipStream_t stream);

/* Batch schedule on the host for an order policy (EBV_ORDER_*):
 * order_host[r] = index of the system taken r-th.  EBV_ORDER_EBV pairs the
 * costliest remaining system (by n^3) with the cheapest, so consecutive
 * pairs carry about equal work (the paper's first-with-last joining).
 *   n_host, order_host: HOST int32[count]. */
int ebv_batched_order(int policy, int64_t count, const int32_t *n_host, int32_t *order_host);

/*
 * ebv_lu_solve_adjoint -- reverse-mode derivative of X = A^{-1} B reusing the
 * factors: Bbar = A^{-T} Xbar (U^T Z = Xbar, then L^T Bbar = Z) and, when
 * Abar != NULL, Abar = -Bbar X^T.
 *   LU (in) factors from ebv_lu_factor; X (in) the solution, ldx >= nrhs;
 *   Bbar (in: Xbar, out: Bbar), ldb >= nrhs; Abar (out) n x n, ldabar >= n.
 *   Strides are element offsets between systems when batch > 1.
 *   info   as for ebv_lu_solve.
 */
int ebv_lu_solve_adjoint(ebv_handle h, ebv_dtype dtype, int64_t n, int64_t nrhs, const void *LU, int64_t lda,
                         const void *X, int64_t ldx, void *Bbar, int64_t ldb, void *Abar,
                         int64_t ldabar, int64_t batch, int64_t strideLU, int64_t strideX,
                         int64_t strideB, int64_t strideAbar, int32_t *info, void *ws, size_t ws_bytes,
                         hipStream_t stream);

/*
 * ebv_lu_solve_mixed -- mixed-precision solve of one dense system: factor a
 * float copy of A (kept in the workspace), solve in float, then refine in
 * double: R = B - A X, X += solve_float(R), until every column c meets the
 * forward-error bound max_i |r_ic| <= tol * m * max_i |x_ic| (m the
 * dominance margin, as for ebv_lu_factor_batched), at most max_iter
 * corrections.
 *   A, B (in, unchanged) double; X (out) double n x nrhs, ldx >= nrhs.
 *   iters  device int32[nrhs] or NULL: corrections used per column (-1 when
 *          not converged after max_iter).
 *   ferr   device double[nrhs] or NULL: the final bound
 *          max_i|r_ic| / (m max_i|x_ic|) per column (+inf when m = 0).
 *   info   device int32 or NULL: zero pivot of the float factor, or -status
 *          when a bounded wait gave up.
 * The refinement loop is a fixed sequence of launches whose kernels exit
 * early once the device-side test has passed, so the call never synchronizes.
 */
int ebv_lu_solve_mixed(ebv_handle h, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
                       int64_t ldb, double *X, int64_t ldx, int32_t max_iter, double tol,
                       int32_t *iters, double *ferr, int32_t *info, void *ws, size_t ws_bytes,
                       hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* EBV_H */
